"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Every case uses seeded synthetic inputs from workloads; the oracle sees the
same float32 inputs converted exactly to float64.  Tolerances (tests/parity.py):
values 1e-5, first derivatives 1e-4, second derivatives and residuals 1e-3,
gradients 1e-3 (relative, with an rms floor).
"""
import numpy as np
import pytest

import workloads as wl
from parity import (TOL_GRAD, TOL_LOSS, TOL_RESIDUAL, assert_close, channel_tolerances,
                    oracle_loss_grad)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_15883_amd as P
    P.lib()
    return P


def ctx_of(P, pb, **kw):
    return P.context_from_problem(pb, device="cuda", **kw)


def gpu_loss_grad(ctx):
    loss, g = ctx.step(1, update=False, want_grad=True)
    torch.cuda.synchronize()
    return loss.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)


def check_channels(P, ctx, orc, pb, x, sub=0, label=""):
    dim = pb.dim
    D = dim + 1
    xt = torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    ch = ctx.query(xt, sub=sub, what="channels").cpu().numpy().reshape(len(x), 2 * dim + 2, D)
    ref = orc.channels(dim, pb.width, pb.depth, pb.subs[sub].theta, x)
    for c, tol in enumerate(channel_tolerances(dim)):
        assert_close(ch[:, c, :], ref[:, c, :], tol, f"{label} channel {c}")
    r = ctx.query(xt, sub=sub, what="residual").cpu().numpy()
    rref = orc.residuals(dim, pb.nu, ref)
    assert_close(r, rref, TOL_RESIDUAL, f"{label} residuals")


# widths cover every tail of the hidden GEMMs' K loop (ceil(W/4) mod 4 = 0..3) and a loop
# with no full chunk of four K-steps (W = 5, 12)
TINY = [(2, 5, 2, 7, 5, 4, 2), (3, 5, 3, 19, 9, 6, 1), (2, 20, 1, 33, 0, 0, 0),
        (2, 16, 2, 16, 3, 0, 2), (3, 33, 2, 40, 100, 130, 3), (2, 50, 3, 1, 1, 1, 1),
        (2, 28, 3, 37, 5, 4, 2), (3, 12, 2, 23, 7, 3, 1)]


@pytest.mark.parametrize("dim,W,H,npde,nobs,ngh,nanc", TINY)
def test_tiny_loss_grad_channels(pkg, orc, dim, W, H, npde, nobs, ngh, nanc):
    pb = wl.tiny(dim=dim, width=W, depth=H, n_pde=npde, n_obs=nobs, n_gh=ngh, n_anc=nanc, seed=W + H)
    ctx = ctx_of(pkg, pb, graph=False)
    L, g = gpu_loss_grad(ctx)
    Lr, gr = oracle_loss_grad(orc, pb)
    assert_close(L[0], Lr, TOL_LOSS, "loss")
    assert_close(g[0], gr, TOL_GRAD, "grad")
    check_channels(pkg, ctx, orc, pb, pb.subs[0].pde_x, label="tiny")
    ctx.close()


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_config1_full_step(pkg, orc, seed):
    pb = wl.config1(seed)
    s = pb.subs[0]
    ctx = ctx_of(pkg, pb, graph=True)
    check_channels(pkg, ctx, orc, pb, s.pde_x, label="config1")
    L, g = gpu_loss_grad(ctx)
    Lr, gr = oracle_loss_grad(orc, pb)
    assert_close(L[0], Lr, TOL_LOSS, "loss")
    assert_close(g[0], gr, TOL_GRAD, "grad")
    # one Adam step (t = 1) from zero moments
    th0 = ctx.subs[0].theta.cpu().numpy().astype(np.float64)
    ctx.step(1, update=True)
    torch.cuda.synchronize()
    th1 = ctx.subs[0].theta.cpu().numpy().astype(np.float64)
    m1 = ctx.subs[0].adam_m.cpu().numpy().astype(np.float64)
    # (1) the Adam update applied to the GPU's own gradient
    t_own, m_own, _ = orc.adam(th0, np.zeros_like(th0), np.zeros_like(th0), g[0], 1, lr=pb.lr)
    assert_close(th1, t_own, 1e-6, "adam on own gradient")
    assert_close(m1, m_own, 1e-6, "adam first moment")
    # (2) against the oracle's gradient, excluding sign-ambiguous entries
    t_ref, _, _ = orc.adam(th0, np.zeros_like(th0), np.zeros_like(th0), gr, 1, lr=pb.lr)
    amb = np.abs(gr) <= TOL_GRAD * (np.abs(gr) + np.sqrt(np.mean(gr * gr)))
    assert amb.mean() < 0.05
    assert_close(th1[~amb], t_ref[~amb], 1e-6, "theta after Adam")
    ctx.close()


@pytest.mark.parametrize("n_pde", [3000, 2999])
def test_config2_reduced(pkg, orc, n_pde):
    pb = wl.config2(0, n_pde=n_pde)
    s = pb.subs[0]
    s.obs_x, s.obs_u = s.obs_x[:700], s.obs_u[:700]
    s.gh_x, s.gh_up, s.gh_kind = s.gh_x[:333], s.gh_up[:333], s.gh_kind[:333]
    ctx = ctx_of(pkg, pb, graph=True)
    L, g = gpu_loss_grad(ctx)
    Lr, gr = oracle_loss_grad(orc, pb)
    assert_close(L[0], Lr, TOL_LOSS, "loss")
    assert_close(g[0], gr, TOL_GRAD, "grad")
    check_channels(pkg, ctx, orc, pb, s.pde_x[:200], label="config2")
    ctx.close()


def test_config4_reduced(pkg, orc):
    pb = wl.config4(0, n_pde=500, n_obs=90, n_gh_face=40)
    ctx = ctx_of(pkg, pb, graph=True)
    L, g = gpu_loss_grad(ctx)
    Lr, gr = oracle_loss_grad(orc, pb)
    assert_close(L[0], Lr, TOL_LOSS, "loss")
    assert_close(g[0], gr, TOL_GRAD, "grad")
    check_channels(pkg, ctx, orc, pb, pb.subs[0].pde_x[:64], label="config4")
    ctx.close()


def test_config4_full_size_sampled_channels(pkg, orc):
    """Full 250k-point problem in the benchmark's launch configuration: the
    channel stacks of sampled points match the oracle point by point."""
    pb = wl.config4(0)
    ctx = ctx_of(pkg, pb, graph=True)
    loss, _ = ctx.step(1, update=False)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(loss.cpu().numpy()))
    rng = np.random.default_rng(0)
    idx = rng.choice(pb.subs[0].pde_x.shape[0], 48, replace=False)
    check_channels(pkg, ctx, orc, pb, pb.subs[0].pde_x[idx], label="config4 full")
    ctx.close()


def test_config3_grouped_equals_per_subdomain_and_oracle(pkg, orc):
    pb = wl.config3(0, pde_range=(300, 1300), n_obs=90, n_gh_face=37)
    ctx = ctx_of(pkg, pb, graph=True)
    L, g = gpu_loss_grad(ctx)
    loss2, g2 = ctx.step(1, update=False, want_grad=True, per_subdomain=True)
    torch.cuda.synchronize()
    L2, g2 = loss2.cpu().numpy(), g2.cpu().numpy()
    for s in range(len(pb.subs)):
        Lr, gr = oracle_loss_grad(orc, pb, sub=s)
        assert_close(L[s], Lr, TOL_LOSS, f"loss sub {s}")
        assert_close(g[s], gr, TOL_GRAD, f"grad sub {s}")
        assert_close(g2[s], gr, TOL_GRAD, f"per-sub grad sub {s}")
        assert_close(L2[s], Lr, TOL_LOSS, f"per-sub loss sub {s}")
    ctx.close()


def test_graph_replay_equals_eager_and_is_deterministic(pkg):
    pb = wl.config1(1)
    outs = []
    for graph in (True, False):
        ctx = ctx_of(pkg, pb, graph=graph)
        for t in range(1, 4):
            loss, _ = ctx.step(t)
            # eager work between replays
            torch.cuda.synchronize()
            _ = (ctx.subs[0].theta * 2).sum().item()
        outs.append((loss.cpu().numpy().copy(), ctx.subs[0].theta.cpu().numpy().copy()))
        ctx.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


def test_query_routing_and_alone_vs_mix(pkg, orc):
    boxes, thetas = wl.serving_nets(seed=3, width=20, depth=3)
    subs = []
    for s in range(len(thetas)):
        sub = wl._sub(2, boxes[s][0], boxes[s][1], thetas[s])
        subs.append(sub)
    pb = wl.Problem("serve", 2, 20, 3, 0.01, np.ones(6), 1e-3, subs)
    ctx = ctx_of(pkg, pb, graph=False)
    rng = np.random.default_rng(1)
    # 20,001 points: the whole batch is routed by the multi-block path, slices of
    # up to 8,192 points by the single-workgroup path; both must agree bitwise
    x = wl.query_points(rng, 20001)
    x[:3] = [[0, 0, 0], [8, 2, 4], [9, 1, 1]]     # corner, global upper corner, outside
    xt = torch.from_numpy(x).cuda()
    out = ctx.query(xt, sub=-1, what="uvpw").cpu().numpy()
    ref = orc.query2d(20, 3, thetas, boxes, x)
    assert np.all(np.isnan(out[2])) and np.all(np.isnan(ref[2]))
    ok = ~np.isnan(ref[:, 0])
    assert_close(out[ok, :3], ref[ok, :3], 1e-5, "query uvp")
    assert_close(out[ok, 3], ref[ok, 3], 1e-4, "query vorticity")
    # each point's result is the same alone, in a small mix and in the full batch
    for lo, hi in [(5, 6), (100, 117), (0, 3001), (3001, 3001 + 8192), (11193, 20001)]:
        part = ctx.query(xt[lo:hi].contiguous(), sub=-1, what="uvpw").cpu().numpy()
        np.testing.assert_array_equal(part, out[lo:hi])
    ctx.close()


def test_small_and_regular_query_tiles_agree(pkg, orc):
    """A request too small to fill the chip runs 16-point tiles; larger ones run
    the regular tiles.  Every column is computed the same way in both, so a
    point's result is bitwise the same whichever tile it lands in; both agree
    with the oracle."""
    W, H = 100, 2
    boxes, thetas = wl.serving_nets(seed=7, width=W, depth=H)
    subs = [wl._sub(2, boxes[s][0], boxes[s][1], thetas[s]) for s in range(len(thetas))]
    pb = wl.Problem("serve_tiles", 2, W, H, 0.01, np.ones(6), 1e-3, subs)
    ctx = ctx_of(pkg, pb, graph=False)
    try:
        x = torch.from_numpy(wl.query_points(np.random.default_rng(4), 50_000)).cuda()
        for what in ("uvpw", "value"):
            full = ctx.query(x, sub=-1, what=what).cpu().numpy()
            for lo in range(0, 50_000, 12_000):
                part = ctx.query(x[lo:lo + 2000].contiguous(), sub=-1, what=what).cpu().numpy()
                np.testing.assert_array_equal(part, full[lo:lo + 2000])
            if what == "uvpw":
                ref = orc.query2d(W, H, thetas, boxes, x[:3000].cpu().numpy())
                ok = ~np.isnan(ref[:, 0])
                assert_close(full[:3000][ok, :3], ref[ok, :3], 1e-5, "uvp")
        # single-subdomain queries take the same two paths
        y = x[:40_000].contiguous()
        one = ctx.query(y, sub=3, what="value").cpu().numpy()
        np.testing.assert_array_equal(ctx.query(y[:1000].contiguous(), sub=3, what="value").cpu().numpy(), one[:1000])
    finally:
        ctx.close()


def test_exchange_matches_oracle(pkg, orc):
    pb = wl.config3(0, pde_range=(100, 200), n_obs=10, n_gh_face=50)
    ctx = ctx_of(pkg, pb, graph=False)
    faces, targets = [], []
    for a, s in enumerate(pb.subs):
        for (b, kind, first, count) in s.faces:
            faces.append((a, b, first, count))
        targets.append(torch.zeros(s.gh_x.shape[0], 3, dtype=torch.float32, device="cuda"))
    ctx.exchange(faces, pb.x_anc, targets)
    torch.cuda.synchronize()
    for (a, b, first, count) in faces:
        x = pb.subs[a].gh_x[first:first + count]
        ref = orc.exchange(2, pb.width, pb.depth, pb.subs[b].theta, pb.subs[b].is_master,
                           pb.x_anc, x)
        got = targets[a][first:first + count].cpu().numpy()
        assert_close(got[:, :2], ref[:, :2], 1e-5, f"exchange u {a}<-{b}")
        assert_close(got[:, 2], ref[:, 2], 1e-4, f"exchange p {a}<-{b}")
    ctx.close()


@pytest.mark.parametrize("act", ["tanh", "sin"])
def test_exchange_3d_matches_oracle(pkg, orc, act):
    """Two 3D subdomains side by side in x, each with a ghost slab inside the
    other's box (a spatial face) plus a temporal ghost slab in the second;
    the first is a master (it holds x_anc), so its sends carry the anchor
    subtraction p - p(x_anc, t)."""
    W, H = 24, 3
    rng = np.random.default_rng(23)
    boxes = [([0, 0, 0, 0], [1, 1, 1, 1]), ([1, 0, 0, 0], [2, 1, 1, 1])]
    x_anc = [0.5, 0.5, 0.5]
    g0 = wl.uniform(rng, 53, [1, 0, 0, 0], [1.4, 1, 1, 1])                 # sub 0's ghosts, owned by sub 1
    g1 = np.concatenate([wl.uniform(rng, 61, [0.6, 0, 0, 0], [1, 1, 1, 1]),  # owned by sub 0
                         wl.uniform(rng, 37, [1, 0, 0, 0.8], [2, 1, 1, 1])])  # sub 1's own later slab
    subs = []
    for k, ((lo, hi), gx) in enumerate(zip(boxes, (g0, g1))):
        th = wl.xavier_theta(3, W, H, 40 + k)
        subs.append(wl._sub(3, np.array(lo, float), np.array(hi, float), th, is_master=(k == 0),
                            pde_x=wl.uniform(rng, 20, lo, hi), gh_x=gx,
                            gh_up=np.zeros((len(gx), 4), np.float32), gh_kind=np.zeros(len(gx), np.uint8)))
    pb = wl.Problem("exchange3d", 3, W, H, 0.01, np.ones(6), 1e-3, subs)
    pb.activation = act
    faces = [(0, 1, 0, 53), (1, 0, 0, 61)]
    orc.set_activation(act)
    ctx = ctx_of(pkg, pb, graph=False)
    try:
        targets = [torch.full((len(g0), 4), -7.0, device="cuda"), torch.full((len(g1), 4), -7.0, device="cuda")]
        ctx.exchange(faces, x_anc, targets)
        torch.cuda.synchronize()
        for (a, b, first, count) in faces:
            xg = pb.subs[a].gh_x[first:first + count]
            ref = orc.exchange(3, W, H, pb.subs[b].theta, pb.subs[b].is_master, x_anc, xg)
            got = targets[a][first:first + count].cpu().numpy()
            assert_close(got[:, :3], ref[:, :3], 1e-5, f"exchange u {a}<-{b}")
            assert_close(got[:, 3], ref[:, 3], 1e-4, f"exchange p {a}<-{b}")
        # ghost points outside every listed face keep their values
        assert np.all(targets[1][61:].cpu().numpy() == -7.0)
    finally:
        ctx.close()
        orc.set_activation("tanh")


def test_empty_sets_and_single_points(pkg, orc):
    pb = wl.tiny(dim=3, width=7, depth=2, n_pde=1, n_obs=0, n_gh=0, n_anc=0)
    ctx = ctx_of(pkg, pb, graph=False)
    L, g = gpu_loss_grad(ctx)
    Lr, gr = oracle_loss_grad(orc, pb)
    assert np.all(L[0, [0, 2, 3, 4, 5]] == 0)
    assert_close(g[0], gr, TOL_GRAD, "grad")
    ctx.close()
    pb = wl.tiny(dim=2, width=7, depth=2, n_pde=0, n_obs=1, n_gh=0, n_anc=0)
    ctx = ctx_of(pkg, pb, graph=True)
    L, g = gpu_loss_grad(ctx)
    Lr, gr = oracle_loss_grad(orc, pb)
    assert_close(g[0], gr, TOL_GRAD, "grad")
    assert_close(L[0], Lr, TOL_LOSS, "loss")
    ctx.close()


def test_many_subdomains_some_empty(pkg, orc):
    """300 small subdomains in one grouped launch, of very uneven size; every
    tenth has no points at all (its losses and gradient are exactly 0), others
    have only collocation, only value or single points.  Each equals the
    oracle, and the grouped launch equals plain per-subdomain launches."""
    rng = np.random.default_rng(17)
    dim, W, H = 2, 16, 2
    lo, hi = np.zeros(3), np.ones(3)
    subs = []
    for k in range(300):
        if k % 10 == 0:
            n = (0, 0, 0, 0)
        else:
            n = (int(rng.choice([0, 1, 5, 17, 40, 130])), int(rng.choice([0, 1, 3, 97])),
                 int(rng.choice([0, 2])), int(rng.choice([0, 1])))
        th = wl.xavier_theta(dim, W, H, k) + (0.05 * rng.standard_normal(wl.n_params(dim, W, H))).astype(np.float32)
        subs.append(wl._sub(dim, lo, hi, th.astype(np.float32), is_master=bool(k % 7 == 0),
                            pde_x=wl.uniform(rng, n[0], lo, hi), obs_x=wl.uniform(rng, n[1], lo, hi),
                            obs_u=rng.standard_normal((n[1], dim)).astype(np.float32),
                            gh_x=wl.uniform(rng, n[2], lo, hi),
                            gh_up=rng.standard_normal((n[2], dim + 1)).astype(np.float32),
                            gh_kind=(np.arange(n[2]) % 2).astype(np.uint8),
                            anc_x=wl.uniform(rng, n[3], lo, hi),
                            anc_p=rng.standard_normal(n[3]).astype(np.float32)))
    pb = wl.Problem("many", dim, W, H, 0.05, np.array([1.0, 1.0, 0.7, 0.6, 0.5, 0.9]), 1e-3, subs)
    ctx = ctx_of(pkg, pb, graph=True)
    try:
        L, g = gpu_loss_grad(ctx)
        loss2, g2 = ctx.step(1, update=False, want_grad=True, per_subdomain=True)
        torch.cuda.synchronize()
        L2, g2 = loss2.cpu().numpy().astype(np.float64), g2.cpu().numpy().astype(np.float64)
    finally:
        ctx.close()
    for k in range(300):
        if k % 10 == 0:
            assert np.all(L[k] == 0) and np.all(g[k] == 0) and np.all(g2[k] == 0), k
            continue
        Lr, gr = oracle_loss_grad(orc, pb, sub=k)
        assert_close(g[k], gr, TOL_GRAD, f"grad sub {k}")
        assert_close(g2[k], gr, TOL_GRAD, f"per-sub grad sub {k}")
        nz = Lr != 0
        assert np.all(L[k][~nz] == 0), k
        assert_close(L[k][nz], Lr[nz], TOL_LOSS, f"loss sub {k}")


def test_failure_paths(pkg):
    """A NaN among the collocation points makes the loss non-finite:
    PINN_CHECK_FINITE reports PINN_E_NONFINITE (without it the step returns and
    the loss holds the NaN).  A routed query above max_query_points is refused
    with PINN_E_BUDGET before anything is enqueued.  Destroying a context with
    steps in flight waits for them."""
    pb = wl.tiny(dim=2, width=20, depth=2, n_pde=50, n_obs=5, n_gh=4, n_anc=1)
    pb.subs[0].pde_x[17, 1] = np.nan
    ctx = ctx_of(pkg, pb, graph=True, max_query_points=100)
    try:
        loss, _ = ctx.step(1, update=False)
        torch.cuda.synchronize()
        assert np.isnan(loss.cpu().numpy()[0, 1]) and np.isnan(loss.cpu().numpy()[0, 6])
        with pytest.raises(pkg.PinnError) as e:
            ctx.step(1, update=False, check_finite=True)
        assert "NONFINITE" in str(e.value)
        x = torch.rand(101, 3, device="cuda")
        with pytest.raises(pkg.PinnError) as e:
            ctx.query(x, sub=-1, what="value")
        assert "BUDGET" in str(e.value)
        assert ctx.query(x[:100].contiguous(), sub=-1, what="value").shape == (100, 3)
    finally:
        ctx.close()
    pb = wl.tiny(dim=2, width=20, depth=2, n_pde=5000, n_obs=50, n_gh=40, n_anc=1)
    ctx = ctx_of(pkg, pb, graph=True)
    for t in range(1, 21):
        ctx.step(t)
    ctx.close()
    torch.cuda.synchronize()


def test_invalid_arguments_rejected(pkg):
    pb = wl.tiny(dim=2, width=5, depth=2)
    with pytest.raises(pkg.PinnError) as e:
        ctx_of(pkg, wl.tiny(dim=2, width=257, depth=1))
    assert "UNSUPPORTED" in str(e.value)
    ctx = ctx_of(pkg, wl.tiny(dim=2, width=5, depth=2), graph=False)
    with pytest.raises(pkg.PinnError):
        ctx.step(0, update=True)
    with pytest.raises(pkg.PinnError):
        ctx.query(torch.zeros(4, 3, device="cuda"), sub=5)
    ctx.close()
    ctx3 = ctx_of(pkg, wl.tiny(dim=3, width=5, depth=2), graph=False)
    with pytest.raises(pkg.PinnError) as e:      # (u, v, p, omega) is defined in 2D only
        ctx3.query(torch.zeros(4, 4, device="cuda"), sub=0, what="uvpw")
    assert "INVAL" in str(e.value)
    ctx3.close()
