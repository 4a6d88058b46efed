"""Networks wider than 128 neurons: each wave of the step, query and exchange
kernels then owns two 16-neuron row blocks (w and w + 8).  Cases span a wave
mix of one and two blocks (W = 150: waves 0-1 hold two; W = 144 in 3D: wave 0),
all waves with two (W = 192, 256), three and seven extra row blocks (W = 176,
240), padding (W = 129 -> 144), both
activations, the paper's cylinder networks (2D 6 x 150 and 3D 8 x 200, sine;
sections 3.2-3.3, appendix B), the column-split LDS plan, several tiles per
workgroup, the largest shape, and the limits."""
import numpy as np
import pytest

import workloads as wl
from parity import TOL_GRAD, TOL_LOSS, TOL_RESIDUAL, assert_close, channel_tolerances, oracle_loss_grad

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_15883_amd as P
    P.lib()
    return P


@pytest.fixture
def act_oracle(orc):
    yield orc
    orc.set_activation("tanh")


# dim, width, depth, activation, collocation points.  Where the two-block
# LDS plan does not fit, the column-split plan runs (one forward activation
# stack, backward by column halves): 2D above 192 (192 from depth 7), 3D
# above 144 (144 from depth 6).
WIDE = [(2, 150, 6, "sin", 87),      # the paper's 2D-cylinder network shape
        (2, 150, 2, "tanh", 8201),   # > 1 tile per workgroup: slab read-modify-write
        (2, 192, 2, "tanh", 87),     # every wave holds two row blocks
        (3, 144, 2, "tanh", 300),
        (3, 129, 3, "sin", 50),      # padded to 144
        (3, 200, 8, "sin", 87),      # the paper's 3D-cylinder network shape (split)
        (3, 200, 2, "tanh", 8201),   # split, > 1 tile per workgroup
        (2, 192, 8, "tanh", 50),     # split
        (2, 256, 2, "sin", 300),     # split, every wave two blocks
        (2, 176, 3, "tanh", 2500),   # three extra row blocks, > 1 tile per workgroup
        (3, 240, 2, "sin", 60),      # split, seven extra row blocks
        (3, 256, 16, "tanh", 40)]    # the largest shape: split plan at the LDS limit


@pytest.mark.parametrize("dim,W,H,act,npde", WIDE)
def test_wide_loss_grad_channels(pkg, act_oracle, dim, W, H, act, npde):
    orc = act_oracle
    orc.set_activation(act)
    pb = wl.tiny(dim=dim, width=W, depth=H, n_pde=npde, n_obs=150, n_gh=30, n_anc=2, seed=W + H)
    pb.activation = act
    print(f"wide step dim={dim} W={W} H={H} act={act} n_pde={npde}", flush=True)
    ctx = pkg.context_from_problem(pb, device="cuda", graph=True)
    try:
        assert ctx.launch_info()["threads"] == 512
        loss, g = ctx.step(1, update=False, want_grad=True)
        torch.cuda.synchronize()
        Lr, gr = oracle_loss_grad(orc, pb)
        assert_close(loss.cpu().numpy()[0].astype(np.float64), Lr, TOL_LOSS, "loss")
        assert_close(g.cpu().numpy()[0].astype(np.float64), gr, TOL_GRAD, "grad")
        x = pb.subs[0].pde_x[:200]
        xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        ch = ctx.query(xt, sub=0, what="channels").cpu().numpy().reshape(len(x), 2 * dim + 2, dim + 1)
        ref = orc.channels(dim, W, H, pb.subs[0].theta, x)
        for c, tol in enumerate(channel_tolerances(dim)):
            assert_close(ch[:, c], ref[:, c], tol, f"channel {c}")
        r = ctx.query(xt, sub=0, what="residual").cpu().numpy()
        assert_close(r, orc.residuals(dim, pb.nu, ref), TOL_RESIDUAL, "residuals")
        v = ctx.query(xt, sub=0, what="value").cpu().numpy()
        assert_close(v, ref[:, 0], 1e-5, "values")
    finally:
        ctx.close()


@pytest.mark.parametrize("W,H", [(150, 2), (200, 2)])
def test_wide_grouped_equals_per_subdomain_and_oracle(pkg, orc, W, H):
    """16 wide subdomains of uneven size (masters, ghost faces of both kinds,
    the anchor term) in one grouped launch and in plain per-subdomain
    launches; W = 200 in 2D takes the column-split plan."""
    pb = wl.config3(1, width=W, depth=H, pde_range=(40, 700), n_obs=30, n_gh_face=20)
    print(f"wide grouped W={W} H={H}", flush=True)
    ctx = pkg.context_from_problem(pb, device="cuda", graph=True)
    try:
        loss, g = ctx.step(1, update=False, want_grad=True)
        loss2, g2 = ctx.step(1, update=False, want_grad=True, per_subdomain=True)
        torch.cuda.synchronize()
        L, G, L2, G2 = (t.cpu().numpy().astype(np.float64) for t in (loss, g, loss2, g2))
    finally:
        ctx.close()
    for s in range(len(pb.subs)):
        Lr, gr = oracle_loss_grad(orc, pb, sub=s)
        assert_close(L[s], Lr, TOL_LOSS, f"loss sub {s}")
        assert_close(G[s], gr, TOL_GRAD, f"grad sub {s}")
        assert_close(L2[s], Lr, TOL_LOSS, f"per-sub loss sub {s}")
        assert_close(G2[s], gr, TOL_GRAD, f"per-sub grad sub {s}")


def test_wide_routed_query_and_exchange(pkg, orc):
    W, H = 150, 2
    boxes, thetas = wl.serving_nets(seed=5, width=W, depth=H)
    subs = [wl._sub(2, boxes[s][0], boxes[s][1], thetas[s]) for s in range(len(thetas))]
    pb = wl.Problem("serve_wide", 2, W, H, 0.01, np.ones(6), 1e-3, subs)
    print("wide routed query", flush=True)
    ctx = pkg.context_from_problem(pb, device="cuda", graph=False)
    try:
        x = wl.query_points(np.random.default_rng(2), 2500)
        out = ctx.query(torch.from_numpy(x).cuda(), sub=-1, what="uvpw").cpu().numpy()
        ref = orc.query2d(W, H, thetas, boxes, x)
        ok = ~np.isnan(ref[:, 0])
        assert_close(out[ok, :3], ref[ok, :3], 1e-5, "query uvp")
        assert_close(out[ok, 3], ref[ok, 3], 1e-4, "query vorticity")
    finally:
        ctx.close()

    pb = wl.config3(0, width=W, depth=H, pde_range=(100, 200), n_obs=10, n_gh_face=50)
    print("wide exchange", flush=True)
    ctx = pkg.context_from_problem(pb, device="cuda", graph=False)
    try:
        faces, targets = [], []
        for a, s in enumerate(pb.subs):
            for (b, kind, first, count) in s.faces:
                faces.append((a, b, first, count))
            targets.append(torch.zeros(s.gh_x.shape[0], 3, dtype=torch.float32, device="cuda"))
        ctx.exchange(faces, pb.x_anc, targets)
        torch.cuda.synchronize()
        for (a, b, first, count) in faces:
            xg = pb.subs[a].gh_x[first:first + count]
            ref = orc.exchange(2, W, H, pb.subs[b].theta, pb.subs[b].is_master, pb.x_anc, xg)
            got = targets[a][first:first + count].cpu().numpy()
            assert_close(got[:, :2], ref[:, :2], 1e-5, f"exchange u {a}<-{b}")
            assert_close(got[:, 2], ref[:, 2], 1e-4, f"exchange p {a}<-{b}")
    finally:
        ctx.close()


def test_wide_limits(pkg):
    """Widths above 256 and depths above 16 are refused with
    PINN_E_UNSUPPORTED, and so are 32-point tiles above 8 row blocks."""
    for dim, W, H, kw in [(3, 257, 2, {}), (2, 64, 17, {}), (2, 150, 2, {"tile_points": 32})]:
        with pytest.raises(pkg.PinnError) as e:
            pkg.context_from_problem(wl.tiny(dim=dim, width=W, depth=H), device="cuda", **kw)
        assert "UNSUPPORTED" in str(e.value), (dim, W, H, str(e.value))


def test_wide_training_loop_reduces_loss(pkg):
    """The domain-decomposed loop (steps, exchange every second step, Adam)
    on four 2D subdomains of width 150 (two row blocks per wave)."""
    from paper_2602_15883_amd.trainer import DDTrainer, faces_of
    pb = wl.config3(2, pde_range=(500, 900), n_obs=200, n_gh_face=50, K=2, M=2, width=150, depth=2)
    print("wide training loop", flush=True)
    ctx = pkg.context_from_problem(pb, device="cuda", graph=True)
    try:
        tr = DDTrainer(ctx, faces_of(pb), pb.x_anc, i_comm=2)
        first = tr.step().cpu().numpy()[:, 6].copy()
        for _ in range(150):
            last = tr.step()
        last = last.cpu().numpy()[:, 6]
    finally:
        ctx.close()
    assert np.all(np.isfinite(last))
    assert last.sum() < 0.8 * first.sum()

