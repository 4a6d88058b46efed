"""Training-loop pieces on the GPU: autograd.Function, finite-difference check
of the GPU adjoint, exchange + step (Algorithm 1 loop), autotuner."""
import numpy as np
import pytest

import workloads as wl
from parity import TOL_GRAD, TOL_LOSS, assert_close, oracle_loss_grad

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_15883_amd as P
    P.lib()
    return P


def test_autograd_function_matches_step_and_torch_adam(pkg):
    from paper_2602_15883_amd.autograd import pinn_loss
    pb = wl.config3(0, pde_range=(200, 600), n_obs=50, n_gh_face=20, K=2, M=2)
    ctx = pkg.context_from_problem(pb, device="cuda", graph=True)
    _, g_ref = ctx.step(1, update=False, want_grad=True)
    g_ref = g_ref.clone()
    thetas = [s.theta.requires_grad_() for s in ctx.subs]
    loss = pinn_loss(ctx)
    w = torch.arange(1, len(thetas) + 1, dtype=torch.float32, device="cuda")
    (loss * w).sum().backward()
    for s, th in enumerate(thetas):
        np.testing.assert_array_equal(th.grad.cpu().numpy(), (w[s] * g_ref[s]).cpu().numpy())
    # torch's Adam on these gradients equals the fused Adam on the same gradient
    before = [th.detach().clone() for th in thetas]
    for th in thetas:
        th.grad = None
    loss = pinn_loss(ctx)
    loss.sum().backward()
    opt = torch.optim.Adam(thetas, lr=pb.lr, betas=(0.9, 0.999), eps=1e-8)
    opt.step()
    torch_after = [th.detach().clone() for th in thetas]
    with torch.no_grad():
        for th, b in zip(thetas, before):
            th.copy_(b)
    ctx.step(1, update=True)
    for th, ta in zip(thetas, torch_after):
        assert_close(th.detach().cpu().numpy(), ta.cpu().numpy(), 1e-6, "fused vs torch Adam")
    ctx.close()


def test_gpu_adjoint_matches_finite_differences(pkg):
    """FP32 central differences of the GPU loss itself (3D 4->8x128->4,
    4,096 collocation points of the 3D workload); loose tolerance for FP32."""
    pb = wl.config4(0, n_pde=4096, n_obs=400, n_gh_face=100)
    ctx = pkg.context_from_problem(pb, device="cuda", graph=False)
    _, g = ctx.step(1, update=False, want_grad=True)
    g = g[0].cpu().numpy().astype(np.float64)
    th = ctx.subs[0].theta
    idx = np.argsort(-np.abs(g))[:12]
    idx = np.concatenate([idx, np.random.default_rng(0).choice(g.size, 12, replace=False)])
    h = 2e-3
    for i in idx:
        v0 = th[i].item()
        th[i] = v0 + h
        Lp = ctx.step(1, update=False)[0][0, 6].item()
        th[i] = v0 - h
        Lm = ctx.step(1, update=False)[0][0, 6].item()
        th[i] = v0
        fd = (Lp - Lm) / (2 * h)
        scale = np.abs(g).max()
        assert abs(fd - g[i]) <= 2e-2 * abs(g[i]) + 2e-3 * scale, (i, fd, g[i])
    ctx.close()


def test_exchange_then_step_matches_oracle(pkg, orc):
    from paper_2602_15883_amd.trainer import DDTrainer, faces_of
    pb = wl.config3(1, pde_range=(150, 400), n_obs=40, n_gh_face=30, K=2, M=2)
    ctx = pkg.context_from_problem(pb, device="cuda", graph=True)
    tr = DDTrainer(ctx, faces_of(pb), pb.x_anc, i_comm=1)
    tr.exchange()
    loss, g = ctx.step(1, update=False, want_grad=True)
    torch.cuda.synchronize()
    L, G = loss.cpu().numpy(), g.cpu().numpy()
    for a, s in enumerate(pb.subs):
        tg = np.zeros_like(s.gh_up, dtype=np.float64)
        for (b, _k, first, count) in s.faces:
            tg[first:first + count] = orc.exchange(2, pb.width, pb.depth, pb.subs[b].theta,
                                                   pb.subs[b].is_master, pb.x_anc,
                                                   s.gh_x[first:first + count])
        s.gh_up = tg.astype(np.float32)
        Lr, gr = oracle_loss_grad(orc, pb, sub=a)
        assert_close(L[a], Lr, TOL_LOSS, f"loss {a}")
        assert_close(G[a], gr, TOL_GRAD, f"grad {a}")
    ctx.close()


def test_training_loop_reduces_loss(pkg):
    from paper_2602_15883_amd.trainer import DDTrainer, faces_of
    pb = wl.config3(2, pde_range=(500, 900), n_obs=200, n_gh_face=50, K=2, M=2, width=32, depth=3)
    ctx = pkg.context_from_problem(pb, device="cuda", graph=True)
    tr = DDTrainer(ctx, faces_of(pb), pb.x_anc, i_comm=2)
    first = tr.step().cpu().numpy()[:, 6].copy()
    for _ in range(150):
        last = tr.step()
    last = last.cpu().numpy()[:, 6]
    assert np.all(np.isfinite(last))
    assert last.sum() < 0.8 * first.sum()
    ctx.close()


def test_autotuner_picks_a_working_candidate(pkg, tmp_path, monkeypatch):
    from paper_2602_15883_amd import tune
    from paper_2602_15883_amd.context import Context, subdomain_to_device
    monkeypatch.setenv("DDPINN_TUNE_CACHE", str(tmp_path / "tune.json"))
    pb = wl.config3(0, pde_range=(2000, 4000), n_obs=100, n_gh_face=50, K=2, M=2)
    subs = [subdomain_to_device(s, "cuda") for s in pb.subs]

    def make(**cand):
        return Context(pb.dim, pb.width, pb.depth, subs, pb.nu, pb.lam, graph=False, **cand)
    best = tune.autotune(make, pb.dim, pb.width, pb.depth, len(subs), pb.n_pde, steps=2)
    assert best["tile_points"] in (16, 32)
    again = tune.autotune(make, pb.dim, pb.width, pb.depth, len(subs), pb.n_pde)
    assert again == best
    # the tuned shape gives the same gradient as the default shape (to FP32 rounding)
    c1 = make(**best)
    c2 = make()
    g1 = c1.step(1, update=False, want_grad=True)[1].cpu().numpy()
    g2 = c2.step(1, update=False, want_grad=True)[1].cpu().numpy()
    assert_close(g1, g2.astype(np.float64), 1e-5, "tuned vs default")
    c1.close()
    c2.close()
