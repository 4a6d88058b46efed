"""Full-size workloads in the benchmark's launch configuration (graph
replay, library launch shape): the fused step's per-subdomain losses and
whole gradients against the FP64 oracle on the entire problem (every
collocation, observation, ghost and anchor point).  The paper's cylinder
networks at full size are beyond what the oracle finishes in a test; for them
a property that holds at any size is checked instead (their kernels are
parity-tested against the oracle at smaller sizes)."""
import dataclasses

import numpy as np
import pytest

import workloads as wl
from parity import TOL_GRAD, TOL_LOSS, assert_close, oracle_loss_grad

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_15883_amd as P
    P.lib()
    return P


def _check(pkg, orc, pb, label):
    ctx = pkg.context_from_problem(pb, device="cuda", graph=True)
    try:
        loss, g = ctx.step(1, update=False, want_grad=True)
        torch.cuda.synchronize()
        L = loss.cpu().numpy().astype(np.float64)
        G = g.cpu().numpy().astype(np.float64)
    finally:
        ctx.close()
    for s in range(len(pb.subs)):
        Lr, gr = oracle_loss_grad(orc, pb, sub=s)
        assert_close(L[s], Lr, TOL_LOSS, f"{label} loss sub {s}")
        assert_close(G[s], gr, TOL_GRAD, f"{label} grad sub {s}")


def test_config2_full_size(pkg, orc):
    """2D 8x100, 100,000 collocation + 10,000 observation + 2,000 ghost points."""
    _check(pkg, orc, wl.config2(0), "config2")


def test_config3_full_size_grouped(pkg, orc):
    """16 subdomains of 2D 6x64 in one grouped launch (ranges taken in turn)."""
    _check(pkg, orc, wl.config3(0), "config3")


def test_config4_full_size(pkg, orc):
    """3D 8x128, 250,000 collocation + 20,000 observation + 12,000 ghost points."""
    _check(pkg, orc, wl.config4(0), "config4")


def test_cylinder3d_recipe_full_size(pkg, orc):
    """The 3D-cylinder recipe: sine network, velocity-component weights."""
    pb = wl.cylinder3d_recipe(0)
    orc.set_activation("sin")
    orc.set_component_weights(pb.comp_w)
    try:
        _check(pkg, orc, pb, "cylinder3d")
    finally:
        orc.set_activation("tanh")
        orc.set_component_weights(None)


def _halves(pkg, pb, label):
    """Every loss term is a mean over its points, so when each point set is
    split into two equal halves the full problem's losses and gradient are the
    means of the halves' (up to float32 summation order).  Checks the work
    partition, the per-workgroup accumulation over many tiles and the slab
    reduction at full size."""
    s = pb.subs[0]
    npde, nobs = s.pde_x.shape[0], s.obs_x.shape[0]
    assert npde % 2 == 0 and nobs % 2 == 0 and s.gh_x.shape[0] == 0 and s.anc_x.shape[0] == 0

    def part(k):
        sp, so = slice(k * npde // 2, (k + 1) * npde // 2), slice(k * nobs // 2, (k + 1) * nobs // 2)
        sub = dataclasses.replace(s, pde_x=np.ascontiguousarray(s.pde_x[sp]),
                                  obs_x=np.ascontiguousarray(s.obs_x[so]), obs_u=np.ascontiguousarray(s.obs_u[so]))
        return dataclasses.replace(pb, subs=[sub])

    runs = []
    for p in (pb, part(0), part(1)):
        print(f"{label}: step on {p.subs[0].pde_x.shape[0]} collocation points", flush=True)
        ctx = pkg.context_from_problem(p, device="cuda", graph=True)
        try:
            loss, g = ctx.step(1, update=False, want_grad=True)
            torch.cuda.synchronize()
            runs.append((loss.cpu().numpy()[0].astype(np.float64), g.cpu().numpy()[0].astype(np.float64)))
        finally:
            ctx.close()
    (Lf, gf), (La, ga), (Lb, gb) = runs
    for k in (0, 1, 6):      # L_obs, L_PDE, total (no interface or anchor points)
        assert_close(Lf[k], (La[k] + Lb[k]) / 2, 1e-5, f"{label} loss term {k}")
    assert_close(gf, (ga + gb) / 2, 1e-4, f"{label} gradient")


def test_cylinder2d_paper_full_size_halves(pkg):
    """The paper's 2D cylinder network (sine 6x150), 500,000 + 10,000 points."""
    _halves(pkg, wl.cylinder2d_paper(0), "cylinder2d_paper")


def test_cylinder3d_paper_full_size_halves(pkg):
    """The paper's 3D cylinder network (sine 8x200, column-split plan),
    600,000 + 100,000 points."""
    _halves(pkg, wl.cylinder3d_paper(0), "cylinder3d_paper")

