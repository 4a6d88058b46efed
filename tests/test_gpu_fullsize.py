"""Full-size workloads in the benchmark's launch configuration (graph
replay, library launch shape): the fused step's per-subdomain losses and
whole gradients against the FP64 oracle on the entire problem (every
collocation, observation, ghost and anchor point)."""
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
