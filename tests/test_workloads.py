"""The synthetic input recipes of the paper's cylinder problems (section
3.2-3.3, appendix B) hold the stated sizes, geometry and training settings."""
import numpy as np
import pytest

import workloads as wl


@pytest.mark.parametrize("make,dim,W,H,n_pde,n_snap,per_snap,lam,nu",
                         [(wl.cylinder2d_paper, 2, 150, 6, 500_000, 50, 200, (10.0, 5.0), 1 / 100),
                          (wl.cylinder3d_paper, 3, 200, 8, 600_000, 80, 1250, (10.0, 10.0), 1 / 300)])
def test_cylinder_recipes(make, dim, W, H, n_pde, n_snap, per_snap, lam, nu):
    pb = make(0)
    assert (pb.dim, pb.width, pb.depth, pb.activation) == (dim, W, H, "sin")
    assert pb.nu == pytest.approx(nu) and tuple(pb.lam[:2]) == lam
    s = pb.subs[0]
    D = dim + 1
    assert s.pde_x.shape == (n_pde, D) and s.pde_x.dtype == np.float32
    assert s.obs_x.shape == (n_snap * per_snap, D) and s.obs_u.shape == (n_snap * per_snap, dim)
    assert s.gh_x.shape[0] == 0 and s.anc_x.shape[0] == 0          # one process: no interfaces
    for x in (s.pde_x, s.obs_x):
        r2 = x[:, 0].astype(np.float64) ** 2 + x[:, 1].astype(np.float64) ** 2
        assert r2.min() >= 0.25                                     # outside the cylinder r < 0.5
        assert np.all(x >= s.lo) and np.all(x <= s.hi)
    # observations: per_snap locations at each snapshot t_k = 0.15 k
    t, counts = np.unique(s.obs_x[:, -1], return_counts=True)
    np.testing.assert_allclose(t, 0.15 * np.arange(n_snap), rtol=0, atol=1e-5)
    assert np.all(counts == per_snap)
    assert np.all(np.isfinite(s.obs_u))
    # the same seed gives the same inputs
    pb2 = make(0)
    np.testing.assert_array_equal(pb2.subs[0].pde_x, s.pde_x)
    np.testing.assert_array_equal(pb2.subs[0].theta, s.theta)


def test_cylinder3d_training_settings():
    pb = wl.cylinder3d_paper(0)
    np.testing.assert_array_equal(pb.comp_w, [1.0, 5.0, 100.0])
    assert pb.clip_norm == 1.0 and (pb.lr_factor, pb.lr_interval) == (0.3, 5000)
    pb = wl.cylinder2d_paper(0)
    assert pb.comp_w is None and pb.clip_norm == 0.0 and (pb.lr_factor, pb.lr_interval) == (0.2, 2000)
