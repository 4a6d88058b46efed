"""Comparison helpers for GPU-vs-oracle parity.

Tolerance reading: a GPU array a matches the FP64 oracle array b at relative
tolerance tol when, elementwise, |a - b| <= tol * (|b| + rms(b)), and
normwise ||a - b||_2 <= tol * ||b||_2.  The rms floor keeps entries near zero
from failing on rounding noise.
"""
import numpy as np

TOL_VALUE = 1e-5
TOL_FIRST = 1e-4
TOL_SECOND = 1e-3
TOL_RESIDUAL = 1e-3
TOL_GRAD = 1e-3
TOL_LOSS = 1e-3


def rel_report(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    if b.size == 0:
        return 0.0, 0.0
    rms = np.sqrt(np.mean(b * b))
    ew = np.max(np.abs(a - b) / (np.abs(b) + rms + 1e-300))
    nb = np.linalg.norm(b)
    nw = np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)
    return float(ew), float(nw)


def assert_close(a, b, tol, name=""):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    assert a.shape == b.shape, f"{name}: shape {a.shape} vs {b.shape}"
    assert np.all(np.isfinite(a)), f"{name}: non-finite values"
    ew, nw = rel_report(a, b)
    assert ew <= tol and nw <= tol, f"{name}: elementwise {ew:.3e}, normwise {nw:.3e} > {tol:.1e}"
    return ew, nw


def channel_tolerances(dim):
    """Per-channel tolerance: value, first derivatives (x_j and t), second."""
    return [TOL_VALUE] + [TOL_FIRST] * (dim + 1) + [TOL_SECOND] * dim


def oracle_loss_grad(orc, pb, sub=0, theta=None, want_grad=True):
    s = pb.subs[sub]
    th = s.theta if theta is None else theta
    return orc.loss_grad(pb.dim, pb.width, pb.depth, pb.nu, pb.lam, th, is_master=s.is_master,
                         pde_x=s.pde_x, obs_x=s.obs_x, obs_u=s.obs_u, gh_x=s.gh_x, gh_up=s.gh_up,
                         gh_kind=s.gh_kind, anc_x=s.anc_x, anc_p=s.anc_p, want_grad=want_grad)
