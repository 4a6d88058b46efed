"""FP64 CPU oracle for the fused subdomain training step (arXiv 2602.15883).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the package smoke
check and by the CPU-baseline leg of the benchmark, never by the product path.
It shares no code with the HIP library.  The arithmetic lives in ``oracle.c``
(plain C, FP64, one point at a time); this module only marshals NumPy arrays.

Functions and the passages they follow:

* :func:`channels`  -- local-expert MLP (section 2.1, network equation) with
  first and second derivatives carried forward (needed by residuals r1-r4).
* :func:`residuals` -- incompressible Navier-Stokes residuals (section 2.1).
* :func:`loss_grad` -- observation, PDE, ghost and anchor losses and the final
  local objective (section 2.1, 2.2; final-loss equation) and its exact
  gradient.
* :func:`adam`      -- optimizer step of Algorithm 1 (Adam, bias-corrected).
* :func:`route`, :func:`query2d` -- stitching of local experts (section 3).
* :func:`exchange`  -- ghost targets with reference anchor normalisation
  (section 2.2, anchor-normalised pressure; Algorithm 1 exchange branch).
* :func:`evaluate`  -- relative L2 errors after stitching, master anchor
  pinning and per-snapshot pressure-mean removal (section 3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_d = ctypes.c_double
_l = ctypes.c_long
_i = ctypes.c_int
_p = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, IEEE double)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.or_nparams.restype = _l
        L.or_nparams.argtypes = [_i, _i, _i]
        L.or_threads.restype = _i
        L.or_threads.argtypes = [_i]
        L.or_channels.argtypes = [_i, _i, _i, _p, _p, _l, _p]
        L.or_values.argtypes = [_i, _i, _i, _p, _p, _l, _p]
        L.or_residuals.argtypes = [_i, _d, _p, _l, _p]
        L.or_loss_grad.argtypes = [_i, _i, _i, _d, _p, _i, _p,
                                   _p, _l, _p, _p, _l, _p, _p, _p, _l, _p, _p, _l,
                                   _p, _p]
        L.or_adam.argtypes = [_p, _p, _p, _p, _l, _l, _d, _d, _d, _d]
        L.or_route.argtypes = [_i, _i, _p, _p, _l, _p]
        L.or_query2d.argtypes = [_i, _i, _i, _p, _p, _p, _l, _p]
        L.or_exchange.argtypes = [_i, _i, _i, _p, _i, _p, _p, _l, _p]
        L.or_evaluate.argtypes = [_i, _i, _i, _i, _p, _p, _p, _p, _p, _l, _p, _p, _i, _p]
        L.or_set_activation.argtypes = [_i]
        L.or_set_component_weights.argtypes = [_p]
        L.or_clip_grad.restype = _d
        L.or_clip_grad.argtypes = [_p, _l, _d]
        L.or_step_lr.restype = _d
        L.or_step_lr.argtypes = [_d, _d, _l, _l]
        _lib = L
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return a.ctypes.data_as(_p) if a is not None and a.size else None


def n_params(dim: int, width: int, depth: int) -> int:
    return int(lib().or_nparams(dim, width, depth))


def threads(n: int = 0) -> int:
    """Set (n > 0) and return the OpenMP thread count the oracle uses."""
    return int(lib().or_threads(n))


def channels(dim, width, depth, theta, x):
    """All channels y[n, C, d+1] at points x[n, d+1]; C = 2d+2 in the order
    value, d/dx_1..d/dx_d, d/dt, d2/dx_1^2..d2/dx_d^2."""
    th = _f64(theta)
    x = _f64(x).reshape(-1, dim + 1)
    n = x.shape[0]
    y = np.zeros((n, 2 * dim + 2, dim + 1))
    lib().or_channels(dim, width, depth, _ptr(th), _ptr(x), n, _ptr(y))
    return y


def values(dim, width, depth, theta, x):
    """Network outputs (u_1..u_d, p) at points x, value channel only."""
    th = _f64(theta)
    x = _f64(x).reshape(-1, dim + 1)
    n = x.shape[0]
    y = np.zeros((n, dim + 1))
    lib().or_values(dim, width, depth, _ptr(th), _ptr(x), n, _ptr(y))
    return y


def residuals(dim, nu, ych):
    """Navier-Stokes residuals r[n, d+1] from a channel stack ych[n, C, d+1]."""
    y = _f64(ych)
    n = y.shape[0]
    r = np.zeros((n, dim + 1))
    lib().or_residuals(dim, float(nu), _ptr(y), n, _ptr(r))
    return r


def loss_grad(dim, width, depth, nu, lam, theta, *, is_master=False,
              pde_x=None, obs_x=None, obs_u=None, gh_x=None, gh_up=None,
              gh_kind=None, anc_x=None, anc_p=None, want_grad=True):
    """Losses [L_obs, L_PDE, L_gh_u, L_gh_p^space, L_gh_p^time, L_anc, L] and
    the gradient dL/dtheta of one subdomain.  lam = (obs, pde, gh_u, gh_p^space,
    gh_p^time, anc)."""
    D = dim + 1
    th = _f64(theta)
    lam = _f64(lam)
    assert lam.size == 6

    def pts(a, cols):
        if a is None:
            return np.zeros((0, cols))
        return _f64(a).reshape(-1, cols)

    px, ox, ou = pts(pde_x, D), pts(obs_x, D), pts(obs_u, dim)
    gx, gu, ax = pts(gh_x, D), pts(gh_up, D), pts(anc_x, D)
    ap = _f64(anc_p if anc_p is not None else np.zeros(0)).reshape(-1)
    gk = np.ascontiguousarray(np.asarray(gh_kind if gh_kind is not None
                                         else np.zeros(gx.shape[0]), dtype=np.uint8))
    assert ox.shape[0] == ou.shape[0] and gx.shape[0] == gu.shape[0] == gk.shape[0]
    assert ax.shape[0] == ap.shape[0]
    P = n_params(dim, width, depth)
    assert th.size == P
    loss = np.zeros(7)
    grad = np.zeros(P) if want_grad else None
    lib().or_loss_grad(dim, width, depth, float(nu), _ptr(lam), int(bool(is_master)),
                       _ptr(th), _ptr(px), px.shape[0], _ptr(ox), _ptr(ou), ox.shape[0],
                       _ptr(gx), _ptr(gu), _ptr(gk), gx.shape[0],
                       _ptr(ax), _ptr(ap), ax.shape[0], _ptr(loss), _ptr(grad))
    return loss, grad


def adam(theta, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam step; returns new (theta, m, v) as float64."""
    th, mm, vv, gg = (_f64(a).copy() for a in (theta, m, v, g))
    lib().or_adam(_ptr(th), _ptr(mm), _ptr(vv), _ptr(gg), th.size, int(t),
                  float(lr), float(beta1), float(beta2), float(eps))
    return th, mm, vv


def route(dim, boxes, x):
    """Subdomain index of each point (half-open boxes, closed global upper
    face); -1 if none.  boxes[s, 2, d+1] = (lo, hi)."""
    b = _f64(boxes)
    n_sub = b.shape[0]
    x = _f64(x).reshape(-1, dim + 1)
    sub = np.zeros(x.shape[0], dtype=np.int32)
    lib().or_route(dim, n_sub, _ptr(b), _ptr(x), x.shape[0], sub.ctypes.data_as(_p))
    return sub


def query2d(width, depth, thetas, boxes, x):
    """(u, v, p, v_x - u_y) at 2D points x[n, 3], each evaluated by the
    subdomain network it routes to."""
    ths = [_f64(t) for t in thetas]
    arr = (_p * len(ths))(*[t.ctypes.data_as(_p) for t in ths])
    b = _f64(boxes)
    x = _f64(x).reshape(-1, 3)
    out = np.zeros((x.shape[0], 4))
    lib().or_query2d(width, depth, len(ths), arr, _ptr(b), _ptr(x), x.shape[0], _ptr(out))
    return out


def exchange(dim, width, depth, theta_nb, nb_is_master, x_anc, x):
    """Neighbour targets (u_nbr, p_nbr) at ghost points x, with the anchor
    subtraction applied when the sending neighbour is a master."""
    th = _f64(theta_nb)
    xa = _f64(x_anc).reshape(-1)
    x = _f64(x).reshape(-1, dim + 1)
    out = np.zeros((x.shape[0], dim + 1))
    lib().or_exchange(dim, width, depth, _ptr(th), int(bool(nb_is_master)), _ptr(xa),
                      _ptr(x), x.shape[0], _ptr(out))
    return out


ACTIVATIONS = {"tanh": 0, "sin": 1}


def set_activation(name: str = "tanh"):
    """Activation of every network the oracle evaluates from now on."""
    lib().or_set_activation(ACTIVATIONS[name])


def set_component_weights(w=None):
    """Weights of the velocity components in L_obs and L_gh_u (None: ones)."""
    if w is None:
        lib().or_set_component_weights(None)
    else:
        a = _f64(list(w) + [1.0] * (3 - len(w)))
        lib().or_set_component_weights(_ptr(a))


def clip_grad(g, c):
    """Global-norm clipping; returns (clipped copy, norm before clipping)."""
    gg = _f64(g).copy()
    nrm = lib().or_clip_grad(_ptr(gg), gg.size, float(c))
    return gg, float(nrm)


def step_lr(lr, factor, interval, t):
    return float(lib().or_step_lr(float(lr), float(factor), int(interval), int(t)))


def evaluate(dim, width, depth, thetas, is_master, boxes, x_anc, x, ref, snap_off):
    """Relative L2 errors after stitching, master anchor pinning and
    per-snapshot pressure mean removal: [u_1..u_d, velocity, p]."""
    ths = [_f64(t) for t in thetas]
    arr = (_p * len(ths))(*[t.ctypes.data_as(_p) for t in ths])
    mst = np.ascontiguousarray(np.asarray(is_master, dtype=np.int32))
    b = _f64(boxes)
    xa = _f64(x_anc).reshape(-1)
    x = _f64(x).reshape(-1, dim + 1)
    r = _f64(ref).reshape(-1, dim + 1)
    so = np.ascontiguousarray(np.asarray(snap_off, dtype=np.int64))
    err = np.zeros(dim + 2)
    lib().or_evaluate(dim, width, depth, len(ths), arr, mst.ctypes.data_as(_p), _ptr(b), _ptr(xa),
                      _ptr(x), x.shape[0], _ptr(r), so.ctypes.data_as(_p), so.size - 1, _ptr(err))
    return err
