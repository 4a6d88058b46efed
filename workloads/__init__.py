"""Seeded synthetic inputs for the fused subdomain training step.

This module is shared by the tests (oracle side and GPU side) and the
benchmark.  It holds no arithmetic of the method itself: only parameter
initialisation, point sampling, analytic flow fields used as data, and the
domain-decomposition geometry (boxes, ghost slabs, anchor, master flags).

The paper's own workloads are CFD datasets that are not available; the
shapes follow its hyperparameter table (appendix B: widths, depths, point
budgets, ghost points per interface, interface thickness, loss weights) and
the data values come from analytic fields:

* 2D Taylor-Green vortex (exact Navier-Stokes solution),
* 3D Ethier-Steinman Beltrami flow (exact Navier-Stokes solution),
* a divergence-free field from a random Fourier stream function (not a
  Navier-Stokes solution; used as generic sparse-velocity data).

All arrays handed to the GPU path and the oracle are float32; the oracle
converts them exactly to float64.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

PI = np.pi


# --------------------------------------------------------------------------
# parameters
# --------------------------------------------------------------------------
def n_params(dim: int, width: int, depth: int) -> int:
    din = dout = dim + 1
    return width * din + width + (depth - 1) * (width * width + width) + dout * width + dout


def xavier_theta(dim: int, width: int, depth: int, seed: int) -> np.ndarray:
    """Packed float32 parameters W1,b1,...,W_{H+1},b_{H+1} ([out][in] row-major).

    Xavier-normal weights N(0, 2/(fan_in+fan_out)) drawn in float64 from
    ``numpy.random.default_rng(seed)`` layer by layer, biases zero, then
    rounded to float32."""
    rng = np.random.default_rng(seed)
    din = dout = dim + 1
    sizes = [din] + [width] * depth + [dout]
    parts = []
    for l in range(len(sizes) - 1):
        fi, fo = sizes[l], sizes[l + 1]
        std = np.sqrt(2.0 / (fi + fo))
        parts.append((rng.standard_normal((fo, fi)) * std).ravel())
        parts.append(np.zeros(fo))
    th = np.concatenate(parts).astype(np.float32)
    assert th.size == n_params(dim, width, depth)
    return th


def uniform(rng: np.random.Generator, n: int, lo, hi) -> np.ndarray:
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return rng.uniform(lo, hi, size=(n, lo.size)).astype(np.float32)


# --------------------------------------------------------------------------
# analytic fields
# --------------------------------------------------------------------------
def taylor_green(x, y, t, Re=100.0, k=2 * PI):
    """2D Taylor-Green vortex: exact incompressible Navier-Stokes solution
    with viscosity 1/Re."""
    F = np.exp(-2.0 * k * k * t / Re)
    u = -np.cos(k * x) * np.sin(k * y) * F
    v = np.sin(k * x) * np.cos(k * y) * F
    p = -0.25 * (np.cos(2 * k * x) + np.cos(2 * k * y)) * F * F
    return u, v, p


def ethier_steinman(x, y, z, t, a=PI / 4, d=PI / 2, nu=1.0):
    """3D Ethier-Steinman Beltrami flow: exact incompressible Navier-Stokes
    solution (viscosity nu)."""
    E = np.exp(-nu * d * d * t)
    u = -a * (np.exp(a * x) * np.sin(a * y + d * z) + np.exp(a * z) * np.cos(a * x + d * y)) * E
    v = -a * (np.exp(a * y) * np.sin(a * z + d * x) + np.exp(a * x) * np.cos(a * y + d * z)) * E
    w = -a * (np.exp(a * z) * np.sin(a * x + d * y) + np.exp(a * y) * np.cos(a * z + d * x)) * E
    p = -(a * a / 2) * (np.exp(2 * a * x) + np.exp(2 * a * y) + np.exp(2 * a * z)
                        + 2 * np.sin(a * x + d * y) * np.cos(a * z + d * x) * np.exp(a * (y + z))
                        + 2 * np.sin(a * y + d * z) * np.cos(a * x + d * y) * np.exp(a * (z + x))
                        + 2 * np.sin(a * z + d * x) * np.cos(a * y + d * z) * np.exp(a * (x + y))) * E * E
    return u, v, w, p


class FourierStream:
    """Divergence-free 2D field from a random stream function
    psi = sum_m (a_m/n_m^2) sin(pi n_m (x cos th_m + y sin th_m) + phi_m) exp(-nu pi^2 n_m^2 t),
    u = dpsi/dy, v = -dpsi/dx.  n_m ~ U{1..8}, th_m, phi_m ~ U[0, 2pi), a_m ~ N(0,1).
    ``p`` is a smooth synthetic pressure-like field of the same modes (used only
    as a fixed interface target)."""

    def __init__(self, seed: int, n_modes: int = 32, nmax: int = 8, nu: float = 0.01):
        rng = np.random.default_rng([seed, 7919])
        self.n = rng.integers(1, nmax + 1, size=n_modes).astype(np.float64)
        self.th = rng.uniform(0, 2 * PI, size=n_modes)
        self.ph = rng.uniform(0, 2 * PI, size=n_modes)
        self.a = rng.standard_normal(n_modes)
        self.nu = nu

    def _arg(self, x, y, t):
        x = np.asarray(x, np.float64)[..., None]
        y = np.asarray(y, np.float64)[..., None]
        t = np.asarray(t, np.float64)[..., None]
        arg = PI * self.n * (x * np.cos(self.th) + y * np.sin(self.th)) + self.ph
        E = np.exp(-self.nu * PI * PI * self.n ** 2 * t)
        return arg, E

    def uv(self, x, y, t):
        arg, E = self._arg(x, y, t)
        c = (self.a / self.n ** 2) * np.cos(arg) * PI * self.n * E
        u = (c * np.sin(self.th)).sum(-1)
        v = -(c * np.cos(self.th)).sum(-1)
        return u, v

    def p(self, x, y, t):
        arg, E = self._arg(x, y, t)
        return ((self.a / self.n ** 2) * np.cos(arg) * E * E).sum(-1)


# --------------------------------------------------------------------------
# problem description
# --------------------------------------------------------------------------
@dataclass
class Subdomain:
    lo: np.ndarray                 # [d+1] interior box, half-open
    hi: np.ndarray
    is_master: bool
    theta: np.ndarray              # [P] float32
    pde_x: np.ndarray              # [N_pde, d+1]
    obs_x: np.ndarray              # [N_obs, d+1]
    obs_u: np.ndarray              # [N_obs, d]
    gh_x: np.ndarray               # [N_gh, d+1]
    gh_up: np.ndarray              # [N_gh, d+1]
    gh_kind: np.ndarray            # [N_gh] uint8: 0 space, 1 time
    anc_x: np.ndarray              # [N_anc, d+1]
    anc_p: np.ndarray              # [N_anc]
    # ghost faces: (neighbour id, kind, first index, count) for the exchange
    faces: list = field(default_factory=list)


@dataclass
class Problem:
    name: str
    dim: int
    width: int
    depth: int
    nu: float
    lam: np.ndarray                # [6] obs, pde, gh_u, gh_p^space, gh_p^time, anc
    lr: float
    subs: List[Subdomain]
    x_anc: Optional[np.ndarray] = None   # spatial anchor location [d]
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    activation: str = "tanh"             # "tanh" or "sin"
    comp_w: Optional[np.ndarray] = None  # velocity-component weights in L_obs, L_gh_u
    clip_norm: float = 0.0               # global-norm gradient clipping (0: off)
    lr_factor: float = 1.0               # step decay of the learning rate
    lr_interval: int = 0

    @property
    def n_params(self) -> int:
        return n_params(self.dim, self.width, self.depth)

    @property
    def n_pde(self) -> int:
        return int(sum(s.pde_x.shape[0] for s in self.subs))


def _empty(D):
    return np.zeros((0, D), np.float32)


def _sub(dim, lo, hi, theta, *, is_master=False, pde_x=None, obs_x=None, obs_u=None,
         gh_x=None, gh_up=None, gh_kind=None, anc_x=None, anc_p=None, faces=None):
    D = dim + 1
    return Subdomain(
        lo=np.asarray(lo, np.float32), hi=np.asarray(hi, np.float32), is_master=is_master,
        theta=theta,
        pde_x=pde_x if pde_x is not None else _empty(D),
        obs_x=obs_x if obs_x is not None else _empty(D),
        obs_u=obs_u if obs_u is not None else np.zeros((0, dim), np.float32),
        gh_x=gh_x if gh_x is not None else _empty(D),
        gh_up=gh_up if gh_up is not None else _empty(D),
        gh_kind=gh_kind if gh_kind is not None else np.zeros(0, np.uint8),
        anc_x=anc_x if anc_x is not None else _empty(D),
        anc_p=anc_p if anc_p is not None else np.zeros(0, np.float32),
        faces=faces or [])


def tiny(dim=2, width=5, depth=3, n_pde=7, n_obs=5, n_gh=4, n_anc=2, seed=0,
         lam=(1.0, 1.0, 0.7, 0.6, 0.5, 0.9), nu=0.05, is_master=False) -> Problem:
    """A small problem with every point set populated (for finite-difference
    checks and edge cases)."""
    rng = np.random.default_rng([seed, 11])
    D = dim + 1
    lo, hi = np.zeros(D), np.ones(D)
    th = xavier_theta(dim, width, depth, seed)
    # non-zero biases so that no term is structurally absent
    th = th + (0.1 * rng.standard_normal(th.size)).astype(np.float32)
    gh_kind = (np.arange(n_gh) % 2).astype(np.uint8)
    s = _sub(dim, lo, hi, th, is_master=is_master,
             pde_x=uniform(rng, n_pde, lo, hi),
             obs_x=uniform(rng, n_obs, lo, hi),
             obs_u=rng.standard_normal((n_obs, dim)).astype(np.float32),
             gh_x=uniform(rng, n_gh, lo, hi),
             gh_up=rng.standard_normal((n_gh, D)).astype(np.float32),
             gh_kind=gh_kind,
             anc_x=uniform(rng, n_anc, lo, hi),
             anc_p=rng.standard_normal(n_anc).astype(np.float32))
    return Problem("tiny", dim, width, depth, nu, np.asarray(lam, np.float64), 1e-3, [s])


def config1(seed: int = 0) -> Problem:
    """One 2D subdomain, 3 -> 4x50 tanh -> 3; 2,000 collocation points in
    [0,1]^3; 200 Taylor-Green (Re=100) velocity samples; one anchor with p=0."""
    rng = np.random.default_rng([seed, 1])
    lo, hi = np.zeros(3), np.ones(3)
    th = xavier_theta(2, 50, 4, seed)
    pde = uniform(rng, 2000, lo, hi)
    obs = uniform(rng, 200, lo, hi)
    x, y, t = (obs[:, i].astype(np.float64) for i in range(3))
    u, v, _ = taylor_green(x, y, t, Re=100.0)
    anc = np.array([[1 / 8, 3 / 8, 1 / 2]], np.float32)
    s = _sub(2, lo, hi, th, is_master=True, pde_x=pde, obs_x=obs,
             obs_u=np.stack([u, v], 1).astype(np.float32),
             anc_x=anc, anc_p=np.zeros(1, np.float32))
    lam = np.array([1.0, 1.0, 0.0, 0.0, 0.0, 1.0])
    return Problem("config1_2d_4x50_2k", 2, 50, 4, 1.0 / 100.0, lam, 1e-3, [s],
                   x_anc=np.array([1 / 8, 3 / 8]))


def config2(seed: int = 0, n_pde: int = 100_000) -> Problem:
    """One 2D subdomain at working size: 3 -> 8x100 tanh -> 3 on
    [0,2]x[0,1]x[0,1]; 100,000 collocation points; 10,000 velocity samples
    from the Fourier stream field; 2,000 ghost points on the x = 2 face
    (slab [2, 2.4]), kind space, with fixed analytic targets; Re = 100."""
    rng = np.random.default_rng([seed, 2])
    lo, hi = np.array([0, 0, 0.]), np.array([2, 1, 1.])
    f = FourierStream(seed, nu=0.01)
    th = xavier_theta(2, 100, 8, seed)
    pde = uniform(rng, n_pde, lo, hi)
    obs = uniform(rng, 10_000, lo, hi)
    u, v = f.uv(obs[:, 0], obs[:, 1], obs[:, 2])
    gh = uniform(rng, 2000, [2, 0, 0], [2.4, 1, 1])
    gu, gv = f.uv(gh[:, 0], gh[:, 1], gh[:, 2])
    gp = f.p(gh[:, 0], gh[:, 1], gh[:, 2])
    s = _sub(2, lo, hi, th, is_master=False, pde_x=pde, obs_x=obs,
             obs_u=np.stack([u, v], 1).astype(np.float32),
             gh_x=gh, gh_up=np.stack([gu, gv, gp], 1).astype(np.float32),
             gh_kind=np.zeros(2000, np.uint8))
    lam = np.array([10.0, 4.0, 1.0, 1.0, 1.0, 0.0])
    return Problem("config2_2d_8x100_100k", 2, 100, 8, 1.0 / 100.0, lam, 1e-3, [s])


def strip_geometry(K=4, M=4, sx=2.0, ly=2.0, st=1.0):
    """K spatial strips [sx k, sx (k+1)] x [0, ly] times M slabs [st m, st (m+1)];
    subdomain id = K m + k.  Returns boxes[n_sub, 2, 3]."""
    boxes = []
    for m in range(M):
        for k in range(K):
            boxes.append([[sx * k, 0.0, st * m], [sx * (k + 1), ly, st * (m + 1)]])
    return np.asarray(boxes, np.float64)


def config3(seed: int = 0, width: int = 64, depth: int = 6, n_gh_face: int = 2000,
            n_obs: int = 1500, pde_range=(20_000, 120_000), K: int = 4, M: int = 4) -> Problem:
    """16 subdomains (4 spatial strips x 4 time slabs of [0,8]x[0,2]x[0,4]),
    each 3 -> 6x64 tanh -> 3; log-uniform collocation counts; 1,500 velocity
    samples each; 2,000 ghost points per face side (slabs dx = 0.4, dt = 0.2);
    anchor x_anc = (1, 1): masters are the k = 0 strip; anchor term in
    subdomain 0 at (1, 1, 0.5) with p = 0.  Ghost targets are analytic (the
    step treats them as fixed inputs; the on-device exchange replaces them)."""
    rng = np.random.default_rng([seed, 3])
    f = FourierStream(seed, nu=0.01)
    boxes = strip_geometry(K, M)
    x_anc = np.array([1.0, 1.0])
    dx, dt = 0.4, 0.2
    lnlo, lnhi = np.log(pde_range[0]), np.log(pde_range[1])
    counts = [int(round(np.exp(rng.uniform(lnlo, lnhi)))) for _ in range(K * M)]
    subs = []
    for sid in range(K * M):
        m, k = divmod(sid, K)
        lo, hi = boxes[sid]
        is_master = bool(lo[0] <= x_anc[0] < hi[0] and lo[1] <= x_anc[1] < hi[1])
        th = xavier_theta(2, width, depth, seed + sid)
        pde = uniform(rng, counts[sid], lo, hi)
        obs = uniform(rng, n_obs, lo, hi)
        u, v = f.uv(obs[:, 0], obs[:, 1], obs[:, 2])
        gx, gk, faces = [], [], []
        nbrs = []
        if k + 1 < K:
            nbrs.append((sid + 1, 0, [hi[0], lo[1], lo[2]], [hi[0] + dx, hi[1], hi[2]]))
        if k - 1 >= 0:
            nbrs.append((sid - 1, 0, [lo[0] - dx, lo[1], lo[2]], [lo[0], hi[1], hi[2]]))
        if m + 1 < M:
            nbrs.append((sid + K, 1, [lo[0], lo[1], hi[2]], [hi[0], hi[1], hi[2] + dt]))
        if m - 1 >= 0:
            nbrs.append((sid - K, 1, [lo[0], lo[1], lo[2] - dt], [hi[0], hi[1], lo[2]]))
        start = 0
        for nb, kind, glo, ghi in nbrs:
            pts = uniform(rng, n_gh_face, glo, ghi)
            gx.append(pts)
            gk.append(np.full(n_gh_face, kind, np.uint8))
            faces.append((nb, kind, start, n_gh_face))
            start += n_gh_face
        gx = np.concatenate(gx)
        gu, gv = f.uv(gx[:, 0], gx[:, 1], gx[:, 2])
        gp = f.p(gx[:, 0], gx[:, 1], gx[:, 2])
        anc_x = anc_p = None
        if sid == 0:
            anc_x = np.array([[1.0, 1.0, 0.5]], np.float32)
            anc_p = np.zeros(1, np.float32)
        subs.append(_sub(2, lo, hi, th, is_master=is_master, pde_x=pde, obs_x=obs,
                         obs_u=np.stack([u, v], 1).astype(np.float32),
                         gh_x=gx, gh_up=np.stack([gu, gv, gp], 1).astype(np.float32),
                         gh_kind=np.concatenate(gk), anc_x=anc_x, anc_p=anc_p, faces=faces))
    lam = np.array([10.0, 4.0, 1.0, 1.0, 1.0, 1.0])
    return Problem(f"config3_16x2d_{depth}x{width}", 2, width, depth, 1.0 / 100.0, lam, 1e-3,
                   subs, x_anc=x_anc)


def config4(seed: int = 0, n_pde: int = 250_000, n_obs: int = 20_000, n_gh_face: int = 4000) -> Problem:
    """One 3D subdomain: 4 -> 8x128 tanh -> 4 on [-1,1]^3 x [0,1];
    250,000 collocation points; 20,000 Ethier-Steinman velocity samples;
    ghost faces x = 1, y = 1 (space, slabs of 0.4) and t = 1 (time, slab 0.2),
    4,000 points each, with exact Ethier-Steinman targets; nu = 1."""
    rng = np.random.default_rng([seed, 4])
    lo, hi = np.array([-1, -1, -1, 0.]), np.array([1, 1, 1, 1.])
    th = xavier_theta(3, 128, 8, seed)
    pde = uniform(rng, n_pde, lo, hi)
    obs = uniform(rng, n_obs, lo, hi)
    u, v, w, _ = ethier_steinman(*(obs[:, i].astype(np.float64) for i in range(4)))
    g1 = uniform(rng, n_gh_face, [1, -1, -1, 0], [1.4, 1, 1, 1])
    g2 = uniform(rng, n_gh_face, [-1, 1, -1, 0], [1, 1.4, 1, 1])
    g3 = uniform(rng, n_gh_face, [-1, -1, -1, 1], [1, 1, 1, 1.2])
    gx = np.concatenate([g1, g2, g3])
    gk = np.concatenate([np.zeros(2 * n_gh_face, np.uint8), np.ones(n_gh_face, np.uint8)])
    gu = np.stack(ethier_steinman(*(gx[:, i].astype(np.float64) for i in range(4))), 1)
    s = _sub(3, lo, hi, th, is_master=False, pde_x=pde, obs_x=obs,
             obs_u=np.stack([u, v, w], 1).astype(np.float32),
             gh_x=gx, gh_up=gu.astype(np.float32), gh_kind=gk)
    lam = np.array([10.0, 10.0, 1.0, 1.0, 1.0, 0.0])
    return Problem("config4_3d_8x128_250k", 3, 128, 8, 1.0, lam, 1e-3, [s])


def serving_nets(seed: int = 0, width: int = 100, depth: int = 8, K: int = 4, M: int = 4):
    """Resident 2D networks for the query server: (boxes[16,2,3], thetas)."""
    boxes = strip_geometry(K, M)
    thetas = [xavier_theta(2, width, depth, seed + s) for s in range(K * M)]
    return boxes, thetas


def query_requests(seed: int, n_req: int, rate_hz: float = 200.0, nmax: int = 200_000,
                   lo=(0, 0, 0), hi=(8, 2, 4)):
    """Open-loop Poisson arrivals (exponential gaps, mean 1/rate) with
    log-uniform sizes in [1, nmax]; returns (arrival_times[s], sizes)."""
    rng = np.random.default_rng([seed, 5])
    gaps = rng.exponential(1.0 / rate_hz, size=n_req)
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes = np.floor(np.exp(rng.uniform(0.0, np.log(nmax), size=n_req))).astype(np.int64)
    sizes = np.clip(sizes, 1, nmax)
    return arrivals, sizes


def query_points(rng: np.random.Generator, n: int, lo=(0, 0, 0), hi=(8, 2, 4)) -> np.ndarray:
    return uniform(rng, n, lo, hi)


def cylinder3d_recipe(seed: int = 0, n_pde: int = 250_000, n_obs: int = 20_000,
                      n_gh_face: int = 4000, width: int = 128, depth: int = 8) -> Problem:
    """The 3D workload trained with the paper's 3D-cylinder recipe (section 3.3,
    appendix B): sin activation, velocity-component weights (1, 5, 100) in
    L_obs and L_gh_u, global-norm clipping at 1.0, learning rate 1e-3 decayed
    by 0.3 every 5,000 steps.  Data as config4 (Ethier-Steinman)."""
    pb = config4(seed, n_pde=n_pde, n_obs=n_obs, n_gh_face=n_gh_face)
    if width != 128 or depth != 8:
        for s in pb.subs:
            s.theta = xavier_theta(3, width, depth, seed)
        pb.width, pb.depth = width, depth
    pb.name = f"cylinder3d_recipe_3d_{depth}x{width}"
    pb.activation = "sin"
    pb.comp_w = np.array([1.0, 5.0, 100.0])
    pb.clip_norm = 1.0
    pb.lr_factor = 0.3
    pb.lr_interval = 5000
    return pb


def _outside_cylinder(rng, n, lo, hi, radius=0.5):
    """n points uniform in the box [lo, hi) with (x, y) outside the cylinder
    of the given radius centred at the origin (rejection sampling)."""
    out = np.zeros((0, len(lo)), np.float32)
    while out.shape[0] < n:
        x = uniform(rng, 2 * (n - out.shape[0]) + 64, lo, hi)
        keep = x[:, 0].astype(np.float64) ** 2 + x[:, 1].astype(np.float64) ** 2 >= radius * radius
        out = np.concatenate([out, x[keep]])
    return np.ascontiguousarray(out[:n])


def _snapshot_points(rng, n_snap, per_snap, lo, hi, dt=0.15):
    """per_snap spatial locations (outside the cylinder) at each of n_snap
    snapshot times t_k = k dt."""
    D = len(lo)
    xs = _outside_cylinder(rng, n_snap * per_snap, list(lo[:-1]) + [0.0], list(hi[:-1]) + [1.0])
    xs[:, D - 1] = np.repeat(np.arange(n_snap) * dt, per_snap).astype(np.float32)
    return xs


def cylinder2d_paper(seed: int = 0) -> Problem:
    """The paper's 2D cylinder-wake training problem on one GPU (section 3.2,
    appendix B, P = 1): 3 -> 6x150 sin -> 3 on [-7.5, 17.5] x [-8, 8] x
    [0, 7.35] with the cylinder r < 0.5 cut out; 500,000 collocation points;
    10,000 velocity observations (200 locations at each of 50 snapshots,
    dt = 0.15); weights (obs, PDE) = (10, 5); Re = 100; learning rate 1e-3
    decayed by 0.2 every 2,000 steps.  The CFD data are not available: the
    observed velocities come from the Fourier stream field."""
    rng = np.random.default_rng([seed, 21])
    lo, hi = np.array([-7.5, -8.0, 0.0]), np.array([17.5, 8.0, 7.35])
    f = FourierStream(seed, nu=0.01)
    th = xavier_theta(2, 150, 6, seed)
    pde = _outside_cylinder(rng, 500_000, lo, hi)
    obs = _snapshot_points(rng, 50, 200, lo, hi)
    u, v = f.uv(obs[:, 0] / 8.0, obs[:, 1] / 8.0, obs[:, 2])
    s = _sub(2, lo, hi, th, pde_x=pde, obs_x=obs, obs_u=np.stack([u, v], 1).astype(np.float32))
    lam = np.array([10.0, 5.0, 1.0, 1.0, 1.0, 0.0])
    pb = Problem("cylinder2d_paper_2d_6x150_500k_sin", 2, 150, 6, 1.0 / 100.0, lam, 1e-3, [s])
    pb.activation = "sin"
    pb.lr_factor, pb.lr_interval = 0.2, 2000
    return pb


def cylinder3d_paper(seed: int = 0) -> Problem:
    """The paper's 3D cylinder-wake training problem on one GPU (section 3.3,
    appendix B, P = 1): 4 -> 8x200 sin -> 4 on [-5, 20] x [-5, 5] x [0, 10] x
    [0, 11.85] with the cylinder r < 0.5 cut out; 600,000 collocation points;
    100,000 velocity observations (1,250 locations at each of 80 snapshots,
    dt = 0.15); weights (obs, PDE) = (10, 10); velocity-component weights
    (1, 5, 100); global-norm clipping at 1.0; Re = 300; learning rate 1e-3
    decayed by 0.3 every 5,000 steps.  The CFD data are not available: the
    observed velocities come from the Ethier-Steinman field on coordinates
    mapped to [-1, 1]^3 x [0, 1]."""
    rng = np.random.default_rng([seed, 22])
    lo, hi = np.array([-5.0, -5.0, 0.0, 0.0]), np.array([20.0, 5.0, 10.0, 11.85])
    th = xavier_theta(3, 200, 8, seed)
    pde = _outside_cylinder(rng, 600_000, lo, hi)
    obs = _snapshot_points(rng, 80, 1250, lo, hi)
    xm = [2.0 * (obs[:, i].astype(np.float64) - lo[i]) / (hi[i] - lo[i]) - 1.0 for i in range(3)]
    u, v, w, _ = ethier_steinman(*xm, obs[:, 3].astype(np.float64) / hi[3])
    s = _sub(3, lo, hi, th, pde_x=pde, obs_x=obs, obs_u=np.stack([u, v, w], 1).astype(np.float32))
    lam = np.array([10.0, 10.0, 1.0, 1.0, 1.0, 0.0])
    pb = Problem("cylinder3d_paper_3d_8x200_600k_sin", 3, 200, 8, 1.0 / 300.0, lam, 1e-3, [s])
    pb.activation = "sin"
    pb.comp_w = np.array([1.0, 5.0, 100.0])
    pb.clip_norm = 1.0
    pb.lr_factor, pb.lr_interval = 0.3, 5000
    return pb

