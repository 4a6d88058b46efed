"""Python handle over one libddpinn context.

PyTorch supplies device memory (tensors) and streams; every computation runs
in the HIP kernels behind the C ABI.  There is no CPU or PyTorch fallback: if
the library is missing or no GPU is present, construction raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import abi
from .abi import PinnConfig, PinnFace, PinnLaunchInfo, PinnSubdomain, check, lib

WHAT = {"value": abi.PINN_Q_VALUE, "uvpw": abi.PINN_Q_UVPW,
        "channels": abi.PINN_Q_CHANNELS, "residual": abi.PINN_Q_RESIDUAL}


@dataclass
class SubTensors:
    """Device tensors of one subdomain (all float32 except gh_kind uint8)."""
    lo: Sequence[float]
    hi: Sequence[float]
    is_master: bool
    theta: torch.Tensor
    adam_m: torch.Tensor
    adam_v: torch.Tensor
    pde_x: torch.Tensor
    obs_x: torch.Tensor
    obs_u: torch.Tensor
    gh_x: torch.Tensor
    gh_up: torch.Tensor
    gh_kind: torch.Tensor
    anc_x: torch.Tensor
    anc_p: torch.Tensor


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None or t.numel() == 0:
        return None
    if not (t.is_cuda and t.is_contiguous()):
        # a host address or a strided view handed to a kernel would be read
        # as a dense device array
        raise ValueError("arrays passed to libddpinn must be contiguous device tensors")
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def subdomain_to_device(s, device) -> SubTensors:
    """Copy one host subdomain description (NumPy arrays with the fields of
    SubTensors) to the device; Adam moments start at zero."""
    def f32(a, cols=None):
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
        return torch.from_numpy(a).to(device)
    th = f32(s.theta)
    return SubTensors(
        lo=list(np.asarray(s.lo, np.float32)), hi=list(np.asarray(s.hi, np.float32)),
        is_master=bool(s.is_master), theta=th,
        adam_m=torch.zeros_like(th), adam_v=torch.zeros_like(th),
        pde_x=f32(s.pde_x), obs_x=f32(s.obs_x), obs_u=f32(s.obs_u),
        gh_x=f32(s.gh_x), gh_up=f32(s.gh_up),
        gh_kind=torch.from_numpy(np.ascontiguousarray(np.asarray(s.gh_kind, np.uint8))).to(device),
        anc_x=f32(s.anc_x), anc_p=f32(s.anc_p))


class Context:
    """One or more subdomain networks of one architecture (section 2.2 local
    experts) and their training data, resident on one GPU."""

    def __init__(self, dim: int, width: int, depth: int, subs: List[SubTensors], nu: float,
                 lam, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, graph: bool = True, tile_points: int = 0,
                 blocks_per_cu: int = 0, max_query_points: int = 1 << 22,
                 activation: str = "tanh", comp_w=None, clip_norm: float = 0.0,
                 lr_factor: float = 1.0, lr_interval: int = 0,
                 gemm_priority: bool = True, ranges_per_wg: int = 0,
                 device=None, stream=None, guard_bytes: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("libddpinn needs a ROCm GPU (gfx950); none is visible")
        L = lib()
        self.dim, self.width, self.depth = dim, width, depth
        self.n_sub = len(subs)
        self.device = torch.device(device) if device is not None else subs[0].theta.device
        self.subs = subs
        self.P = abi.num_params(dim, width, depth)
        cfg = PinnConfig()
        cfg.dim, cfg.width, cfg.depth, cfg.n_sub = dim, width, depth, self.n_sub
        if activation not in ("tanh", "sin"):
            raise ValueError(f"activation must be 'tanh' or 'sin', got {activation!r}")
        cfg.activation = {"tanh": 0, "sin": 1}[activation]
        self.activation = activation
        if comp_w is not None:
            for k, v in enumerate(list(comp_w)[:3]):
                cfg.comp_w[k] = float(v)
        cfg.clip_norm = float(clip_norm)
        cfg.lr_factor = float(lr_factor)
        cfg.lr_interval = int(lr_interval)
        cfg.flags = abi.PINN_GRAPH if graph else 0
        cfg.nu = float(nu)
        for k in range(6):
            cfg.lam[k] = float(lam[k])
        cfg.lr, cfg.beta1, cfg.beta2, cfg.eps = lr, beta1, beta2, eps
        cfg.tile_points = tile_points
        cfg.blocks_per_cu = blocks_per_cu
        cfg.gemm_priority_off = 0 if gemm_priority else 1
        cfg.ranges_per_wg = int(ranges_per_wg)
        cfg.guard_bytes = int(guard_bytes)
        cfg.max_query_points = max_query_points
        self.cfg = cfg
        arr = (PinnSubdomain * self.n_sub)()
        for i, s in enumerate(subs):
            if s.theta.numel() != self.P:
                raise ValueError(f"subdomain {i}: theta has {s.theta.numel()} entries, the network has {self.P}")
            d = arr[i]
            for q in range(4):
                d.lo[q] = float(s.lo[q]) if q < len(s.lo) else 0.0
                d.hi[q] = float(s.hi[q]) if q < len(s.hi) else 0.0
            d.is_master = int(bool(s.is_master))
            d.theta, d.adam_m, d.adam_v = _ptr(s.theta), _ptr(s.adam_m), _ptr(s.adam_v)
            d.pde_x, d.n_pde = _ptr(s.pde_x), s.pde_x.shape[0]
            d.obs_x, d.obs_u, d.n_obs = _ptr(s.obs_x), _ptr(s.obs_u), s.obs_x.shape[0]
            d.gh_x, d.gh_up, d.gh_kind, d.n_gh = (_ptr(s.gh_x), _ptr(s.gh_up), _ptr(s.gh_kind),
                                                  s.gh_x.shape[0])
            d.anc_x, d.anc_p, d.n_anc = _ptr(s.anc_x), _ptr(s.anc_p), s.anc_x.shape[0]
        self._subs_c = arr
        nbytes = ctypes.c_size_t(0)
        st = _stream(stream)
        with torch.cuda.device(self.device):
            check(L.pinn_create(ctypes.byref(cfg), arr, None, ctypes.byref(nbytes), st, None))
            self.workspace = torch.empty(max(int(nbytes.value), 256) + 256, dtype=torch.uint8,
                                         device=self.device)
            base = self.workspace.data_ptr()
            off = (-base) % 256
            self._ws_ptr = base + off
            avail = ctypes.c_size_t(self.workspace.numel() - off)
            h = ctypes.c_void_p()
            check(L.pinn_create(ctypes.byref(cfg), arr, self._ws_ptr, ctypes.byref(avail), st,
                                ctypes.byref(h)))
        self._h = h
        self.workspace_bytes = int(avail.value)
        self._loss = torch.zeros(self.n_sub, 7, dtype=torch.float32, device=self.device)
        self._scratch = None

    # ------------------------------------------------------------------ step
    def step(self, t: int, update: bool = True, check_finite: bool = False,
             per_subdomain: bool = False, want_grad: bool = False, grad_out=None, stream=None,
             time_kernel: bool = False):
        """One training step of every subdomain.  Returns (loss [n_sub, 7],
        grad [n_sub, P] or None); loss rows are (L_obs, L_PDE, L_gh_u,
        L_gh_p^space, L_gh_p^time, L_anc, L)."""
        flags = 0
        if not update:
            flags |= abi.PINN_NO_UPDATE
        if check_finite:
            flags |= abi.PINN_CHECK_FINITE
        if per_subdomain:
            flags |= abi.PINN_PER_SUBDOMAIN
        if time_kernel:
            flags |= abi.PINN_TIME_KERNEL
        g = grad_out
        if want_grad and g is None:
            g = torch.empty(self.n_sub, self.P, dtype=torch.float32, device=self.device)
        check(lib().pinn_step(self._h, int(t), flags, self._loss.data_ptr(),
                              g.data_ptr() if g is not None else None, _stream(stream)))
        return self._loss, g

    # ----------------------------------------------------------------- query
    def query_scratch_bytes(self, n: int) -> int:
        return int(lib().pinn_query_scratch_bytes(self._h, int(n)))

    def query(self, x: torch.Tensor, sub: int = -1, what: str = "uvpw", out=None,
              scratch: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Evaluate the networks at points x[n, d+1] (routed to subdomains when
        sub == -1)."""
        n = x.shape[0]
        D = self.dim + 1
        kind = WHAT[what]
        cols = {"value": D, "uvpw": 4, "channels": (2 * self.dim + 2) * D, "residual": D}[what]
        if out is None:
            out = torch.empty(n, cols, dtype=torch.float32, device=self.device)
        sptr, sbytes = None, 0
        if sub < 0:
            need = self.query_scratch_bytes(n)
            if scratch is None:
                if self._scratch is None or self._scratch.numel() < need + 256:
                    self._scratch = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
                scratch = self._scratch
            base = scratch.data_ptr()
            off = (-base) % 256
            sptr, sbytes = base + off, scratch.numel() - off
        check(lib().pinn_query(self._h, _ptr(x) if n else None, n, sub, kind,
                               _ptr(out) if n else None, sptr, sbytes, _stream(stream)))
        return out

    def query_noalloc(self, x: torch.Tensor, out: torch.Tensor, sub: int = -1, what: str = "uvpw",
                      stream=None) -> torch.Tensor:
        """pinn_query_noalloc: the same query into the caller's `out`, routed
        through the library-held scratch (no allocation anywhere)."""
        n = x.shape[0]
        check(lib().pinn_query_noalloc(self._h, _ptr(x) if n else None, n, sub, WHAT[what],
                                       _ptr(out) if n else None, _stream(stream)))
        return out

    # -------------------------------------------------------------- exchange
    def exchange(self, faces, x_anc, targets: List[Optional[torch.Tensor]], stream=None):
        """Write neighbour targets (u, p~) at ghost points (section 2.2);
        faces = [(a, b, first, count), ...]."""
        arr = (PinnFace * max(len(faces), 1))()
        for i, (a, b, first, count) in enumerate(faces):
            arr[i].a, arr[i].b, arr[i].first, arr[i].count = int(a), int(b), int(first), int(count)
        xa = (ctypes.c_float * 3)(*[float(v) for v in list(x_anc)[:3]])
        tg = (ctypes.c_void_p * self.n_sub)(*[(_ptr(t) if t is not None else None) for t in targets])
        check(lib().pinn_exchange(self._h, arr, len(faces), xa, tg, _stream(stream)))

    def kernel_time(self):
        """(total milliseconds, launches) of the fused-kernel launches timed
        with HIP events since the previous call (waits for them)."""
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        check(lib().pinn_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    def check_guards(self, stream=None) -> int:
        """Memory-check mode (guard_bytes > 0): bytes of the workspace's guard
        zones that no longer hold their fill pattern (waits for the stream)."""
        bad = ctypes.c_int64(0)
        check(lib().pinn_check_guards(self._h, ctypes.byref(bad), _stream(stream)))
        return int(bad.value)

    def evaluate(self, x: torch.Tensor, ref: torch.Tensor, snap_off, x_anc, stream=None):
        """Relative L2 errors [u_1..u_d, velocity, p] after stitching, master
        anchor pinning and per-snapshot pressure-mean removal (section 3)."""
        n = x.shape[0]
        off = np.ascontiguousarray(np.asarray(snap_off, dtype=np.int64))
        n_snap = off.size - 1
        max_snap = int(np.max(np.diff(off))) if n_snap else 0
        need = int(lib().pinn_evaluate_scratch_bytes(self._h, n, n_snap, max_snap))
        scratch = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        base = scratch.data_ptr()
        adj = (-base) % 256
        err = torch.empty(self.dim + 2, dtype=torch.float32, device=self.device)
        xa = (ctypes.c_float * 3)(*[float(v) for v in list(x_anc)[:3]])
        check(lib().pinn_evaluate(self._h, _ptr(x), _ptr(ref), n,
                                  off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n_snap, xa,
                                  _ptr(err), base + adj, scratch.numel() - adj, _stream(stream)))
        return err

    def refresh(self, stream=None):
        check(lib().pinn_refresh(self._h, _stream(stream)))

    def launch_info(self) -> dict:
        info = PinnLaunchInfo()
        check(lib().pinn_get_launch_info(self._h, ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in PinnLaunchInfo._fields_}

    def close(self):
        if getattr(self, "_h", None):
            check(lib().pinn_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().pinn_destroy(self._h)
                self._h = None
        except Exception:
            pass


def context_from_problem(pb, device="cuda", **kw) -> Context:
    """Build a Context from a host problem description (an object with dim,
    width, depth, nu, lam, lr, beta1, beta2, eps and subs of NumPy arrays)."""
    subs = [subdomain_to_device(s, device) for s in pb.subs]
    opts = dict(activation=getattr(pb, "activation", "tanh"), comp_w=getattr(pb, "comp_w", None),
                clip_norm=getattr(pb, "clip_norm", 0.0), lr_factor=getattr(pb, "lr_factor", 1.0),
                lr_interval=getattr(pb, "lr_interval", 0))
    opts.update(kw)
    return Context(pb.dim, pb.width, pb.depth, subs, pb.nu, pb.lam, lr=pb.lr, beta1=pb.beta1,
                   beta2=pb.beta2, eps=pb.eps, device=device, **opts)
