"""Continuous-batching query server over resident subdomain networks.

Stitching of local experts (section 3): every query point is evaluated by the
subdomain network whose box contains it; the server returns (u, v, p) and the
vorticity v_x - u_y.  All networks stay resident on the GPU.  Requests arrive
open loop; a dispatcher admits them while earlier batches are still on the
GPU (as long as the HBM budget allows), packs whole requests into batches and
issues each batch on one of several HIP streams: host-to-device copy, routed
query (pinn_query), device-to-host copy, completion event.  Per-point results
do not depend on the batch a point lands in, so a request's result is the same
alone and in the mix.

Device memory: the server allocates one arena at construction and never
again.  The arena holds one batch slot per stream (input points, outputs and
routing scratch for max_batch_points points); the number of slots is the
number of streams, reduced until the arena fits the HBM budget.  A batch
occupies a slot until its completion event has fired, so the memory the
requests in flight use is bounded by the budget, not just counted against it.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from .context import Context, SubTensors

def _align(n: int) -> int:
    return (int(n) + 255) & ~255


def serving_context(boxes, thetas, width: int, depth: int, dim: int = 2, nu: float = 0.01,
                    device="cuda", max_query_points: int = 1 << 22, masters=None,
                    activation: str = "tanh") -> Context:
    """A context holding only resident networks (no training data); masters[s]
    marks the subdomains that hold the pressure anchor."""
    subs = []
    dev = torch.device(device)
    D = dim + 1
    for s, th in enumerate(thetas):
        t = torch.from_numpy(np.ascontiguousarray(th, np.float32)).to(dev)
        eD = torch.zeros(0, D, device=dev)
        subs.append(SubTensors(lo=list(boxes[s][0]), hi=list(boxes[s][1]),
                               is_master=bool(masters[s]) if masters is not None else False,
                               theta=t, adam_m=torch.zeros_like(t), adam_v=torch.zeros_like(t),
                               pde_x=eD, obs_x=eD, obs_u=torch.zeros(0, dim, device=dev),
                               gh_x=eD, gh_up=eD,
                               gh_kind=torch.zeros(0, dtype=torch.uint8, device=dev),
                               anc_x=eD, anc_p=torch.zeros(0, device=dev)))
    return Context(dim, width, depth, subs, nu, np.zeros(6), graph=False, device=dev,
                   max_query_points=max_query_points, activation=activation)


@dataclass
class Request:
    rid: int
    arrival: float                 # scheduled arrival (s, relative to start)
    x: np.ndarray                  # [n, 3] float32 host points
    out: Optional[np.ndarray] = None
    done: float = -1.0             # completion visible on host (s)
    admitted: float = -1.0
    deferred: bool = False         # waited for a free batch slot


@dataclass
class _Batch:
    reqs: List[Request]
    n: int
    slot: int
    event: torch.cuda.Event
    start_ev: torch.cuda.Event
    keep: list = field(default_factory=list)
    nbytes: int = 0


class QueryServer:
    """Open-loop, continuously batching server over one Context."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 32 << 30, n_streams: int = 4,
                 max_batch_points: int = 1 << 20, min_batch_points: int = 1):
        self.ctx = ctx
        self.budget = int(hbm_budget_bytes)
        self.max_batch = int(max_batch_points)
        cap = self.max_batch
        # one batch slot: points in, outputs, routing scratch (256-byte aligned parts)
        self.in_bytes = _align(cap * 3 * 4)
        self.out_bytes = _align(cap * 4 * 4)
        self.scratch_bytes = _align(ctx.query_scratch_bytes(cap))
        self.slot_bytes = self.in_bytes + self.out_bytes + self.scratch_bytes
        n_slots = min(int(n_streams), self.budget // self.slot_bytes)
        if n_slots < 1:
            raise ValueError(f"an HBM budget of {self.budget} bytes holds no batch slot of "
                             f"{cap} points ({self.slot_bytes} bytes); lower max_batch_points")
        self.n_slots = n_slots
        self.streams = [torch.cuda.Stream(device=ctx.device) for _ in range(n_slots)]
        self.free_slots = deque(range(n_slots))
        self.h_in = [torch.empty(cap, 3, dtype=torch.float32, pin_memory=True) for _ in range(n_slots)]
        self.h_out = [torch.empty(cap, 4, dtype=torch.float32, pin_memory=True) for _ in range(n_slots)]
        # the only device allocation of the server: n_slots slots in one arena
        self.arena = torch.empty(n_slots * self.slot_bytes, dtype=torch.uint8, device=ctx.device)
        self.d_in, self.d_out, self.d_scratch = [], [], []
        for k in range(n_slots):
            base = k * self.slot_bytes
            seg = self.arena[base:base + self.slot_bytes]
            self.d_in.append(seg[:cap * 12].view(torch.float32).view(cap, 3))
            o = self.in_bytes
            self.d_out.append(seg[o:o + cap * 16].view(torch.float32).view(cap, 4))
            o += self.out_bytes
            self.d_scratch.append(seg[o:o + self.scratch_bytes])
        self.inflight: List[_Batch] = []
        self.inflight_bytes = 0
        self.busy_intervals = []
        self.deferred = 0

    @property
    def device_bytes(self) -> int:
        """Device memory the server holds (the arena)."""
        return self.arena.numel()

    def request_bytes(self, n: int) -> int:
        """Device bytes a request of n points uses inside its batch slot."""
        return _align(n * 12) + _align(n * 16) + _align(self.ctx.query_scratch_bytes(n))

    # -------------------------------------------------------------- dispatch
    def _launch(self, reqs: List[Request], t0: float):
        slot = self.free_slots.popleft()
        s = self.streams[slot]
        n = sum(len(r.x) for r in reqs)
        hin, hout = self.h_in[slot], self.h_out[slot]
        o = 0
        for r in reqs:
            hin[o:o + len(r.x)].numpy()[:] = r.x
            o += len(r.x)
        with torch.cuda.stream(s):
            start_ev = torch.cuda.Event(enable_timing=True)
            start_ev.record(s)
            x = self.d_in[slot][:n]
            x.copy_(hin[:n], non_blocking=True)
            out = self.d_out[slot][:n]
            scratch = self.d_scratch[slot]
            self.ctx.query(x, sub=-1, what="uvpw", out=out, scratch=scratch, stream=s)
            hout[:n].copy_(out, non_blocking=True)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
        b = _Batch(reqs=reqs, n=n, slot=slot, event=ev, start_ev=start_ev, keep=[x, out, scratch])
        b.nbytes = sum(self.request_bytes(len(r.x)) for r in reqs)
        self.inflight.append(b)

    def _poll(self, t0: float) -> int:
        done = 0
        still = []
        for b in self.inflight:
            if b.event.query():
                now = time.perf_counter() - t0
                hout = self.h_out[b.slot]
                o = 0
                for r in b.reqs:
                    r.out = hout[o:o + len(r.x)].numpy().copy()
                    o += len(r.x)
                    r.done = now
                self.busy_intervals.append((b.start_ev, b.event))
                self.inflight_bytes -= b.nbytes
                self.free_slots.append(b.slot)
                done += len(b.reqs)
            else:
                still.append(b)
        self.inflight = still
        return done

    def run(self, requests: List[Request], time_scale: float = 1.0, idle_sleep: float = 1e-3):
        """Serve `requests` (sorted by arrival) open loop; returns wall seconds."""
        for r in requests:
            if len(r.x) > self.max_batch:
                raise ValueError(f"request {r.rid} of {len(r.x)} points exceeds a batch slot "
                                 f"({self.max_batch} points) of the HBM budget")
        pending = deque(requests)
        waiting: deque = deque()
        remaining = len(requests)
        t0 = time.perf_counter()
        while remaining:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival * time_scale <= now:
                waiting.append(pending.popleft())
            remaining -= self._poll(t0)
            # admission: whole requests, oldest first, while a batch slot (its
            # share of the HBM budget) is free; a request that does not fit the
            # slot being filled waits for the next one
            while waiting and self.free_slots:
                batch, n, nbytes = [], 0, 0
                while waiting:
                    r = waiting[0]
                    rb = self.request_bytes(len(r.x))
                    if n + len(r.x) > self.max_batch:
                        break
                    batch.append(waiting.popleft())
                    n += len(r.x)
                    nbytes += rb
                if not batch:
                    break
                for r in batch:
                    r.admitted = now
                self.inflight_bytes += nbytes
                self._launch(batch, t0)
            # requests still waiting had no free batch slot: count each once
            for r in reversed(waiting):
                if r.deferred:
                    break
                r.deferred = True
                self.deferred += 1
            # with batches in flight, poll their events without sleeping (a
            # sleep of a few microseconds lasts tens in practice); when idle,
            # sleep until shortly before the next arrival (at most idle_sleep)
            # and spin from there
            if remaining and not self.inflight and not (waiting and self.free_slots):
                gap = pending[0].arrival * time_scale - (time.perf_counter() - t0) if pending else 0.0
                if gap > 3e-4:
                    time.sleep(min(gap - 2e-4, idle_sleep))
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def busy_seconds(self) -> float:
        """Union of the batches' device intervals (from their events)."""
        if not self.busy_intervals:
            return 0.0
        base = self.busy_intervals[0][0]
        iv = sorted((base.elapsed_time(a) / 1e3, base.elapsed_time(b) / 1e3)
                    for a, b in self.busy_intervals)
        tot, cs, ce = 0.0, iv[0][0], iv[0][1]
        for a, b in iv[1:]:
            if a > ce:
                tot += ce - cs
                cs, ce = a, b
            else:
                ce = max(ce, b)
        return tot + ce - cs


def latency_stats(requests: List[Request], time_scale: float = 1.0) -> dict:
    lat = np.array([(r.done - r.arrival * time_scale) * 1e3 for r in requests])
    pts = sum(len(r.x) for r in requests)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "p999_ms": float(np.percentile(lat, 99.9)), "mean_ms": float(lat.mean()),
            "requests": len(requests), "points": int(pts)}
