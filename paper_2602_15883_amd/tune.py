"""Autotuner for the fused step's launch shape.

Knobs: collocation points per tile (16, or 32 when the workgroup has at most
four waves), persistent workgroups per compute unit, whether the younger half
of a workgroup's waves raises its priority for its GEMMs, and how many item
ranges each workgroup takes in turn when several share a compute unit.  Each
candidate is a fresh context over the same device tensors; its fused-kernel
time is measured with HIP events tied to the kernel's dispatch
(PINN_TIME_KERNEL) over a few steps without the Adam update.  Winners are
cached in JSON keyed by (arch, dim, width, depth, subdomain count, log2 of
the collocation point count, activation).  Candidates that the library maps
to the same launch (points per tile, workgroup count, priority, ranges) are
timed once.  Lookup order: the user cache
(DDPINN_TUNE_CACHE or ~/.cache/ddpinn/tune.json), then the table shipped with
the package (tuned.json), else the library defaults.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Optional

import torch

from .abi import PINN_E_INVAL, PINN_E_UNSUPPORTED, PinnError
from .context import Context

# statuses of a launch shape the library refuses before enqueueing any work
REJECTED = (PINN_E_INVAL, PINN_E_UNSUPPORTED)

HERE = os.path.dirname(os.path.abspath(__file__))
SHIPPED = os.path.join(HERE, "tuned.json")


def user_cache_path() -> str:
    return os.environ.get("DDPINN_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ddpinn", "tune.json"))


def arch_name() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def tune_key(dim, width, depth, n_sub, n_pde, activation: str = "tanh") -> str:
    b = int(math.floor(math.log2(max(n_pde, 1))))
    return f"{arch_name()}|d{dim}|w{width}|h{depth}|s{n_sub}|n2^{b}|{activation}"


def _load(path) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(key: str) -> Optional[dict]:
    for path in (user_cache_path(), SHIPPED):
        e = _load(path).get(key)
        if e:
            return e
    return None


def store(key: str, entry: dict, path: Optional[str] = None):
    path = path or user_cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tab = _load(path)
    tab[key] = entry
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def ctx_cu_count() -> int:
    try:
        return int(torch.cuda.get_device_properties(0).multi_processor_count)
    except Exception:
        return 0


def shape_of(entry: dict) -> dict:
    """The launch-shape keyword arguments of a tuning-table entry (entries
    from before the priority and range knobs default to the library's)."""
    return {"tile_points": int(entry["tile_points"]), "blocks_per_cu": int(entry["blocks_per_cu"]),
            "gemm_priority": bool(entry.get("gemm_priority", True)),
            "ranges_per_wg": int(entry.get("ranges_per_wg", 0))}


def candidates(width: int) -> List[dict]:
    """Launch shapes: collocation points per tile (32 only up to four waves),
    persistent workgroups per compute unit, the GEMM wave priority, and the
    item ranges each workgroup takes in turn when several share a compute
    unit (one workgroup per compute unit takes one range)."""
    waves = (width + 15) // 16
    out = []
    for tp in (16, 32):
        if tp == 32 and waves > 4:
            continue
        for bpc in (1, 2, 3, 4):
            for prio in (True, False):
                for rpw in ((0,) if bpc == 1 else (2, 4, 8)):
                    out.append({"tile_points": tp, "blocks_per_cu": bpc, "gemm_priority": prio,
                                "ranges_per_wg": rpw})
    return out


def measure(make_ctx, cand: dict, steps: int = 3, warmup: int = 1, seen: Optional[dict] = None) -> float:
    """Average fused-kernel milliseconds of one candidate (no Adam update).
    Candidates whose launch (points per tile, workgroup count) equals one in
    `seen` are not timed again."""
    ctx: Context = make_ctx(**cand)
    try:
        info = ctx.launch_info()
        if info["tile_points"] != cand["tile_points"]:
            return float("inf")
        launch = (info["tile_points"], info["n_wg"], bool(cand.get("gemm_priority", True)),
                  int(cand.get("ranges_per_wg", 0)) if info["n_wg"] > ctx_cu_count() else 0)
        if seen is not None and launch in seen:
            return seen[launch]
        for _ in range(warmup):
            ctx.step(1, update=False, time_kernel=True)
        ctx.kernel_time()
        for _ in range(steps):
            ctx.step(1, update=False, time_kernel=True)
        ms, n = ctx.kernel_time()
        ms /= max(n, 1)
        if seen is not None:
            seen[launch] = ms
        return ms
    finally:
        ctx.close()


def autotune(make_ctx, dim, width, depth, n_sub, n_pde, steps: int = 3,
             cache: bool = True, force: bool = False, verbose: bool = False,
             path: Optional[str] = None, activation: str = "tanh") -> dict:
    """Return the best launch shape {tile_points, blocks_per_cu,
    gemm_priority, ranges_per_wg} for this network and problem size, from the
    caches or by timing every candidate.  make_ctx(**cand) builds a Context.
    With cache, the winner and every trial are stored in `path` (default: the
    user cache)."""
    key = tune_key(dim, width, depth, n_sub, n_pde, activation)
    if not force:
        e = lookup(key)
        if e:
            return shape_of(e)
    best, best_ms, trials = None, float("inf"), []
    seen: dict = {}
    cands = candidates(width)
    try:   # one untimed pass first: the first launch of a process pays start-up costs
        measure(make_ctx, cands[0], steps=1)
    except PinnError as ex:
        if ex.status not in REJECTED:
            raise
    for cand in cands:
        try:
            ms = measure(make_ctx, cand, steps=steps, seen=seen)
        except PinnError as ex:
            # only a candidate the library rejects before launching anything is
            # skipped; any other failure (a device error) ends the tuning run
            # without storing a result
            if ex.status not in REJECTED:
                raise
            if verbose:
                print("tune: skip", cand, ex)
            continue
        trials.append({**cand, "ms": ms})
        if verbose:
            print("tune:", cand, f"{ms:.3f} ms")
        if ms < best_ms:
            best, best_ms = cand, ms
    if best is None:
        raise RuntimeError("no launch candidate worked")
    if cache:
        store(key, {**best, "ms": best_ms, "trials": trials}, path=path)
    return dict(best)
