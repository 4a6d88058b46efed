#!/usr/bin/env python
"""Benchmark of the fused subdomain training step on one MI355X.

Prints ONE JSON line.  `value` is collocation points per second of the whole
fused training step (forward with first and second derivative channels,
Navier-Stokes residuals, losses, hand-written adjoint, gradient reduction and
Adam), inputs resident in HBM, timed over exactly --steps hipGraph replays
after --warmup untimed ones.  The default workload is the width-128 3D
network (4->8x128->4, 250,000 collocation and 32,000 value points).  The line
also carries:

  roofline          the fused step kernel's algorithmic FP32 FLOPs per launch
                    divided by its average duration (HIP events tied to the
                    kernel's dispatch: its start and end time stamps), against
                    the FP32 MFMA peak, plus HBM traffic from rocprofv3
                    counters when a matching profile is committed under
                    profiles/
  config2           the same figures for the 2D 3->8x100->3 network at 100,000
                    collocation points (extra leg)
  grouped_vs_plain  16 uneven 2D 3->6x64->3 subdomains: one grouped persistent
                    launch against one plain launch per subdomain (extra leg)
  exchange          the on-device ghost-target exchange of those subdomains
  cpu_baseline      the FP64 oracle timed on this host's cores on a bounded
                    sample of the headline workload (a baseline, not the
                    target)
  query             p50/p99/p99.9 latency and points/s of the continuous-
                    batching query server (16 resident 3->8x100->3 networks,
                    Poisson arrivals at 200 req/s; 5 s warm-up, 30 s window)
  evaluate          timing of the evaluation post-processing

Only one GPU is used: --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3     # MI355X dense FP32 matrix
PEAK_HBM_GBS = 8000.0
COPY_BYTES = 256 << 20            # size of the counter-calibration copy (each way)

WORKLOADS = {
    "config1": "config1_2d_4x50_2k",
    "config2": "config2_2d_8x100_100k",
    "config3": "config3_16x2d_6x64",
    "config4": "config4_3d_8x128_250k",
    "cylinder3d": "cylinder3d_recipe_3d_8x128_250k_sin",
    "cylinder2d_paper": "cylinder2d_paper_2d_6x150_500k_sin",
    "cylinder3d_paper": "cylinder3d_paper_3d_8x200_600k_sin",
}


def flops_per_point(dim, W, H, C):
    """Algorithmic FLOPs of one point with C channels: 3 x forward GEMM FLOPs
    (forward, input adjoint, weight gradient) at the true width."""
    D = dim + 1
    return 3 * (2 * D * W + 2 * C * W * W * (H - 1) + 2 * C * W * D)


def step_flops(pb):
    C = 2 * pb.dim + 2
    fc = flops_per_point(pb.dim, pb.width, pb.depth, C)
    fv = flops_per_point(pb.dim, pb.width, pb.depth, 1)
    n_pde = sum(s.pde_x.shape[0] for s in pb.subs)
    n_val = sum(s.obs_x.shape[0] + s.gh_x.shape[0] + s.anc_x.shape[0] for s in pb.subs)
    return n_pde * fc + n_val * fv, fc


def algorithmic_bytes(pb):
    """Inputs the step must read plus parameter/moment/gradient traffic:
    points and targets once, theta/m/v read and written, gradient once."""
    D = pb.dim + 1
    b = 0
    for s in pb.subs:
        b += s.pde_x.size * 4 + s.obs_x.size * 4 + s.obs_u.size * 4
        b += s.gh_x.size * 4 + s.gh_up.size * 4 + s.gh_kind.size + s.anc_x.size * 4 + s.anc_p.size * 4
        b += 7 * s.theta.size * 4
    return b


def make_problem(name, seed=0):
    import workloads as wl
    return {"config1": wl.config1, "config2": wl.config2, "config3": wl.config3,
            "config4": wl.config4, "cylinder3d": wl.cylinder3d_recipe,
            "cylinder2d_paper": wl.cylinder2d_paper, "cylinder3d_paper": wl.cylinder3d_paper}[name](seed)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("ddpinn_kernels.hip", "ddpinn_internal.h"):
        with open(os.path.join(ROOT, "paper_2602_15883_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload):
    """HBM bytes per launch of the fused kernel from committed rocprofv3
    counter runs, if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            tab = json.load(f)
    except (OSError, ValueError):
        return None
    e = tab.get(workload)
    if not e or e.get("kernel_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(pb, budget_s=12.0, one_core_s=5.0):
    """FP64 oracle (loss + gradient [+ clipping] + Adam) on a bounded sample of
    the workload, sized to roughly budget_s seconds from a short calibration
    run: a prefix of the collocation points with the same per-point mix of
    observation and ghost points, repeated over several steps when the whole
    workload takes less than the budget.  Same activation and component
    weights as the workload.  Timed on all the host cores the oracle uses,
    then on one core (a smaller sample of about one_core_s seconds)."""
    import oracle
    prev = oracle.threads(0)
    n_aff = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS", "")
    cores = min(n_aff, int(omp)) if omp.isdigit() and int(omp) > 0 else n_aff
    oracle.threads(cores)
    s = pb.subs[0]
    n_all = s.pde_x.shape[0]
    frac_obs = s.obs_x.shape[0] / max(n_all, 1)
    frac_gh = s.gh_x.shape[0] / max(n_all, 1)

    def run(n, reps=1):
        no, ng = int(round(n * frac_obs)), int(round(n * frac_gh))
        t0 = time.perf_counter()
        for _ in range(reps):
            L, g = oracle.loss_grad(pb.dim, pb.width, pb.depth, pb.nu, pb.lam, s.theta,
                                    is_master=s.is_master, pde_x=s.pde_x[:n], obs_x=s.obs_x[:no],
                                    obs_u=s.obs_u[:no], gh_x=s.gh_x[:ng], gh_up=s.gh_up[:ng],
                                    gh_kind=s.gh_kind[:ng], anc_x=s.anc_x, anc_p=s.anc_p)
            if pb.clip_norm > 0:
                g, _ = oracle.clip_grad(g, pb.clip_norm)
            oracle.adam(s.theta, np.zeros(g.size), np.zeros(g.size), g, 1, lr=pb.lr)
        return time.perf_counter() - t0, no, ng

    def measure(budget):
        n0 = min(n_all, 256)
        t0, _, _ = run(n0)
        n = int(min(n_all, max(n0, n0 * budget / max(t0, 1e-3))))
        reps = 1
        if n == n_all:
            t_all, _, _ = run(n_all)
            reps = max(1, int(round(budget / max(t_all, 1e-3))))
        dt, no, ng = run(n, reps)
        return (n * reps / dt,
                (f"first {n} of {n_all} collocation points of subdomain 0 with {no} observation and "
                 f"{ng} ghost points (same per-point mix), {reps} step(s): FP64 loss, gradient and "
                 f"Adam, {pb.activation} network, {dt:.1f} s"))

    oracle.set_activation(pb.activation)
    oracle.set_component_weights(pb.comp_w)
    try:
        value, sample = measure(budget_s)
        oracle.threads(1)
        v1, s1 = measure(one_core_s)
    finally:
        oracle.threads(prev)
        oracle.set_activation("tanh")
        oracle.set_component_weights(None)
    return {"value": value, "unit": "collocation pts/s", "cores": cores, "kind": "oracle", "sample": sample,
            "affinity_cores": n_aff,
            "threads_note": "OpenMP threads = cores in this process's affinity mask, capped by "
                            "OMP_NUM_THREADS when set",
            "one_core": {"value": v1, "unit": "collocation pts/s", "cores": 1, "sample": s1}}


def query_bench(seconds, seed=0, rate=200.0, budget=32 << 30, warmup_seconds=0.0):
    """The serving protocol: 16 resident 3->8x100->3 networks, open-loop
    Poisson arrivals at `rate`, 1-200,000 points per request (log-uniform),
    warmup_seconds of untimed traffic of the same kind, then `seconds` timed."""
    import workloads as wl
    from paper_2602_15883_amd.serve import QueryServer, Request, latency_stats, serving_context
    boxes, thetas = wl.serving_nets(seed, width=100, depth=8)
    ctx = serving_context(boxes, thetas, 100, 8, device="cuda")
    n_req = max(1, int(seconds * rate))
    arrivals, sizes = wl.query_requests(seed, n_req, rate_hz=rate)
    rng = np.random.default_rng([seed, 9])
    pool = wl.query_points(rng, int(min(sizes.sum(), 4_000_000)))
    reqs, o = [], 0
    for i in range(n_req):
        n = int(sizes[i])
        if o + n > pool.shape[0]:
            o = 0
        reqs.append(Request(i, float(arrivals[i]), pool[o:o + n]))
        o += n
    srv = QueryServer(ctx, hbm_budget_bytes=budget, n_streams=4, max_batch_points=1 << 20)
    # warm-up: a few requests through the same path, then an open-loop stream
    # of the same kind for warmup_seconds (untimed)
    warm = [Request(-1 - i, 0.0, pool[:1000 * (i + 1)]) for i in range(4)]
    if warmup_seconds > 0:
        n_w = int(warmup_seconds * rate)
        wa, ws = wl.query_requests(seed + 1000, n_w, rate_hz=rate)
        ow = 0
        for i in range(n_w):
            m = int(ws[i])
            if ow + m > pool.shape[0]:
                ow = 0
            warm.append(Request(-100 - i, float(wa[i]), pool[ow:ow + m]))
            ow += m
    srv.run(warm)
    srv.busy_intervals.clear()
    srv.deferred = 0
    wall = srv.run(reqs)
    st = latency_stats(reqs)
    busy = srv.busy_seconds()
    ctx.close()
    st.update({"points_per_s": st["points"] / wall, "wall_s": wall, "rate_hz": rate,
               "warmup_s": warmup_seconds, "window_s": seconds,
               "gpu_busy_frac": busy / wall, "server_device_bytes": srv.device_bytes,
               "deferred": srv.deferred,
               "workload": "16 x 2d 3->8x100->3, Poisson 200 req/s, "
               "1-200000 pts/request log-uniform, 4 streams, 32 GB budget"})
    return st


def eval_bench(seed=0, n_snap=40, per_snap=50_000, reps=5):
    """Timing of the evaluation post-processing (section 3) over the resident
    serving networks: n_snap snapshots of per_snap points.  The networks are
    untrained, so the error values are not results and are not reported."""
    import torch

    import workloads as wl
    from paper_2602_15883_amd.serve import serving_context
    boxes, thetas = wl.serving_nets(seed, width=100, depth=8)
    masters = [s % 4 == 0 for s in range(len(thetas))]
    n = n_snap * per_snap
    ctx = serving_context(boxes, thetas, 100, 8, device="cuda", masters=masters,
                          max_query_points=max(n, 1 << 22))
    rng = np.random.default_rng([seed, 11])
    x = wl.uniform(rng, n, (0, 0, 0), (8, 2, 4))
    x[:, 2] = np.repeat((np.arange(n_snap) + 0.5) * 4.0 / n_snap, per_snap)
    u, v, p = wl.taylor_green(x[:, 0].astype(np.float64), x[:, 1], x[:, 2])
    ref = np.stack([u, v, p], axis=1).astype(np.float32)
    off = np.arange(n_snap + 1, dtype=np.int64) * per_snap
    xd, rd = torch.from_numpy(x).cuda(), torch.from_numpy(ref).cuda()
    ctx.evaluate(xd, rd, off, [1.0, 1.0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.evaluate(xd, rd, off, [1.0, 1.0])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ctx.close()
    return {"ms": dt * 1e3, "points": n, "snapshots": n_snap, "points_per_s": n / dt,
            "timing_only": True,
            "workload": "16 x 2d 3->8x100->3 (untrained: timing only), masters = first strip, "
                        f"{n_snap} snapshots x {per_snap} points"}


def launch_shape(args, pb, name, P):
    """Launch shape: command line, tuning now, the tuning table, or the
    library default."""
    from paper_2602_15883_amd import tune
    n_pde = pb.n_pde
    key = tune.tune_key(pb.dim, pb.width, pb.depth, len(pb.subs), n_pde, pb.activation)
    if args.tile_points:
        return {"tile_points": args.tile_points}, "command line"
    if args.tune:
        shape = tune.autotune(lambda **c: P.context_from_problem(pb, device="cuda:0", graph=False, **c),
                              pb.dim, pb.width, pb.depth, len(pb.subs), n_pde, steps=3,
                              cache=args.tune_out is not None, force=True, path=args.tune_out,
                              activation=pb.activation)
        return shape, "tuned now"
    e = tune.lookup(key)
    if e:
        return tune.shape_of(e), "tuning table"
    return {}, "library default"


def time_workload(args, name, steps, warmup, per_subdomain=False):
    """Graph replays of the whole step (the throughput), HIP events around
    each replay (the per-step distribution), and the fused kernel's own
    duration from events tied to its dispatches (the roofline); optionally the
    same kernel launched once per subdomain."""
    import torch

    import paper_2602_15883_amd as P
    pb = make_problem(name, args.seed)
    flops, fc = step_flops(pb)
    n_pde = pb.n_pde
    shape, shape_src = launch_shape(args, pb, name, P)
    ctx = P.context_from_problem(pb, device="cuda:0", graph=True, **shape)
    info = ctx.launch_info()

    # ---- throughput: graph replays of the whole step
    for t in range(1, warmup + 1):
        ctx.step(t)
    torch.cuda.synchronize()
    t_begin = time.perf_counter()
    for t in range(warmup + 1, warmup + steps + 1):
        ctx.step(t)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_begin
    ms_per_step = elapsed / steps * 1e3
    loss = ctx._loss.cpu().numpy()
    finite = bool(np.all(np.isfinite(loss)))

    # ---- a second pass, interleaving two measurements so that both see the
    # same clocks: HIP events around each graph replay (the per-step
    # distribution of the whole step: prep, fused kernel, reduction, Adam),
    # and, for the roofline, the fused kernel's own duration from HIP events
    # tied to its dispatch (start and end time stamps of the kernel itself)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    base_t = warmup + steps
    ctx.kernel_time()
    for k, (e0, e1) in enumerate(evs):
        e0.record()
        ctx.step(base_t + 2 * k + 1)
        e1.record()
        ctx.step(base_t + 2 * k + 2, time_kernel=True)
    torch.cuda.synchronize()
    k_ms, k_n = ctx.kernel_time()
    k_avg_ms = k_ms / max(k_n, 1)
    st = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    step_ms = {"p10": float(np.percentile(st, 10)), "p50": float(np.median(st)),
               "p90": float(np.percentile(st, 90)), "steps": int(st.size)}
    res = {"pb": pb, "name": name, "flops": flops, "fc": fc, "n_pde": n_pde, "info": info,
           "shape_src": shape_src, "ms_per_step": ms_per_step, "value": n_pde * steps / elapsed,
           "step_ms": step_ms, "kernel_ms": k_avg_ms, "launches": k_n, "finite": finite,
           "achieved": flops / (k_avg_ms * 1e-3) / 1e12}
    faces = [(a, b, first, count) for a, sd in enumerate(pb.subs) for (b, _k, first, count) in sd.faces]
    if faces:
        # on-device ghost-target exchange (value forward of every neighbour on
        # its faces, anchor subtraction for master senders), HIP events
        targets = [sd.gh_up if sd.gh_up.numel() else None for sd in ctx.subs]
        ctx.exchange(faces, pb.x_anc, targets)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            ctx.exchange(faces, pb.x_anc, targets)
        e1.record()
        torch.cuda.synchronize()
        n_gh = sum(c for (_a, _b, _f, c) in faces)
        ms = e0.elapsed_time(e1) / steps
        res["exchange"] = {"ms": ms, "ghost_points": n_gh, "faces": len(faces),
                           "points_per_s": n_gh / (ms * 1e-3)}
    if per_subdomain and len(pb.subs) > 1:
        # grouped and plain launches alternate, so both see the same clocks
        base_t = warmup + 4 * steps
        ctx.kernel_time()
        g_sum = p_sum = 0.0
        for k in range(steps):
            ctx.step(base_t + 2 * k + 1, time_kernel=True)
            g_sum += ctx.kernel_time()[0]
            ctx.step(base_t + 2 * k + 2, time_kernel=True, per_subdomain=True)
            p_sum += ctx.kernel_time()[0]
        grouped, plain = g_sum / steps, p_sum / steps
        res["grouped_vs_plain"] = {
            "workload": WORKLOADS[name], "n_sub": len(pb.subs), "n_pde": n_pde,
            "grouped_kernel_ms": grouped, "plain_launches_ms": plain, "speedup": plain / grouped,
            "grouped_step_ms": ms_per_step, "grouped_pts_per_s": res["value"],
            "grouped_frac": res["achieved"] / PEAK_FP32_MFMA_TFLOPS,
            "note": "kernel spans from dispatch-tied HIP events: one grouped persistent launch vs "
                    f"{len(pb.subs)} plain launches of the same kernel in a row on one stream"}
    ctx.close()
    return res


def summary(res):
    """A compact record of one timed workload (for the extra keys)."""
    return {"workload": WORKLOADS[res["name"]], "value": res["value"], "unit": "collocation pts/s",
            "ms_per_step": res["ms_per_step"], "kernel_ms": res["kernel_ms"],
            "achieved_tflops": res["achieved"], "frac": res["achieved"] / PEAK_FP32_MFMA_TFLOPS,
            "gflop_per_step": res["flops"] / 1e9, "tile_points": res["info"]["tile_points"],
            "workgroups": res["info"]["n_wg"], "traffic": traffic_from_profiles(res["name"]),
            "losses_finite": res["finite"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="config4", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tile-points", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--query-seconds", type=float, default=30.0)
    ap.add_argument("--query-warmup", type=float, default=5.0,
                    help="seconds of untimed Poisson traffic before the timed query window")
    ap.add_argument("--no-query", action="store_true")
    ap.add_argument("--no-eval", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra legs (the 2D working-size workload and the grouped-vs-plain "
                         "comparison on the 16-subdomain workload)")
    ap.add_argument("--tune", action="store_true",
                    help="time every launch shape (points per tile, workgroups per CU) first and "
                         "use the fastest; --tune-out FILE records it in a tuning table")
    ap.add_argument("--tune-out", default=None)
    ap.add_argument("--per-subdomain", action="store_true",
                    help="also time one plain launch per subdomain (grouped vs plain) on --workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain elementwise copy of 256 MiB (reads and writes "
                         "268435456 bytes) three times, for scaling HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(subdomains are grouped inside one launch on one device)", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    print(f"bench: {args.workload}, {args.steps} steps after {args.warmup} warm-up", file=sys.stderr, flush=True)
    r = time_workload(args, args.workload, args.steps, args.warmup, per_subdomain=args.per_subdomain)
    pb = r["pb"]
    traffic = traffic_from_profiles(args.workload)
    k_s = r["kernel_ms"] * 1e-3
    alg_bytes = algorithmic_bytes(pb)
    out = {
        "metric": "collocation pts/s per fused train step (fwd+2nd-deriv+bwd); query p50/p99 ms",
        "value": r["value"],
        "unit": "collocation pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "step_ms": r["step_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "dim": pb.dim, "width": pb.width,
                   "depth": pb.depth, "n_sub": len(pb.subs), "n_pde": r["n_pde"],
                   "n_value_points": int(sum(s.obs_x.shape[0] + s.gh_x.shape[0] + s.anc_x.shape[0]
                                             for s in pb.subs)),
                   "gflop_per_step": r["flops"] / 1e9, "tile_points": r["info"]["tile_points"],
                   "launch_shape": r["shape_src"],
                   "activation": pb.activation,
                   "workgroups": r["info"]["n_wg"], "graph": True, "losses_finite": r["finite"]},
        "roofline": {"bound": "mfma", "achieved": r["achieved"], "peak": PEAK_FP32_MFMA_TFLOPS,
                     "unit": "TFLOP/s", "frac": r["achieved"] / PEAK_FP32_MFMA_TFLOPS,
                     "traffic": traffic, "kernel": "step_kernel", "kernel_ms": r["kernel_ms"],
                     "kernel_timing": "HIP events tied to the kernel's dispatch (start and end "
                                      "time stamps), averaged over the launches",
                     "launches_timed": r["launches"], "flop_per_launch": r["flops"],
                     "flop_per_collocation_point": r["fc"],
                     "hbm": {"algorithmic_bytes": alg_bytes,
                             "algorithmic_gbs": alg_bytes / k_s / 1e9,
                             "measured_gbs": (traffic / k_s / 1e9) if traffic else None,
                             "peak_gbs": PEAK_HBM_GBS,
                             "measured_frac": (traffic / k_s / 1e9 / PEAK_HBM_GBS) if traffic else None}},
    }
    if "exchange" in r:
        out["exchange"] = r["exchange"]
    if "grouped_vs_plain" in r:
        out["grouped_vs_plain"] = r["grouped_vs_plain"]
    del r
    if not args.no_extra:
        steps_x = max(10, min(args.steps, 50))
        warm_x = max(3, min(args.warmup, 10))
        if args.workload != "config2":
            print("bench: config2 (extra leg)", file=sys.stderr, flush=True)
            out["config2"] = summary(time_workload(args, "config2", steps_x, warm_x))
        if args.workload != "config3":
            print("bench: config3 grouped vs plain (extra leg)", file=sys.stderr, flush=True)
            r3 = time_workload(args, "config3", steps_x, warm_x, per_subdomain=True)
            out["grouped_vs_plain"] = r3["grouped_vs_plain"]
            out["exchange"] = r3["exchange"]
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pb)
    if not args.no_query:
        print(f"bench: query server ({args.query_warmup:g} s warm-up, {args.query_seconds:g} s)",
              file=sys.stderr, flush=True)
        out["query"] = query_bench(args.query_seconds, seed=args.seed, warmup_seconds=args.query_warmup)
    if not args.no_eval:
        out["evaluate"] = eval_bench(seed=args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
