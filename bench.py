"""Benchmark: large-number add/sub/mul on one MI355X.

One JSON line on stdout.  The headline `value` is add/sub operand throughput on
the batched workload (2^20 pairs of 64-limb operands): a step is one batched add
plus one batched subtract over that batch, inputs resident in HBM, and `value` is
the algorithmic bytes of the step (24 B per limb: two operands read, one result
written, plus 8 B per pair of carry/borrow) divided by the step time.  The other
workloads are measured in the same run and reported under "workloads": 4-limb
pairs (latency, graph replay), one 2^26-limb pair (look-back scan), 2^16 ragged
multiply pairs (persistent launch, graph replay, mad vs MFMA), 64 products of
16384-limb operands (mad vs MFMA) and a square-size sweep for the mad/MFMA
crossover.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
INT8_PEAK_TOPS = 5000.0        # MI355X dense int8 MFMA, published (ops = 2 x MAC)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "flat_scan_c2_traffic.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(per_launch_bytes_alg: float):
    """HBM bytes per launch of the scan kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    from paper_2604_21566_amd.rocprof_summary import kernel_source_hash
    if vals.get("kernel_src_sha") != kernel_source_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def ci95(ts) -> float:
    """Half-width of the 95% confidence interval of the mean of the samples ts
    (Student t with n - 1 degrees of freedom)."""
    n = len(ts)
    if n < 2:
        return float("nan")
    try:
        from scipy.stats import t as student_t
        q = float(student_t.ppf(0.975, n - 1))
    except ImportError:
        q = 1.96
    return q * float(np.std(ts, ddof=1)) / np.sqrt(n)


REPS = 20   # timed repetitions of each secondary workload (mean and 95% CI), after warm-ups


def gpu_time(fn, reps: int, warmup: int = 1):
    """Mean and per-rep ms of fn() on torch's current stream (HIP events)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in evs:
        e0.record()
        fn()
        e1.record()
    torch.cuda.synchronize()
    ts = [e0.elapsed_time(e1) for e0, e1 in evs]
    return float(np.mean(ts)), ts


def queued_time(torch, fn, k: int, reps: int = 20):
    """Median device-side ms per fn() when k calls sit in the stream behind a spin
    kernel (about 1 ms): the events then time the GPU's work and its dispatch gaps,
    not the host's enqueue.  None when this torch has no spin kernel (torch.cuda._sleep)."""
    if not hasattr(torch.cuda, "_sleep"):
        return None
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        torch.cuda._sleep(3_000_000)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / k)
    return float(np.median(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tuning", default=None, help="tuning JSON written by bn_autotune")
    ap.add_argument("--only", default=None,
                    help="comma-separated secondary workloads to run alone (copy, c1, c3, c4, c4auto: the "
                         "full C4 batch in its automatic plan only, c5: the schoolbook forms, c5k: Karatsuba "
                         "levels on C5, crossover); prints their figures only, for profiling runs")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a plain 512 MiB device-to-device copy 3 times (the known-size reference "
                         "for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_21566_amd as bn
    from paper_2604_21566_amd import workloads as wl

    torch.cuda.set_device(0)
    # compute calls never allocate: every workload's workspace is reserved before it runs
    ctx = bn.bn_create(0, tuning=args.tuning)
    D = bn.to_device
    if args.only:
        res = extra_workloads(ctx, bn, wl, torch, only=set(args.only.split(",")))
        bn.bn_destroy(ctx)
        print(json.dumps({"workloads": res}), flush=True)
        return

    # ------------------------------------------------------------ headline: c2 add + sub
    n, npairs = 64, 1 << 20
    N = n * npairs
    log("generating c2 operands")
    a_add, b_add = wl.c2("add", npairs=npairs, n=n)
    a_sub, b_sub = wl.c2("sub", npairs=npairs, n=n)
    ta, tb, sa, sb = D(a_add), D(b_add), D(a_sub), D(b_sub)
    tr = torch.empty(N, dtype=torch.int64, device="cuda")
    tc = torch.empty(npairs, dtype=torch.int64, device="cuda")
    bytes_per_launch = 24.0 * N + 8.0 * npairs

    bn.bn_reserve_for(ctx, bn.BN_OP_ADDSUB, n, 0, npairs)

    def add():
        bn.bn_add_n_batch(ctx, tr, ta, tb, n, npairs, tc)

    def sub():
        bn.bn_sub_n_batch(ctx, tr, sa, sb, n, npairs, tc)

    if args.calibrate:
        for _ in range(3):
            tr.copy_(ta)
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        add()
        sub()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[3 * k].record()
        add()
        ev[3 * k + 1].record()
        sub()
        ev[3 * k + 2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = []
    step_ms = []
    for k in range(args.steps):
        launch_ms += [ev[3 * k].elapsed_time(ev[3 * k + 1]), ev[3 * k + 1].elapsed_time(ev[3 * k + 2])]
        step_ms.append(ev[3 * k].elapsed_time(ev[3 * k + 2]))
    ms_per_step = wall * 1e3 / args.steps
    value = 2 * bytes_per_launch / (ms_per_step * 1e-3) / 1e9
    avg_launch = float(np.mean(launch_ms))
    achieved = bytes_per_launch / (avg_launch * 1e-3) / 1e9
    traffic = measured_traffic(bytes_per_launch)
    workloads_latch = bn.bn_check(ctx)
    log(f"c2: step {ms_per_step:.4f} ms, kernel {avg_launch:.4f} ms, {achieved:.1f} GB/s")
    workloads = {"c2_addsub": {"GBps_add": bytes_per_launch / (np.mean(launch_ms[0::2]) * 1e-3) / 1e9,
                               "GBps_sub": bytes_per_launch / (np.mean(launch_ms[1::2]) * 1e-3) / 1e9,
                               "kernel_ms_mean": avg_launch, "kernel_ms_min": float(np.min(launch_ms)),
                               "ci95_ms": float(1.96 * np.std(launch_ms) / np.sqrt(len(launch_ms))),
                               "lookback_self_help_latch": workloads_latch}}

    # ------------------------------------------------------------ CPU oracle baseline (same workload)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_oracle_baseline(a_add, b_add, a_sub, b_sub, n, npairs, bytes_per_launch)
        workloads["cpu_dot_c2"] = cpu_dot_baseline(a_add, b_add, a_sub, b_sub, n, npairs, bytes_per_launch)
    del a_sub, b_sub, sa, sb

    if not args.quick:
        workloads.update(extra_workloads(ctx, bn, wl, torch))
        workloads["c2_addsub"]["frac_of_measured_copy"] = achieved / workloads["hbm_copy_GBps"]
        workloads["c2_addsub"]["frac_of_nt_copy"] = achieved / workloads["measured_rates"]["nt_copy_GBps"]

    bn.bn_destroy(ctx)
    out = {
        "metric": "add/sub operand GB/s vs HBM peak; mul products/s by size, MFMA vs plain form",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "batched add+sub: 2^20 pairs x 64 u64 limbs (10% adversarial carry runs)",
                   "pairs": npairs, "limbs_per_operand": n, "bytes_per_step": 2 * bytes_per_launch},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
        "cpu_baseline": cpu,
        "workloads": workloads,
    }
    print(json.dumps(out), flush=True)


def host_threads() -> int:
    """Host cores this process may use (at most 16, the CPU share of one GPU)."""
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(16, os.cpu_count() or 1))


def cpu_oracle_baseline(a_add, b_add, a_sub, b_sub, n, npairs, bytes_per_launch):
    """The CPU oracle on the same 2^20 x 64-limb add + sub step: pairs split into
    contiguous chunks, one oracle call per chunk on a pool of threads (the oracle's
    C loops run without the interpreter lock), and once more on one thread."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle._load()
    threads = host_threads()
    bounds = np.linspace(0, npairs, threads + 1).astype(np.int64)

    def step(pool):
        if pool is None:
            oracle.add_batch(a_add, b_add, n)
            oracle.sub_batch(a_sub, b_sub, n)
            return
        jobs = []
        for f, x, y in ((oracle.add_batch, a_add, b_add), (oracle.sub_batch, a_sub, b_sub)):
            for p0, p1 in zip(bounds[:-1], bounds[1:]):
                jobs.append(pool.submit(f, x[p0 * n:p1 * n], y[p0 * n:p1 * n], n))
        for j in jobs:
            j.result()

    def timed(pool, budget_s, max_reps):
        reps, t0 = 0, time.perf_counter()
        while True:
            step(pool)
            reps += 1
            if time.perf_counter() - t0 > budget_s or reps >= max_reps:
                return (time.perf_counter() - t0) / reps, reps

    log(f"timing the CPU oracle on the full c2 batch (add + sub), {threads} threads and one thread")
    with ThreadPoolExecutor(threads) as pool:
        step(pool)
        dt_mt, reps_mt = timed(pool, 8.0, 40)
    dt_1, reps_1 = timed(None, 8.0, 20)
    return {"value": 2 * bytes_per_launch / dt_mt / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"full 2^20 x 64-limb batch, add + sub, {reps_mt} repetitions, pairs split over "
                      f"{threads} threads",
            "ms_per_step": dt_mt * 1e3,
            "one_thread": {"value": 2 * bytes_per_launch / dt_1 / 1e9, "ms_per_step": dt_1 * 1e3,
                           "repetitions": reps_1},
            "host_cpu": host_cpu_model()}


def cpu_dot_baseline(a_add, b_add, a_sub, b_sub, n, npairs, bytes_per_launch):
    """The paper's own CPU method (DoT add/sub with AVX-512 or AVX2, and the scalar
    carry chain) on the same full 2^20 x 64-limb add + sub step, host arrays: context
    for the GPU rate, not the oracle."""
    from paper_2604_21566_amd import host as H
    threads = host_threads()
    r = np.empty_like(a_add)
    c = np.empty(npairs, np.uint64)

    def rate(isa, nthreads, budget_s=2.0, max_reps=20):
        def step():
            H.bnh_add_n_batch(r, a_add, b_add, n, npairs, c, isa, nthreads)
            H.bnh_sub_n_batch(r, a_sub, b_sub, n, npairs, c, isa, nthreads)
        step()
        reps, t0 = 0, time.perf_counter()
        while True:
            step()
            reps += 1
            if time.perf_counter() - t0 > budget_s or reps >= max_reps:
                dt = (time.perf_counter() - t0) / reps
                return {"GBps": 2 * bytes_per_launch / dt / 1e9, "ms_per_step": dt * 1e3, "repetitions": reps}

    best = H.bnh_isa_best()
    log(f"timing host DoT ({H.ISA_NAMES[best]}) on the full c2 batch, {threads} threads and one thread per ISA")
    out = {"isa": H.ISA_NAMES[best], "threads": threads, "host_cpu": host_cpu_model(),
           "all_threads": rate(best, threads)}
    for isa in range(best + 1):
        out[f"one_thread_{H.ISA_NAMES[isa]}"] = rate(isa, 1)
    # cache-resident operands (16384 limbs = 384 KiB per call over r, a, b; one thread):
    # the arithmetic itself, where the paper's SIMD-versus-scalar comparison lives.  The
    # pointers are converted once and the cost of an empty call is subtracted.
    import ctypes
    g = np.random.default_rng(1)
    L = H.lib()
    cached = {}
    for m in (8, 64, 1024):
        np_ = 16384 // m
        x = g.integers(0, 2 ** 64 - 1, m * np_, dtype=np.uint64, endpoint=True)
        y = g.integers(0, 2 ** 64 - 1, m * np_, dtype=np.uint64, endpoint=True)
        z = np.empty_like(x)
        cc = np.empty(np_, np.uint64)
        px, py, pz, pc = (v.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)) for v in (x, y, z, cc))

        def per_call(isa, pairs, reps=400):
            L.bnh_add_n_batch(pz, px, py, m, pairs, pc, isa, 1)
            t0 = time.perf_counter()
            for _ in range(reps):
                L.bnh_add_n_batch(pz, px, py, m, pairs, pc, isa, 1)
            return (time.perf_counter() - t0) / reps

        row = {}
        for isa in range(best + 1):
            dt = min(per_call(isa, np_) for _ in range(3)) - min(per_call(isa, 0) for _ in range(3))
            row[f"{H.ISA_NAMES[isa]}_ns_per_limb"] = dt / (m * np_) * 1e9
        row["simd_speedup_over_scalar"] = row["scalar_ns_per_limb"] / row[f"{H.ISA_NAMES[best]}_ns_per_limb"]
        cached[f"{m}_limbs"] = row
    out["cache_resident_add_one_thread"] = cached
    return out


def host_cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def extra_workloads(ctx, bn, wl, torch, only=None):
    """Secondary workloads (all, or those named in `only`)."""
    D = bn.to_device
    res = {}
    s = torch.cuda.Stream()

    # ---- measured HBM reference: a plain 512 MiB device-to-device copy
    if only is None or "copy" in only:
        src = torch.empty(1 << 26, dtype=torch.int64, device="cuda").random_()
        dst = torch.empty_like(src)
        ms, _ = gpu_time(lambda: dst.copy_(src), 20, 3)
        res["hbm_copy_GBps"] = 2.0 * src.numel() * 8 / (ms * 1e-3) / 1e9
        del src, dst

    # ---- c1: 1088 pairs of 4 limbs, graph replay (latency)
    if only is None or "c1" in only:
        log("c1")
        c1 = {}
        for op in ("add", "sub", "mul_mad", "mul_mfma"):
            a, b = wl.c1("sub" if op == "sub" else "add")
            ta, tb = D(a), D(b)
            if op.startswith("mul"):
                tr = torch.empty(1088 * 8, dtype=torch.int64, device="cuda")
                g = bn.bn_graph_capture_batch(ctx, 2, tr, ta, tb, 4, 4, 1088, None, op[4:], s)
            else:
                tr = torch.empty(1088 * 4, dtype=torch.int64, device="cuda")
                tc = torch.empty(1088, dtype=torch.int64, device="cuda")
                g = bn.bn_graph_capture_batch(ctx, 0 if op == "add" else 1, tr, ta, tb, 4, 0, 1088, tc, 0, s)
            with torch.cuda.stream(s):
                ms, _ = gpu_time(lambda: bn.bn_graph_launch(g, s), 50, 5)
            bn.bn_graph_destroy(g)
            c1[op + "_us"] = ms * 1e3
            c1[op + "_pairs_per_s"] = 1088 / (ms * 1e-3)
            # the same call launched directly
            if op.startswith("mul"):
                fn = lambda: bn.bn_mul_n_batch(ctx, tr, ta, tb, 4, 4, 1088, op[4:])
            else:
                f = bn.bn_add_n_batch if op == "add" else bn.bn_sub_n_batch
                fn = lambda: f(ctx, tr, ta, tb, 4, 1088, tc)
            ms, _ = gpu_time(fn, 50, 5)
            c1[op + "_direct_us"] = ms * 1e3
            # device side: the same work queued behind a spin kernel, so that the host's
            # enqueue time is hidden; 8 back to back per event pair.  Then 8 calls
            # captured into one graph (the runtime's per-graph launch cost shared by 8).
            g = bn.bn_graph_capture_batch(ctx, 2, tr, ta, tb, 4, 4, 1088, None, op[4:], s) if op.startswith("mul") \
                else bn.bn_graph_capture_batch(ctx, 0 if op == "add" else 1, tr, ta, tb, 4, 0, 1088, tc, 0, s)
            us = lambda ms, per=1: None if ms is None else ms * 1e3 / per
            with torch.cuda.stream(s):
                c1[op + "_device_us"] = us(queued_time(torch, lambda: bn.bn_graph_launch(g, s), 8))
                c1[op + "_direct_device_us"] = us(queued_time(torch, fn, 8))
            bn.bn_graph_destroy(g)
            torch.cuda.synchronize()
            ref = tr.clone()
            tr.zero_()
            g8 = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g8, stream=s, capture_error_mode="thread_local"):
                for _ in range(8):
                    fn()
            with torch.cuda.stream(s):
                c1[op + "_graph8_us_per_batch"] = us(queued_time(torch, g8.replay, 1), 8)
                ms, _ = gpu_time(g8.replay, 50, 5)
            c1[op + "_graph8_alone_us_per_batch"] = ms * 1e3 / 8
            torch.cuda.synchronize()
            if not torch.equal(tr, ref):
                raise SystemExit(f"c1 {op}: the 8-call graph's output differs from the direct launch's")
            del g8
        res["c1"] = c1

    # ---- c3: one pair of 2^26 limbs (random with runs, and the all-propagate worst case)
    if only is None or "c3" in only:
        log("c3")
        c3 = {}
        n3 = 1 << 26
        bn.bn_reserve_for(ctx, bn.BN_OP_ADDSUB, n3, 0, 1)
        tr = torch.empty(n3, dtype=torch.int64, device="cuda")
        tc = torch.empty(1, dtype=torch.int64, device="cuda")
        defer_default = bn.bn_get_param(ctx, "addsub.defer_tiles")
        c3["defer_tiles"] = defer_default
        for op in ("add", "sub"):
            for worst in (False, True):
                a, b = wl.c3(op, n=n3, worst=worst)
                ta, tb = D(a), D(b)
                f = bn.bn_add if op == "add" else bn.bn_sub
                key = f"{op}{'_worst' if worst else ''}"
                # the default (all-propagate tiles deferred to a fill pass at this size)
                # and the form in which every tile waits for its look-back
                for form, dt in (("", defer_default), ("_waiting", 0)):
                    bn.bn_set_param(ctx, "addsub.defer_tiles", dt)
                    ms, ts = gpu_time(lambda: f(ctx, tr, ta, tb, tc), REPS, 2)
                    c3[key + form + "_GBps"] = 24.0 * n3 / (ms * 1e-3) / 1e9
                    c3[key + form + "_ms"] = ms
                    c3[key + form + "_ci95_ms"] = ci95(ts)
                # look-back distances of one more (untimed) run of the waiting form
                # (deferred launches record none)
                bn.bn_lookback_stats(ctx)
                bn.bn_set_param(ctx, "debug.flags", 2)
                f(ctx, tr, ta, tb, tc)
                h = bn.bn_lookback_stats(ctx)
                bn.bn_set_param(ctx, "debug.flags", 0)
                bn.bn_set_param(ctx, "addsub.defer_tiles", defer_default)
                top = max([k for k, v in enumerate(h) if v] or [0])
                c3[key + "_waiting_lookback_hist_log2"] = h[:top + 1]
                del ta, tb
        res["c3"] = c3

    # ---- c4: 2^16 ragged products, persistent launch captured in a graph
    if only is None or "c4" in only or "c4auto" in only:
        log("c4")
        a, b, desc, rsz = wl.c4()
        work = float((desc[:, 3].astype(np.float64) * desc[:, 4].astype(np.float64)).sum())
        ta, tb = D(a), D(b)
        tr = torch.empty(rsz, dtype=torch.int64, device="cuda")
        c4 = {"limb_products": work}
        auto_only = only is not None and "c4" not in only
        for form in (("auto",) if auto_only else ("mad", "mfma", "auto")):
            plan = bn.bn_plan_mul_ragged(ctx, desc, form)
            g = bn.bn_graph_capture_mul_ragged(ctx, plan, tr, ta, tb, s)
            with torch.cuda.stream(s):
                ms, ts = gpu_time(lambda: bn.bn_graph_launch(g, s), REPS, 3)
            bn.bn_graph_destroy(g)
            bn.bn_plan_destroy(plan)
            c4[f"{form}_ms"] = ms
            c4[f"{form}_ci95_ms"] = ci95(ts)
            c4[f"{form}_limb_products_per_s"] = work / (ms * 1e-3)
            c4[f"{form}_pairs_per_s"] = len(desc) / (ms * 1e-3)
        # the same batch launched directly (no graph)
        plan = bn.bn_plan_mul_ragged(ctx, desc, "auto")
        ms, ts = gpu_time(lambda: bn.bn_mul_ragged(ctx, plan, tr, ta, tb), REPS, 3)
        bn.bn_plan_destroy(plan)
        c4["auto_direct_ms"] = ms
        c4["auto_direct_ci95_ms"] = ci95(ts)
        if auto_only:
            res["c4"] = c4
    if only is None or "c4" in only:
        # per size bucket (larger operand length in [lo, 2 lo), the last one [64, 128]: the
        # 128-limb operands alone are a few hundred pairs, too few to time), each bucket
        # its own graph
        big = np.maximum(desc[:, 3], desc[:, 4])
        buckets = {}
        crossover = None
        lo = 4
        while lo <= 64:
            sel = desc[(big >= lo) & (big < 2 * lo)] if lo < 64 else desc[big >= lo]
            if len(sel):
                w = float((sel[:, 3].astype(np.float64) * sel[:, 4].astype(np.float64)).sum())
                row = {"pairs": int(len(sel)), "limb_products": w}
                for form in ("mad", "mfma"):
                    plan = bn.bn_plan_mul_ragged(ctx, sel, form)
                    g = bn.bn_graph_capture_mul_ragged(ctx, plan, tr, ta, tb, s)
                    with torch.cuda.stream(s):
                        ms, ts = gpu_time(lambda: bn.bn_graph_launch(g, s), REPS, 3)
                    bn.bn_graph_destroy(g)
                    bn.bn_plan_destroy(plan)
                    row[f"{form}_us"] = ms * 1e3
                    row[f"{form}_ci95_us"] = ci95(ts) * 1e3
                    row[f"{form}_limb_products_per_s"] = w / (ms * 1e-3)
                # the smallest bucket from which MFMA is faster in every larger bucket
                if row["mfma_limb_products_per_s"] > row["mad_limb_products_per_s"]:
                    crossover = lo if crossover is None else crossover
                else:
                    crossover = None
                buckets[f"{lo}-{2 * lo - 1 if lo < 64 else 128}"] = row
            lo *= 2
        c4["buckets_by_longer_operand_limbs"] = buckets
        c4["mfma_faster_from_bucket"] = crossover
        res["c4"] = c4

    # ---- measured ceilings of the two multiplication forms' inner operations
    if only is None or "c5" in only:
        mac_rate, mfma_rate, copy_rate = bn.bn_probe_rates(ctx)
        res["measured_rates"] = {"mac96_per_s": mac_rate, "mfma_i8_ops_per_s": mfma_rate,
                                 "nt_copy_GBps": copy_rate / 1e9,
                                 "mad_form_limb_products_per_s_ceiling": mac_rate / 4,
                                 "mfma_form_limb_products_per_s_ceiling": mfma_rate / 128}

    # ---- c5: 64 products of 16384-limb operands
    n5 = 16384
    c5 = None
    if only is None or "c5" in only or "c5k" in only:
        a, b = wl.c5()
        ta, tb = D(a), D(b)
        tr = torch.empty(64 * 2 * n5, dtype=torch.int64, device="cuda")
    if only is None or "c5" in only:
        log("c5")
        c5 = {"limb_products": 64.0 * n5 * n5}
        for form in ("mad", "mfma"):
            bn.bn_reserve_for(ctx, bn.BN_OP_MUL, n5, n5, 64, form)
            ms, ts = gpu_time(lambda: bn.bn_mul_n_batch(ctx, tr, ta, tb, n5, n5, 64, form), REPS, 2)
            c5[f"{form}_ms"] = ms
            c5[f"{form}_ci95_ms"] = ci95(ts)
            c5[f"{form}_limb_products_per_s"] = 64.0 * n5 * n5 / (ms * 1e-3)
            c5[f"{form}_products_per_s"] = 64 / (ms * 1e-3)
        c5["mfma_int8_TOPS"] = 2 * 64.0 * 64.0 * n5 * n5 / (c5["mfma_ms"] * 1e-3) / 1e12
        c5["mfma_frac_of_int8_peak"] = c5["mfma_int8_TOPS"] / INT8_PEAK_TOPS
        c5["mfma_frac_of_measured_int8"] = c5["mfma_int8_TOPS"] * 1e12 / mfma_rate
        c5["mad_frac_of_measured_mac96"] = c5["mad_limb_products_per_s"] * 4 / mac_rate
        c5["mfma_over_mad"] = c5["mad_ms"] / c5["mfma_ms"]
        res["c5"] = c5
    if only is None or "c5k" in only:
        # Karatsuba levels above the MFMA schoolbook kernel (same products; the rate is
        # stated in schoolbook limb products per second for comparison)
        log("c5 Karatsuba")
        kar = {}
        for levels in (1, 2, 3):
            bn.bn_reserve_for(ctx, bn.BN_OP_MUL_KARATSUBA, n5, n5, 64, "mfma", levels)
            ms, ts = gpu_time(lambda: bn.bn_mul_karatsuba_n_batch(ctx, tr, ta, tb, n5, 64, levels, "mfma"), REPS, 2)
            kar[f"levels{levels}_ms"] = ms
            kar[f"levels{levels}_ci95_ms"] = ci95(ts)
            kar[f"levels{levels}_limb_products_per_s"] = 64.0 * n5 * n5 / (ms * 1e-3)
        best = min((1, 2, 3), key=lambda l: kar[f"levels{l}_ms"])
        kar["best_levels"] = best
        kar["auto_levels"] = bn.bn_karatsuba_auto_levels(n5, bn.bn_get_param(ctx, "mul.karatsuba_limbs"))
        if c5 is not None:
            kar["best_over_schoolbook_mfma"] = c5["mfma_ms"] / kar[f"levels{best}_ms"]
            c5["karatsuba_mfma"] = kar
        else:
            res["c5_karatsuba_mfma"] = kar

    # ---- crossover sweep: square products
    if only is None or "crossover" in only:
        log("crossover sweep")
        sweep = {}
        crossover = None
        n = 4
        big = torch.empty(1 << 25, dtype=torch.int64, device="cuda").random_()
        out = torch.empty(1 << 26, dtype=torch.int64, device="cuda")
        while n <= 16384:
            # about 2^32 limb products per size (fewer where the 2^25-limb operand
            # buffer runs out), so that every size fills the device
            npairs = int(max(1, min((1 << 32) // (n * n), (1 << 25) // n)))
            row = {}
            for form in ("mad", "mfma", "auto"):
                bn.bn_reserve_for(ctx, bn.BN_OP_MUL, n, n, npairs, form)
                ms, ts = gpu_time(lambda: bn.bn_mul_n_batch(ctx, out, big, big, n, n, npairs, form), REPS, 2)
                row[form + "_limb_products_per_s"] = npairs * n * n / (ms * 1e-3)
                row[form + "_ms"] = ms
                row[form + "_ci95_ms"] = ci95(ts)
            row["pairs"] = npairs
            # the automatic form against the faster of the two (1.0: it picked the faster)
            row["auto_over_best"] = row["auto_ms"] / min(row["mad_ms"], row["mfma_ms"])
            sweep[str(n)] = row
            faster = row["mfma_limb_products_per_s"] > row["mad_limb_products_per_s"]
            if faster and crossover is None:
                crossover = n
            elif not faster:
                crossover = None
            n *= 2
        res["crossover"] = {"sweep": sweep, "mfma_faster_from_limbs": crossover,
                            "auto_over_best_max": max(r["auto_over_best"] for r in sweep.values())}

    res["lookback_self_help_latch"] = bn.bn_check(ctx)
    return res


if __name__ == "__main__":
    main()
