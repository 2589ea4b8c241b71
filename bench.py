"""Benchmark: batched FP32 multilevel W1 solves on one MI355X.

Default workload (the uniform-batch configuration): 256 pairs on a 256-grid
(257^2 nodes), each density a union of 1-5 random rectangles/disks on a 1e-4
floor, L2 ground metric, 3-level cascade (64 -> 128 -> 256), plain PDHG
(Algorithm 3) with the paper's stop rule (eq. (stop_tol), alpha = -1), FP32
iterates with FP64 reductions.  One step = one w1_solve of the whole batch,
masses already resident in HBM.

Besides the headline solves/s it reports node updates/s, the plain FP64
one-pair-at-a-time GPU path on a sample (its solves/s and the W1 agreement of
the batched FP32 results with it at 1e-4), the dominant kernel's roofline
from HIP-event timing inside the timed region, and the FP64 CPU oracle timed
on this host's cores on a bounded sample.

    python bench.py [--gpus 1] [--steps 6] [--warmup 1] [--no-cpu]
    python bench.py --ground linf       # the uniform batch under another ground metric
    python bench.py --workload uneven   # 1024 pairs, n in {64..512}, Algorithm 4
    python bench.py --workload served   # Poisson arrivals, n in {128..2048}
    python bench.py --workload single   # one 512-grid pair, both algorithms
    python bench.py --workload tolerance  # the tolerance-rule / level-count study
    python bench.py --workload cube     # d = 3, one 129^3 pair

Each workload prints one JSON line of the same layout.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "W1 solves/s + cell-updates/s, batched FP32 vs plain FP64 at rel err 1e-4"
HBM_PEAK_GBS = 8000.0
# launches timed with HIP events in the timed region: a timed dispatch ends
# with a cache flush (~6 us each), so about one launch in 8 of the tiled and
# Algorithm 2 families is timed (a pseudo-random sample) and the rest run as
# they do untimed; whole-level resident launches are all timed
TILED_TIMING_EVERY = 8
RESIDENT_FAMILIES = ("plain_resident", "prox_resident")
TIMING_NOTE = (f"HIP events on a pseudo-random sample of about 1 in {TILED_TIMING_EVERY} launches "
               "(whole-level resident launches: all); launches and ms are the sample's")


def _est_ms(kstats, k):
    """A family's summed launch time scaled from its timed sample."""
    return kstats[k]["ms"] * (1 if k in RESIDENT_FAMILIES else TILED_TIMING_EVERY)
FP32_VALU_TFLOPS = 157.3
# VALU issue rate without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9
# VALU issue cycles per node update of the plain tiled kernel's step loop
# (FP32), counted in its compiled code per region shape (width, wavefronts):
# instructions of the loop body (two steps) over the node updates a thread
# makes in it (16; 8 for the 64 x 64 region over 16 wavefronts), v_rsq_f32
# (the l_2 shrink's reciprocal square root, quarter rate) at 4 cycles
TILED_VALU_CYCLES = {
    (128, 16): {"l1": 482 / 16, "l2": (514 + 3 * 16) / 16, "linf": 626 / 16},
    (64, 8): {"l1": 470 / 16, "l2": (502 + 3 * 16) / 16, "linf": 615 / 16},
    (64, 16): {"l1": 230 / 8, "l2": (250 + 3 * 8) / 8, "linf": 308 / 8},
}
# VALU issue slots the node update itself needs (the algorithmic figure):
# flux half per component 3 (difference, times 1/h, m + mu g), dual-norm
# prox (l_1: 3 per component; l_2: |v|^2 2, test 1, rsq 4 slots, factor 1,
# select 1, scaling 2; l_inf: 14), extrapolation 2, potential half 6
# (two differences, their sum, times 1/h, minus rho, phi + tau (.))
ALG_VALU_SLOTS = {"l1": 6 + 6 + 2 + 6, "l2": 6 + 11 + 2 + 6, "linf": 6 + 14 + 2 + 6}


def measured_traffic(kernel, workload):
    """HBM bytes per useful node update of `kernel` from the committed
    counter summary (profiles/<kernel minus k_>_traffic.md, its JSON block),
    or None when that summary is missing or was taken on another version of
    the kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", kernel.replace("k_", "", 1) + "_traffic.md")
    src = os.path.join(ROOT, "paper_1810_00118_amd", "csrc", "kernels.hip")
    try:
        txt = open(path).read()
        block = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except (OSError, IndexError, ValueError):
        return None
    if block.get("kernels_hip_sha256_16") != sha or block.get("workload") != workload:
        return None
    return block


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_solve(job):
    """One FP64 oracle solve of the uniform workload (a pool worker)."""
    a, b, n, L, p, scale = job
    import oracle.w1_oracle as o
    t = time.perf_counter()
    r = o.solve(a, b, n, L=L, p=p, algo=1, stop="fpr", step_scale=scale or None,
                eps_L=o.paper_stop_tolerance(1, n, True), alpha=-1.0, max_iters=20000, check_every=10,
                return_fields=False)
    return time.perf_counter() - t, r["w1"], r["iters"]


def oracle_pool(pairs, n, L, p, scale, rounds=2):
    """The FP64 CPU oracle as it stands, one process per host core (at most
    16), each solving `rounds` pairs of the workload: solves/s of the pool.
    Runs before the process touches the GPU (the workers are forked)."""
    import multiprocessing as mp
    cores = min(16, len(os.sched_getaffinity(0)))
    jobs = [(a, b, n, L, p, scale) for a, b in pairs[:cores * rounds]]
    cores = min(cores, len(jobs))
    log(f"[bench] CPU oracle: {len(jobs)} pairs on {cores} processes")
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env:
        os.environ[k] = "1"
    t = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        out = pool.map(_oracle_solve, jobs, chunksize=1)
    wall = time.perf_counter() - t
    for k, v in env.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v
    per = [o_[0] for o_ in out]
    log(f"[bench] CPU oracle: {len(jobs) / wall:.2f} solves/s ({wall:.1f} s wall)")
    return {"value": len(jobs) / wall, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(jobs)} pairs of the workload (full {L}-level cascade each), one process per core, "
                      f"{wall:.1f} s wall; {float(np.median(per)):.1f} s per pair on one core",
            "seconds_per_pair_median": float(np.median(per)), "w1_pair0": out[0][1], "iters_pair0": out[0][2]}


def workload_pairs(count, n):
    import w1data
    return [w1data.pair_shapes(i, n=n) for i in range(count)]



FP32_MFMA_TFLOPS = 157.3


def _levels(n):
    return int(round(np.log2(n // 32))) + 1


def _mfma_roofline(kstats):
    """Dominant-kernel roofline for Algorithm 2 runs: the Poisson solves'
    DCT passes, with the flops they execute (matrix passes on the matrix
    cores, folded: 4 N^3 per solve; for N >= 1025 the FFT passes, 5 M log2 M
    per complex FFT of length M = 2N - 2, two per line pair and transform,
    plus the pre- and post-twiddles); other families by time only (the
    dominant one by its summed time scaled from the timed sample)."""
    dom = max(kstats, key=lambda k: _est_ms(kstats, k))
    st = kstats[dom]
    if dom == "dct" and st["ms"] > 0:
        ach = st["flops"] / (st["ms"] * 1e-3) / 1e12
        return {"kernel": "dct", "bound": "mfma", "achieved": ach, "peak": FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / FP32_MFMA_TFLOPS, "traffic": None, "avg_launch_ms": st["ms"] / max(st["launches"], 1),
                "launches": st["launches"]}
    return {"kernel": dom, "bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None,
            "traffic": None, "avg_launch_ms": st["ms"] / max(st["launches"], 1), "launches": st["launches"]}


def _serve_all(w1, srv, items, prm_for):
    """Submit every (n, metric, p0, p1) item, wait, return results in order."""
    tickets = [srv.submit(a, b, prm_for(n, m)) for n, m, a, b in items]
    srv.drain()
    out = []
    for t in tickets:
        r = None
        while r is None:
            r = srv.poll(t)
        out.append(r[0])
    return out


def run_uneven(args, w1):
    """Uneven batch: 1024 pairs, n in {64,128,256,512} (p = .4,.3,.2,.1), L1 for
    even pairs and L2 for odd ones, Gaussian mixtures with 2..10 components,
    FP32 Algorithm 4 with L = log2(n/32)+1 levels and the paper's stop rule;
    one step = the whole batch through the served entry points."""
    import torch
    import w1data
    P = args.pairs if args.pairs != 256 else 1024
    log(f"[bench] uneven: generating {P} pairs")
    items = [w1data.pair_uneven(i) for i in range(P)]
    dev = [(n, m, torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for n, m, a, b in items]

    def prm_for(n, m, precision=w1.FP32):
        # W1 only: the served requests keep no output fields
        return w1.params(n=n, levels=_levels(n), metric=m, algo=w1.ALGO_PROX, precision=precision,
                         stop_rule=w1.STOP_FPR, tol=0.0, alpha=-1.0, max_iters=20000, check_every=10,
                         flags=w1.FLAG_NO_FIELDS)

    srv = w1.Solver(prm_for(512, 2), capacity=P)
    for k in range(args.warmup):
        _serve_all(w1, srv, dev, prm_for)
        log(f"[bench] warmup {k} done")
    srv.profile(True, every=TILED_TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        res = _serve_all(w1, srv, dev, prm_for)
        log(f"[bench] step {k} done")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ks = srv.kernel_stats()
    srv.close()
    ups = sum(sum(it * ((n >> (len(r["iters"]) - 1 - l)) + 1) ** 2 for l, it in enumerate(r["iters"]))
              for (n, _, _, _), r in zip(dev, res))
    # every counted solve against the FP64 path of the same requests
    # (outside the timed region): a solve counts only within 1e-4
    t = time.perf_counter()
    s64all = w1.Solver(prm_for(512, 2, w1.FP64), capacity=P)
    ref_all = _serve_all(w1, s64all, dev, lambda n_, m_: prm_for(n_, m_, w1.FP64))
    s64all.close()
    rel_all = [abs(r["w1"] - q["w1"]) / abs(q["w1"]) for r, q in zip(res, ref_all)]
    good = sum(x <= 1e-4 for x in rel_all)
    log(f"[bench] FP64 reference of all {P} requests: {time.perf_counter() - t:.1f} s, {good} within 1e-4")
    # FP64 one-at-a-time reference on a sample (first pairs of each size)
    sample = []
    for size in (64, 128, 256, 512):
        sample += [i for i, it in enumerate(items) if it[0] == size][:max(1, args.fp64_sample // 4)]
    s64 = w1.Solver(prm_for(512, 2, w1.FP64), capacity=1)
    rel, t64 = [], 0.0
    for i in sample:
        n, m, a, b = dev[i]
        torch.cuda.synchronize()
        t = time.perf_counter()
        r64 = _serve_all(w1, s64, [(n, m, a, b)], lambda n_, m_: prm_for(n_, m_, w1.FP64))[0]
        torch.cuda.synchronize()
        t64 += time.perf_counter() - t
        rel.append(abs(res[i]["w1"] - r64["w1"]) / abs(r64["w1"]))
    s64.close()
    cpu = None
    if not args.no_cpu:
        # one pair of each size, weighted by the size mix: expected seconds
        # per solve of the workload on one host core
        import oracle.w1_oracle as o
        probs = {64: 0.4, 128: 0.3, 256: 0.2, 512: 0.1}
        exp_t, parts = 0.0, []
        for size, pr in probs.items():
            i = next(j for j, it in enumerate(items) if it[0] == size)
            n, m, a, b = items[i]
            t = time.perf_counter()
            o.solve(a, b, n, L=_levels(n), p=m, algo=2, stop="fpr", eps_L=o.paper_stop_tolerance(2, n, True),
                    alpha=-1.0, max_iters=20000, check_every=10, return_fields=False)
            dt = time.perf_counter() - t
            exp_t += pr * dt
            parts.append(f"n={n}: {dt:.2f} s")
            log(f"[bench] CPU oracle pair {i} n={n}: {dt:.2f} s")
        cpu = {"value": 1.0 / exp_t, "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": "one pair of each size, weighted by the size mix (" + ", ".join(parts) + ")"}
    sps = good * args.steps / el
    return {"metric": METRIC, "value": sps, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"uneven batch: {P} pairs, n in {{64,128,256,512}} w.p. {{.4,.3,.2,.1}}, "
                                   "L1/L2 alternating, Gaussian mixtures K~U{2..10}, Algorithm 4 (DCT Poisson), "
                                   "L=log2(n/32)+1, paper stop rule, FP32 iterates / FP64 reductions",
                       "global_batch": P, "parallelism": "batch"},
            "cell_updates_per_s": ups * args.steps / el,
            "fp64_single": {"solves_per_s": len(sample) / t64 if t64 else None, "sample": len(sample)},
            "accuracy": {"reference": "FP64 served path, every request", "checked": len(rel_all),
                         "within_1e-4": good, "max_rel": max(rel_all), "median_rel": float(np.median(rel_all)),
                         "fp64_single_sample": {"checked": len(rel), "within_1e-4": sum(x <= 1e-4 for x in rel),
                                                "max_rel": max(rel) if rel else None}},
            "solves_per_s_all": P * args.steps / el,
            "roofline": _mfma_roofline(ks),
            "kernel_timing": TIMING_NOTE,
            "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 3)} for k, v in ks.items()
                        if v["launches"]},
            "cpu_baseline": cpu}


def run_served(args, w1):
    """Served stream: Poisson arrivals at --rate for --duration seconds, grid
    side uniform over --sizes, densities 50/50 Gaussian mixtures or unions of
    rectangles/disks, FP32 Algorithm 4 with L = log2(n/32)+1 and the paper's
    stop rule tested every iteration; each result is checked against the FP64
    solve of the same request (relative difference 1e-4).  Requests join the
    running batch as slots and HBM budget free up; latency is submission to
    completion."""
    import torch
    import w1data
    sizes = tuple(int(x) for x in args.sizes.split(","))
    count = int(args.rate * args.duration)
    reqs = w1data.served_requests(count, rate=args.rate, sizes=sizes)
    # a pool of distinct pairs per size, reused round robin (the solver keeps
    # no state between requests, so repeats cost the same as new inputs)
    POOL = 4
    pool, seen = {}, {}
    for r in reqs:
        k = seen.get(r.n, 0)
        if k < POOL:
            a, b = w1data.served_pair(r)
            pool[(r.n, k)] = (torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
        seen[r.n] = k + 1
    torch.cuda.synchronize()

    def prm_for(n, precision=w1.FP32):
        return w1.params(n=n, levels=_levels(n), metric=w1.METRIC_L2, algo=w1.ALGO_PROX, precision=precision,
                         stop_rule=w1.STOP_FPR, tol=0.0, alpha=-1.0, max_iters=20000, check_every=1,
                         flags=w1.FLAG_NO_FIELDS)

    srv = w1.Solver(prm_for(max(sizes)), capacity=256)
    srv.serve_config(1 << 30)
    srv.profile(True, every=TILED_TIMING_EVERY)
    out, pend, cnt = [], {}, {}
    last = [0.0]
    t0 = time.perf_counter()

    def sweep():
        for tk in list(pend):
            r = srv.poll(tk)
            if r is not None:
                out.append((pend.pop(tk), r[0]))
        now = time.perf_counter() - t0
        if now - last[0] > 2.0:
            last[0] = now
            log(f"[bench] served t={now:.1f}s done {len(out)} pending {len(pend)}")

    for r in reqs:
        while True:
            now = time.perf_counter() - t0
            if now >= r.arrival:
                break
            sweep()
            time.sleep(min(0.0005, r.arrival - now))
        k = cnt.get(r.n, 0)
        cnt[r.n] = k + 1
        a, b = pool[(r.n, k % POOL)]
        pend[srv.submit(a, b, prm_for(r.n))] = (r, k % POOL)
    deadline = args.duration * 6 + 30
    while pend and time.perf_counter() - t0 < deadline:
        sweep()
        time.sleep(0.001)
    el = time.perf_counter() - t0
    unfinished = len(pend)
    ks = srv.kernel_stats()
    srv.close()
    lat = np.array([x[1]["seconds"] for x in out])
    per = {}
    for n in sizes:
        l = np.array([x[1]["seconds"] for x in out if x[0][0].n == n])
        if len(l):
            per[str(n)] = {"count": int(len(l)), "p50_ms": float(np.percentile(l, 50) * 1e3),
                           "p99_ms": float(np.percentile(l, 99) * 1e3)}
    # FP64 one-at-a-time reference on one request of each size
    s64 = w1.Solver(prm_for(max(sizes), w1.FP64), capacity=1)
    rel, t64, n64 = [], 0.0, 0
    for n in sizes:
        mine = [x for x in out if x[0][0].n == n]
        if not mine:
            continue
        (r, slot), res = mine[0]
        a, b = pool[(n, slot)]
        torch.cuda.synchronize()
        t = time.perf_counter()
        tk = s64.submit(a, b, prm_for(n, w1.FP64))
        s64.drain()
        r64 = None
        while r64 is None:
            r64 = s64.poll(tk)
        torch.cuda.synchronize()
        t64 += time.perf_counter() - t
        n64 += 1
        rel.append(abs(res["w1"] - r64[0]["w1"]) / abs(r64[0]["w1"]))
    s64.close()
    return {"metric": METRIC, "value": len(out) / el, "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": el * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"served stream: Poisson arrivals at {args.rate:g}/s for {args.duration:g} s, "
                                   f"n uniform over {{{args.sizes}}}, mixtures or rectangles/disks, Algorithm 4, "
                                   "L=log2(n/32)+1, paper stop rule every iteration, FP32 iterates",
                       "requests": count, "parallelism": "continuous batching"},
            "latency": {"p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
                        "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
                        "per_size": per, "unfinished": unfinished},
            "fp64_single": {"solves_per_s": n64 / t64 if t64 else None, "sample": n64},
            "accuracy": {"reference": "FP64 solve of a sample of the requests (first of each size)",
                         "checked": len(rel), "within_1e-4": sum(x <= 1e-4 for x in rel),
                         "max_rel": max(rel) if rel else None},
            "roofline": _mfma_roofline(ks),
            "kernel_timing": TIMING_NOTE,
            "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 3)} for k, v in ks.items()
                        if v["launches"]},
            "cpu_baseline": None}


def run_poisson(args, w1):
    """The FP32 Neumann Poisson solve of eq. (pdhg) alone (w1_op_poisson,
    one pair of sides per size in --sizes): FFT path for sides 1024..4096,
    folded matrix passes below.  Each call also sets up its tables and
    planes, so the per-call wall time is an upper bound; the kernels' own
    times come from a kernel trace of this run."""
    import torch
    sizes = [int(x) for x in args.sizes.split(",")]
    out = {}
    for n in sizes:
        rng = np.random.default_rng(n)
        r = rng.standard_normal((n + 1, n + 1))
        r -= r.mean()
        gr = torch.from_numpy(r).float().cuda()
        gu = torch.zeros_like(gr)
        for _ in range(max(1, args.warmup)):
            w1.op_poisson(n, w1.FP32, gr, gu)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            w1.op_poisson(n, w1.FP32, gr, gu)
        torch.cuda.synchronize()
        out[str(n)] = {"ms_per_call_wall": (time.perf_counter() - t) * 1e3 / args.steps,
                       "path": "fft" if n + 1 >= 1025 else "matrix passes"}
        log(f"[bench] poisson n={n}: {out[str(n)]['ms_per_call_wall']:.2f} ms per call")
    return {"workload": "Neumann Poisson solve, FP32, one grid per call", "steps": args.steps, "sizes": out}


def run_tiled(args, w1):
    """The plain tiled kernel alone on one stream (w1_op_plain_steps): one
    grid of side --n, FP32, l_2, 64 x --tiled-width regions over
    --tiled-waves wavefronts, 10 steps per launch, --steps launches per call.
    For counter collection (HBM bytes per launch) and kernel traces of a
    single, fixed launch shape."""
    import torch
    n = args.n
    rng = np.random.default_rng(n)
    r = rng.random((n + 1, n + 1))
    r -= r.mean()
    rho = torch.from_numpy(r).float().cuda()
    m1, m2, phi = (torch.zeros_like(rho) for _ in range(3))
    torch.cuda.synchronize()
    t = time.perf_counter()
    w1.op_plain_steps(n, w1.METRIC_L2, w1.FP32, 10 * args.steps, m1, m2, phi, rho, block_steps=10,
                      waves=args.tiled_waves, width=args.tiled_width)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    ups = float(n + 1) ** 2 * 10 * args.steps
    log(f"[bench] tiled n={n}: {args.steps} launches, {el * 1e3:.2f} ms")
    return {"workload": f"plain tiled kernel, one {n + 1}^2 grid, FP32, l_2, 64 x {args.tiled_width} regions, "
                        f"{args.tiled_waves} wavefronts, 10 steps per launch",
            "launches": args.steps, "useful_updates_per_launch": ups / args.steps, "wall_ms": el * 1e3}


def run_single(args, w1):
    """Single pair at n = 512: eight anisotropic Gaussians and the same
    mixture shifted by up to 0.1 (W1 close to the shift length), L2, 4-level
    cascade; plain (Algorithm 3) and prox (Algorithm 4), FP32 and FP64,
    paper stop rule; seconds per solve."""
    import torch
    import w1data
    n = 512
    a, b, shift = w1data.pair_shift8(0, n=n)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    out = {}
    for algo, name in ((w1.ALGO_PLAIN, "plain"), (w1.ALGO_PROX, "prox")):
        for prec, pn in ((w1.FP32, "f32"), (w1.FP64, "f64")):
            prm = w1.params(n=n, levels=4, metric=w1.METRIC_L2, algo=algo, precision=prec, stop_rule=w1.STOP_FPR,
                            tol=0.0, alpha=-1.0, max_iters=20000, check_every=10)
            with w1.Solver(prm, capacity=1) as s:
                s.solve([(da, db)])
                torch.cuda.synchronize()
                t = time.perf_counter()
                reps = max(1, args.steps)
                for _ in range(reps):
                    r = s.solve([(da, db)])[0]
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t) / reps
            out[f"{name}_{pn}"] = {"seconds": dt, "w1": r["w1"], "iters": r["iters"], "lo": r["lo"], "hi": r["hi"]}
            log(f"[bench] single {name} {pn}: {dt*1e3:.1f} ms W1 {r['w1']:.6f} iters {r['iters']}")
    sec = out["prox_f32"]["seconds"]
    return {"metric": METRIC, "value": 1.0 / sec, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "single pair n=512: 8 anisotropic Gaussians and a shifted copy (|s| <= 0.1), "
                                   "L2, 4 levels, paper stop rule; value = Algorithm 4 FP32",
                       "global_batch": 1, "parallelism": "none"},
            "shift_length": float(np.hypot(*shift)), "runs": out,
            "context": "paper: 0.2-1.5 s per 512x512 W1 on one i7-2600 (MATLAB, Algorithm 4)",
            "cpu_baseline": None}


def run_tolerance(args, w1):
    """The tolerance-rule study of Sec. 5.2 (Tables tab:1m and tab:2m) and
    the level-count comparison of Sec. 5.1 (Table tab:pd_comparel) on
    synthetic pairs: Algorithm 3 at n = 256 and Algorithm 4 at n = 512, six
    levels, l_1 ground metric, FP32 iterates.

    Per level, the optimum f(m*_{h_l}) is taken from an FP64 Algorithm 4
    cascade run to a normalised KKT residual of 1e-8 at every level.  For
    each alpha in {1, 0, -1, -5}, eps_L walks down the paper's grid
    (1e-6 2^p, p = 0..-10 for Algorithm 3; 1e-4 2^p, p = 5..-10 for
    Algorithm 4; both extended upwards, to p = 6 and p = 10, so that the
    largest passing value is inside the grid), with an iteration cap of
    200000 per level, until condition (cond_f) holds at levels 2..L:
    |f(m*_{h_l}) - f(m^{K_l}_{h_l})| < |f(m*_{h_l}) - f(m*_{h_{l-1}})|.
    The single-level baseline takes the largest eps on the same grid whose
    error on the finest level is below the finest grid error.  Times are
    wall seconds of one w1_solve (median of three; per level: host steps
    that saw the level end); K_l, errors and the speedup over the baseline
    are reported, then L = 1..6 at the alpha = -1 tolerance (Sec. 5.1)."""
    import torch
    import w1data
    L = 6
    study = {}
    cap = 200000
    for algo, n, grid in ((w1.ALGO_PLAIN, 256, [1e-6 * 2.0 ** p for p in range(6, -11, -1)]),
                          (w1.ALGO_PROX, 512, [1e-4 * 2.0 ** p for p in range(10, -11, -1)])):
        a, b = w1data.pair_shapes(0, n=n)
        pair = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())]
        ref_prm = w1.params(n=n, levels=L, metric=w1.METRIC_L1, algo=w1.ALGO_PROX, precision=w1.FP64,
                            stop_rule=w1.STOP_KKT, tol=1e-8, alpha=0.0, max_iters=100000, check_every=10,
                            flags=w1.FLAG_LEVEL_COST)
        with w1.Solver(ref_prm, capacity=1) as s:
            ref = s.solve(pair)[0]
        # stop tests every iteration for Algorithm 4, whose finer levels stop
        # after one or two (as in the paper); every 10 for Algorithm 3
        ce = 10 if algo == w1.ALGO_PLAIN else 1
        fstar = ref["level_w1"]
        gerr = [None] + [abs(fstar[l] - fstar[l - 1]) for l in range(1, L)]
        log(f"[bench] tolerance study algo {algo} n={n}: level optima {['%.7f' % f for f in fstar]} "
            f"(reference iters {ref['iters']}, level KKT {['%.1e' % x for x in ref['measure']]}, "
            f"bracket [{ref['lo']:.8f}, {ref['hi']:.8f}])")

        def run(levels, eps, alpha, caps=None):
            extra = {"level_caps": caps} if caps else {}
            prm = w1.params(n=n, levels=levels, metric=w1.METRIC_L1, algo=algo, precision=w1.FP32,
                            stop_rule=w1.STOP_FPR, tol=eps, alpha=alpha, max_iters=cap, check_every=ce,
                            flags=w1.FLAG_LEVEL_COST, **extra)
            with w1.Solver(prm, capacity=1) as s:
                s.solve(pair)                        # shapes settled by the autotuner
                walls = []
                for _ in range(3):
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    r = s.solve(pair)[0]
                    torch.cuda.synchronize()
                    walls.append(time.perf_counter() - t)
                r["wall"] = float(np.median(walls))
            off = L - levels
            r["err"] = [abs(fstar[off + l] - r["level_w1"][l]) for l in range(levels)]
            ls = r["level_seconds"]
            r["level_time"] = [ls[0]] + [ls[l] - ls[l - 1] for l in range(1, levels)]
            return r

        def row(r, eps, alpha, levels):
            # eps_l = eps_L (h_l / h)^alpha, h_l = 2^(levels - 1 - l) h (l = 0 coarsest)
            return {"eps_L": eps, "alpha": alpha, "levels": levels,
                    "eps_l": [eps * 2.0 ** ((levels - 1 - l) * alpha) for l in range(levels)],
                    "K": r["iters"], "error": r["err"], "level_seconds": r["level_time"], "seconds": r["wall"],
                    "w1": r["w1"]}

        base = None
        for eps in grid:
            r = run(1, eps, 0.0)
            if r["err"][0] < gerr[L - 1]:
                base = row(r, eps, 0.0, 1)
                break
        if base:
            log(f"[bench]   baseline (L=1): eps {base['eps_L']:.3g} K {base['K']} {base['seconds']:.3f}s")
        else:
            log("[bench]   baseline (L=1): no eps on the grid reaches the finest grid error")
        rules = []
        for alpha in (1.0, 0.0, -1.0, -5.0):
            best = None
            for eps in grid:
                r = run(L, eps, alpha)
                if all(r["err"][l] < gerr[l] for l in range(1, L)):
                    best = row(r, eps, alpha, L)
                    break
            if best is not None:
                best["speedup"] = base["seconds"] / best["seconds"] if base else None
                log(f"[bench]   alpha {alpha:+.0f}: eps_L {best['eps_L']:.3g} K {best['K']} "
                    f"{best['seconds']:.3f}s speedup {best['speedup']}")
            else:
                log(f"[bench]   alpha {alpha:+.0f}: no eps_L on the grid meets (cond_f)")
            rules.append({"alpha": alpha, "best": best})
        levels_rows = []
        eps_m1 = next((x["best"]["eps_L"] for x in rules if x["alpha"] == -1.0 and x["best"]), grid[-1])
        for levels in range(1, L + 1):
            r = run(levels, eps_m1, -1.0)
            levels_rows.append(row(r, eps_m1, -1.0, levels))
            log(f"[bench]   L={levels}: K {r['iters']} {r['wall']:.3f}s")
        # per-level caps from the study: twice the alpha = -1 rule's K_l,
        # rounded up to the check cadence; the capped run must keep the
        # (cond_f) errors of the uncapped one (a bounded worst case per
        # level for served requests of this kind)
        derived = None
        best_m1 = next((x["best"] for x in rules if x["alpha"] == -1.0 and x["best"]), None)
        if best_m1:
            caps = [int(math.ceil(2.0 * k / ce)) * ce for k in best_m1["K"]]
            rc = run(L, best_m1["eps_L"], -1.0, caps)
            derived = {"rule": "caps = 2 K_l of the alpha = -1 row, rounded up to check_every", "caps": caps,
                       "K": rc["iters"], "status": rc["status"], "error": rc["err"],
                       "cond_f_holds": all(rc["err"][l] < gerr[l] for l in range(1, L)),
                       "seconds": rc["wall"]}
            log(f"[bench]   derived caps {caps}: K {rc['iters']} {rc['wall']:.3f}s "
                f"(cond_f {'holds' if derived['cond_f_holds'] else 'fails'})")
        study["plain" if algo == w1.ALGO_PLAIN else "prox"] = {
            "n": n, "grid_error": gerr[1:], "level_optima": fstar, "derived_caps": derived,
            "reference": {"iters": ref["iters"], "level_kkt": ref["measure"], "lo": ref["lo"], "hi": ref["hi"]},
            "eps_grid": [grid[0], grid[-1]], "cap": cap, "check_every": ce, "baseline": base, "rules": rules, "levels": levels_rows}
    sp = [x["best"]["speedup"] for x in study["prox"]["rules"] if x["alpha"] == -1.0 and x["best"]]
    return {"metric": "speedup of the multilevel cascade over one level at equal accuracy (Sec. 5.2 protocol)",
            "value": sp[0] if sp else None, "unit": "x", "n_gpus": 1, "steps": 1, "warmup": 1,
            "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "tolerance-rule study: one rectangles/disks pair, Algorithm 3 at n=256 and "
                                   "Algorithm 4 at n=512, 6 levels, l_1 metric, FP32, alpha in {1, 0, -1, -5}, "
                                   "eps_L on the paper's grids; value = Algorithm 4 speedup at alpha = -1"},
            "study": study}


def run_cube(args, w1):
    """d = 3 (the method for general d, Sec. 2.2 / 3.3): one pair of
    isotropic Gaussian mixtures on the unit cube at n = 128 (129^3 nodes),
    3 levels (33^3, 65^3, 129^3), l_2 metric, Algorithm 3 (FPR eps_L 1e-7)
    and Algorithm 4 (FPR eps_L 1e-5), alpha = -1, FP32 iterates; against the
    same solves in FP64 on the GPU, and the FP64 oracle's Algorithm 1
    node-update rate on this host.  `value` is Algorithm 3's."""
    import torch
    import w1data
    n, L = 128, 3
    p0, p1 = w1data.pair_gauss_3d(0, n=n)
    d0, d1 = torch.from_numpy(p0).cuda(), torch.from_numpy(p1).cuda()
    out = {}
    for algo, an, tol in ((w1.ALGO_PLAIN, "plain", 1e-7), (w1.ALGO_PROX, "prox", 1e-5)):
        for prec, name in ((w1.FP32, "f32"), (w1.FP64, "f64")):
            prm = w1.params(n=n, levels=L, metric=w1.METRIC_L2, algo=algo, precision=prec,
                            stop_rule=w1.STOP_FPR, tol=tol, alpha=-1.0, max_iters=20000, check_every=10)
            w1.solve3d(prm, d0, d1)
            torch.cuda.synchronize()
            reps = max(1, args.steps) if prec == w1.FP32 else 1
            t = time.perf_counter()
            for _ in range(reps):
                r = w1.solve3d(prm, d0, d1)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / reps
            key = name if algo == w1.ALGO_PLAIN else f"prox_{name}"
            out[key] = {"seconds": dt, "w1": r["w1"], "iters": r["iters"], "lo": r["lo"], "hi": r["hi"],
                        "kkt": r["kkt"]}
            log(f"[bench] cube {an} {name}: {dt*1e3:.1f} ms W1 {r['w1']:.7f} [{r['lo']:.6f}, {r['hi']:.6f}] "
                f"iters {r['iters']}")
    # many pairs at once: w1_solve3d_batch on 8 concurrent streams
    B = 16
    bpairs = [tuple(torch.from_numpy(x).cuda() for x in w1data.pair_gauss_3d(i, n=n)) for i in range(B)]
    batch = {}
    for algo, an, tol in ((w1.ALGO_PLAIN, "plain", 1e-7), (w1.ALGO_PROX, "prox", 1e-5)):
        prm = w1.params(n=n, levels=L, metric=w1.METRIC_L2, algo=algo, precision=w1.FP32,
                        stop_rule=w1.STOP_FPR, tol=tol, alpha=-1.0, max_iters=20000, check_every=10)
        w1.solve3d_batch(prm, bpairs[:8], workers=8)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rs = w1.solve3d_batch(prm, bpairs, workers=8)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        batch[an] = {"pairs": B, "workers": 8, "seconds": dt, "solves_per_s": B / dt,
                     "iters_median": [float(np.median([r["iters"][l] for r in rs])) for l in range(L)]}
        log(f"[bench] cube batch {an}: {B} pairs in {dt:.3f} s, {B / dt:.1f} solves/s")
    sides = [n >> (L - 1 - l) for l in range(L)]
    nodes = [(s_ + 1) ** 3 for s_ in sides]
    upd = sum(k * nd for k, nd in zip(out["f32"]["iters"], nodes))
    sec = out["f32"]["seconds"]
    cups = upd / sec
    # 9 words per node update: read m1, m2, m3, phi, rho; write m1, m2, m3, phi
    alg = 36.0
    roof = {"kernel": "k3_flux + k3_pot (whole solve, wall time)", "bound": "hbm", "achieved": cups * alg / 1e9,
            "peak": 8000.0, "unit": "GB/s", "frac": cups * alg / 8e12, "traffic": None,
            "alg_bytes_per_node_update": alg}
    cpu = None
    if not args.no_cpu:
        os.environ.setdefault("OMP_NUM_THREADS", "1")
        import oracle.w1_oracle3d as o3
        rho = o3.prepare_levels(p0, p1, n, 1)[0]
        h = 1.0 / n
        mu, tau = o3.plain_step_sizes(h, 3)
        m = tuple(np.zeros((n + 1,) * 3) for _ in range(3))
        phi = np.zeros((n + 1,) * 3)
        k, t = 0, time.perf_counter()
        while time.perf_counter() - t < 15.0:
            m, phi, _ = o3.pd_step(m, phi, rho, h, mu, tau, 2)
            k += 1
        dt = time.perf_counter() - t
        rate = k * (n + 1) ** 3 / dt
        cpu = {"value": rate / upd, "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": f"{k} iterations of eq. (primaldual) on the 129^3 level in {dt:.1f} s, scaled by the "
                         "node updates of the GPU solve", "node_updates_per_s": rate}
        log(f"[bench] cube CPU oracle: {rate:.3e} node updates/s")
    rel = abs(out["f32"]["w1"] - out["f64"]["w1"]) / out["f64"]["w1"]
    return {"metric": METRIC, "value": 1.0 / sec, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "d=3: one pair of 3-Gaussian mixtures on the unit cube, n=128 (129^3 nodes), "
                                   "3 levels, L2 metric, Algorithm 3, FPR eps_L 1e-7 alpha -1, FP32"},
            "cell_updates_per_s": cups, "fp64_single": {"solves_per_s": 1.0 / out["f64"]["seconds"],
                                                        "speedup_fp32": out["f64"]["seconds"] / sec},
            "accuracy": {"rel_w1_fp32_vs_fp64": rel,
                         "prox_rel_w1_fp32_vs_fp64": abs(out["prox_f32"]["w1"] - out["prox_f64"]["w1"])
                         / out["prox_f64"]["w1"]},
            "solves": out, "batch": batch, "roofline": roof, "cpu_baseline": cpu}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pairs", type=int, default=256)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--levels", type=int, default=3)
    ap.add_argument("--fp64-sample", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64-ref", action="store_true",
                    help="uniform: skip the FP64 reference of every pair (traced runs); the value then counts "
                         "every solve and says so")
    ap.add_argument("--block-steps", type=int, default=0)
    ap.add_argument("--graph", action="store_true",
                    help="uniform: plain-only steps replay captured HIP graphs (W1_GRAPH=1); "
                         "launches untimed, so no roofline")
    ap.add_argument("--tiled-width", type=int, default=128, choices=[64, 128], help="tiled: region columns")
    ap.add_argument("--tiled-waves", type=int, default=16, choices=[8, 16], help="tiled: wavefronts per region")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only copy this many bytes device-to-device (HBM counter calibration)")
    ap.add_argument("--workload", default="uniform",
                    choices=["uniform", "uneven", "served", "single", "tolerance", "cube", "poisson", "tiled"])
    ap.add_argument("--ground", default="l2", choices=["l1", "l2", "linf"],
                    help="uniform: ground metric of the flux cost (the headline figure is l2)")
    ap.add_argument("--step-scale", type=float, default=0.0,
                    help="uniform: step_scale of every solve (0: the paper's 1/2; 1: its practical steps)")
    ap.add_argument("--rate", type=float, default=200.0, help="served: arrivals per second")
    ap.add_argument("--duration", type=float, default=10.0, help="served: seconds of arrivals")
    ap.add_argument("--sizes", default="128,256,512,1024,2048", help="served: grid sides")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solves shard across GPUs "
              "as independent batches, which this build does not launch", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        src = torch.empty(args.copy_calibration // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4}))
        return

    import paper_1810_00118_amd as w1

    if args.workload != "uniform":
        assert torch.cuda.is_available(), "bench.py needs a HIP device"
        run = {"uneven": run_uneven, "served": run_served, "single": run_single, "poisson": run_poisson, "tiled": run_tiled,
               "tolerance": run_tolerance, "cube": run_cube}[args.workload]
        print(json.dumps(run(args, w1)), flush=True)
        return
    n, L, P = args.n, args.levels, args.pairs
    log(f"[bench] generating {P} pairs n={n}")
    pairs = workload_pairs(P, n)
    p_or = {"l1": 1, "l2": 2, "linf": math.inf}[args.ground]
    cpu_pool = None if args.no_cpu else oracle_pool(pairs, n, L, p_or, args.step_scale)
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev_pairs = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b in pairs]
    torch.cuda.synchronize()

    w1.lib()
    gm = {"l1": w1.METRIC_L1, "l2": w1.METRIC_L2, "linf": w1.METRIC_LINF}[args.ground]
    prm = w1.params(n=n, levels=L, metric=gm, algo=w1.ALGO_PLAIN, precision=w1.FP32,
                    stop_rule=w1.STOP_FPR, tol=0.0, alpha=-1.0, max_iters=20000, check_every=10,
                    block_steps=args.block_steps, step_scale=args.step_scale)
    if args.graph:
        os.environ["W1_GRAPH"] = "1"
    solver = w1.Solver(prm, capacity=P)
    for k in range(args.warmup):
        t = time.perf_counter()
        solver.solve(dev_pairs)
        log(f"[bench] warmup {k} {time.perf_counter() - t:.3f}s")
    solver.profile(not args.graph, every=TILED_TIMING_EVERY)
    c0 = solver.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = None
    step_s = []
    for k in range(args.steps):
        ts = time.perf_counter()
        results = solver.solve(dev_pairs)   # returns once the batch's results are on the host
        step_s.append(time.perf_counter() - ts)
        log(f"[bench] step {k} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kstats = solver.kernel_stats()
    counters = {k: (v - c0[k]) / args.steps for k, v in solver.counters().items()}   # per step
    solver.profile(False)
    sides = [n >> (L - 1 - l) for l in range(L)]
    nodes = [(s + 1) ** 2 for s in sides]
    cell_updates = sum(sum(it * nd for it, nd in zip(r["iters"], nodes)) for r in results)
    its = np.array([r["iters"] for r in results])
    iter_stats = {f"level{l + 1}": {"min": int(its[:, l].min()), "median": float(np.median(its[:, l])),
                                    "max": int(its[:, l].max())} for l in range(L)}
    ms_per_step = elapsed / args.steps * 1e3
    solves_per_s = P * args.steps / elapsed
    cups = cell_updates * args.steps / elapsed
    log(f"[bench] batched FP32: {solves_per_s:.1f} solves/s, {cups:.3e} node-updates/s, "
        f"{ms_per_step:.1f} ms/step, iters pair0 {results[0]['iters']}")

    # ---- every counted solve against the FP64 batched GPU path (outside
    # the timed region): a solve counts only within 1e-4 of its FP64 W1 ----
    prm64b = w1.params(n=n, levels=L, metric=gm, algo=w1.ALGO_PLAIN, precision=w1.FP64,
                       step_scale=args.step_scale, stop_rule=w1.STOP_FPR, tol=0.0, alpha=-1.0, max_iters=20000,
                       check_every=10, flags=w1.FLAG_NO_CERT)
    t = time.perf_counter()
    if args.no_fp64_ref:
        ref_all = results
    else:
        with w1.Solver(prm64b, capacity=P) as s64b:
            ref_all = s64b.solve(dev_pairs)
        log(f"[bench] FP64 batched reference of all {P} pairs: {time.perf_counter() - t:.1f} s")
    rel_all = [abs(r["w1"] - q["w1"]) / abs(q["w1"]) for r, q in zip(results, ref_all)]
    good = sum(x <= 1e-4 for x in rel_all)
    # a pair outside 1e-4: is it the stop decision (an integer FP32 decides,
    # R19)?  FP64 run to the FP32 path's own per-level iteration counts
    same_iter = []
    for i in [k for k, x in enumerate(rel_all) if x > 1e-4][:8]:
        q = w1.params(n=n, levels=L, metric=gm, algo=w1.ALGO_PLAIN, precision=w1.FP64,
                      step_scale=args.step_scale, stop_rule=w1.STOP_FPR, tol=1e-300, alpha=-1.0, max_iters=20000,
                      check_every=10, flags=w1.FLAG_NO_CERT, level_caps=results[i]["iters"])
        with w1.Solver(q, capacity=1) as s1:
            r1 = s1.solve([dev_pairs[i]])[0]
        same_iter.append({"pair": i, "rel_own_stops": rel_all[i], "iters_fp32": results[i]["iters"],
                          "iters_fp64": ref_all[i]["iters"],
                          "rel_same_iters": abs(results[i]["w1"] - r1["w1"]) / abs(r1["w1"])})
    capped = sum(r["status"] == w1.SOLVE_MAXITER for r in results)
    solves_counted_per_s = good * args.steps / elapsed

    # ---- plain FP64 one-pair-at-a-time GPU path on a sample ----
    prm64 = w1.params(n=n, levels=L, metric=gm, algo=w1.ALGO_PLAIN, precision=w1.FP64, step_scale=args.step_scale,
                      stop_rule=w1.STOP_FPR, tol=0.0, alpha=-1.0, max_iters=20000, check_every=10,
                      block_steps=1, flags=w1.FLAG_NO_RESIDENT)
    s64 = w1.Solver(prm64, capacity=1)
    ref, t64 = [], 0.0
    for i in range(args.fp64_sample):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ref.append(s64.solve([dev_pairs[i]])[0])
        torch.cuda.synchronize()
        t64 += time.perf_counter() - t
    s64.close()
    fp64_sps = args.fp64_sample / t64 if args.fp64_sample else None
    rel = [abs(results[i]["w1"] - ref[i]["w1"]) / abs(ref[i]["w1"]) for i in range(args.fp64_sample)]
    if rel:
        log(f"[bench] FP64 single: {fp64_sps:.2f} solves/s; max rel W1 diff {max(rel):.2e}")

    # launch shapes the autotuner settled on (per size class of the active set)
    tuned = []
    for e in w1.tuner_table():
        if e["best"] >= 0:
            a = e["arms"][e["best"]]
            tuned.append({"precision": e["precision"], "class": e["class"], "waves": a["waves"], "T": a["T"],
                          "width": a.get("width", 128), "height": a.get("height", 64),
                          "ns_per_update": a["ns_per_update"]})

    # ---- dominant kernel roofline (HIP events in the timed region) ----
    # (tiled and Algorithm 2 launches are timed on a sample of about one in
    # TILED_TIMING_EVERY: their summed time is scaled up to compare families)
    dom = max(kstats, key=lambda k: _est_ms(kstats, k))
    st = kstats[dom]
    roof = None
    if st["launches"]:
        avg_ms = st["ms"] / st["launches"]
        if dom == "plain_tiled":
            # temporal blocking keeps T steps in registers, so the kernel is
            # bound by VALU issue, not HBM: achieved = the VALU issue slots
            # the algorithm's node updates need (halo recomputation and the
            # kernel's own index and lane-shift work not counted) per second
            # of its launches; issue_frac_computed is the compiled loop's
            # slots over every node it computes, halo included.
            # The launches' number is exact (`issued`), their mean duration
            # the timed sample's; the useful node updates come from the
            # solves' own iteration counts (all node updates of the timed
            # solves minus those of the resident levels, which are all
            # timed), not from the launches' slot lists: a slot that stops
            # inside a step's queued blocks is skipped on the device but
            # stays in the list it was issued with.
            issued = max(st["issued"], st["launches"])
            sec = avg_ms * 1e-3 * issued
            useful = cell_updates * args.steps - kstats["plain_resident"]["node_updates"]
            halo = st["flops"] / st["node_updates"]   # computed per useful update, as issued
            computed = useful * halo
            # the compiled count of the shape the autotuner chose for the
            # largest active set (the launches that carry most of the work)
            big = max((a for a in tuned if a["precision"] == 1), key=lambda a: a["class"], default=None)
            shape = (big["width"], big["waves"]) if big else (128, 16)
            cyc = TILED_VALU_CYCLES.get(shape, {}).get(args.ground)
            alg = ALG_VALU_SLOTS[args.ground]
            achieved = useful * alg / sec
            T_ = [a["T"] for a in tuned] or [10]
            Tm = float(np.median(T_))
            dram = (16.0 * halo + 12.0) / Tm   # per useful update: read m1 m2 phi rho per region node, write m1 m2 phi
            # HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE
            # counts (per useful update, scaled to this run's launches)
            tr = measured_traffic("k_plain_tiled", "uniform256") if (n, P, args.ground) == (256, 256, "l2") else None
            traffic = tr["bytes_per_useful_update"] * useful / issued if tr else None
            roof = {"kernel": dom, "bound": "alu", "achieved": achieved / 1e12, "peak": VALU_LANE_OPS_PEAK / 1e12,
                    "unit": "TOP/s (VALU lane-ops, non-packed FP32)", "frac": achieved / VALU_LANE_OPS_PEAK,
                    "traffic": traffic, "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                    "traffic_gbs": traffic / (avg_ms * 1e-3) / 1e9 if traffic else None,
                    "avg_launch_ms": avg_ms, "launches": issued, "launches_timed": st["launches"],
                    "timed_launches": f"pseudo-random sample of about 1 in {TILED_TIMING_EVERY} launches "
                                      "(events bound to the dispatch: kernel start to end)",
                    "alg_valu_slots_per_update": alg,
                    "valu_cycles_per_update": cyc,
                    "region_shape": f"64 x {shape[0]}, {shape[1]} wavefronts",
                    "issue_frac_computed": computed * cyc / sec / VALU_LANE_OPS_PEAK if cyc else None,
                    "useful_updates_per_launch": useful / issued,
                    "computed_updates_per_launch": computed / issued,
                    "halo_factor": halo,
                    "useful_updates_per_s": useful / sec,
                    "modelled_dram_bytes_per_useful_update": dram,
                    "modelled_dram_gbs": dram * useful / sec / 1e9,
                    "effective_alg_gbs_28B": 28.0 * useful / sec / 1e9}
        elif dom == "prox_elem":
            achieved = st["alg_bytes"] / (st["ms"] * 1e-3) / 1e9
            roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None, "avg_launch_ms": avg_ms,
                    "launches": st["launches"]}
        elif dom == "dct":
            achieved = st["flops"] / (st["ms"] * 1e-3) / 1e12
            # the matrix passes (N <= 513) run on the FP32 matrix cores,
            # whose dense peak equals the FP32 vector figure
            roof = {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": FP32_VALU_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved / FP32_VALU_TFLOPS, "traffic": None,
                    "avg_launch_ms": avg_ms, "launches": st["launches"]}
        else:
            # LDS-resident levels: node updates per second against the
            # FP32 VALU issue rate (one node update ~ 40 VALU instructions)
            ups = st["node_updates"] / (st["ms"] * 1e-3)
            roof = {"kernel": dom, "bound": "alu", "achieved": ups, "peak": None, "unit": "node-updates/s",
                    "frac": None, "traffic": None, "avg_launch_ms": avg_ms, "launches": st["launches"]}
    kernels = {k: {"launches": v["launches"], "ms": round(v["ms"], 3)} for k, v in kstats.items() if v["launches"]}

    # ---- FP64 CPU oracle on this host (timed before the first GPU call) ----
    cpu = cpu_pool
    if cpu is not None:
        cpu["w1_rel_vs_gpu_pair0"] = abs(cpu.pop("w1_pair0") - results[0]["w1"]) / results[0]["w1"]

    line = {
        "metric": METRIC, "value": solves_counted_per_s, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step,
        "step_ms": {"median": float(np.median(step_s)) * 1e3, "min": min(step_s) * 1e3, "max": max(step_s) * 1e3},
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"uniform batch: {P} pairs, n={n} ({n + 1}^2 nodes), rectangles/disks on 1e-4 "
                               f"floor, {args.ground.upper()} metric, {L}-level cascade{' step_scale ' + str(args.step_scale) if args.step_scale else ''}, plain PDHG (Algorithm 3), paper stop rule "
                               "eq. (stop_tol) alpha=-1, FP32 iterates / FP64 reductions",
                   "global_batch": P, "grid": n, "levels": L, "parallelism": "batch"},
        "cell_updates_per_s": cups,
        "fp64_single": {"solves_per_s": fp64_sps, "sample": args.fp64_sample,
                        "speedup_batched_fp32": solves_counted_per_s / fp64_sps if fp64_sps else None},
        "solves_per_s_all": solves_per_s,
        "accuracy": {"reference": "none (--no-fp64-ref): every solve counted" if args.no_fp64_ref
                     else "FP64 batched GPU path, every pair", "checked": 0 if args.no_fp64_ref else len(rel_all),
                     "within_1e-4": good, "max_rel": max(rel_all), "median_rel": float(np.median(rel_all)),
                     "capped_solves": capped, "outside_1e-4": same_iter,
                     "fp64_single_sample": {"checked": len(rel), "within_1e-4": sum(x <= 1e-4 for x in rel),
                                            "max_rel": max(rel) if rel else None}},
        "iterations": iter_stats, "roofline": roof, "kernel_timing": TIMING_NOTE, "kernels": kernels, "autotune": tuned,
        "engine_counters": counters, "cpu_baseline": cpu,
        "context": "paper: 0.2-1.5 s per 512x512 W1 on one i7-2600 (MATLAB, Algorithm 4)",
    }
    solver.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
