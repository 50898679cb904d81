"""Throughput of the Kalman-MPC hot path on one MI355X.

One step = one closed-loop MPC step: a full solve (Algorithm 1: rollout, means,
pooled statistics, FP64 gain, analysis of every stored slice) through the C ABI
with device-resident inputs and device-generated noise, followed by the plant
step X_{k+1} = CNN(X_k, U_hat_k).  Default workload: the largest one-GPU
configuration, a 256x256 field, l = 64, CNN 2-64-64-64-64-1 (GELU), N = 512
members, horizon H = 20.

Prints one JSON line: metric member-steps/s (= N H solves/s) of the FP32 path (the
headline `value`), with solves/s, p50/p99 solve latency, the roofline of the dominant
kernel class (from HIP events recorded by the library on its stream) and the FP64 CPU
oracle timed on a bounded sample of the same workload; beside it, under `precisions`,
the same figures for the BF16 and FP8 rollouts with their smoothed-control error and
closed-loop tracking cost against the FP32 path.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"hbm": 8.0e12, "fp32": 157.3e12, "fp64": 78.6e12, "bf16": 2.5e15, "fp8": 5.0e15}


def workload_name(p):
    ch = "-".join(str(c) for c in p.channels)
    act = "tanh" if p.activation == 0 else "gelu"
    return (f"{p.name}: {p.n}x{p.m} field, l={p.l}, CNN {ch} ({act}), N={p.N}, H={p.H}, "
            f"closed-loop MPC steps")


def algorithmic_work(p, H, precision="fp32"):
    """Per kernel class: (FLOP, HBM bytes) the method needs in one solve, summed over
    the launches of that class.  FLOPs count multiply-adds as 2; bytes are the operands
    each launch must read and write once (activations 2 B in BF16/FP8, 4 B in FP32)."""
    n, m, l, N = p.n, p.m, p.l, p.N
    rr = pp = n + l
    NM = N * m
    ab = 4 if precision == "fp32" else 2
    work = {}

    def add(k, f, b):
        f0, b0 = work.get(k, (0.0, 0.0))
        work[k] = (f0 + f, b0 + b)

    L = len(p.channels) - 1
    folded = last_layer_folded(p, precision)
    px = n * m * N
    # a 64-channel first layer takes its lift channel B U precomputed: the lift reads U and
    # writes B U, the layer reads X and B U
    lifted = L > 1 and p.channels[1] >= 64
    for t in range(1, H + 1):
        if lifted:
            add("lift", 2.0 * l * px, 4.0 * (l * m * N + px))
        Ma = (t + 1) * rr
        for k, (ci, co) in enumerate(zip(p.channels[:-1], p.channels[1:])):
            cls = "conv_first" if k == 0 else ("conv_last" if k == L - 1 else "conv_mid")
            rd = (4.0 * (2 * px if lifted else (n + l) * m * N)) if k == 0 else ab * ci * px
            wr = 4.0 * px if k == L - 1 else ab * co * px
            f = 2.0 * 9 * ci * co * px
            if folded and k == L - 2:
                # the last layer's products run in this launch's epilogue, which writes the
                # nine FP32 tap planes instead of the activations
                f += 2.0 * 9 * co * px
                wr = 4.0 * 9 * px
            if folded and k == L - 1:
                # the remaining tap sum: nine planes read, the state written
                f, rd = 9.0 * px, 4.0 * 9 * px
            add(cls, f, rd + wr)
        add("stats", 2.0 * (Ma + pp) * pp * NM, 4.0 * (Ma + pp) * NM)
        # time at peak: Sigma^{XY} on the FP32 matrix cores in every mode, Sigma^Y on the
        # FP64 ones in the FP32 mode (FP32 otherwise); the class's peak is the FLOP-weighted one
        yy_peak = PEAK["fp64"] if precision == "fp32" else PEAK["fp32"]
        add("stats_t_peak", 2.0 * Ma * pp * NM / PEAK["fp32"] + 2.0 * pp * pp * NM / yy_peak, 0.0)
        add("update", 2.0 * Ma * pp * NM, 4.0 * (2 * Ma + pp) * NM)
        add("means", float(pp) * NM, 4.0 * pp * NM)
        add("chol", float(pp) ** 3, 16.0 * pp * pp)  # Cholesky, triangular inverse, W^T W
        add("gain", 2.0 * pp * pp * Ma, 8.0 * (Ma * pp + pp * pp) + 4.0 * Ma * pp)
    add("means", float((H + 1) * rr) * NM, 4.0 * (H + 1) * rr * NM)  # final smoothed means
    return work


def last_layer_folded(p, precision):
    """Whether the library folds the last layer (C -> 1) into the last hidden layer's
    epilogue: every rollout precision, with a last hidden layer of 32 or 64 inputs and 64
    outputs (the library's conv_last_folds / conv_last_folds_bf16)."""
    ch = p.channels
    return precision in ("fp32", "bf16", "fp8") and len(ch) >= 4 and ch[-2] == 64 and ch[-3] in (32, 64)


MATRIX_CLASSES = ("conv_first", "conv_mid", "stats", "gain", "update")
SOURCE_OF = {"conv_first": "rollout.hip", "conv_mid": "rollout.hip", "conv_last": "rollout.hip",
             "stats": "stats.hip", "stats_reduce": "stats.hip",
             "means": "stats.hip", "chol": "gain.hip", "gain": "gain.hip", "update": "update.hip",
             "noise": "noise.hip", "assemble": "noise.hip", "observe": "noise.hip", "init": "noise.hip",
             "lift": "rollout.hip"}


def roofline_for(cls, flops, nbytes, ms, launches, precision, tag=None, t_peak=None):
    sec = ms * 1e-3
    if t_peak:  # a class whose launches run on matrix cores of different precisions
        fpeak = flops / t_peak
    elif cls in ("gain", "chol"):
        fpeak = PEAK["fp64"]
    elif cls.startswith("conv"):
        fpeak = {"bf16": PEAK["bf16"], "fp8": PEAK["fp8"]}.get(precision, PEAK["fp32"])
    else:
        fpeak = PEAK["fp32"]
    t_f = flops / fpeak
    t_b = nbytes / PEAK["hbm"]
    common = {"traffic": measured_traffic(cls, tag), "kernel_class": cls, "launches": launches,
              "avg_launch_us": 1e3 * ms / max(launches, 1),
              "algorithmic_bytes_per_launch": nbytes / max(launches, 1),
              "algorithmic_flop_per_launch": flops / max(launches, 1)}
    if t_b > t_f:
        ach = nbytes / sec / 1e9
        return dict({"bound": "hbm", "achieved": ach, "peak": PEAK["hbm"] / 1e9, "unit": "GB/s",
                     "frac": ach / (PEAK["hbm"] / 1e9)}, **common)
    ach = flops / sec / 1e12
    kind = "mfma" if cls in MATRIX_CLASSES else "alu"
    return dict({"bound": kind, "achieved": ach, "peak": fpeak / 1e12, "unit": "TFLOP/s",
                 "frac": ach / (fpeak / 1e12)}, **common)


def measured_traffic(cls, tag):
    """HBM bytes per launch of the class from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes of the same workload (each scaled by what the counter reads for a
    plain device copy of known size), or None when there are none, they were taken on
    another workload, or the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(tag, {}).get(cls)
    except (OSError, ValueError, AttributeError):
        return None
    if not rec:
        return None
    src = os.path.join(ROOT, "paper_2410_09663_amd", "csrc", SOURCE_OF.get(cls, ""))
    try:
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if sha != rec.get("source_sha256"):
        return None
    return rec["hbm_bytes_per_launch"]


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        return len(os.sched_getaffinity(0))


def cpu_baseline(p, prob, seconds_budget=25.0):
    """The FP64 oracle on the host cores: closed-loop solves of the same workload
    until about `seconds_budget` seconds of work (at least one)."""
    from oracle import enks, philox
    from paper_2410_09663_amd import workloads as wl
    threads = _blas_threads()
    X = prob.X0.astype(np.float64)
    Up = np.zeros((p.l, p.m))
    t0 = time.perf_counter()
    solves = 0
    first = None
    while True:
        z = philox.solve_noise(p.noise_seed_base + solves, p.n, p.m, p.l, p.N, p.H)
        res = enks.solve(prob.B, prob.weights, p.activation, X, wl.reference_window(p, solves),
                         prob.Q, prob.Q, prob.R, p.N, p.H, *z, U_prev=Up)
        if first is None:
            first = res
        Up = res.U_mean[0]
        X = enks.plant_step(X, Up, prob.B, prob.weights, p.activation)
        solves += 1
        if time.perf_counter() - t0 > seconds_budget or solves >= 20:
            break
    el = time.perf_counter() - t0
    return {"value": p.N * p.H * solves / el, "unit": "member-steps/s", "cores": int(threads),
            "kind": "oracle", "solves_per_s": solves / el,
            "sample": f"{solves} closed-loop solve(s) of the same workload, FP64 NumPy, "
                      f"{el:.1f} s wall"}, first


def cpu_baseline_sampled(p, prob, members, members_one_thread=None):
    """The FP64 oracle on a bounded sample of a workload whose full solve takes the
    oracle minutes: one oracle solve with one horizon step (H = 1: the rollout of every
    sampled member, then one analysis of the two stored slices) on the full grid and CNN
    with `members` of the N members, i.e. `members` member-steps of the same per-member
    work; member-steps/s = members / wall time.  The analysis's share of a member-step
    grows with the stored slices (j = 2 here, up to H + 1 in a full solve), which this
    sample does not include.  Beside it the same sample with `members_one_thread` members
    (default: the fewest whose pooled covariance can be positive definite, at least 3) on
    one BLAS thread."""
    from oracle import enks, philox
    from paper_2410_09663_amd import workloads as wl
    threads = _blas_threads()
    if members_one_thread is None:
        members_one_thread = max(3, -(-(p.n + p.l) // p.m) + 1)

    def timed(k):
        z = philox.solve_noise(p.noise_seed_base, p.n, p.m, p.l, k, 1)
        t0 = time.perf_counter()
        enks.solve(prob.B, prob.weights, p.activation, prob.X0, wl.reference_window(p, 0, 1), prob.Q, prob.Q,
                   prob.R, k, 1, *z)
        return time.perf_counter() - t0

    el = timed(members)
    out = {"value": members / el, "unit": "member-steps/s", "cores": int(threads), "kind": "oracle",
           "solves_per_s": members / el / (p.N * p.H),
           "sample": f"one FP64 NumPy oracle solve with H = 1 and {members} of the {p.N} members on the "
                     f"full {p.n}x{p.m} grid and CNN ({members} member-steps, one analysis at j = 2), "
                     f"{el:.1f} s wall; solves/s scaled by N H = {p.N * p.H}"}
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        return out
    with threadpool_limits(limits=1):
        el1 = timed(members_one_thread)
    out["one_thread"] = {"value": members_one_thread / el1, "unit": "member-steps/s", "cores": 1,
                         "sample": f"the same with {members_one_thread} members on one BLAS thread, "
                                   f"{el1:.1f} s wall"}
    return out


def serve_main(args):
    """Serving workload: many independent controllers (grids 32^2..256^2, N 64..256, H 5..20,
    BF16 rollout) behind one request loop with continuous admission by HBM footprint and
    grouped solves of same-shape requests.  Runs over the same request list: (1) every
    request submitted at once (capacity, solves/s); (2) Poisson arrivals at the offered rate
    (default 400 solves/s, above capacity: latency is queue-dominated); (3) Poisson arrivals
    at 70% of the measured capacity; (4) the requests of the grids below 256^2 alone, all at
    once.  Runs (1) and (4) again on a server with one slot per pack (every request its own
    solve, overlapping only as concurrent streams) give the gain of the grouped solves.
    Then each distinct shape solved alone (resident, graph warm), summed over the request
    list.  Last, the same requests in the plain FP32 single-request form (one solve at a
    time, FP32 rollout), whose solves/s gives the speed-up."""
    from paper_2410_09663_amd import oic
    from paper_2410_09663_amd import workloads as wl

    mix = wl.serving_mix(args.controllers)
    probs = [wl.make_problem(p) for p in mix]
    rng = np.random.default_rng(99)
    ctrl_of = rng.integers(0, len(probs), args.requests)
    step_of = np.zeros(args.requests, np.int64)
    seen = {}
    for r, c in enumerate(ctrl_of):
        step_of[r] = seen.get(int(c), 0) + 1  # step 0 is the warm-up request
        seen[int(c)] = step_of[r]
    budget = int(args.hbm_gb * (1 << 30))

    def inputs(c, k):
        p = probs[c].preset
        return (probs[c].X0 * (1.0 + 0.02 * k)).astype(np.float32), wl.reference_window(p, k), \
            p.noise_seed_base + k

    def run(srv, ids, rate, seed, reqs=None):
        reqs = list(range(args.requests)) if reqs is None else reqs
        arr = np.zeros(len(reqs))
        if rate:
            arr = np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, len(reqs)))
        t0 = time.perf_counter()
        sub = []
        for j, r in enumerate(reqs):
            while time.perf_counter() - t0 < arr[j]:
                time.sleep(min(1e-3, max(0.0, arr[j] - (time.perf_counter() - t0))))
            c = int(ctrl_of[r])
            X0, ref, sd = inputs(c, int(step_of[r]))
            sub.append((c, time.perf_counter() - t0, srv.submit(ids[c], X0, ref, sd)))
        lat, svc, done = [], [], []
        for j, (c, ts, t) in enumerate(sub):
            if j % 50 == 0:
                print(f"[serve] {j}/{len(sub)} results", file=sys.stderr, flush=True)
            _, _, ms, q = srv.wait(ids[c], t)
            lat.append(ms)
            svc.append(ms - q)
            done.append(ts + 1e-3 * ms)
        span = max(done)
        return {"solves_per_s": len(reqs) / span, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "service_p50_ms": float(np.percentile(svc, 50)),
                "service_p99_ms": float(np.percentile(svc, 99)), "makespan_s": span}

    def warm(srv, ids):
        print(f"[serve] warm-up: one request per controller ({len(probs)})", file=sys.stderr, flush=True)
        for c in range(len(probs)):
            if c % 25 == 0:
                print(f"[serve] warm-up {c}/{len(probs)}", file=sys.stderr, flush=True)
            X0, ref, sd = inputs(c, 0)
            srv.wait(ids[c], srv.submit(ids[c], X0, ref, sd))

    out = {"metric": "solves/s (served mix)", "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": f"serving: {args.controllers} controllers, grids "
                                  f"{list(wl.SERVE_GRIDS)}, N {list(wl.SERVE_N)}, H {list(wl.SERVE_H)}, "
                                  f"BF16 rollout, FP64 gain; {args.requests} requests",
                      "hbm_budget_gb": args.hbm_gb, "max_inflight": args.inflight}}
    # the requests of the controllers below 256x256 (whose solves leave the GPU partly idle)
    small = [r for r in range(args.requests) if probs[int(ctrl_of[r])].preset.n < 256]
    with oic.Server(budget, max_inflight=args.inflight) as srv:
        ids = [srv.add(pr, pr.preset.N, pr.preset.H) for pr in probs]
        warm(srv, ids)
        cap = run(srv, ids, None, 0)
        offered = run(srv, ids, args.rate, 1)
        sustain_rate = 0.7 * cap["solves_per_s"]
        sustained = run(srv, ids, sustain_rate, 2)
        small_cap = run(srv, ids, None, 3, small)
        st = srv.stats()
    out.update({"value": cap["solves_per_s"], "capacity": cap,
                "offered": dict(offered, rate=args.rate),
                "sustainable": dict(sustained, rate=sustain_rate),
                "small_grids_capacity": dict(small_cap, requests=len(small)), "server": st})
    # the same server with one slot per pack: every request its own solve, requests overlapping
    # only as concurrent streams (no shared launches)
    print("[serve] one slot per pack (no grouped solves)", file=sys.stderr, flush=True)
    with oic.Server(budget, max_inflight=args.inflight, group_slots=1) as srv:
        ids = [srv.add(pr, pr.preset.N, pr.preset.H) for pr in probs]
        warm(srv, ids)
        ung_cap = run(srv, ids, None, 0)
        ung_small = run(srv, ids, None, 3, small)
    out["one_slot_per_pack"] = {"capacity": ung_cap, "small_grids_capacity": ung_small,
                                "grouped_over_one_slot": cap["solves_per_s"] / ung_cap["solves_per_s"],
                                "small_grids_grouped_over_one_slot":
                                    small_cap["solves_per_s"] / ung_small["solves_per_s"]}
    # each distinct (grid, N, H) solved alone on a resident controller (graph warm), summed
    # over the request list: the GPU time the requests need without any overlap
    print("[serve] solo solve times per shape", file=sys.stderr, flush=True)
    shape_ms = {}
    for c, pr in enumerate(probs):
        p = pr.preset
        key = (p.n, p.N, p.H)
        if key in shape_ms:
            continue
        with oic.controller_for(pr, precision=wl.PREC_BF16) as h:
            X0, ref, _ = inputs(c, 0)
            ts = []
            for k in range(4):
                t0 = time.perf_counter()
                h.solve(X0, ref, pr.Q, pr.R, p.N, p.H, 1 + k, want_X=True)
                ts.append(time.perf_counter() - t0)
        shape_ms[key] = 1e3 * float(np.median(ts[1:]))
    solo_by_grid = {}
    for c in ctrl_of:
        p = probs[int(c)].preset
        solo_by_grid[p.n] = solo_by_grid.get(p.n, 0.0) + 1e-3 * shape_ms[(p.n, p.N, p.H)]
    solo_sum = sum(solo_by_grid.values())
    out["solo"] = {"sum_s": solo_sum, "by_grid_s": {str(g): v for g, v in sorted(solo_by_grid.items())},
                   "capacity_makespan_over_sum": cap["makespan_s"] / solo_sum,
                   "shape_ms": {f"{g}x{g} N={N} H={H}": v for (g, N, H), v in sorted(shape_ms.items())}}
    if not args.no_fp32_baseline:
        with oic.Server(budget, max_inflight=1) as srv:
            ids = [srv.add(pr, pr.preset.N, pr.preset.H, precision=wl.PREC_FP32) for pr in probs]
            warm(srv, ids)
            single = run(srv, ids, None, 0)
        out["fp32_single_request"] = single
        out["speedup_solves_per_s"] = cap["solves_per_s"] / single["solves_per_s"]
        out["p99_ms_fp32_single_service"] = single["service_p99_ms"]
    print(json.dumps(out), flush=True)


PRECISIONS = ("fp32", "bf16", "fp8")
DTYPE = {"fp32": "f32", "bf16": "bf16", "fp8": "fp8-e4m3"}


def run_precision(p, prob, precision, K, W, eager_steps, dev):
    """W warm-up and K timed closed-loop steps of one precision, then `eager_steps` more
    launched kernel by kernel with HIP events around every launch (per-class durations
    for the roofline).  Returns the figures of the run and the first solve's U_hat."""
    import torch
    from paper_2410_09663_amd import oic
    from paper_2410_09663_amd import workloads as wl

    prec = {"fp32": oic.OIC_PREC_FP32, "bf16": oic.OIC_PREC_BF16, "fp8": oic.OIC_PREC_FP8}[precision]
    steps = W + K + eager_steps
    refs = torch.from_numpy(np.stack([wl.reference_window(p, k) for k in range(steps + 1)])).to(dev)
    stream = torch.cuda.current_stream().cuda_stream
    ctrl = oic.controller_for(prob, precision=prec, mem_mode=oic.OIC_MEM_DEVICE, stream=stream)
    # the plant step runs on a handle of its own, so that the per-kernel durations of the
    # solve handle hold the solve's launches only
    plant = oic.controller_for(prob, max_N=2, max_H=1, precision=oic.OIC_PREC_FP32,
                               mem_mode=oic.OIC_MEM_DEVICE, stream=stream)
    Ubufs = torch.empty((steps, p.H + 1, p.l, p.m), dtype=torch.float32, device=dev)
    Xbuf = torch.empty((p.H + 1, p.n, p.m), dtype=torch.float32, device=dev)

    def step(k, X):
        # full smoother output: U_hat and X_hat of every slice (Algorithm 1, line 13)
        ctrl.solve(X, refs[k], prob.Q, prob.R, p.N, p.H, p.noise_seed_base + k, U_out=Ubufs[k],
                   X_out=Xbuf)
        return plant.plant_step(X, Ubufs[k][0])

    X = torch.from_numpy(prob.X0).to(dev)
    states = [X]
    for k in range(W):
        X = step(k, X)
        states.append(X)
    torch.cuda.synchronize()
    # Timed region: K closed-loop steps, each solve replayed from its captured graph.
    lat = []
    t0 = time.perf_counter()
    for k in range(W, W + K):
        ts = time.perf_counter()
        X = step(k, X)
        lat.append(time.perf_counter() - ts)
        states.append(X)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # Per-kernel durations: more steps of the same loop, launched kernel by kernel with HIP
    # events around every launch on the library's stream (events cannot sit inside a
    # replayed graph); the per-class totals feed the roofline.
    ctrl.timing(True)
    for k in range(W + K, steps):
        X = step(k, X)
        states.append(X)
    torch.cuda.synchronize()
    stats = ctrl.kernel_stats()
    ctrl.timing(False)
    ctrl.close()
    plant.close()

    # closed-loop tracking cost of every realised step (problem-setup stage cost, FP64 host)
    Xs = torch.stack(states).cpu().numpy()
    Us = Ubufs[:, 0].cpu().numpy()
    first_U = Ubufs[0].cpu().numpy()
    loop_cost = 0.0
    Uprev = np.zeros((p.l, p.m), np.float32)
    for k in range(steps):
        loop_cost += oic.stage_cost(Xs[k + 1], wl.reference_at(p, k + 1), Us[k], Us[k] - Uprev, prob.Q, prob.R)
        Uprev = Us[k]
    mse_last = float(np.mean((Xs[-1].astype(np.float64) - wl.reference_at(p, steps)) ** 2))

    work = algorithmic_work(p, p.H, precision)
    per_class = {}
    for cls, (cnt, ms) in stats.items():
        if cnt == 0:
            continue
        f, b = work.get(cls, (0.0, 0.0))
        per_class[cls] = {"launches": cnt, "total_ms": ms, "flop": f * eager_steps, "bytes": b * eager_steps,
                          "t_peak": work.get(cls + "_t_peak", (0.0, 0.0))[0] * eager_steps}
    dom = max(per_class, key=lambda c: per_class[c]["total_ms"])
    d = per_class[dom]
    roof = roofline_for(dom, d["flop"], d["bytes"], d["total_ms"], d["launches"], precision,
                        f"{p.name}_{precision}", d["t_peak"])
    roof["measured"] = ("HIP events around each launch on the library stream, over "
                        f"{eager_steps} closed-loop steps launched kernel by kernel right after the timed region")
    # every class that does matrix work, and the two figures the method's targets name:
    # the whole rollout against the MFMA peak of its precision, the update against HBM
    by_class = {}
    for cls in ("lift", "conv_first", "conv_mid", "conv_last", "stats", "gain", "update"):
        if cls in per_class and per_class[cls]["flop"] > 0:
            c = per_class[cls]
            r = roofline_for(cls, c["flop"], c["bytes"], c["total_ms"], c["launches"], precision,
                             t_peak=c["t_peak"])
            by_class[cls] = {k: r[k] for k in ("bound", "achieved", "peak", "unit", "frac", "avg_launch_us")}
    conv = [per_class[c] for c in ("lift", "conv_first", "conv_mid", "conv_last") if c in per_class]
    conv_s = sum(c["total_ms"] for c in conv) * 1e-3
    mfma_peak = {"bf16": PEAK["bf16"], "fp8": PEAK["fp8"]}.get(precision, PEAK["fp32"])
    rollout_frac = sum(c["flop"] for c in conv) / conv_s / mfma_peak if conv_s > 0 else None
    upd = per_class.get("update")
    update_frac = upd["bytes"] / (upd["total_ms"] * 1e-3) / PEAK["hbm"] if upd else None
    lat_ms = np.array(lat) * 1e3
    solves_per_s = K / el
    out = {"member_steps_per_s": p.N * p.H * solves_per_s, "solves_per_s": solves_per_s,
           "ms_per_step": 1e3 * el / K, "p50_ms": float(np.percentile(lat_ms, 50)),
           "p99_ms": float(np.percentile(lat_ms, 99)), "dtype": DTYPE[precision],
           "closed_loop_steps": steps, "closed_loop_cost": loop_cost, "tracking_mse_last": mse_last,
           "tracking_rmse_last": float(np.sqrt(mse_last)), "roofline": roof, "roofline_by_class": by_class,
           "rollout_mfma_frac": rollout_frac, "update_hbm_frac": update_frac,
           "kernel_ms_per_solve": {c: v["total_ms"] / eager_steps for c, v in sorted(per_class.items())}}
    return out, first_U


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)  # at least 1
    ap.add_argument("--workload", default="C4")
    ap.add_argument("--precision", default="all", choices=["all", *PRECISIONS],
                    help="all: FP32 (the headline value) and, beside it, BF16 and FP8")
    ap.add_argument("--eager-steps", type=int, default=2,
                    help="closed-loop steps launched kernel by kernel for the per-kernel durations")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    ap.add_argument("--cpu-members", type=int, default=64,
                    help="members of the oracle's one-step sample on workloads it cannot solve in seconds")
    # serving workload (--workload C5)
    ap.add_argument("--controllers", type=int, default=200)
    ap.add_argument("--requests", type=int, default=400)
    ap.add_argument("--rate", type=float, default=400.0)
    ap.add_argument("--hbm-gb", type=float, default=200.0)
    ap.add_argument("--inflight", type=int, default=8)
    ap.add_argument("--no-fp32-baseline", action="store_true")
    # a plain 256 MiB device-to-device copy, three times: the reference that scales the
    # FETCH_SIZE / WRITE_SIZE counters of a rocprofv3 --pmc run into HBM bytes
    ap.add_argument("--calibrate-copy", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 (sharding the ensemble members "
                                   "over several GPUs is not implemented)"}))
        sys.exit(2)

    import torch
    from paper_2410_09663_amd import oic
    from paper_2410_09663_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        x = torch.ones(64 << 20, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each": x.numel() * 4, "copies": 3}), flush=True)
        return
    if args.workload == "C5":
        serve_main(args)
        return
    dev = torch.device("cuda:0")
    p = wl.PRESETS[args.workload]
    prob = wl.make_problem(p)
    K, W, E = args.steps, max(1, args.warmup), max(1, args.eager_steps)
    precs = PRECISIONS if args.precision == "all" else (args.precision,)
    runs, firsts = {}, {}
    for prec in precs:
        print(f"[bench] {p.name} {prec}: {W} warm-up, {K} timed, {E} per-kernel steps", file=sys.stderr,
              flush=True)
        runs[prec], firsts[prec] = run_precision(p, prob, prec, K, W, E, dev)
    head = precs[0]
    r0 = runs[head]
    out = {
        "metric": "member-steps/s", "value": r0["member_steps_per_s"], "unit": "member-steps/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": r0["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": r0["dtype"], "data": "synthetic",
        "config": {"workload": workload_name(p), "n": p.n, "m": p.m, "l": p.l, "N": p.N, "H": p.H,
                   "channels": p.channels, "precision": head},
        "solves_per_s": r0["solves_per_s"], "p50_ms": r0["p50_ms"], "p99_ms": r0["p99_ms"],
        "roofline": r0["roofline"],
    }
    out.update({k: r0[k] for k in ("roofline_by_class", "rollout_mfma_frac", "update_hbm_frac",
                                   "kernel_ms_per_solve", "closed_loop_steps", "closed_loop_cost",
                                   "tracking_mse_last", "tracking_rmse_last")})
    if len(precs) > 1:
        # reduced-precision rollouts beside FP32: the same closed loop (same X_0, seeds and
        # references), their first solve's U_hat against FP32's (identical inputs), and the
        # closed-loop tracking cost over the same steps
        j32 = r0["closed_loop_cost"]
        u32 = firsts[head].astype(np.float64)
        out["precisions"] = {}
        for prec in precs[1:]:
            r = runs[prec]
            u = firsts[prec].astype(np.float64)
            keep = ("member_steps_per_s", "solves_per_s", "ms_per_step", "p50_ms", "p99_ms", "dtype",
                    "rollout_mfma_frac", "update_hbm_frac", "closed_loop_cost", "kernel_ms_per_solve")
            e = {k: r[k] for k in keep}
            e["roofline"] = {k: r["roofline"][k] for k in ("kernel_class", "bound", "achieved", "peak",
                                                          "unit", "frac")}
            e["relerr_U_vs_fp32_gpu"] = float(np.linalg.norm(u - u32) / np.linalg.norm(u32))
            e["max_relerr_U_vs_fp32_gpu"] = float(np.max(np.abs(u - u32)) / np.max(np.abs(u32)))
            e["cost_rel_vs_fp32"] = abs(r["closed_loop_cost"] - j32) / j32
            e["speedup_vs_fp32"] = r["member_steps_per_s"] / r0["member_steps_per_s"]
            out["precisions"][prec] = e
    if not args.no_cpu_baseline:
        if p.n * p.m * p.N <= 64 * 64 * 128:
            cb, first = cpu_baseline(p, prob, args.cpu_seconds)
            out["cpu_baseline"] = cb
            # parity of the first closed-loop solve of the same stream, for the record
            c2 = oic.controller_for(prob, precision={"fp32": oic.OIC_PREC_FP32, "bf16": oic.OIC_PREC_BF16,
                                                     "fp8": oic.OIC_PREC_FP8}[head])
            U, _ = c2.solve(prob.X0, wl.reference_window(p, 0), prob.Q, prob.R, p.N, p.H,
                            p.noise_seed_base)
            c2.close()
            out["relerr_U_vs_fp64_oracle"] = float(np.linalg.norm(U - first.U_mean) /
                                                   np.linalg.norm(first.U_mean))
        else:
            out["cpu_baseline"] = cpu_baseline_sampled(p, prob, min(args.cpu_members, p.N))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
