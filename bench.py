#!/usr/bin/env python3
"""Benchmark: macro-particle-turns/s of the plain FP64 GPU tracker on one MI355X.

Workload (default): the current-scan configuration -- eight single-bunch jobs
of 1e6 macro-particles each (bunch currents 0.1-5 mA), 3rd-harmonic cavity at
90% of its flat-potential voltage, broadband-resonator wake on 512 bins,
run as one launch set per turn.  A step is one turn of the whole hot path
(between-turn kernel: moments, wake potential; push kernel: kick, damping,
noise, drift, histogram, deposits, moment sums; moment output).  Inputs are
resident in HBM before the timed region.

Prints one JSON line with the throughput, the push kernel's roofline figures
(algorithmic bytes per launch / average launch duration from HIP events over
the timed region) and the oracle timed on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, vendor figure
# Vector issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64 VALU
# instruction occupies a SIMD for four cycles), in lane-instructions/s.
VALU_PEAK = 256 * 4 * 16 * 2.4e9
BYTES_PER_PARTICLE_TURN = 32  # read tau, delta + write tau, delta (FP64)
PMC_FILE = os.path.join(ROOT, "profiles", "push_c2_pmc.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_1809_00391_amd", "csrc", f)
               for f in ("mbt_kernels.hip", "mbt_fastmath.h", "mbt_internal.h")]


def kernel_sha():
    """Hash of the device code: every source the kernels are built from, with
    comments and blank lines removed (a comment changes no kernel)."""
    import re
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def pmc_record(particles_per_launch):
    """The committed rocprofv3 counter record of the push (FETCH_SIZE and
    WRITE_SIZE scaled by a copy kernel of known size, SQ instruction counts),
    or None when it is missing or was taken on a different kernel source or
    workload."""
    if not os.path.exists(PMC_FILE):
        return None
    d = json.load(open(PMC_FILE))
    if d.get("kernel_sha") != kernel_sha() or d.get("particles_per_launch") != particles_per_launch:
        return None
    return d


def make_tracker(w):
    from paper_1809_00391_amd import tracker as tr
    t = tr.Tracker(w.ring)
    if w.hc_flat:
        t.set_harmonic_cavity(tr.hc_flat_fraction(w.ring, *w.hc_flat))
    t.set_fill(w.buckets, w.currents_A, w.streams)
    if w.grid is not None:
        t.set_short_range(list(w.short_range), w.grid)
    if w.long_range:
        t.set_long_range(list(w.long_range))
    t.bind(w.N)
    t.init_gaussian(w.sigma_tau0, w.sigma_delta0, w.seed)
    return t


def cpu_baseline(w, budget_s):
    """The oracle (as it stands) on this host's cores, on a bounded number of
    turns of the same workload; then the same with one thread."""
    from oracle import ref
    allc = ref.threads()
    out = _oracle_rate(w, budget_s)
    ref.set_threads(1)
    try:
        one = _oracle_rate(w, budget_s / 3)
    finally:
        ref.set_threads(allc)
    out["single_thread"] = {"value": one["value"], "cores": 1, "sample": one["sample"]}
    return out


def _oracle_rate(w, budget_s):
    from oracle import ref
    s = ref.RefSim(w.ring)
    if w.hc_flat:
        s.set_harmonic_cavity(ref.hc_flat_fraction(w.ring, *w.hc_flat))
    s.set_fill(w.buckets, w.currents_A, w.streams)
    if w.grid is not None:
        s.set_short_range(list(w.short_range), w.grid)
    if w.long_range:
        s.set_long_range(list(w.long_range))
    s.init_gaussian(w.N, w.sigma_tau0, w.sigma_delta0, w.seed)
    t0 = time.perf_counter()
    s.track(2)
    per_turn = (time.perf_counter() - t0) / 2
    turns = int(max(2, min(1000, budget_s / max(per_turn, 1e-9))))
    t0 = time.perf_counter()
    s.track(turns)
    dt = time.perf_counter() - t0
    return {"value": w.M * w.N * turns / dt, "unit": "macro-particle-turns/s",
            "cores": ref.threads(), "kind": "oracle",
            "sample": f"{turns} turns of the same workload ({w.M} x {w.N} particles) after 2 "
                      f"warm-up turns, {dt:.1f} s"}


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Device-to-device bandwidth of the library's own streaming copy kernel
    (mbt_stream_copy) over a buffer four times the Infinity Cache: bytes read
    plus bytes written per second, best of `reps` timed copies."""
    import torch
    from paper_1809_00391_amd import tracker as tr
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    s = torch.cuda.current_stream()
    tr.stream_copy(a, b, s)
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        tr.stream_copy(a, b, s)
        e1.record(s)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    ok = bool(torch.equal(a, b))
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / best / 1e9, ok


def full_fill(turns, wake, copy_gbs=None):
    """The full-fill configuration (484 bunches x 1e5 particles, BB wake on
    256 bins, HOM long-range resonator) tracked `turns` turns twice: by the
    plain FP64 tracker (eager launches, FP64 VALU convolution) and in the
    batched mixed-precision form (captured 16-turn graphs, launch shape tuned
    online, wake potential on the matrix cores in `wake`).  Moments are
    copied out in both.  Returns both throughputs."""
    import torch
    from paper_1809_00391_amd import tracker as tr
    from paper_1809_00391_amd import workloads as wl
    w = wl.PRESETS["c4"]
    particles = w.M * w.N
    res = {"workload": w.name, "turns_timed": turns, "unit": "macro-particle-turns/s"}
    for form in ("plain_fp64", "batched_mixed"):
        t = make_tracker(w)
        b = None
        if form == "batched_mixed":
            t.set_wake_precision(wake)
            b = tr.Batch([t], stream=t.stream, graph_turns=16, autotune=True)
            run = lambda n: b.track(n, moments=True)
        else:
            run = lambda n: t.track(n, moments=True)
        run(64)   # warm-up; the tuner measures its candidates here
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(turns)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[form] = {"value": particles * turns / dt, "ms_per_turn": dt * 1e3 / turns}
        if b is None:
            # this state (774 MB) is three times the Infinity Cache: the HBM
            # case.  The push is timed on further turns, every one bracketed
            # by HIP events, outside the throughput measurement above.
            t.set_timing(1)
            run(min(turns, 200))
            torch.cuda.synchronize()
            push_ms, push_n, _, _ = t.get_timing()
            if push_n:
                push_s = push_ms / 1e3 / push_n
                gbs = BYTES_PER_PARTICLE_TURN * particles / push_s / 1e9
                res[form]["push_roofline"] = {
                    "bound": "hbm", "avg_launch_us": push_s * 1e6, "launches_timed": push_n,
                    "bytes_per_launch": BYTES_PER_PARTICLE_TURN * particles, "achieved": gbs,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                    "frac_of_copy": gbs / copy_gbs if copy_gbs else None}
        if b is not None:
            res[form].update({"wake": wake, "graph_turns": 16, "autotune": True,
                              "launch_groups": [list(g) for g in b.launch_info()]})
            b.close()
        t.close()
        torch.cuda.empty_cache()
    res["batched_over_plain"] = res["batched_mixed"]["value"] / res["plain_fp64"]["value"]
    return res


# Table 4 of the paper: wall time of 20,000 turns of bunches of 1e5
# macro-particles (radiation damping and quantum excitation on) on an 8-core
# workstation (2x Intel E5-2609 v2), a 36-core workstation (2x Intel E5-2697
# v4), a 576-core cluster (32x Intel Xeon Gold 6140) running the CPU code,
# and an NVIDIA Tesla K40c running the GPU code; None where it gives none.
PAPER_TABLE4_S = {
    1: (810, 549, 232, 93),
    2: (814, 558, 236, 157),
    3: (832, 562, 240, 221),
    10: (3596, 577, 266, 546),
    20: (None, 757, 312, 1006),
    121: (None, 2883, 922, 5860),
    363: (None, 10931, 3165, 18754),
}


def paper_table4(turns):
    """The bunch counts of Table 4 (1e5 macro-particles per bunch, radiation
    damping and quantum excitation on, consecutive buckets of the 480-bucket
    ring, broadband-resonator wake on 256 bins) tracked by the plain FP64
    tracker for `turns` turns; the time of 20,000 turns is extrapolated
    linearly (the per-turn cost is constant) and set beside the paper's."""
    import torch
    from paper_1809_00391_amd import workloads as wl
    rows = []
    for m, paper in PAPER_TABLE4_S.items():
        w = wl.C3.with_(name=f"{m} bunches", buckets=tuple(range(m)), currents_A=(1e-3,) * m,
                        long_range=(), N=100_000, seed=4)
        t = make_tracker(w)
        t.track(50, moments=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t.track(turns, moments=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        t.close()
        torch.cuda.empty_cache()
        rows.append({"bunches": m, "value": m * w.N * turns / dt,
                     "s_per_20000_turns": dt * 20000 / turns,
                     "paper_s": dict(zip(("cpu_8core", "cpu_36core", "cluster_576core", "k40c"), paper))})
    return {"turns_timed": turns, "unit": "macro-particle-turns/s", "rows": rows}


def serving_sample(scale, budget_gb, wake, fill):
    """The serving mix (64 jobs with Poisson arrivals at 2/s, bunch counts
    {1, 3, 40, 121, 363, 484}, 1e4-2e5 particles, 1000-20000 turns) with turns
    and arrival times scaled by `scale` so a sample takes seconds: once
    through the continuous-batching server (matrix-core wake `wake`), once as
    the plain per-job FP64 tracker running the jobs one after another in
    arrival order.  Returns throughput and p50/p99 job latency of both."""
    import numpy as np
    import torch
    from paper_1809_00391_amd import serve
    from paper_1809_00391_amd import workloads as wl
    reqs = []
    for i, (t, w) in enumerate(wl.serving_mix()):
        turns = max(50, int(round(w.turns * scale)))
        reqs.append(serve.Request(i, t * scale, w, turns))
    total = sum(r.workload.M * r.workload.N * r.turns for r in reqs)
    srv = serve.Server(hbm_budget=int(budget_gb * 2 ** 30), quantum=max(64, int(1000 * scale)),
                       graph_turns=16, autotune=False, wake=wake, fill_particles=fill)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = srv.run(reqs, keep_moments=False)
    span = time.perf_counter() - t0
    lat = serve.latency_percentiles(res)
    # plain FP64 tracker, one job at a time in arrival order
    t0 = time.perf_counter()
    done = []
    for r in sorted(reqs, key=lambda r: r.arrival_s):
        now = time.perf_counter() - t0
        if now < r.arrival_s:
            time.sleep(r.arrival_s - now)
        trk = serve.make_job(r.workload)
        trk.track(r.turns, moments=False)
        trk.close()
        done.append(time.perf_counter() - t0 - r.arrival_s)
    span_plain = time.perf_counter() - t0
    return {"jobs": len(reqs), "scale": scale, "particle_turns": total,
            "batched": {"value": total / span, "p50_s": lat["p50"], "p99_s": lat["p99"],
                        "wake": wake, "hbm_budget_gb": budget_gb, "fill_particles": fill,
                        "slices": srv.slices,
                        "batches_built": srv.batches_built, "peak_bytes": srv.peak_bytes},
            "plain_fp64_per_job": {"value": total / span_plain,
                                   "p50_s": float(np.percentile(done, 50)),
                                   "p99_s": float(np.percentile(done, 99))},
            "unit": "macro-particle-turns/s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000, help="timed turns")
    ap.add_argument("--warmup", type=int, default=200, help="untimed turns first")
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--timing-every", type=int, default=32,
                    help="bracket every k-th turn's launches with HIP events (each bracketed "
                         "turn costs about 12 us of event records at c2; 0: none)")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle time for the CPU baseline (0: skip)")
    ap.add_argument("--serve-scale", type=float, default=0.05,
                    help="turn and arrival-time scale of the serving sample (0: skip)")
    ap.add_argument("--serve-budget-gb", type=float, default=24.0,
                    help="HBM budget of the serving sample's admission")
    ap.add_argument("--serve-wake", default="bf16x2", choices=["fp64", "fp32", "bf16x2", "bf16x3"])
    ap.add_argument("--serve-fill", type=float, default=3.2e7,
                    help="admit while the admitted jobs hold fewer particles than this (0: no limit)")
    ap.add_argument("--table4-turns", type=int, default=1000,
                    help="turns of the paper's Table 4 bunch counts (0: skip)")
    ap.add_argument("--full-fill-turns", type=int, default=2000,
                    help="turns of the full-fill plain vs batched comparison (0: skip)")
    ap.add_argument("--copy-bw", type=int, default=1,
                    help="measure the library copy kernel's bandwidth (0: skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (counter scale for rocprofv3 --pmc)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the tracker is a "
              "single-GPU library; see DESIGN.md for how it would shard.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1809_00391_amd import workloads as wl

    w = wl.PRESETS[args.workload]
    torch.cuda.set_device(0)
    t = make_tracker(w)
    stream = t.stream
    with torch.cuda.stream(stream):
        if args.copy_probe:
            a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
            torch.cuda.synchronize()
            del a, b
        if args.warmup:
            t.track(args.warmup, moments=True)
        t.set_timing(args.timing_every)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        ev0.record(stream)
        mom = t.track(args.steps, moments=True)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
    gpu_ms = ev0.elapsed_time(ev1)
    elapsed = max(wall, gpu_ms / 1e3)
    push_ms, push_n, _, _ = t.get_timing()
    particles = w.M * w.N
    value = particles * args.steps / elapsed
    push_avg_s = push_ms / 1e3 / push_n if push_n else float("nan")
    achieved = BYTES_PER_PARTICLE_TURN * particles / push_avg_s / 1e9 if push_n else float("nan")
    pmc = pmc_record(particles)
    traffic = pmc["hbm_bytes_per_launch"] if pmc else None
    alu = None
    if pmc and push_n:
        lane_instr = pmc["valu_instructions_per_pair"] * particles / 2 / push_avg_s
        alu = {"bound": "alu", "valu_instructions_per_pair": pmc["valu_instructions_per_pair"],
               "achieved": lane_instr / 1e12, "peak": VALU_PEAK / 1e12,
               "unit": "T lane-instructions/s", "frac": lane_instr / VALU_PEAK,
               "source": "profiles/push_c2_pmc.json (SQ_INSTS_VALU of the same kernel source)"}
    finite = bool(torch.isfinite(torch.from_numpy(mom[-1])).all())
    copy_gbs, copy_ok = copy_bandwidth() if args.copy_bw else (None, None)

    out = {
        "metric": "macro-particle-turns/s (FP64 plain vs batched mixed-prec) at 1 GPU; "
                  "p50/p99 job lat",
        "value": value,
        "unit": "macro-particle-turns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "form": "plain FP64 tracker (one job per launch set, no graphs, no MFMA)",
            "bunches": w.M, "particles_per_bunch": w.N,
            "bins": w.grid[0] if w.grid else 0,
            "long_range_resonators": len(w.long_range),
            "turns_timed": args.steps,
        },
        "roofline": {
            "bound": "hbm", "kernel": "k_push",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "avg_launch_us": push_avg_s * 1e6, "launches_timed": push_n,
            "bytes_per_launch": BYTES_PER_PARTICLE_TURN * particles,
            "alu": alu,
            "copy_GBs": copy_gbs, "copy_exact": copy_ok,
            "frac_of_copy": achieved / copy_gbs if copy_gbs else None,
        },
        "moments_finite": finite,
    }
    if args.cpu_budget > 0:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    if args.full_fill_turns > 0:
        out["full_fill"] = full_fill(args.full_fill_turns, args.serve_wake, copy_gbs)
    if args.table4_turns > 0:
        out["paper_table4"] = paper_table4(args.table4_turns)
    if args.serve_scale > 0:
        out["serving"] = serving_sample(args.serve_scale, args.serve_budget_gb, args.serve_wake,
                                        args.serve_fill or None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
