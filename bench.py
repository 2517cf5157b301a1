#!/usr/bin/env python3
"""Benchmark: macro-particle-turns/s on one MI355X, the batched mixed-precision
tracker against the plain FP64 tracker, plus p50/p99 job latency of the
serving mix.

Headline workload (default): the full fill of the 484-bucket ring of the
paper's Table 1 -- 484 bunches of 1e5 macro-particles at 1 mA, broadband
resonator wake on 256 bins, one long-range higher-order-mode resonator.  Its
particle state (774 MB) is three times the 256 MB Infinity Cache, so the push
kernel streams from HBM.  A step is one turn of the whole hot path for every
bunch: phasor scan; push (kick, damping, noise, drift, histogram, deposits,
moment sums); between-turn kernel (moments, deposit sums, wake potential);
moment output.  Inputs are resident in HBM before the timed region.

Two forms, both set up first (untimed: the batch's tuner and graph capture,
as many turns of the plain form), then each timed over exactly K turns after
W warm-up turns:
  batched_mixed (the `value`): a batch (captured 16-turn HIP graphs, push
      launch shape tuned online during set-up), wake potential as a BF16x2
      Toeplitz product on the matrix cores; FP64 coordinates and phasors;
  plain_fp64: one job per launch set, eager launches, FP64 VALU convolution.
Outside the timed windows: a sustained comparison of the two forms (1000
turns each, twice, interleaved), and the roofline of the push kernel from
further turns whose every launch is bracketed by HIP events.

Prints one JSON line; progress goes to stderr as each part finishes.
"""
import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, vendor figure
# Vector issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64 VALU
# instruction occupies a SIMD for four cycles), in lane-instructions/s.
VALU_PEAK = 256 * 4 * 16 * 2.4e9
BYTES_PER_PARTICLE_TURN = 32  # read tau, delta + write tau, delta (FP64)
PMC_FILES = {"c2": os.path.join(ROOT, "profiles", "push_c2_pmc.json"),
             "c4": os.path.join(ROOT, "profiles", "push_c4_pmc.json")}
KERNEL_SRCS = [os.path.join(ROOT, "paper_1809_00391_amd", "csrc", f)
               for f in ("mbt_kernels.hip", "mbt_fastmath.h", "mbt_internal.h")]
_T0 = time.perf_counter()


def progress(msg):
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


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


def pmc_record(key, particles_per_launch):
    """The committed rocprofv3 counter record of the push on workload `key`
    (FETCH_SIZE and WRITE_SIZE scaled by a copy kernel of known size, SQ
    instruction counts), or None when it is missing or was taken on a
    different kernel source or workload."""
    path = PMC_FILES.get(key)
    if not path or not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_sha") != kernel_sha() or d.get("particles_per_launch") != particles_per_launch:
        return None
    d["_path"] = path
    return d


def make_tracker(w, wake="fp64"):
    from paper_1809_00391_amd import tracker as tr
    t = tr.Tracker(w.ring)
    if w.hc_flat:
        t.set_harmonic_cavity(tr.hc_flat_fraction(w.ring, *w.hc_flat))
    t.set_fill(w.buckets, w.currents_A, w.streams)
    if w.grid is not None:
        t.set_short_range(list(w.short_range), w.grid)
    if w.long_range:
        t.set_long_range(list(w.long_range))
    if wake != "fp64" and w.grid is not None:
        t.set_wake_precision(wake)
    t.bind(w.N)
    t.init_gaussian(w.sigma_tau0, w.sigma_delta0, w.seed)
    return t


def push_roofline(push_ms, push_n, particles, copy_gbs, pmc):
    """Roofline figures of the push from HIP-event timings: algorithmic bytes
    (32 B per macro-particle) per launch over the average launch duration."""
    if not push_n:
        return None
    push_s = push_ms / 1e3 / push_n
    gbs = BYTES_PER_PARTICLE_TURN * particles / push_s / 1e9
    out = {"bound": "hbm", "kernel": "k_push", "achieved": gbs, "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
           "traffic": pmc["hbm_bytes_per_launch"] if pmc else None,
           "avg_launch_us": push_s * 1e6, "launches_timed": push_n,
           "bytes_per_launch": BYTES_PER_PARTICLE_TURN * particles,
           "copy_GBs": copy_gbs, "frac_of_copy": gbs / copy_gbs if copy_gbs else None}
    if pmc:
        lane_instr = pmc["valu_instructions_per_pair"] * particles / 2 / push_s
        out["alu"] = {"bound": "alu",
                      "valu_instructions_per_pair": pmc["valu_instructions_per_pair"],
                      "achieved": lane_instr / 1e12, "peak": VALU_PEAK / 1e12,
                      "unit": "T lane-instructions/s", "frac": lane_instr / VALU_PEAK,
                      "source": os.path.relpath(pmc["_path"], ROOT)}
    return out


class Form:
    """One form of the headline workload, set up and warm: the plain FP64
    tracker (one job per launch set, eager launches, FP64 VALU convolution),
    or the batched mixed-precision form (a batch: the push launch shape tuned
    online on real turns, 16-turn HIP graphs, BF16x2 wake on the matrix
    cores).  Set-up turns are untimed: the batch's tuner candidates and graph
    capture, and the same number of turns for the plain form, so that both
    reach their timed window equally warm."""

    def __init__(self, w, key, form, wake, graph_turns):
        from paper_1809_00391_amd import tracker as tr
        self.w, self.key, self.form = w, key, form
        self.wake, self.graph_turns = (wake, graph_turns) if form == "batched_mixed" else ("fp64", 0)
        self.t = make_tracker(w, self.wake)
        self.b = None
        if form == "batched_mixed":
            self.b = tr.Batch([self.t], stream=self.t.stream, graph_turns=graph_turns, autotune=True)
            self.run = lambda n: self.b.track(n, moments=True)
        else:
            self.run = lambda n: self.t.track(n, moments=True)
        self.run(64 + 2 * max(graph_turns, 16))

    def timed(self, steps):
        """Exactly `steps` turns between HIP events on the stream, also timed
        by the wall clock; returns the larger elapsed time and the moments."""
        import torch
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        ev0.record(self.t.stream)
        mom = self.run(steps)
        ev1.record(self.t.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        return max(wall, ev0.elapsed_time(ev1) / 1e3), (mom[0] if isinstance(mom, list) else mom)

    def roofline(self, turns, copy_gbs):
        """Push launches of `turns` further turns, each bracketed by HIP
        events on the tracker's stream (eager launches)."""
        import torch
        timer = self.b if self.b is not None else self.t
        timer.set_timing(1)
        self.run(turns)
        torch.cuda.synchronize()
        push_ms, push_n, btw_ms, btw_n = timer.get_timing()
        timer.set_timing(0)
        particles = self.w.M * self.w.N
        pmc = pmc_record(self.key, particles)
        return (push_roofline(push_ms, push_n, particles, copy_gbs, pmc),
                btw_ms * 1e3 / btw_n if btw_n else None)

    def info(self):
        d = {"wake": self.wake, "graph_turns": self.graph_turns, "autotune": self.b is not None}
        if self.b is not None:
            d["launch_groups"] = [list(g) for g in self.b.launch_info()]
        return d

    def close(self):
        import torch
        if self.b is not None:
            self.b.close()
        self.t.close()
        torch.cuda.empty_cache()


def run_forms(w, key, names, steps, warmup, roofline_turns, wake, graph_turns, copy_gbs,
              sustained_turns):
    """Both forms set up and warmed first; then each form's `warmup` turns and
    exactly `steps` timed turns; then, outside the timed windows, a sustained
    comparison (`sustained_turns` turns of each form, twice, interleaved) and
    the push roofline of each form."""
    import torch
    particles = w.M * w.N
    forms = {n: Form(w, key, n, wake, graph_turns) for n in names}
    progress("forms set up: " + ", ".join(names))
    res = {}
    for n, f in forms.items():
        if warmup:
            f.run(warmup)
        elapsed, m = f.timed(steps)
        res[n] = {"value": particles * steps / elapsed, "ms_per_step": elapsed * 1e3 / steps,
                  "moments_finite": bool(torch.isfinite(torch.from_numpy(m[-1])).all())}
        progress(f"{n}: {res[n]['value']:.4g} macro-particle-turns/s over {steps} turns")
    sustained = None
    if sustained_turns > 0:
        rates = {n: [] for n in forms}
        for _ in range(2):
            for n, f in forms.items():
                elapsed, _m = f.timed(sustained_turns)
                rates[n].append(particles * sustained_turns / elapsed)
        sustained = {"turns": sustained_turns, "repetitions": 2,
                     "unit": "macro-particle-turns/s",
                     **{n: max(r) for n, r in rates.items()}}
        if "batched_mixed" in rates and "plain_fp64" in rates:
            sustained["batched_over_plain"] = max(rates["batched_mixed"]) / max(rates["plain_fp64"])
        progress(f"sustained: {sustained}")
    for n, f in forms.items():
        if roofline_turns:
            res[n]["push_roofline"], res[n]["between_turn_us"] = f.roofline(roofline_turns, copy_gbs)
        res[n].update(f.info())
        f.close()
    return res, sustained


def cache_resident(turns, roofline_turns, copy_gbs):
    """The eight-current scan (8 x 1e6 particles, 3rd-harmonic cavity, BB
    wake on 512 bins) in the plain FP64 tracker.  Its 128 MB of state fits in
    the 256 MB Infinity Cache, so its push fraction is not an HBM figure."""
    from paper_1809_00391_amd import workloads as wl
    w = wl.PRESETS["c2"]
    f = Form(w, "c2", "plain_fp64", "fp64", 0)
    f.run(200)
    elapsed, m = f.timed(turns)
    res = {"value": w.M * w.N * turns / elapsed, "ms_per_step": elapsed * 1e3 / turns}
    if roofline_turns:
        res["push_roofline"], res["between_turn_us"] = f.roofline(roofline_turns, copy_gbs)
    f.close()
    res["workload"] = w.name
    res["note"] = "state 128 MB, inside the 256 MB Infinity Cache: not an HBM measurement"
    return res


# The physics variants measured on the full fill (the plane and wakes of the
# transverse GPU parity test, a copper wall, a beam-driven harmonic cavity).
TRANSVERSE_PLANE = dict(tune=18.2137, chromaticity=2.5, alpha=-0.7, beta_m=7.5, disp_m=0.12,
                        disp_prime=-0.031, emittance_m=1e-9, tau_damp_s=8e-3)
TRANSVERSE_WAKE = [(2e6, 1.0, 1.2e10)]     # broadband transverse resonator (Ohm/m, Q, Hz)
COPPER = (0.01, 5.8e7)                      # pipe radius (m), conductivity (S/m)


def physics_variants(turns, copy_gbs):
    """The full fill (484 bunches x 1e5) with each physics variant of the
    turn map, in the plain FP64 tracker: throughput over `turns` turns and
    the push from HIP events over as many more.
      resistive_wall: the broadband wake plus the short-range wake of a
        copper pipe (10 mm, the whole ring) in the same wake table, so the
        same push as the headline;
      passive_hc: the HOM and a beam-driven third-harmonic resonator as two
        long-range resonators (the two-resonator push);
      transverse: one transverse plane with dispersion, chromaticity and
        noise, a broadband transverse resonator and a copper wall remembered
        for 8 turns (k_push_tr; 64 B per macro-particle-turn: tau, delta,
        x and x' read and written)."""
    import numpy as np
    import torch
    from paper_1809_00391_amd import tracker as tr
    from paper_1809_00391_amd import workloads as wl
    w = wl.PRESETS["c4"]
    ring_m = w.ring["harmonic"] * 299792458.0 / w.ring["f_rf_Hz"]
    out = {}
    for name in ("resistive_wall", "passive_hc", "transverse"):
        t = tr.Tracker(w.ring)
        t.set_fill(w.buckets, w.currents_A, w.streams)
        t.set_short_range(list(w.short_range), w.grid)
        lr = list(w.long_range)
        if name == "passive_hc":
            lr.append((2.0e3, 2.0e4, 3 * w.ring["f_rf_Hz"] + 0.1e6))
        t.set_long_range(lr)
        if name == "resistive_wall":
            t.set_resistive_wall((COPPER[0], COPPER[1], ring_m))
        tr_on = name == "transverse"
        if tr_on:
            t.set_transverse(TRANSVERSE_PLANE)
            t.set_transverse_wake(TRANSVERSE_WAKE)
            t.set_transverse_rw((COPPER[0], COPPER[1], ring_m, 8))
        t.bind(w.N)
        t.init_gaussian(w.sigma_tau0, w.sigma_delta0, w.seed)
        if tr_on:
            t.init_transverse(TRANSVERSE_PLANE["emittance_m"])
        run = (lambda n: t.track2(n)[0]) if tr_on else (lambda n: t.track(n))
        run(50)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        ev0.record(t.stream)
        m = run(turns)
        ev1.record(t.stream)
        torch.cuda.synchronize()
        elapsed = max(time.perf_counter() - wall0, ev0.elapsed_time(ev1) / 1e3)
        t.set_timing(1)
        run(turns)
        torch.cuda.synchronize()
        push_ms, push_n, btw_ms, btw_n = t.get_timing()
        t.set_timing(0)
        bpp = 64 if tr_on else 32
        push_s = push_ms / 1e3 / push_n
        gbs = bpp * w.M * w.N / push_s / 1e9
        out[name] = {"value": w.M * w.N * turns / elapsed, "ms_per_step": elapsed * 1e3 / turns,
                     "moments_finite": bool(np.isfinite(m).all()),
                     "push": {"kernel": "k_push_tr" if tr_on else "k_push", "avg_launch_us": push_s * 1e6,
                              "bytes_per_particle_turn": bpp, "achieved": gbs, "unit": "GB/s",
                              "frac": gbs / HBM_PEAK_GBS,
                              "frac_of_copy": gbs / copy_gbs if copy_gbs else None},
                     "between_turn_us": btw_ms * 1e3 / btw_n if btw_n else None}
        t.close()
        torch.cuda.empty_cache()
        progress(f"physics variant {name} done")
    out["workload"] = w.name
    out["unit"] = "macro-particle-turns/s"
    return out


def cpu_info():
    model = platform.processor() or ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return model, os.cpu_count()


def cpu_baseline(w, budget_s):
    """The oracle (as it stands) on this host's cores for a bounded number of
    turns of the same workload (all bunches), then on one thread over the
    first 44 of its bunches (a sample of the same per-bunch work)."""
    from oracle import ref
    model, nproc = cpu_info()
    allc = ref.threads()
    out = _oracle_rate(w, budget_s)
    ref.set_threads(1)
    try:
        k = min(w.M, 44)
        sub = w.with_(buckets=w.buckets[:k], currents_A=w.currents_A[:k])
        one = _oracle_rate(sub, budget_s / 3)
    finally:
        ref.set_threads(allc)
    out["single_thread"] = {"value": one["value"], "cores": 1, "sample": one["sample"]}
    out["cpu_model"] = model
    out["nproc"] = nproc
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
    s.track(1)
    per_turn = time.perf_counter() - t0
    turns = int(max(2, min(1000, budget_s / max(per_turn, 1e-9))))
    t0 = time.perf_counter()
    s.track(turns)
    dt = time.perf_counter() - t0
    return {"value": w.M * w.N * turns / dt, "unit": "macro-particle-turns/s",
            "cores": ref.threads(), "kind": "oracle",
            "sample": f"{turns} turns of {w.M} bunches x {w.N} particles (same ring, wakes "
                      f"and seed) after 1 warm-up turn, {dt:.1f} s"}


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
    {1, 3, 40, 121, 363, 484}, 1e4-2e5 particles, 1000-20000 turns), with
    turns and arrival times multiplied by `scale` (1.0: the mix as stated):
    once through the continuous-batching server (matrix-core wake `wake`),
    once as the plain per-job FP64 tracker running the jobs one after another
    in arrival order.  Returns throughput and p50/p99 job latency of both."""
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
    progress(f"serving: batched form done ({span:.1f} s)")
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
    progress(f"serving: plain per-job form done ({span_plain:.1f} s)")
    return {"jobs": len(reqs), "scale": scale, "particle_turns": total,
            "arrival_window_s": max(r.arrival_s for r in reqs),
            "batched": {"value": total / span, "p50_s": lat["p50"], "p99_s": lat["p99"],
                        "span_s": span, "wake": wake, "hbm_budget_gb": budget_gb,
                        "fill_particles": fill, "slices": srv.slices,
                        "batches_built": srv.batches_built, "batch_build_s": srv.build_s,
                        "peak_bytes": srv.peak_bytes},
            "plain_fp64_per_job": {"value": total / span_plain, "span_s": span_plain,
                                   "p50_s": float(np.percentile(done, 50)),
                                   "p99_s": float(np.percentile(done, 99))},
            "batched_over_plain": span_plain / span,
            "unit": "macro-particle-turns/s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000, help="timed turns of each form")
    ap.add_argument("--warmup", type=int, default=50, help="untimed turns of each form first")
    ap.add_argument("--workload", default="c4", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--wake", default="bf16x2", choices=["fp32", "bf16x2", "bf16x3"],
                    help="matrix-core wake arithmetic of the batched form")
    ap.add_argument("--graph-turns", type=int, default=16)
    ap.add_argument("--sustained-turns", type=int, default=1000,
                    help="turns of each form (twice, interleaved) for the sustained comparison (0: skip)")
    ap.add_argument("--roofline-turns", type=int, default=200,
                    help="turns after the timed window with every push bracketed by HIP events")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle time for the CPU baseline (0: skip)")
    ap.add_argument("--cache-resident-turns", type=int, default=2000,
                    help="turns of the cache-resident eight-current scan (0: skip)")
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="turn and arrival-time scale of the serving mix (1: as stated; 0: skip)")
    ap.add_argument("--serve-budget-gb", type=float, default=24.0,
                    help="HBM budget of the serving admission")
    ap.add_argument("--serve-fill", type=float, default=3.2e7,
                    help="admit while the admitted jobs hold fewer particles than this (0: no limit)")
    ap.add_argument("--table4-turns", type=int, default=1000,
                    help="turns of the paper's Table 4 bunch counts (0: skip)")
    ap.add_argument("--physics-turns", type=int, default=100,
                    help="turns of each physics variant on the full fill (0: skip)")
    ap.add_argument("--copy-bw", type=int, default=1,
                    help="measure the library copy kernel's bandwidth (0: skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (counter scale for rocprofv3 --pmc)")
    ap.add_argument("--forms", default="plain_fp64,batched_mixed",
                    help="forms of the headline workload to run")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the tracker is a "
              "single-GPU library; see DESIGN.md for how it would shard.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1809_00391_amd import workloads as wl

    w = wl.PRESETS[args.workload]
    torch.cuda.set_device(0)
    if args.copy_probe:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    copy_gbs, copy_ok = copy_bandwidth() if args.copy_bw else (None, None)
    progress(f"copy bandwidth {copy_gbs}")
    forms, sustained = run_forms(w, args.workload, args.forms.split(","), args.steps, args.warmup,
                                 args.roofline_turns, args.wake, args.graph_turns, copy_gbs,
                                 args.sustained_turns)
    head = forms.get("batched_mixed") or forms[next(iter(forms))]
    head_form = "batched_mixed" if "batched_mixed" in forms else next(iter(forms))
    particles = w.M * w.N
    out = {
        "metric": "macro-particle-turns/s (FP64 plain vs batched mixed-prec) at 1 GPU; "
                  "p50/p99 job lat",
        "value": head["value"],
        "unit": "macro-particle-turns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "form": head_form,
            "bunches": w.M, "particles_per_bunch": w.N,
            "bins": w.grid[0] if w.grid else 0,
            "long_range_resonators": len(w.long_range),
            "turns_timed": args.steps,
            "precision": ("FP64 coordinates, sums and long-range phasors; short-range wake "
                          f"potential in {args.wake} on the matrix cores")
                         if head_form == "batched_mixed" else "FP64 throughout",
        },
        "roofline": head.get("push_roofline"),
        "forms": forms,
        "moments_finite": all(f["moments_finite"] for f in forms.values()),
    }
    if "batched_mixed" in forms and "plain_fp64" in forms:
        out["batched_over_plain"] = forms["batched_mixed"]["value"] / forms["plain_fp64"]["value"]
    if sustained:
        out["sustained"] = sustained
    out["copy_exact"] = copy_ok
    if args.cpu_budget > 0:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
        progress("cpu baseline done")
    if args.cache_resident_turns > 0:
        out["cache_resident"] = cache_resident(args.cache_resident_turns, args.roofline_turns,
                                               copy_gbs)
        progress("cache-resident scan done")
    if args.table4_turns > 0:
        out["paper_table4"] = paper_table4(args.table4_turns)
        progress("table 4 done")
    if args.physics_turns > 0:
        out["physics_variants"] = physics_variants(args.physics_turns, copy_gbs)
    if args.serve_scale > 0:
        out["serving"] = serving_sample(args.serve_scale, args.serve_budget_gb, args.wake,
                                        args.serve_fill or None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
