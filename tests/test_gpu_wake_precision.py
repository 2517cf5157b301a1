"""Mixed-precision wake potential on the matrix cores (MBT_WAKE_FP32,
MBT_WAKE_BF16X2, MBT_WAKE_BF16X3) against the FP64 oracle.

The wake potential V[k] = qpp sum_{m<=k} W[k-m] c[m] (Sec. 2.3) is checked
element by element against an error bound derived from the arithmetic:
  |V - V_exact| <= qpp (u_W + n_terms 2^-24) sum_{m<=k} |W[k-m]| c[m]
with u_W the relative error of the stored W (2^-24 for FP32, 2^-16 and 2^-24
for two and three BF16 terms of 8 significant bits each) and 2^-24 the unit
roundoff of the FP32 accumulation over at most n_terms products (the counts
themselves are exact in every mode).  Tracking with each mode is then
compared with the FP64 oracle: the deviations of centroid, rms length and
energy spread are printed and bounded, and a coupled-bunch growth rate is
compared with the FP64 tracker's.
"""
import numpy as np
import pytest

from paper_1809_00391_amd import workloads as wl
from oracle import ref

import theory as th
from helpers import make_oracle, make_tracker, set_same_particles

pytestmark = pytest.mark.gpu

MODES = {"fp32": 2.0 ** -24, "bf16x2": 2.0 ** -16, "bf16x3": 2.0 ** -24}

# Full-ring-like shape (c4's grid and wakes) at a size the oracle runs in seconds.
W4 = wl.C4.with_(name="c4-like", buckets=tuple(range(40)), currents_A=tuple(
    1e-3 * (1 + 0.4 * np.sin(b)) for b in range(40)), N=20_000)


def print_case(name, **kw):
    print(f"[gpu case] {name} {kw}", flush=True)


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("case", ["c4-like", "mb-ragged", "wide-600", "max-4096"])
def test_wake_potential_within_bound(cuda, mode, case):
    if case == "c4-like":
        w = W4
    elif case == "mb-ragged":  # 200 bins (not a multiple of 16 or 64), 5 bunches, an empty one
        w = wl.Workload(name="mb", ring=wl.RING_R480, buckets=(0, 3, 4, 9, 200),
                        currents_A=(1e-3, 2.5e-3, 0.0, 1.5e-3, 4e-3), N=70_001, turns=0, seed=7,
                        sigma_tau0=20e-12, sigma_delta0=8.6e-4, short_range=(wl.BB,),
                        grid=(200, -150e-12, 150e-12), long_range=(wl.HOM,))
    elif case == "wide-600":  # histograms staged in three blocks (256, 256, 88 bins)
        w = wl.C1.with_(name="wide", buckets=(0, 1, 2), currents_A=(1e-3, 2e-3, 0.5e-3),
                        N=60_000, grid=(600, -80e-12, 80e-12))
    else:  # the largest grid the library accepts, 17 bunches (a second, one-bunch tile)
        w = wl.C1.with_(name="max bins", buckets=tuple(range(17)),
                        currents_A=tuple(1e-3 * (1 + 0.1 * b) for b in range(17)),
                        N=30_000, grid=(4096, -80e-12, 80e-12))
    print_case("wake bound", mode=mode, case=case, M=w.M, N=w.N)
    g = make_tracker(w, init=False)
    g.set_wake_precision(mode)
    parts = set_same_particles(w, [g], w.N)
    V = g.wake_potential()
    W = ref.wake_table(list(w.short_range) + list(w.long_range), w.grid)
    T0 = w.ring["harmonic"] / w.ring["f_rf_Hz"]
    nb = w.grid[0]
    worst = 0.0
    for b, (tau, _) in enumerate(parts):
        c, _ = ref.histogram(w.grid, tau)
        qpp = w.currents_A[b] * T0 / w.N
        V_o = ref.wake_potential(W, c, qpp)
        absconv = ref.wake_potential(np.abs(W), c, abs(qpp))
        bound = (MODES[mode] + nb * 2.0 ** -24) * absconv * 1.01 + 1e-300
        err = np.abs(V[b] - V_o)
        assert np.all(err <= bound), (b, np.max(err / bound))
        if np.max(absconv) > 0:
            worst = max(worst, float(np.max(err) / np.max(absconv)))
    print(f"[wake error] mode={mode} case={case} max|dV|/max(|W|*c) = {worst:.3e}", flush=True)


def _moments(w, mode, turns):
    g = make_tracker(w)
    if mode != "fp64":
        g.set_wake_precision(mode)
    return g.track(turns)


def test_tracking_error_vs_oracle(cuda):
    """100 turns of the c4-like case in every mode against the oracle:
    centroid, rms length and energy spread deviations relative to the
    bunch's rms (printed; bounded well below the physics tolerances)."""
    turns = 100
    o = make_oracle(W4)
    mo = o.track(turns)
    sig = np.concatenate([mo[..., 2:4], mo[..., 2:4]], axis=-1)
    report = {}
    for mode in ["fp64"] + sorted(MODES):
        mg = _moments(W4, mode, turns)
        dev = np.abs(mg - mo) / sig
        report[mode] = [float(np.max(dev[..., i])) for i in range(4)]
        print(f"[tracking error] mode={mode} max rel dev: centroid tau {report[mode][0]:.2e} "
              f"delta {report[mode][1]:.2e} rms tau {report[mode][2]:.2e} "
              f"rms delta {report[mode][3]:.2e}", flush=True)
    assert max(report["fp64"]) <= 1e-9
    for mode in MODES:
        assert max(report[mode]) <= 1e-4, (mode, report[mode])


def test_growth_rate_bf16_matches_fp64(cuda):
    """Coupled-bunch growth of a seeded mode in a uniform fill of Gaussian
    bunches (BB short-range wake on 64 bins, HOM long range, noise and
    damping on): the growth rate with the wake potential in BF16x2 agrees
    with the FP64 run of the same seed within 2%."""
    ring = wl.RING_R480
    M, mu, turns, A = 480, 19, 3000, 2e-12
    T0 = ring["harmonic"] / ring["f_rf_Hz"]
    omega_s = 2 * np.pi * th.synchrotron_tune(ring) / T0
    w = wl.Workload(name="cb+bb", ring=ring, buckets=tuple(range(M)), currents_A=(1e-3,) * M,
                    N=2000, turns=turns, seed=5, sigma_tau0=10e-12, sigma_delta0=8.6e-4,
                    short_range=(wl.BB,), grid=(64, -60e-12, 60e-12), long_range=(wl.HOM,))
    rates = {}
    for mode in ["fp64", "bf16x2"]:
        g = make_tracker(w)
        if mode != "fp64":
            g.set_wake_precision(mode)
        for b in range(M):
            tau, delta = g.get_particles(b)
            ph = 2 * np.pi * mu * b / M
            g.set_particles(b, tau + A * np.cos(ph), delta - A * omega_s / ring["alpha_c"] * np.sin(ph))
        m = g.track(turns)
        amp = th.mode_amplitudes(m[:, :, 0], m[:, :, 1], ring["alpha_c"], omega_s)[:, mu]
        t = np.arange(turns) * T0
        sel = slice(turns // 5, turns)
        rates[mode] = th.fit_growth(t[sel], amp[sel])
    print(f"[growth rate] fp64 {rates['fp64']:.6g} /s  bf16x2 {rates['bf16x2']:.6g} /s", flush=True)
    assert rates["fp64"] > 0  # the mode grows (HOM drive above radiation damping)
    assert rates["bf16x2"] == pytest.approx(rates["fp64"], rel=2e-2)


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", ["40 bunches", "71 tiles"])
def test_matrix_core_job_between_turn_work(cuda, mode, case):
    """A job whose wake potential comes from the matrix cores has no prep
    launch: its moments, deposit sums, profile rows, histogram clearing and
    turn counter come from the wake kernel (the sums by one wavefront per
    bunch).  With the grid placed beside the bunches every histogram is
    empty and the wake potential is zero in every arithmetic, so the job
    must give the same doubles as the FP64 job, whose prep sums by whole
    workgroups: moments, particles, phasors and profiles over 30 turns, in
    two calls.  Cases: 40 bunches (a ragged 16-bunch tile, 200 bins in
    four ragged 64-bin tiles, two long-range resonators) and 3 bunches of 71
    push tiles (more tiles than one 64-lane slice sums)."""
    if case == "40 bunches":
        w = wl.Workload(name="lr, empty grid", ring=wl.RING_R480, buckets=tuple(range(0, 480, 12)),
                        currents_A=tuple(1e-3 * (1 + 0.5 * np.sin(b)) for b in range(40)),
                        N=3 * 8192 + 101, turns=0, seed=9, sigma_tau0=12e-12,
                        sigma_delta0=8.6e-4, short_range=(wl.BB,),
                        grid=(200, 300e-12, 400e-12), long_range=(wl.HOM, (3e5, 5e3, 2.21e9)))
    else:
        w = wl.Workload(name="many tiles, empty grid", ring=wl.RING_R480, buckets=(0, 5, 9),
                        currents_A=(2e-3, 1e-3, 3e-3), N=70 * 8192 + 5, turns=0, seed=10,
                        sigma_tau0=12e-12, sigma_delta0=8.6e-4, short_range=(wl.BB,),
                        grid=(64, -400e-12, -300e-12), long_range=(wl.HOM,))
    print_case("matrix-core between-turn work", mode=mode, case=case, M=w.M, N=w.N)
    ref_job = make_tracker(w)
    mc_job = make_tracker(w)
    mc_job.set_wake_precision(mode)
    for part in (17, 13):
        m_ref, p_ref = ref_job.track(part, profiles_stride=4)
        m_mc, p_mc = mc_job.track(part, profiles_stride=4)
        assert np.array_equal(m_mc, m_ref)
        assert np.array_equal(p_mc, p_ref) and not p_ref.any()
    for b in (0, w.M - 1):
        t_ref, d_ref = ref_job.get_particles(b)
        t_mc, d_mc = mc_job.get_particles(b)
        assert np.array_equal(t_mc, t_ref) and np.array_equal(d_mc, d_ref)
    s_ref, s_mc = ref_job.get_state(), mc_job.get_state()
    assert s_ref[0] == s_mc[0] == 30
    assert np.array_equal(s_ref[2], s_mc[2])
