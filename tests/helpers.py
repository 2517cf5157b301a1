"""Shared test helpers: configure the oracle and the GPU tracker from one
workload preset, and the parity tolerances.

Each side computes its own derived quantities (harmonic-cavity solution,
synchronous phase, wake tables); only the preset values are shared.
"""
import numpy as np

from paper_1809_00391_amd import workloads as wl

# Tolerances (stated for the tracker against the FP64 oracle).
COORD_RTOL = 1e-12     # one turn from identical input, relative to max(|x|, sigma_x)
MOMENT_RTOL = 1e-9     # first 100 turns, relative to max(|m|, sigma)


def make_oracle(w, N=None, init=True, hc_override=None):
    from oracle import ref
    s = ref.RefSim(w.ring)
    if w.hc_flat is not None or hc_override is not None:
        hc = hc_override or ref.hc_flat_fraction(w.ring, *w.hc_flat)
        s.set_harmonic_cavity(hc)
    s.set_fill(w.buckets, w.currents_A, w.streams)
    if w.grid is not None:
        s.set_short_range(list(w.short_range), w.grid)
    if w.long_range:
        s.set_long_range(list(w.long_range))
    if w.rw is not None:
        s.set_resistive_wall(w.rw)
    n = N or w.N
    if init:
        s.init_gaussian(n, w.sigma_tau0, w.sigma_delta0, w.seed)
    else:
        s.alloc_particles(n, w.seed)
    return s


def make_tracker(w, N=None, init=True, hc_override=None):
    from paper_1809_00391_amd import tracker as tr
    t = tr.Tracker(w.ring)
    if w.hc_flat is not None or hc_override is not None:
        hc = hc_override or tr.hc_flat_fraction(w.ring, *w.hc_flat)
        t.set_harmonic_cavity(hc)
    t.set_fill(w.buckets, w.currents_A, w.streams)
    if w.grid is not None:
        t.set_short_range(list(w.short_range), w.grid)
    if w.long_range:
        t.set_long_range(list(w.long_range))
    if w.rw is not None:
        t.set_resistive_wall(w.rw)
    n = N or w.N
    t.bind(n)
    if init:
        t.init_gaussian(w.sigma_tau0, w.sigma_delta0, w.seed)
    else:
        t.set_state(0, w.seed, None)
    return t


def set_same_particles(w, sims, N, seed=1234, scale=1.0):
    """Give every side identical seeded Gaussian particles (from workloads)."""
    out = []
    for b in range(w.M):
        tau, delta = wl.gaussian_particles(seed + b, N, scale * w.sigma_tau0,
                                           scale * w.sigma_delta0)
        for s in sims:
            s.set_particles(b, tau, delta)
        out.append((tau, delta))
    return out


def coord_excess(x_gpu, x_ref):
    """max |dx| / max(|x|, sigma_x); parity holds when <= COORD_RTOL."""
    sig = np.std(x_ref)
    scale = np.maximum(np.abs(x_ref), sig)
    return float(np.max(np.abs(x_gpu - x_ref) / scale))


def moment_excess(m_gpu, m_ref):
    """Moments [T][M][4] = mean tau, mean delta, rms tau, rms delta; the
    deviation of each relative to max(|m|, the bunch's rms of that coordinate)."""
    m_gpu = np.asarray(m_gpu)
    m_ref = np.asarray(m_ref)
    sig = np.concatenate([m_ref[..., 2:4], m_ref[..., 2:4]], axis=-1)
    scale = np.maximum(np.abs(m_ref), sig)
    return float(np.max(np.abs(m_gpu - m_ref) / scale))
