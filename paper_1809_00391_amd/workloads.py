"""Workload presets and seeded input generators.

This module is the only code shared by the GPU path's tests and benchmark and
by the oracle's tests.  It holds parameter values and random-number recipes
only -- none of the tracking method's arithmetic (no synchronous phase, no
harmonic-cavity solution, no wake, no map).  Each side derives those itself.

Rings.  R480 is the single- and coupled-bunch test ring: E0 = 2.4 GeV,
f_RF = 500 MHz, h = 480, V_RF = 1.5 MV, alpha_c = 6e-4, U0 = 0.5 MeV/turn,
longitudinal damping time 4 ms, equilibrium energy spread 8.6e-4 (taken equal
to the stated initial spread, since no other is given).  R484 is the same with
h = 484, the harmonic number of the paper's Table 1 ring, for full-ring fills
of 484 bunches.

Resonators are (R_s [Ohm], Q, f_r [Hz]) tuples; grids are
(nbins, tau_min [s], tau_max [s]).
"""
from dataclasses import dataclass, field, replace

import numpy as np

RING_R480 = dict(energy_eV=2.4e9, f_rf_Hz=500e6, v_rf_V=1.5e6, alpha_c=6e-4, u0_eV=0.5e6,
                 tau_long_s=4e-3, sigma_delta=8.6e-4, harmonic=480)
RING_R484 = dict(RING_R480, harmonic=484)

# Broadband resonator (short-range wake) and a high-Q cavity higher-order mode.
BB = (10e3, 1.0, 20e9)
HOM = (1e6, 2e4, 1.52e9)


@dataclass(frozen=True)
class Workload:
    name: str
    ring: dict
    buckets: tuple
    currents_A: tuple
    N: int
    turns: int
    seed: int
    sigma_tau0: float
    sigma_delta0: float
    short_range: tuple = ()
    grid: tuple = None
    long_range: tuple = ()
    hc_flat: tuple = None  # (n, fraction of the flat-potential voltage)
    streams: tuple = None
    rw: tuple = None       # resistive wall (radius m, conductivity S/m, length m)
    notes: str = field(default="", compare=False)

    @property
    def M(self):
        return len(self.buckets)

    @property
    def particle_turns(self):
        return self.M * self.N * self.turns

    def with_(self, **kw):
        return replace(self, **kw)


def current_scan_mA():
    """Eight bunch currents spread geometrically over 0.1-5 mA."""
    return tuple(0.1 * 50.0 ** (k / 7.0) for k in range(8))


# Single bunch, plain FP64: 10,000 macro-particles, 128 bins over +-75.85 ps
# (+-5 times the 15.17 ps zero-current bunch length of R480), 0.5 mA, BB wake.
C1 = Workload(
    name="single bunch 1e4 particles, BB wake, 128 bins, 2000 turns",
    ring=RING_R480, buckets=(0,), currents_A=(0.5e-3,), N=10_000, turns=2000, seed=1,
    sigma_tau0=10e-12, sigma_delta0=8.6e-4, short_range=(BB,),
    grid=(128, -75.85e-12, 75.85e-12))

# Single bunch at scale: 1e6 macro-particles with a 3rd-harmonic cavity at 90%
# of its flat-potential voltage, 512 bins over +-200 ps (about +-5 times the
# 39.7 ps zero-current bunch length in that potential), BB wake, eight
# currents 0.1-5 mA, 20,000 turns each, one seed for all currents.  The eight
# currents run as eight independent single-bunch jobs in one launch: no
# long-range wake couples them, and each gets random-stream ordinal 0.
C2 = Workload(
    name="current scan: 8 x single bunch 1e6 particles, 3rd-harmonic cavity, BB wake, "
         "512 bins, 20000 turns",
    ring=RING_R480, buckets=tuple(range(8)), currents_A=tuple(i * 1e-3 for i in current_scan_mA()),
    N=1_000_000, turns=20_000, seed=1, sigma_tau0=10e-12, sigma_delta0=8.6e-4,
    short_range=(BB,), grid=(512, -200e-12, 200e-12), hc_flat=(3, 0.9),
    streams=(0,) * 8)

# Coupled bunch: 360 consecutive bunches of 480 buckets (120-bucket gap),
# 1e5 macro-particles and 1 mA each, BB wake on 256 bins, HOM long-range.
C3 = Workload(
    name="3/4 fill 360 x 1e5 particles, BB 256 bins + HOM, 10000 turns",
    ring=RING_R480, buckets=tuple(range(360)), currents_A=(1e-3,) * 360, N=100_000,
    turns=10_000, seed=3, sigma_tau0=10e-12, sigma_delta0=8.6e-4, short_range=(BB,),
    grid=(256, -75.85e-12, 75.85e-12), long_range=(HOM,))

# Full fill of R484: 484 x 1e5 macro-particles at 1 mA, BB 256 bins + HOM.
C4 = Workload(
    name="full fill 484 x 1e5 particles, BB 256 bins + HOM, 20000 turns",
    ring=RING_R484, buckets=tuple(range(484)), currents_A=(1e-3,) * 484, N=100_000,
    turns=20_000, seed=4, sigma_tau0=10e-12, sigma_delta0=8.6e-4, short_range=(BB,),
    grid=(256, -76.15e-12, 76.15e-12), long_range=(HOM,))

# The paper's wake validation: copper chamber, 10 mm radius, whole ring.
RW_COPPER_10MM = (0.010, 5.8e7, 288.0)

PRESETS = {"c1": C1, "c2": C2, "c3": C3, "c4": C4}


def serving_mix(n_jobs=64, rate_per_s=2.0, seed=5):
    """Tracking jobs with Poisson arrivals for the serving workload: bunch
    count from {1, 3, 40, 121, 363, 484} in consecutive buckets of R484,
    particles per bunch log-uniform in [1e4, 2e5], turns uniform in
    [1000, 20000], current uniform in [0.2, 3] mA per bunch, HOM frequency
    uniform in [1.4, 1.6] GHz, seed = job id."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, size=n_jobs))
    jobs = []
    for i in range(n_jobs):
        M = int(rng.choice([1, 3, 40, 121, 363, 484]))
        N = int(round(np.exp(rng.uniform(np.log(1e4), np.log(2e5)))))
        turns = int(rng.integers(1000, 20001))
        cur = float(rng.uniform(0.2e-3, 3e-3))
        fr = float(rng.uniform(1.4e9, 1.6e9))
        w = Workload(name=f"job{i}", ring=RING_R484, buckets=tuple(range(M)),
                     currents_A=(cur,) * M, N=N, turns=turns, seed=i, sigma_tau0=10e-12,
                     sigma_delta0=8.6e-4, short_range=(BB,), grid=(256, -76.15e-12, 76.15e-12),
                     long_range=((1e6, 2e4, fr),))
        jobs.append((float(t[i]), w))
    return jobs


def gaussian_particles(seed, N, sigma_tau, sigma_delta, mean_tau=0.0, mean_delta=0.0):
    """Independent Gaussian (tau, delta) for N particles from numpy's PCG64."""
    rng = np.random.default_rng(seed)
    tau = mean_tau + sigma_tau * rng.standard_normal(N)
    delta = mean_delta + sigma_delta * rng.standard_normal(N)
    return tau, delta


def correlated_gaussian(seed, N, cov, mean=(0.0, 0.0)):
    """N samples of (tau, delta) with the given 2x2 covariance."""
    rng = np.random.default_rng(seed)
    x = rng.multivariate_normal(np.asarray(mean, float), np.asarray(cov, float), size=N)
    return np.ascontiguousarray(x[:, 0]), np.ascontiguousarray(x[:, 1])
