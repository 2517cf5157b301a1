"""Pins of the oracle to things other than itself: a library implementation of
the same random generator, textbook impedance and loss-factor integrals,
closed-form linear-map results (tune, damping, Lyapunov equilibrium), the
Boltzmann and Haissinski equilibria, a brute-force sum over all earlier
passages for the long-range wake, and coupled-bunch growth rates (two
independent closed forms, one of them the paper's Eq. 7).  CPU only.
"""
import json
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import ref
from paper_1809_00391_amd import workloads as wl

import theory as th

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
R480 = wl.RING_R480
T0 = R480["harmonic"] / R480["f_rf_Hz"]


# ---------------------------------------------------------------------------
# Random numbers
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.fail("hipcc is needed to build the rocRAND Philox pin")
    exe = str(tmp_path_factory.mktemp("pin") / "philox_pin")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "philox_rocrand_pin.cpp")],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_pin):
    rng = np.random.default_rng(2024)
    rows = rng.integers(0, 2**32, size=(3000, 6), dtype=np.uint64)
    rows[0] = 0
    rows[1] = 2**32 - 1
    rows[2] = [0, 1, 2, 3, 0xDEADBEEF, 0xCAFEBABE]
    text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_pin], input=text, capture_output=True, text=True, check=True)
    lib = np.array([[int(v) for v in line.split()] for line in out.stdout.strip().splitlines()],
                   dtype=np.uint64)
    assert lib.shape == (len(rows), 4)
    for r, expect in zip(rows, lib):
        got = ref.philox4x32_10(r[:4].astype(np.uint32), r[4:].astype(np.uint32))
        assert np.array_equal(got.astype(np.uint64), expect), r


def test_normal_deviates_statistics():
    # init_gaussian with unit sigmas returns the two Box-Muller branches.
    ring = dict(R480)
    s = ref.RefSim(ring)
    s.set_fill([0], [0.0])
    s.init_gaussian(400_000, 1.0, 1.0, 99)
    z0, z1 = s.get_particles(0)
    for z in (z0, z1):
        assert abs(z.mean()) < 5 / np.sqrt(z.size)
        assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
        assert stats.kstest(z, "norm").pvalue > 1e-4
        assert abs(stats.kurtosis(z)) < 5 * np.sqrt(24 / z.size)
    assert abs(np.corrcoef(z0, z1)[0, 1]) < 5 / np.sqrt(z0.size)
    # the noise of a particle pair is the same two branches (counter = pair index)
    zp = ref.normal_pair(99, [0, 0, 0, 1])
    assert zp[0] == z0[0] and zp[1] == z1[0]


# ---------------------------------------------------------------------------
# Wakes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("res", [wl.BB, (1e6, 200.0, 1.52e9), (3e5, 50.0, 2.21e9)])
def test_resonator_wake_transforms_to_impedance(res):
    """int_0^inf W(t) exp(-i w t) dt equals the textbook Rs/(1+iQ(w/wr-wr/w)),
    from Q = 1 (strongly damped) to Q = 200 (sharp)."""
    rs, q, fr = res
    wr = 2 * np.pi * fr
    alpha = wr / (2 * q)
    T = 36.0 / alpha  # exp(-36): the tail is negligible
    for w in (0.37 * wr, wr, 1.9 * wr):
        n = max(4001, int(100 * T * (w + wr) / (2 * np.pi))) // 2 * 2 + 1
        t = np.linspace(0.0, T, n)
        W = np.array([ref.resonator_wake(rs, q, fr, x) for x in t])
        re = integrate.simpson(W * np.cos(w * t), x=t)
        im = -integrate.simpson(W * np.sin(w * t), x=t)
        Z = th.resonator_impedance(rs, q, fr, w)
        assert abs(complex(re, im) - Z) <= 1e-5 * rs, (w / wr, complex(re, im), Z)


def test_wake_table_self_term_and_samples():
    grid = (64, -50e-12, 50e-12)
    W = ref.wake_table([wl.BB, wl.HOM], grid)
    a_bb = 2 * np.pi * wl.BB[2] / (2 * wl.BB[1])
    a_hom = 2 * np.pi * wl.HOM[2] / (2 * wl.HOM[1])
    # W[0] is half of W(0+) = 2 alpha Rs (beam-loading theorem)
    assert W[0] == pytest.approx(a_bb * wl.BB[0] + a_hom * wl.HOM[0], rel=1e-15)
    dt = 100e-12 / 64
    for k in (1, 5, 63):
        assert W[k] == pytest.approx(ref.resonator_wake(*wl.BB, k * dt)
                                     + ref.resonator_wake(*wl.HOM, k * dt), rel=1e-14)


def test_wake_potential_is_causal_convolution():
    rng = np.random.default_rng(3)
    grid = (300, -75e-12, 75e-12)
    W = ref.wake_table([wl.BB], grid)
    c = rng.integers(0, 5000, size=300).astype(np.uint32)
    q = 0.5e-3 * T0 / 1e6
    V = ref.wake_potential(W, c, q)
    expect = q * np.convolve(c.astype(float), W)[:300]
    assert np.max(np.abs(V - expect)) <= 1e-13 * np.max(np.abs(expect))


def test_binning_edges():
    g = (10, -1e-11, 1e-11)
    assert ref.bin_index(g, -1e-11) == 0
    assert ref.bin_index(g, np.nextafter(-1e-11, -1)) == -1
    assert ref.bin_index(g, 1e-11) == -1
    assert ref.bin_index(g, np.nextafter(1e-11, -1)) == 9
    assert ref.bin_index(g, float("nan")) == -1
    assert ref.bin_index(g, float("inf")) == -1
    centres = -1e-11 + (np.arange(10) + 0.5) * 2e-12
    assert [ref.bin_index(g, x) for x in centres] == list(range(10))
    tau = np.concatenate([centres, [5e-11, -5e-11, centres[3]]])
    counts, oog = ref.histogram(g, tau)
    assert oog == 2 and counts.sum() == 11 and counts[3] == 2
    # brute force on random input
    x = np.random.default_rng(1).normal(0, 1e-11, 20000)
    counts, oog = ref.histogram(g, x)
    k = np.floor((x - (-1e-11)) * (10 / 2e-11))
    inside = (k >= 0) & (k < 10)
    assert oog == int((~inside).sum())
    assert np.array_equal(counts, np.bincount(k[inside].astype(int), minlength=10))


def test_gaussian_loss_factor():
    """Mean energy change of a frozen Gaussian bunch from one turn with the
    wake minus one without = -Q k(sigma) (k: loss-factor integral of Re Z)."""
    N = 1_000_000
    sig = 15.17e-12
    I = 0.5e-3
    grid = (512, -5 * sig, 5 * sig)
    tau, delta = wl.gaussian_particles(5, N, sig, 0.0)
    ring = dict(R480, tau_long_s=float("inf"), sigma_delta=0.0)
    ends = []
    for with_wake in (True, False):
        s = ref.RefSim(ring)
        s.set_fill([0], [I])
        s.set_short_range([wl.BB] if with_wake else [], grid)
        s.alloc_particles(N, 1)
        s.set_particles(0, tau, delta)
        s.track(1)
        ends.append(s.get_particles(0)[1])
    dE = (ends[0] - ends[1]).mean() * R480["energy_eV"]
    k = th.gaussian_loss_factor([wl.BB], np.std(tau))
    assert dE == pytest.approx(-I * T0 * k, rel=1e-2)


# ---------------------------------------------------------------------------
# Single-particle map
# ---------------------------------------------------------------------------

def _single_particle(ring, tau0, delta0, turns, hc=None):
    s = ref.RefSim(ring)
    if hc:
        s.set_harmonic_cavity(hc)
    s.set_fill([0], [0.0])
    s.alloc_particles(1, 1)
    s.set_particles(0, [tau0], [delta0])
    m = s.track(turns)
    return m[:, 0, 0], m[:, 0, 1]


def test_synchrotron_tune_closed_form():
    ring = dict(R480, u0_eV=0.0, tau_long_s=float("inf"), sigma_delta=0.0)
    tau, _ = _single_particle(ring, 2e-12, 0.0, 20000)
    nu0 = th.synchrotron_tune(ring)
    n = np.arange(tau.size)
    # refine the FFT peak with a least-squares fit of a sinusoid
    from scipy.optimize import curve_fit
    f = lambda n, A, nu, ph: A * np.cos(2 * np.pi * nu * n + ph)
    spec = np.abs(np.fft.rfft(tau, 8 * tau.size))
    nu_fft = np.argmax(spec) / (8 * tau.size)
    (A, nu, ph), _ = curve_fit(f, n, tau, p0=[2e-12, nu_fft, 0.0])
    assert nu == pytest.approx(nu0, rel=1e-4)
    # with U0 on, the slope of the RF at phi_s sets the tune
    ring2 = dict(ring, u0_eV=R480["u0_eV"])
    tau2, _ = _single_particle(ring2, 2e-12, 0.0, 20000)
    (A2, nu2, ph2), _ = curve_fit(f, n, tau2, p0=[2e-12, th.synchrotron_tune(ring2), 0.0])
    assert nu2 == pytest.approx(th.synchrotron_tune(ring2), rel=1e-4)


def test_table1_tune_golden():
    """Table 1 prints nu_s for its ring; the small-amplitude tune of the map
    with the radiated energy off reproduces it within 0.5%."""
    t1 = json.load(open(os.path.join(HERE, "golden", "dc12c_table1.json")))
    ring = dict(energy_eV=t1["energy_eV"], f_rf_Hz=500e6, v_rf_V=t1["v_rf_V"],
                alpha_c=t1["alpha_c"], u0_eV=0.0, tau_long_s=float("inf"), sigma_delta=0.0,
                harmonic=t1["harmonic"])
    tau, _ = _single_particle(ring, 2e-12, 0.0, 8000)
    spec = np.abs(np.fft.rfft(tau - tau.mean(), 16 * tau.size))
    nu = np.argmax(spec) / (16 * tau.size)
    assert nu == pytest.approx(t1["nu_s"], rel=5e-3)
    assert nu == pytest.approx(th.synchrotron_tune(ring), rel=2e-4)


def test_damping_decrement_is_exact():
    """Kicks that depend on tau only and the drift preserve area; damping
    scales it by 1 - D per turn: tau_n delta_{n+1} - tau_{n+1} delta_n
    shrinks by exactly that factor for the linearised motion."""
    ring = dict(R480, sigma_delta=0.0)
    tau, delta = _single_particle(ring, 1e-14, 0.0, 3000)
    A = tau[:-1] * delta[1:] - tau[1:] * delta[:-1]
    D = 2 * T0 / R480["tau_long_s"]
    ratio = A[1:] / A[:-1]
    assert np.max(np.abs(ratio - (1 - D))) < 1e-6
    # envelope decay rate against the stated damping time (amplitude)
    assert th.radiation_damping_rate(ring) == pytest.approx(1 / R480["tau_long_s"], rel=1e-3)


def test_equilibrium_matches_lyapunov():
    cov = th.equilibrium_covariance(R480)
    N = 50_000
    tau, delta = wl.correlated_gaussian(17, N, cov)
    s = ref.RefSim(R480)
    s.set_fill([0], [0.0])
    s.alloc_particles(N, 11)
    s.set_particles(0, tau, delta)
    m = s.track(3000)
    st, sd = m[-1000:, 0, 2].mean(), m[-1000:, 0, 3].mean()
    assert st == pytest.approx(np.sqrt(cov[0, 0]), rel=1e-2)
    assert sd == pytest.approx(np.sqrt(cov[1, 1]), rel=1e-2)
    # and the energy spread relaxes to sigma_E from a cold start
    s2 = ref.RefSim(R480)
    s2.set_fill([0], [0.0])
    s2.init_gaussian(N, 0.0, 0.0, 12)
    m2 = s2.track(12000)
    assert m2[-2000:, 0, 3].mean() == pytest.approx(np.sqrt(cov[1, 1]), rel=1e-2)


def test_harmonic_cavity_flat_potential():
    hc = ref.hc_flat_fraction(R480, 3, 1.0)
    v0, v1, v2 = th.flat_potential_derivatives(R480, hc)
    w = 2 * np.pi * R480["f_rf_Hz"]
    V = R480["v_rf_V"]
    assert abs(v0) < 1e-9 * V
    assert abs(v1) < 1e-6 * V * w
    assert abs(v2) < 1e-4 * V * w * w
    # the oracle's synchronous phase with the cavity restores U0 at tau = 0
    s = ref.RefSim(R480)
    s.set_harmonic_cavity(hc)
    phi = s.derived()["phi_s"]
    tot = V * np.sin(phi) + hc["v_ratio"] * V * np.sin(hc["phase_n_rad"])
    assert tot == pytest.approx(R480["u0_eV"], rel=1e-13)


def test_harmonic_cavity_zero_current_profile():
    """Equilibrium in the 90%-flat potential = Boltzmann quadrature."""
    hc = ref.hc_flat_fraction(R480, 3, 0.9)
    tgrid = np.linspace(-300e-12, 300e-12, 6001)
    rho = th.boltzmann_profile(R480, hc, tgrid)
    m_th, s_th = th.profile_moments(tgrid, rho)
    N = 50_000
    tau = th.sample_profile(21, N, tgrid, rho)
    delta = np.random.default_rng(22).normal(0, R480["sigma_delta"], N)
    s = ref.RefSim(R480)
    s.set_harmonic_cavity(hc)
    s.set_fill([0], [0.0])
    s.alloc_particles(N, 23)
    s.set_particles(0, tau, delta)
    m = s.track(3000)
    assert m[-1500:, 0, 2].mean() == pytest.approx(s_th, rel=1e-2)
    assert abs(m[-1500:, 0, 0].mean() - m_th) < 0.02 * s_th


@pytest.mark.parametrize("alpha_sign", [1, -1])
def test_haissinski_below_threshold(alpha_sign):
    """Potential-well distortion by the BB wake at 0.5 mA: the tracked
    equilibrium matches the Haissinski fixed point (lengthening for
    alpha_c > 0; shortening for alpha_c < 0 with this inductive wake, as the
    paper observes for its ring), and the energy spread stays sigma_E."""
    ring = dict(R480, alpha_c=alpha_sign * R480["alpha_c"])
    I = 0.5e-3
    tgrid = np.linspace(-250e-12, 250e-12, 4001)
    rho = th.haissinski(ring, None, [wl.BB], I * T0, tgrid)
    m_th, s_th = th.profile_moments(tgrid, rho)
    s0 = th.profile_moments(tgrid, th.boltzmann_profile(ring, None, tgrid))[1]
    assert (s_th > s0) == (alpha_sign > 0)
    N = 50_000
    tau = th.sample_profile(31, N, tgrid, rho)
    delta = np.random.default_rng(32).normal(0, R480["sigma_delta"], N)
    s = ref.RefSim(ring)
    s.set_fill([0], [I])
    s.set_short_range([wl.BB], (512, -100e-12, 100e-12))
    s.alloc_particles(N, 33)
    s.set_particles(0, tau, delta)
    m = s.track(3000)
    assert m[-1500:, 0, 2].mean() == pytest.approx(s_th, rel=1e-2)
    assert abs(m[-1500:, 0, 0].mean() - m_th) < 0.02 * s_th
    assert m[-1500:, 0, 3].mean() == pytest.approx(R480["sigma_delta"], rel=1e-2)


# ---------------------------------------------------------------------------
# Long-range wake
# ---------------------------------------------------------------------------

def _brute_force_long_range(ring, buckets, currents, res_list, tau0, delta0, turns):
    """Direct tracker: every particle sees the sum of the resonator wakes of
    all particles of all earlier bunch passages (no phasors), with times
    measured from turn 0 in extended precision."""
    k = th.ring_constants(ring)
    E0, Vrf, w, phi, U0 = k["E0"], k["Vrf"], k["w"], k["phi_s"], k["U0"]
    D, b = k["D"], k["b"]
    T0l = np.longdouble(ring["harmonic"]) / np.longdouble(ring["f_rf_Hz"])
    Trf = np.longdouble(1) / np.longdouble(ring["f_rf_Hz"])
    M, N = tau0.shape
    tau = tau0.copy()
    delta = delta0.copy()
    src_t, src_q = [], []
    out = []
    for n in range(turns):
        for bb in range(M):
            t_nom = n * T0l + buckets[bb] * Trf
            tp = t_nom + tau[bb].astype(np.longdouble)
            V = np.zeros(N, dtype=np.longdouble)
            if src_t:
                st = np.concatenate(src_t)
                sq = np.concatenate(src_q)
                dt = tp[:, None] - st[None, :]
                for rs, q, fr in res_list:
                    wr = 2 * np.pi * np.longdouble(fr)
                    al = wr / (2 * q)
                    wb = np.sqrt(wr * wr - al * al)
                    Wt = 2 * al * rs * np.exp(-al * dt) * (np.cos(wb * dt) - al / wb * np.sin(wb * dt))
                    V += (Wt * sq[None, :]).sum(axis=1)
            qpp = currents[bb] * float(T0l) / N
            src_t.append(tp.copy())
            src_q.append(np.full(N, qpp, dtype=np.longdouble))
            dE = Vrf * np.sin(phi - w * tau[bb]) - U0 - V.astype(float)
            d = (delta[bb] + dE / E0) * (1 - D)
            delta[bb] = d
            tau[bb] = tau[bb] + b * d
        out.append((tau.copy(), delta.copy()))
    return out


def test_long_range_matches_brute_force():
    ring = dict(R480, sigma_delta=0.0)
    buckets = [2, 5, 6, 300]
    currents = [2e-3, 1e-3, 3e-3, 0.5e-3]
    res = [wl.HOM, (5e5, 300.0, 0.83e9)]
    N, turns = 16, 50
    rng = np.random.default_rng(8)
    tau0 = rng.normal(0, 15e-12, (4, N))
    delta0 = rng.normal(0, 8e-4, (4, N))
    s = ref.RefSim(ring)
    s.set_fill(buckets, currents)
    s.set_long_range(res)
    s.alloc_particles(N, 1)
    for bb in range(4):
        s.set_particles(bb, tau0[bb], delta0[bb])
    s.track(turns)
    got = np.array([s.get_particles(bb) for bb in range(4)])  # [M][2][N]
    bf = _brute_force_long_range(ring, buckets, currents, res, tau0, delta0, turns)[-1]
    # the long-range kicks move delta by ~1e-4 relative over these turns; the
    # two routes agree far below that
    assert np.max(np.abs(got[:, 0, :] - bf[0])) <= 1e-10 * 15e-12
    assert np.max(np.abs(got[:, 1, :] - bf[1])) <= 1e-10 * 8e-4
    # and the long-range wake is not negligible here
    s0 = ref.RefSim(ring)
    s0.set_fill(buckets, currents)
    s0.alloc_particles(N, 1)
    for bb in range(4):
        s0.set_particles(bb, tau0[bb], delta0[bb])
    s0.track(turns)
    free = np.array([s0.get_particles(bb) for bb in range(4)])
    assert np.max(np.abs(free[:, 1, :] - bf[1])) > 1e-6 * 8e-4


def test_passive_harmonic_cavity_beam_loading():
    """A passive harmonic cavity is a high-Q long-range resonator near n f_RF
    driven only by the beam.  For a uniform fill of point bunches (charge q,
    spacing T_rf, current I0 = q / T_rf) its steady-state voltage at a bunch,
    counting the bunch's own half charge (W(0+)/2 = alpha Rs per unit charge),
    is by Poisson summation over the bunch train 2 I0 sum_{p>=1} Re Z(p w_b)
    (Z(0) = 0 for a resonator).  The oracle gets it by rotating and depositing
    into one phasor bucket by bucket; the frequency-domain sum is independent
    of that recursion.  Particles are held at tau = 0 by a vanishing momentum
    compaction."""
    ring = dict(R480, alpha_c=1e-12, sigma_delta=0.0)
    h = ring["harmonic"]
    f_rf = ring["f_rf_Hz"]
    T_rf = 1.0 / f_rf
    I_b = 0.4e-3
    q = I_b * T0
    rs, Q = 2.0e3, 2.0e4
    fr = 3 * f_rf + 0.1e6               # third harmonic, detuned by 100 kHz
    s = ref.RefSim(ring)
    s.set_fill(list(range(h)), [I_b] * h)
    s.set_long_range([(rs, Q, fr)])
    s.alloc_particles(1, 1)
    for b in range(h):
        s.set_particles(b, [0.0], [0.0])
    s.track(300)                         # the fill time is a few turns
    _, _, ph = s.get_state()
    V = complex(ph[0], ph[1])            # just after the last bunch's deposit
    wr = 2 * np.pi * fr
    a = wr / (2 * Q)
    wb = np.sqrt(wr * wr - a * a)
    seen = (np.exp((-a + 1j * wb) * T_rf) * V).real   # at the next bucket
    got = seen + q * a * rs
    I0 = q / T_rf
    P = 2_000_000
    p = np.arange(1, P + 1, dtype=float)
    w = p * 2 * np.pi * f_rf
    reZ = th.resonator_impedance(rs, Q, fr, w).real
    tail = rs * (fr / f_rf) ** 2 / (Q * Q * P)       # sum over p > P of Rs / (Q p / n)^2
    want = 2 * I0 * (np.sum(reZ) + tail)
    assert got == pytest.approx(want, rel=1e-9)
    # the detuned cavity's fundamental term dominates: Rs cos^2(psi)
    tan_psi = Q * (3 * f_rf / fr - fr / (3 * f_rf))
    assert want == pytest.approx(2 * I0 * rs / (1 + tan_psi ** 2), rel=1e-3)


def _cb_oracle_growth(ring, M, mu, current, turns, res=wl.HOM, A=1e-13):
    """Seed the single mode z_b = tau_b - i (alpha_c/omega_s) delta_b =
    A exp(2 pi i mu b / M) and fit the growth of its amplitude."""
    omega_s = 2 * np.pi * th.synchrotron_tune(ring) / T0
    s = ref.RefSim(ring)
    s.set_fill(list(range(M)), [current] * M)
    s.set_long_range([res])
    s.alloc_particles(1, 1)
    for b in range(M):
        ph = 2 * np.pi * mu * b / M
        s.set_particles(b, [A * np.cos(ph)], [-A * omega_s / ring["alpha_c"] * np.sin(ph)])
    m = s.track(turns)
    amp = th.mode_amplitudes(m[:, :, 0], m[:, :, 1], ring["alpha_c"], omega_s)[:, mu]
    t = np.arange(turns) * T0
    sel = slice(turns // 5, turns)
    return th.fit_growth(t[sel], amp[sel])


@pytest.mark.parametrize("mu", [19, 461])
def test_coupled_bunch_growth_rate_exact(mu):
    """Uniform fill of 480 point bunches with the HOM at 1 mA per bunch: the
    oracle's mode grows (mu = 19) or decays (mu = 461) at the rate of the
    exact linearised per-turn map (self-consistent coherent tune), with
    radiation damping.  Here the coherent tune shift is ~9% of nu_s, so the
    first-order (Sacherer / Eq. 7) rate is 8% high; that form is pinned at
    weak coupling below."""
    M = 480
    ring = dict(R480, sigma_delta=0.0)
    g_ex, nu_ex = th.cb_growth_discrete(ring, wl.HOM, 1e-3, M, mu)
    g = _cb_oracle_growth(ring, M, mu, 1e-3, 6000 if g_ex > 0 else 2000)
    assert g == pytest.approx(g_ex, rel=2e-3), (g, g_ex)


def test_coupled_bunch_growth_rate_sacherer():
    """At 0.1 mA per bunch (coherent shift < 1% of nu_s) the first-order
    growth rate -- the paper's Eq. 7 summed over all revolution lines, equal
    to the time-domain sum -- matches the oracle within 2% (damping off)."""
    M, mu = 480, 19
    ring = dict(R480, sigma_delta=0.0, tau_long_s=float("inf"))
    g_eq7 = th.cb_growth_frequency_domain(ring, wl.HOM, 0.1e-3, M, mu)
    assert th.cb_growth_time_domain(ring, wl.HOM, 0.1e-3, M, mu) == pytest.approx(g_eq7, rel=1e-6)
    g = _cb_oracle_growth(ring, M, mu, 0.1e-3, 12000)
    assert g == pytest.approx(g_eq7, rel=2e-2), (g, g_eq7)


# ---------------------------------------------------------------------------
# Determinism, resume, validation
# ---------------------------------------------------------------------------

def _mb_oracle():
    s = ref.RefSim(R480)
    s.set_harmonic_cavity(ref.hc_flat_fraction(R480, 3, 0.9))
    s.set_fill([0, 4, 9], [1e-3, 2e-3, 0.5e-3])
    s.set_short_range([wl.BB], (128, -120e-12, 120e-12))
    s.set_long_range([wl.HOM])
    s.init_gaussian(5000, 20e-12, 8.6e-4, 3)
    return s


def test_checkpoint_resume_bitwise():
    a = _mb_oracle()
    full = a.track(40)
    b = _mb_oracle()
    first = b.track(20)
    turn, seed, ph = b.get_state()
    parts = [b.get_particles(i) for i in range(3)]
    c = _mb_oracle()
    for i, (t, d) in enumerate(parts):
        c.set_particles(i, t, d)
    c.set_state(turn, seed, ph)
    second = c.track(20)
    assert np.array_equal(np.concatenate([first, second]), full)


# ---------------------------------------------------------------------------
# Bunch moments (Sec. 2.4): means and population rms of the state after a turn
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N", [2001, 7])
def test_moments_match_numpy_definition(N):
    # Three bunches with wakes, long range and noise on; bunch 1 sits 5 sigma
    # off in both coordinates, so a one-pass or shifted-reference slip would
    # show, and bunch 2 is nearly a point (rms 1e-6 of its offset).  The
    # oracle's moments of the state after the turn must be numpy's mean and
    # std with ddof=0 of the particles it returns (a 1/(N-1) variance is off
    # by 1/(2N) relative: 2.5e-4 at N = 2001, 7e-2 at N = 7).
    s = ref.RefSim(R480)
    s.set_fill([0, 3, 8], [1e-3, 2e-3, 0.5e-3])
    s.set_short_range([wl.BB], (128, -120e-12, 120e-12))
    s.set_long_range([wl.HOM])
    s.alloc_particles(N, 11)
    offs = [(0.0, 0.0, 1.0), (5 * 15e-12, 5 * 8.6e-4, 1.0), (40e-12, 1e-3, 1e-6)]
    for b, (mt, md, scale) in enumerate(offs):
        tau, delta = wl.gaussian_particles(70 + b, N, scale * 15e-12, scale * 8.6e-4,
                                           mean_tau=mt, mean_delta=md)
        s.set_particles(b, tau, delta)
    mom = s.track(1)
    assert mom.shape == (1, 3, 4)
    for b in range(3):
        tau, delta = s.get_particles(b)
        expect = np.array([np.mean(tau), np.mean(delta), np.std(tau, ddof=0),
                           np.std(delta, ddof=0)])
        scale = np.array([np.std(tau), np.std(delta)] * 2)
        scale = np.maximum(np.abs(expect), scale)
        assert np.all(np.abs(mom[0, b] - expect) <= 1e-14 * scale), (b, mom[0, b], expect)
        # the rms is the population one, not the sample one
        sample = np.array([np.std(tau, ddof=1), np.std(delta, ddof=1)])
        assert np.all(np.abs(mom[0, b, 2:] - sample) > 1e-6 * sample)


def test_thread_count_does_not_change_results():
    code = (
        "import sys, numpy as np; sys.path.insert(0, %r); sys.path.insert(0, %r);"
        "from test_oracle_pins import _mb_oracle; s = _mb_oracle(); m = s.track(10);"
        "sys.stdout.write(m.tobytes().hex())" % (ROOT, HERE))
    outs = []
    for nt in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=nt)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           check=True)
        outs.append(r.stdout)
    assert outs[0] == outs[1] and len(outs[0]) > 0


def test_validation_errors():
    bad = [dict(R480, energy_eV=0.0), dict(R480, v_rf_V=0.4e6), dict(R480, alpha_c=0.0),
           dict(R480, harmonic=0), dict(R480, tau_long_s=-1.0), dict(R480, sigma_delta=-1e-4),
           dict(R480, f_rf_Hz=float("nan"))]
    for r in bad:
        with pytest.raises(ref.OracleError):
            ref.RefSim(r)
    s = ref.RefSim(R480)
    with pytest.raises(ref.OracleError):
        s.set_fill([3, 3], [1e-3, 1e-3])
    with pytest.raises(ref.OracleError):
        s.set_fill([0, 480], [1e-3, 1e-3])
    with pytest.raises(ref.OracleError):
        s.set_short_range([(1.0, 0.5, 1e9)], (64, -1e-11, 1e-11))
    with pytest.raises(ref.OracleError):
        s.set_short_range([wl.BB], (0, -1e-11, 1e-11))
    with pytest.raises(ref.OracleError):
        s.track(1)  # no fill, no particles
    with pytest.raises(ref.OracleError):
        s.set_harmonic_cavity({"n": 3, "v_ratio": 10.0, "phase_n_rad": -1.5})


# ---------------------------------------------------------------------------
# Short-range resistive-wall wake (the paper's validation: copper, 10 mm)
# ---------------------------------------------------------------------------

RW_CU = (0.010, 5.8e7, 288.0)     # radius m, conductivity S/m, length m
C_LIGHT, Z0 = 299792458.0, 376.730313668


def test_resistive_wall_wake_limits():
    """W(0+) = Z0 c L / (pi b^2), independent of the conductivity; far behind
    the charge the classic thick-wall wake -(c L / (4 pi b)) sqrt(Z0 / (pi
    sigma)) z^-3/2, which follows from the thick-wall impedance alone."""
    b, sig, L = RW_CU
    assert ref.rw_wake(RW_CU, 0.0) == pytest.approx(Z0 * C_LIGHT * L / (np.pi * b * b), rel=1e-13)
    assert ref.rw_wake((b, 10 * sig, L), 0.0) == pytest.approx(ref.rw_wake(RW_CU, 0.0), rel=1e-13)
    s0 = (2 * b * b / (Z0 * sig)) ** (1 / 3)
    for u in (1e3, 1e4):
        z = u * s0
        classic = -(C_LIGHT * L / (4 * np.pi * b)) * np.sqrt(Z0 / (np.pi * sig)) * z ** -1.5
        assert ref.rw_wake(RW_CU, z / C_LIGHT) == pytest.approx(classic, rel=3.0 / u ** 3 + 1e-11)
    assert ref.rw_wake(RW_CU, -1e-12) == 0.0


@pytest.mark.parametrize("kappa", [0.05, 0.2, 1.0, 3.0, 10.0])
def test_resistive_wall_wake_transforms_to_impedance(kappa):
    """The Fourier transform of the wake is the round-pipe impedance with DC
    conductivity, Z(w) = (L / (2 pi b)) / (1/Z_s + i w eps0 b / 2) with the
    surface impedance Z_s = (1 + i) sqrt(w mu0 / (2 sigma)), at w = kappa c/s0
    where the short-range term matters."""
    import warnings
    b, sig, L = RW_CU
    s0 = (2 * b * b / (Z0 * sig)) ** (1 / 3)
    W = lambda u: ref.rw_wake(RW_CU, u * s0 / C_LIGHT)
    U = 60.0
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        re = integrate.quad(lambda u: W(u) * np.cos(kappa * u), 0, U, limit=400, epsabs=0,
                            epsrel=1e-11)[0]
        im = -integrate.quad(lambda u: W(u) * np.sin(kappa * u), 0, U, limit=400, epsabs=0,
                             epsrel=1e-11)[0]
        re += integrate.quad(W, U, np.inf, weight="cos", wvar=kappa, limlst=200)[0]
        im -= integrate.quad(W, U, np.inf, weight="sin", wvar=kappa, limlst=200)[0]
    z_num = (s0 / C_LIGHT) * complex(re, im)
    w = kappa * C_LIGHT / s0
    zs = (1 + 1j) * np.sqrt(w * (Z0 / C_LIGHT) / (2 * sig))
    z_th = (L / (2 * np.pi * b)) / (1 / zs + 1j * w * b / (2 * Z0 * C_LIGHT))
    assert abs(z_num - z_th) <= 1e-9 * abs(z_th)


def test_resistive_wall_table_and_tracking_hook():
    """The table adds the wall's samples (self term W(0+)/2) to the
    resonators', and a simulation with the wall set kicks differently from
    one without."""
    grid = (128, -60e-12, 60e-12)
    W_res = ref.wake_table([wl.BB], grid)
    W_all = ref.wake_table([wl.BB], grid, rw=RW_CU)
    dt = 120e-12 / 128
    assert W_all[0] - W_res[0] == pytest.approx(0.5 * ref.rw_wake(RW_CU, 0.0), rel=1e-14)
    k = np.arange(1, 128)
    extra = np.array([ref.rw_wake(RW_CU, kk * dt) for kk in k])
    assert np.allclose(W_all[1:] - W_res[1:], extra, rtol=1e-12, atol=1e-12 * np.max(np.abs(extra)))
    moms = []
    for rw in (None, RW_CU):
        s = ref.RefSim(R480)
        s.set_fill([0], [5e-3])
        s.set_short_range([wl.BB], grid)
        s.set_resistive_wall(rw)
        s.init_gaussian(2000, 10e-12, 8.6e-4, 3)
        moms.append(s.track(20))
    assert not np.allclose(moms[0], moms[1], rtol=1e-6, atol=0)
