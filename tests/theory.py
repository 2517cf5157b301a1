"""Closed forms and textbook results that pin the oracle (and, through it, the
GPU tracker).  Nothing here calls the oracle: each function is the physics or
mathematics the tracking must reproduce, written independently.

Ring notation: E0 [eV], V_rf [V], w_rf = 2 pi f_rf, alpha_c, T0 = h/f_rf,
D = 2 T0 / tau_L (per-turn damping of delta, the paper's Eq. 5 read with a
single coefficient), sigma_E the equilibrium energy spread.
"""
import numpy as np
from scipy import integrate, linalg

TWO_PI = 2.0 * np.pi


def ring_constants(ring, u0=None, hc=None):
    E0, Vrf, frf, h = ring["energy_eV"], ring["v_rf_V"], ring["f_rf_Hz"], ring["harmonic"]
    U0 = ring["u0_eV"] if u0 is None else u0
    T0 = h / frf
    w = TWO_PI * frf
    s = U0 / Vrf - (hc["v_ratio"] * np.sin(hc["phase_n_rad"]) if hc else 0.0)
    phi = np.arcsin(s) if ring["alpha_c"] > 0 else np.pi - np.arcsin(s)
    D = 2.0 * T0 / ring["tau_long_s"]
    return dict(E0=E0, Vrf=Vrf, w=w, T0=T0, phi_s=phi, U0=U0, D=D,
                b=ring["alpha_c"] * T0, noise=ring["sigma_delta"] * np.sqrt(2.0 * D))


def linear_map(ring, u0=None, with_damping=True):
    """One-turn matrix of (tau, delta) near the synchronous particle for
    kick -> damping -> drift with the new delta: M = Drift * Damp * Kick."""
    k = ring_constants(ring, u0)
    a = k["Vrf"] * k["w"] * np.cos(k["phi_s"]) / k["E0"]  # -d(kick)/d(tau)
    kick = np.array([[1.0, 0.0], [-a, 1.0]])
    damp = np.diag([1.0, 1.0 - (k["D"] if with_damping else 0.0)])
    drift = np.array([[1.0, k["b"]], [0.0, 1.0]])
    return drift @ damp @ kick, a, k["b"]


def synchrotron_tune(ring, u0=None):
    """Closed form for the symplectic kick-drift map: cos(2 pi nu) = 1 - a b / 2."""
    _, a, b = linear_map(ring, u0, with_damping=False)
    return float(np.arccos(1.0 - a * b / 2.0) / TWO_PI)


def equilibrium_covariance(ring):
    """Stationary covariance of (tau, delta) under the linear damped map with
    the noise sigma_E sqrt(2D) z added to delta before the drift:
    Sigma = M Sigma M^T + Q, Q = B diag(0, s^2) B^T with B the drift."""
    M, a, b = linear_map(ring)
    k = ring_constants(ring)
    B = np.array([[1.0, k["b"]], [0.0, 1.0]])
    Q = B @ np.diag([0.0, k["noise"] ** 2]) @ B.T
    # solve in coordinates of comparable size (tau in units of sqrt(b/a))
    S = np.diag([np.sqrt(abs(b / a)), 1.0])
    Si = np.linalg.inv(S)
    X = linalg.solve_discrete_lyapunov(Si @ M @ S, Si @ Q @ Si.T)
    return S @ X @ S.T


def resonator_impedance(rs, q, fr, w):
    """Textbook resonator impedance Z(w) = Rs / (1 + i Q (w/wr - wr/w))."""
    wr = TWO_PI * fr
    w = np.asarray(w, dtype=float)
    return rs / (1.0 + 1j * q * (w / wr - wr / w))


def gaussian_loss_factor(resonators, sigma):
    """k(sigma) = (1/pi) int_0^inf Re Z(w) exp(-w^2 sigma^2) dw  [V/C]."""
    tot = 0.0
    for rs, q, fr in resonators:
        wr = TWO_PI * fr
        f = lambda w: resonator_impedance(rs, q, fr, w).real * np.exp(-(w * sigma) ** 2)
        pts = [wr * 0.5, wr, wr * 1.5]
        val, _ = integrate.quad(f, 0.0, 12.0 / sigma + 4 * wr, points=pts, limit=400)
        tot += val / np.pi
    return tot


def total_voltage(ring, hc, tau):
    k = ring_constants(ring, hc=hc)
    v = k["Vrf"] * np.sin(k["phi_s"] - k["w"] * tau)
    if hc:
        v = v + hc["v_ratio"] * k["Vrf"] * np.sin(hc["phase_n_rad"] - hc["n"] * k["w"] * tau)
    return v - k["U0"]


def boltzmann_profile(ring, hc, tau, wake_voltage=None):
    """Equilibrium line density of the Fokker-Planck equation for a kick F
    per turn and drift b delta: rho ~ exp(int_0^tau F dtau' / (b sigma_E^2)),
    F = (V_rf + V_hc - U0 - V_wake)/E0.  Returns the normalised rho on tau."""
    k = ring_constants(ring, hc=hc)
    F = total_voltage(ring, hc, tau)
    if wake_voltage is not None:
        F = F - wake_voltage
    F = F / k["E0"]
    U = integrate.cumulative_trapezoid(F, tau, initial=0.0)
    U -= U[np.argmin(np.abs(tau))]
    expo = U / (k["b"] * ring["sigma_delta"] ** 2)
    rho = np.exp(expo - expo.max())
    return rho / np.trapezoid(rho, tau)


def profile_moments(tau, rho):
    m = np.trapezoid(tau * rho, tau)
    return m, np.sqrt(np.trapezoid((tau - m) ** 2 * rho, tau))


def haissinski(ring, hc, resonators, charge, tau, iters=3000, relax=0.1):
    """Fixed point of the potential-well distortion (Haissinski): the line
    density in the RF potential plus the wake potential of the density itself,
    V_w(tau) = Q int rho(tau') W(tau - tau') dtau' with the causal resonator
    wake; solved by damped iteration on the grid tau (uniform)."""
    dt = tau[1] - tau[0]
    n = tau.size
    lags = np.arange(n) * dt
    W = np.zeros(n)
    for rs, q, fr in resonators:
        wr = TWO_PI * fr
        al = wr / (2 * q)
        wb = np.sqrt(wr * wr - al * al)
        W += 2 * al * rs * np.exp(-al * lags) * (np.cos(wb * lags) - al / wb * np.sin(wb * lags))
    W[0] *= 0.5  # the distribution's own point: half the jump (trapezoid rule)
    rho = boltzmann_profile(ring, hc, tau)
    for _ in range(iters):
        Vw = charge * dt * np.convolve(rho, W)[:n]
        new = boltzmann_profile(ring, hc, tau, Vw)
        rho = relax * new + (1 - relax) * rho
    return rho


def flat_potential_derivatives(ring, hc, h=1e-13):
    """Total voltage and its first two tau-derivatives at tau = 0 (centred
    finite differences of the analytic voltage)."""
    v0 = total_voltage(ring, hc, 0.0)
    v1 = (total_voltage(ring, hc, h) - total_voltage(ring, hc, -h)) / (2 * h)
    v2 = (total_voltage(ring, hc, h) - 2 * v0 + total_voltage(ring, hc, -h)) / h ** 2
    return v0, v1, v2


# ---------------------------------------------------------------------------
# Coupled-bunch growth rates (uniform fill of M point bunches).
# ---------------------------------------------------------------------------

def cb_growth_time_domain(ring, resonator, current_per_bunch, M, mu, omega_s=None):
    """Linear growth rate [1/s] of coupled-bunch mode mu (bunch b oscillating
    as exp(i omega_s t + 2 pi i mu b / M)) for M equal point bunches in a
    uniform fill, from the wake of all earlier passages:
        g = alpha_c q / (2 omega_s E0 T0) * Im sum_{k>=1} W'(k Tb) exp(-i k (omega_s Tb + 2 pi mu / M)),
    with the resonator's W(t) = Re[c exp(s t)], s = -alpha + i wbar, summed as a
    geometric series.  Radiation damping is not included."""
    k = ring_constants(ring)
    T0 = k["T0"]
    Tb = T0 / M
    if omega_s is None:
        omega_s = TWO_PI * synchrotron_tune(ring) / T0
    rs, q, fr = resonator
    wr = TWO_PI * fr
    al = wr / (2 * q)
    wb = np.sqrt(wr * wr - al * al)
    c = 2 * al * rs * (1 + 1j * al / wb)
    s = -al + 1j * wb
    theta = omega_s * Tb + TWO_PI * mu / M
    x = np.exp(s * Tb - 1j * theta)
    y = np.exp(np.conj(s) * Tb - 1j * theta)
    F = 0.5 * c * s * x / (1 - x) + 0.5 * np.conj(c) * np.conj(s) * y / (1 - y)
    charge = current_per_bunch * T0
    return ring["alpha_c"] * charge / (2 * omega_s * k["E0"] * T0) * F.imag


def cb_growth_frequency_domain(ring, resonator, current_per_bunch, M, mu, omega_s=None,
                               sigma_tau=0.0, pmax=None):
    """The same growth rate in the frequency domain (the paper's Eq. 7 with
    omega_p in place of its omega_r prefactor, summed over all lines):
        g = alpha_c q M / (2 omega_s E0 T0^2) * sum_p omega_p Re Z(|omega_p|) F(omega_p),
    omega_p = (p M + mu) omega_0 + omega_s, with the dipole form factor
    F = exp(-(omega_p sigma)^2) of a Gaussian bunch (1 for point bunches)."""
    k = ring_constants(ring)
    T0 = k["T0"]
    w0 = TWO_PI / T0
    if omega_s is None:
        omega_s = TWO_PI * synchrotron_tune(ring) / T0
    rs, q, fr = resonator
    wr = TWO_PI * fr
    pc = int(round(wr / (M * w0)))
    if pmax is None:
        pmax = 2000
    p = np.arange(-pc - pmax, pc + pmax + 1)
    wp = (p * M + mu) * w0 + omega_s
    ReZ = resonator_impedance(rs, q, fr, np.abs(wp)).real
    term = wp * ReZ * np.exp(-(wp * sigma_tau) ** 2)
    charge = current_per_bunch * T0
    return ring["alpha_c"] * charge * M / (2 * omega_s * k["E0"] * T0 ** 2) * term.sum()


def cb_growth_discrete(ring, resonator, current_per_bunch, M, mu, damping=True, iters=200):
    """Exact linear growth rate [1/s] and tune of coupled-bunch mode mu for M
    equal point bunches in a uniform fill under the per-turn map (kick with
    the RF slope and the wake of all earlier passages, damping, drift).  With
    every coordinate of bunch b at turn n proportional to
    Lam^(n + b/M) exp(2 pi i mu b / M), the wake of the source k passages
    earlier enters through F(Lam) = sum_k W'(k Tb) Lam^(-k/M) exp(-2 pi i mu k / M);
    the one-turn 2x2 matrix then has det = 1 - D and
    trace = 2 - D - b (1 - D) (a - q (F(Lam) - F0) / E0), and Lam is the
    self-consistent root (fixed-point iteration from the bare tune).  Unlike
    the first-order forms above it keeps the coherent frequency shift."""
    k = ring_constants(ring)
    T0 = k["T0"]
    Tb = T0 / M
    a = k["Vrf"] * k["w"] * np.cos(k["phi_s"]) / k["E0"]
    b = k["b"]
    D = k["D"] if damping else 0.0
    rs, q, fr = resonator
    wr = TWO_PI * fr
    al = wr / (2 * q)
    wb = np.sqrt(wr * wr - al * al)
    c = 2 * al * rs * (1 + 1j * al / wb)
    s = -al + 1j * wb
    phase = np.exp(-1j * TWO_PI * mu / M)

    def wake_sum(rot):
        x = np.exp(s * Tb) * rot
        y = np.exp(np.conj(s) * Tb) * rot
        return 0.5 * c * s * x / (1 - x) + 0.5 * np.conj(c) * np.conj(s) * y / (1 - y)

    F0 = wake_sum(1.0).real
    charge = current_per_bunch * T0
    lam = np.exp(1j * np.arccos(1 - a * b / 2))
    for _ in range(iters):
        K = charge / k["E0"] * (wake_sum(lam ** (-1.0 / M) * phase) - F0)
        tr = 2 - D - b * (1 - D) * (a - K)
        roots = np.roots([1.0, -tr, 1 - D])
        lam = roots[np.argmin(np.abs(roots - lam))]
    return float(np.log(abs(lam)) / T0), float(np.angle(lam) / TWO_PI)


def radiation_damping_rate(ring):
    """Amplitude decay rate of the damped linear map: -ln(1 - D) / (2 T0)."""
    k = ring_constants(ring)
    return -np.log(1.0 - k["D"]) / (2.0 * k["T0"])


def mode_amplitudes(tau, delta, alpha_c, omega_s):
    """Complex mode amplitudes a_mu(t) of M bunch centroids (arrays [T][M]):
    z_b = tau_b - i (alpha_c/omega_s) delta_b rotates as exp(+i omega_s t);
    a_mu = (1/M) sum_b z_b exp(-2 pi i mu b / M)."""
    z = tau - 1j * (alpha_c / omega_s) * delta
    return np.fft.fft(z, axis=-1) / z.shape[-1]


def fit_growth(t, amp):
    """Least-squares slope of ln|amp| against t."""
    A = np.vstack([t, np.ones_like(t)]).T
    slope, _ = np.linalg.lstsq(A, np.log(np.abs(amp)), rcond=None)[0]
    return slope


def sample_profile(seed, N, tau, rho):
    """N samples from a tabulated line density by inverse CDF."""
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (rho[1:] + rho[:-1]) * np.diff(tau))])
    cdf /= cdf[-1]
    u = np.random.default_rng(seed).uniform(size=N)
    return np.interp(u, cdf, tau)
