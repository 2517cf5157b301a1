"""ctypes binding of the oracle library (plain FP64 CPU tracker).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  Nothing in the GPU library or its Python
binding imports this module.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class RefRing(C.Structure):
    _fields_ = [("energy_eV", C.c_double), ("f_rf_Hz", C.c_double), ("v_rf_V", C.c_double),
                ("alpha_c", C.c_double), ("u0_eV", C.c_double), ("tau_long_s", C.c_double),
                ("sigma_delta", C.c_double), ("harmonic", C.c_int32)]


class RefHC(C.Structure):
    _fields_ = [("n", C.c_int32), ("v_ratio", C.c_double), ("phase_n_rad", C.c_double)]


class RefResonator(C.Structure):
    _fields_ = [("rs_ohm", C.c_double), ("q", C.c_double), ("fr_Hz", C.c_double)]


class RefGrid(C.Structure):
    _fields_ = [("nbins", C.c_int32), ("tau_min_s", C.c_double), ("tau_max_s", C.c_double)]


class RefRW(C.Structure):
    _fields_ = [("radius_m", C.c_double), ("conductivity_S_m", C.c_double),
                ("length_m", C.c_double)]


class RefTransverse(C.Structure):
    _fields_ = [("tune", C.c_double), ("chromaticity", C.c_double), ("alpha", C.c_double),
                ("beta_m", C.c_double), ("disp_m", C.c_double), ("disp_prime", C.c_double),
                ("emittance_m", C.c_double), ("tau_damp_s", C.c_double)]


class RefLRRW(C.Structure):
    _fields_ = [("radius_m", C.c_double), ("conductivity_S_m", C.c_double),
                ("length_m", C.c_double), ("turns", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = C.CDLL(path)
        P = C.POINTER
        dp, up, ip = P(C.c_double), P(C.c_uint32), P(C.c_int32)
        sims = C.c_void_p
        sig = {
            "mbt_ref_philox4x32_10": (None, [up, up, up]),
            "mbt_ref_normal_pair": (None, [C.c_uint64, up, dp]),
            "mbt_ref_resonator_wake": (C.c_double, [P(RefResonator), C.c_double]),
            "mbt_ref_wake_table": (C.c_int, [C.c_int32, P(RefResonator), P(RefGrid), dp]),
            "mbt_ref_rw_wake": (C.c_double, [P(RefRW), C.c_double]),
            "mbt_ref_wake_table_rw": (C.c_int, [C.c_int32, P(RefResonator), P(RefRW), P(RefGrid), dp]),
            "mbt_ref_set_resistive_wall": (C.c_int, [sims, P(RefRW)]),
            "mbt_ref_bin_index": (C.c_int32, [P(RefGrid), C.c_double]),
            "mbt_ref_histogram": (C.c_int, [P(RefGrid), C.c_int64, dp, up, P(C.c_int64)]),
            "mbt_ref_wake_potential": (C.c_int, [C.c_int32, dp, up, C.c_double, dp]),
            "mbt_ref_hc_flat_fraction": (C.c_int, [P(RefRing), C.c_int32, C.c_double, P(RefHC)]),
            "mbt_ref_create": (C.c_int, [P(RefRing), P(sims)]),
            "mbt_ref_destroy": (None, [sims]),
            "mbt_ref_last_error": (C.c_char_p, [sims]),
            "mbt_ref_set_harmonic_cavity": (C.c_int, [sims, P(RefHC)]),
            "mbt_ref_set_fill": (C.c_int, [sims, C.c_int32, ip, dp, ip]),
            "mbt_ref_set_short_range": (C.c_int, [sims, C.c_int32, P(RefResonator), P(RefGrid)]),
            "mbt_ref_set_long_range": (C.c_int, [sims, C.c_int32, P(RefResonator)]),
            "mbt_ref_init_gaussian": (C.c_int, [sims, C.c_int64, C.c_double, C.c_double, C.c_uint64]),
            "mbt_ref_alloc_particles": (C.c_int, [sims, C.c_int64, C.c_uint64]),
            "mbt_ref_set_particles": (C.c_int, [sims, C.c_int32, dp, dp]),
            "mbt_ref_get_particles": (C.c_int, [sims, C.c_int32, dp, dp]),
            "mbt_ref_track": (C.c_int, [sims, C.c_int64, dp, up, C.c_int32]),
            "mbt_ref_get_state": (C.c_int, [sims, P(C.c_int64), P(C.c_uint64), dp]),
            "mbt_ref_set_state": (C.c_int, [sims, C.c_int64, C.c_uint64, dp]),
            "mbt_ref_derived": (C.c_int, [sims, dp]),
            "mbt_ref_threads": (C.c_int, []),
            "mbt_ref_set_threads": (C.c_int, [C.c_int]),
            "mbt_ref_transverse_resonator_wake": (C.c_double, [P(RefResonator), C.c_double]),
            "mbt_ref_transverse_rw_wake": (C.c_double, [P(RefRW), C.c_double]),
            "mbt_ref_transverse_wake_table": (C.c_int, [C.c_int32, P(RefResonator), P(RefGrid), dp]),
            "mbt_ref_dipole_histogram": (C.c_int, [P(RefGrid), C.c_int64, dp, dp, up, dp]),
            "mbt_ref_transverse_kicks": (C.c_int, [C.c_int32, dp, dp, C.c_double, dp]),
            "mbt_ref_set_transverse": (C.c_int, [sims, P(RefTransverse)]),
            "mbt_ref_set_transverse_wake": (C.c_int, [sims, C.c_int32, P(RefResonator)]),
            "mbt_ref_set_transverse_rw": (C.c_int, [sims, P(RefLRRW)]),
            "mbt_ref_init_transverse": (C.c_int, [sims, C.c_double, C.c_double]),
            "mbt_ref_set_transverse_particles": (C.c_int, [sims, C.c_int32, dp, dp]),
            "mbt_ref_get_transverse_particles": (C.c_int, [sims, C.c_int32, dp, dp]),
            "mbt_ref_track2": (C.c_int, [sims, C.c_int64, dp, dp, up, C.c_int32]),
            "mbt_ref_get_rw_history": (C.c_int, [sims, dp]),
            "mbt_ref_set_rw_history": (C.c_int, [sims, dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _up(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


# ---- free functions -------------------------------------------------------

def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().mbt_ref_philox4x32_10(_up(c), _up(k), _up(out))
    return out


def normal_pair(seed, ctr):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    z = np.zeros(2)
    lib().mbt_ref_normal_pair(C.c_uint64(seed), _up(c), _dp(z))
    return z


def resonator_wake(rs, q, fr, t):
    r = RefResonator(rs, q, fr)
    return lib().mbt_ref_resonator_wake(C.byref(r), float(t))


def rw_wake(rw, t):
    """Short-range resistive-wall wake W(t) in V/C; rw = (radius, conductivity, length)."""
    return lib().mbt_ref_rw_wake(C.byref(RefRW(*map(float, rw))), float(t))


def wake_table(resonators, grid, rw=None):
    arr = (RefResonator * max(1, len(resonators)))(*[RefResonator(*r) for r in resonators])
    g = RefGrid(*grid)
    W = np.zeros(g.nbins)
    r = None if rw is None else C.byref(RefRW(*map(float, rw)))
    rc = lib().mbt_ref_wake_table_rw(len(resonators), arr, r, C.byref(g), _dp(W))
    if rc:
        raise OracleError(rc, "wake_table")
    return W


def bin_index(grid, tau):
    g = RefGrid(*grid)
    return lib().mbt_ref_bin_index(C.byref(g), float(tau))


def histogram(grid, tau):
    g = RefGrid(*grid)
    t = np.ascontiguousarray(tau, dtype=np.float64)
    counts = np.zeros(g.nbins, dtype=np.uint32)
    oog = C.c_int64(0)
    rc = lib().mbt_ref_histogram(C.byref(g), t.size, _dp(t), _up(counts), C.byref(oog))
    if rc:
        raise OracleError(rc, "histogram")
    return counts, oog.value


def wake_potential(W, counts, q_per_particle):
    W = np.ascontiguousarray(W, dtype=np.float64)
    c = np.ascontiguousarray(counts, dtype=np.uint32)
    V = np.zeros_like(W)
    rc = lib().mbt_ref_wake_potential(W.size, _dp(W), _up(c), float(q_per_particle), _dp(V))
    if rc:
        raise OracleError(rc, "wake_potential")
    return V


def hc_flat_fraction(ring, n, frac):
    r = RefRing(**ring)
    out = RefHC()
    rc = lib().mbt_ref_hc_flat_fraction(C.byref(r), n, frac, C.byref(out))
    if rc:
        raise OracleError(rc, "hc_flat_fraction")
    return {"n": out.n, "v_ratio": out.v_ratio, "phase_n_rad": out.phase_n_rad}


def transverse_resonator_wake(rs, q, fr, t):
    """Transverse resonator wake in V/(C m) (R_s in Ohm/m)."""
    return lib().mbt_ref_transverse_resonator_wake(C.byref(RefResonator(rs, q, fr)), float(t))


def transverse_rw_wake(rw, t):
    """Long-range transverse resistive-wall wake; rw = (radius, conductivity, length)."""
    return lib().mbt_ref_transverse_rw_wake(C.byref(RefRW(*map(float, rw))), float(t))


def transverse_wake_table(resonators, grid):
    arr = (RefResonator * max(1, len(resonators)))(*[RefResonator(*r) for r in resonators])
    g = RefGrid(*grid)
    T = np.zeros(g.nbins)
    rc = lib().mbt_ref_transverse_wake_table(len(resonators), arr, C.byref(g), _dp(T))
    if rc:
        raise OracleError(rc, "transverse_wake_table")
    return T


def dipole_histogram(grid, tau, x):
    g = RefGrid(*grid)
    t = np.ascontiguousarray(tau, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    counts = np.zeros(g.nbins, dtype=np.uint32)
    X = np.zeros(g.nbins)
    rc = lib().mbt_ref_dipole_histogram(C.byref(g), t.size, _dp(t), _dp(xx), _up(counts), _dp(X))
    if rc:
        raise OracleError(rc, "dipole_histogram")
    return counts, X


def transverse_kicks(T, X, scale):
    T = np.ascontiguousarray(T, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    U = np.zeros_like(T)
    rc = lib().mbt_ref_transverse_kicks(T.size, _dp(T), _dp(X), float(scale), _dp(U))
    if rc:
        raise OracleError(rc, "transverse_kicks")
    return U


def threads():
    return lib().mbt_ref_threads()


def set_threads(n):
    """Threads of the oracle's per-particle loop from now on; returns the number in effect."""
    return lib().mbt_ref_set_threads(int(n))


# ---- simulation object ----------------------------------------------------

class RefSim:
    """One oracle simulation: ring, optional harmonic cavity, fill, wakes."""

    def __init__(self, ring):
        self._h = C.c_void_p()
        r = RefRing(**ring)
        rc = lib().mbt_ref_create(C.byref(r), C.byref(self._h))
        if rc:
            raise OracleError(rc, "create: invalid ring parameters")
        self.M = 0
        self.N = 0
        self.nbins = 0
        self.n_lr = 0

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().mbt_ref_destroy(self._h)
            self._h = C.c_void_p()

    def _check(self, rc):
        if rc:
            raise OracleError(rc, lib().mbt_ref_last_error(self._h).decode())

    def set_harmonic_cavity(self, hc):
        if hc is None:
            self._check(lib().mbt_ref_set_harmonic_cavity(self._h, None))
        else:
            h = RefHC(hc["n"], hc["v_ratio"], hc["phase_n_rad"])
            self._check(lib().mbt_ref_set_harmonic_cavity(self._h, C.byref(h)))

    def set_fill(self, buckets, currents_A, streams=None):
        b = np.ascontiguousarray(buckets, dtype=np.int32)
        c = np.ascontiguousarray(currents_A, dtype=np.float64)
        s = None if streams is None else np.ascontiguousarray(streams, dtype=np.int32)
        self._check(lib().mbt_ref_set_fill(self._h, b.size, _ip(b), _dp(c),
                                           None if s is None else _ip(s)))
        self.M = int(b.size)

    def set_short_range(self, resonators, grid):
        if grid is None:
            self._check(lib().mbt_ref_set_short_range(self._h, 0, None, None))
            self.nbins = 0
            return
        arr = (RefResonator * max(1, len(resonators)))(*[RefResonator(*r) for r in resonators])
        g = RefGrid(*grid)
        self._check(lib().mbt_ref_set_short_range(self._h, len(resonators), arr, C.byref(g)))
        self.nbins = g.nbins

    def set_long_range(self, resonators):
        arr = (RefResonator * max(1, len(resonators)))(*[RefResonator(*r) for r in resonators])
        self._check(lib().mbt_ref_set_long_range(self._h, len(resonators), arr))
        self.n_lr = len(resonators)

    def set_resistive_wall(self, rw):
        r = None if rw is None else C.byref(RefRW(*map(float, rw)))
        self._check(lib().mbt_ref_set_resistive_wall(self._h, r))

    def init_gaussian(self, N, sigma_tau, sigma_delta, seed):
        self._check(lib().mbt_ref_init_gaussian(self._h, N, sigma_tau, sigma_delta, seed))
        self.N = N

    def alloc_particles(self, N, seed):
        self._check(lib().mbt_ref_alloc_particles(self._h, N, seed))
        self.N = N

    def set_particles(self, bunch, tau, delta):
        t = np.ascontiguousarray(tau, dtype=np.float64)
        d = np.ascontiguousarray(delta, dtype=np.float64)
        assert t.size == self.N and d.size == self.N
        self._check(lib().mbt_ref_set_particles(self._h, bunch, _dp(t), _dp(d)))

    def get_particles(self, bunch):
        t = np.zeros(self.N)
        d = np.zeros(self.N)
        self._check(lib().mbt_ref_get_particles(self._h, bunch, _dp(t), _dp(d)))
        return t, d

    def track(self, nturns, profiles_stride=0):
        mom = np.zeros((nturns, self.M, 4))
        counts = None
        if profiles_stride:
            rows = -(-nturns // profiles_stride)
            counts = np.zeros((rows, self.M, self.nbins), dtype=np.uint32)
        self._check(lib().mbt_ref_track(self._h, nturns, _dp(mom),
                                        None if counts is None else _up(counts),
                                        int(profiles_stride)))
        return (mom, counts) if profiles_stride else mom

    def get_state(self):
        turn = C.c_int64()
        seed = C.c_uint64()
        ph = np.zeros(2 * max(1, self.n_lr))
        self._check(lib().mbt_ref_get_state(self._h, C.byref(turn), C.byref(seed), _dp(ph)))
        return turn.value, seed.value, ph[:2 * self.n_lr].copy()

    def set_state(self, turn, seed, phasors):
        ph = np.zeros(2 * max(1, self.n_lr))
        if phasors is not None and len(phasors):
            ph[:2 * self.n_lr] = np.asarray(phasors, dtype=np.float64)[:2 * self.n_lr]
        self._check(lib().mbt_ref_set_state(self._h, turn, seed, _dp(ph)))

    # ---- transverse plane --------------------------------------------
    def set_transverse(self, tr):
        """tr: dict of RefTransverse fields, or None."""
        if tr is None:
            self._check(lib().mbt_ref_set_transverse(self._h, None))
            self.tr = None
            return
        t = RefTransverse(**{k: float(v) for k, v in tr.items()})
        self._check(lib().mbt_ref_set_transverse(self._h, C.byref(t)))
        self.tr = dict(tr)

    def set_transverse_wake(self, resonators):
        arr = (RefResonator * max(1, len(resonators)))(*[RefResonator(*r) for r in resonators])
        self._check(lib().mbt_ref_set_transverse_wake(self._h, len(resonators), arr))

    def set_transverse_rw(self, rw):
        """rw = (radius m, conductivity S/m, length m, turns), or None."""
        if rw is None:
            self._check(lib().mbt_ref_set_transverse_rw(self._h, None))
            self.rw_turns = 0
            return
        r = RefLRRW(float(rw[0]), float(rw[1]), float(rw[2]), int(rw[3]))
        self._check(lib().mbt_ref_set_transverse_rw(self._h, C.byref(r)))
        self.rw_turns = int(rw[3])

    def init_transverse(self, emittance, offset=0.0):
        self._check(lib().mbt_ref_init_transverse(self._h, float(emittance), float(offset)))

    def set_transverse_particles(self, bunch, x, xp):
        a = np.ascontiguousarray(x, dtype=np.float64)
        b = np.ascontiguousarray(xp, dtype=np.float64)
        assert a.size == self.N and b.size == self.N
        self._check(lib().mbt_ref_set_transverse_particles(self._h, bunch, _dp(a), _dp(b)))

    def get_transverse_particles(self, bunch):
        x = np.zeros(self.N)
        xp = np.zeros(self.N)
        self._check(lib().mbt_ref_get_transverse_particles(self._h, bunch, _dp(x), _dp(xp)))
        return x, xp

    def track2(self, nturns, profiles_stride=0):
        """Track; returns (moments [T][M][4], transverse moments [T][M][4]) and
        the profiles when profiles_stride is given."""
        mom = np.zeros((nturns, self.M, 4))
        tmom = np.zeros((nturns, self.M, 4))
        counts = None
        if profiles_stride:
            rows = -(-nturns // profiles_stride)
            counts = np.zeros((rows, self.M, self.nbins), dtype=np.uint32)
        self._check(lib().mbt_ref_track2(self._h, nturns, _dp(mom), _dp(tmom),
                                         None if counts is None else _up(counts),
                                         int(profiles_stride)))
        return (mom, tmom, counts) if profiles_stride else (mom, tmom)

    def get_rw_history(self):
        H = np.zeros((self.rw_turns, self.M))
        self._check(lib().mbt_ref_get_rw_history(self._h, _dp(H)))
        return H

    def set_rw_history(self, H):
        h = np.ascontiguousarray(H, dtype=np.float64)
        assert h.size == self.rw_turns * self.M
        self._check(lib().mbt_ref_set_rw_history(self._h, _dp(h)))

    def derived(self):
        out = np.zeros(5)
        self._check(lib().mbt_ref_derived(self._h, _dp(out)))
        return dict(zip(["phi_s", "T0", "D", "noise", "drift"], out.tolist()))


def lib_path():
    return os.path.abspath(_build.LIB)
