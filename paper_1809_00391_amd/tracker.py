"""Python binding of the tracker's C ABI (include/mbt.h).

Argument marshalling only: every step of the turn runs in the HIP kernels of
libmbt.so.  PyTorch provides the device memory (uint8 tensors handed over as
raw pointers) and the stream.
"""
import ctypes as C

import numpy as np
import torch

from . import _abi
from ._abi import HC, Grid, Moments, Resonator, Ring

__all__ = ["Batch", "MbtError", "Tracker", "hc_flat_fraction", "philox4x32_10", "strerror"]


class MbtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mbt error {code} ({strerror(code)}): {msg}")
        self.code = code


def strerror(code):
    return _abi.lib().mbt_strerror(code).decode()


def _ring(r):
    return Ring(float(r["energy_eV"]), float(r["f_rf_Hz"]), float(r["v_rf_V"]),
                float(r["alpha_c"]), float(r["u0_eV"]), float(r["tau_long_s"]),
                float(r["sigma_delta"]), int(r["harmonic"]))


def _resonators(res):
    res = list(res)
    return (Resonator * max(1, len(res)))(*[Resonator(*map(float, r)) for r in res]), len(res)


def hc_flat_fraction(ring, n, frac):
    """mbt_hc_flat_fraction: harmonic cavity at frac of the flat-potential voltage."""
    out = HC()
    rc = _abi.lib().mbt_hc_flat_fraction(C.byref(_ring(ring)), int(n), float(frac), C.byref(out))
    if rc:
        raise MbtError(rc, "no flat-potential solution")
    return {"n": out.n, "v_ratio": out.v_ratio, "phase_n_rad": out.phase_n_rad}


def philox4x32_10(ctr, key0, key1, stream=None):
    """mbt_philox4x32_10 on a uint32 CUDA tensor ctr of shape [n, 4]."""
    assert ctr.is_cuda and ctr.dtype in (torch.int32, torch.uint32)
    ctr = ctr.contiguous()
    out = torch.empty_like(ctr)
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = _abi.lib().mbt_philox4x32_10(ctr.shape[0], C.c_void_p(ctr.data_ptr()), key0 & 0xFFFFFFFF,
                                      key1 & 0xFFFFFFFF, C.c_void_p(out.data_ptr()),
                                      C.c_void_p(s.cuda_stream))
    if rc:
        raise MbtError(rc, "philox")
    return out


def stream_copy(src, dst, stream=None):
    """mbt_stream_copy: copy the bytes of CUDA tensor src into dst (same byte
    size, contiguous, 16-byte aligned) with the library's streaming kernel."""
    assert src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = _abi.lib().mbt_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                    nbytes, C.c_void_p(s.cuda_stream))
    if rc:
        raise MbtError(rc, "stream copy")


class Tracker:
    """One tracking job: a context of the C ABI plus its device buffers."""

    def __init__(self, ring):
        self._L = _abi.lib()
        self._h = C.c_void_p()
        rc = self._L.mbt_create(C.byref(_ring(ring)), C.byref(self._h))
        if rc:
            raise MbtError(rc, "mbt_create: invalid ring parameters")
        self.M = 0
        self.N = 0
        self.nbins = 0
        self.n_lr = 0
        self.tr_on = False
        self.rw_turns = 0
        self.state = None
        self.work = None
        self.stream = None

    def close(self):
        """Destroy the context (mbt_destroy drains its stream first), then
        drop the device buffers it was bound to."""
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.mbt_destroy(self._h)
            self._h = C.c_void_p()
        self.state = None
        self.work = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc:
            raise MbtError(rc, self._L.mbt_last_error(self._h).decode())

    # ---- configuration ---------------------------------------------------
    def set_harmonic_cavity(self, hc):
        if hc is None:
            self._check(self._L.mbt_set_harmonic_cavity(self._h, None))
        else:
            h = HC(int(hc["n"]), float(hc["v_ratio"]), float(hc["phase_n_rad"]))
            self._check(self._L.mbt_set_harmonic_cavity(self._h, C.byref(h)))

    def set_fill(self, buckets, currents_A, streams=None):
        b = np.ascontiguousarray(buckets, dtype=np.int32)
        c = np.ascontiguousarray(currents_A, dtype=np.float64)
        s = None if streams is None else np.ascontiguousarray(streams, dtype=np.int32)
        self._check(self._L.mbt_set_fill(
            self._h, b.size, b.ctypes.data_as(C.POINTER(C.c_int32)),
            c.ctypes.data_as(C.POINTER(C.c_double)),
            None if s is None else s.ctypes.data_as(C.POINTER(C.c_int32))))
        self.M = int(b.size)

    def set_short_range(self, resonators, grid):
        if grid is None:
            self._check(self._L.mbt_set_short_range(self._h, 0, None, None))
            self.nbins = 0
            return
        arr, n = _resonators(resonators)
        g = Grid(int(grid[0]), float(grid[1]), float(grid[2]))
        self._check(self._L.mbt_set_short_range(self._h, n, arr, C.byref(g)))
        self.nbins = g.nbins

    def set_long_range(self, resonators):
        arr, n = _resonators(resonators)
        self._check(self._L.mbt_set_long_range(self._h, n, arr))
        self.n_lr = n

    def set_resistive_wall(self, rw):
        """Short-range resistive wall (radius m, conductivity S/m, length m), or None."""
        if rw is None:
            self._check(self._L.mbt_set_resistive_wall(self._h, None))
        else:
            r = _abi.ResistiveWall(*map(float, rw))
            self._check(self._L.mbt_set_resistive_wall(self._h, C.byref(r)))

    # ---- transverse plane ----------------------------------------------
    def set_transverse(self, plane):
        """One transverse plane (dict with tune, chromaticity, alpha, beta_m,
        disp_m, disp_prime, emittance_m, tau_damp_s), or None."""
        if plane is None:
            self._check(self._L.mbt_set_transverse(self._h, None))
            self.tr_on = False
            return
        t = _abi.Transverse(*[float(plane[k]) for k in (
            "tune", "chromaticity", "alpha", "beta_m", "disp_m", "disp_prime", "emittance_m",
            "tau_damp_s")])
        self._check(self._L.mbt_set_transverse(self._h, C.byref(t)))
        self.tr_on = True

    def set_transverse_wake(self, resonators):
        """Transverse short-range resonators (R_s in Ohm/m, Q, f_r)."""
        arr, n = _resonators(resonators)
        self._check(self._L.mbt_set_transverse_wake(self._h, n, arr))

    def set_transverse_rw(self, rw):
        """Long-range transverse resistive wall (radius m, conductivity S/m,
        length m, turns), or None."""
        self.rw_turns = 0 if rw is None else int(rw[3])
        if rw is None:
            self._check(self._L.mbt_set_transverse_rw(self._h, None))
            return
        r = _abi.TransverseRW(float(rw[0]), float(rw[1]), float(rw[2]), int(rw[3]))
        self._check(self._L.mbt_set_transverse_rw(self._h, C.byref(r)))

    def init_transverse(self, emittance, offset=0.0):
        self._check(self._L.mbt_init_transverse(self._h, float(emittance), float(offset)))

    def set_transverse_particles(self, bunch, x, xp):
        a = np.ascontiguousarray(x, dtype=np.float64)
        b = np.ascontiguousarray(xp, dtype=np.float64)
        assert a.size == self.N and b.size == self.N
        self._check(self._L.mbt_set_transverse_particles(
            self._h, int(bunch), C.c_void_p(a.ctypes.data), C.c_void_p(b.ctypes.data),
            _abi.MBT_HOST))

    def get_transverse_particles(self, bunch):
        x = np.empty(self.N)
        xp = np.empty(self.N)
        self._check(self._L.mbt_get_transverse_particles(
            self._h, int(bunch), C.c_void_p(x.ctypes.data), C.c_void_p(xp.ctypes.data),
            _abi.MBT_HOST))
        return x, xp

    def track2(self, nturns, profiles_stride=0):
        """Track nturns; returns (moments [T][M][4], transverse moments
        [T][M][4] = mean x, mean x', rms x, rms x') (and profiles)."""
        mom = np.zeros((nturns, self.M, 4))
        tmom = np.zeros((nturns, self.M, 4))
        counts = None
        if profiles_stride:
            rows = -(-nturns // profiles_stride)
            counts = np.zeros((rows, self.M, self.nbins), dtype=np.uint32)
        self._check(self._L.mbt_track2(
            self._h, int(nturns), C.c_void_p(mom.ctypes.data), C.c_void_p(tmom.ctypes.data),
            None if counts is None else C.c_void_p(counts.ctypes.data), int(profiles_stride)))
        return (mom, tmom, counts) if profiles_stride else (mom, tmom)

    def get_rw_history(self):
        H = np.zeros((self.rw_turns, self.M))
        self._check(self._L.mbt_get_rw_history(self._h, C.c_void_p(H.ctypes.data)))
        return H

    def set_rw_history(self, H):
        a = np.ascontiguousarray(H, dtype=np.float64)
        assert a.size == self.rw_turns * self.M
        self._check(self._L.mbt_set_rw_history(self._h, C.c_void_p(a.ctypes.data)))

    def query_bytes(self, N):
        sb, wb = C.c_size_t(), C.c_size_t()
        self._check(self._L.mbt_query_bytes(self._h, int(N), C.byref(sb), C.byref(wb)))
        return sb.value, wb.value

    def bind(self, N, device="cuda", stream=None):
        """Allocate state and workspace as torch tensors and bind them."""
        sb, wb = self.query_bytes(N)
        self.state = torch.empty(sb + 256, dtype=torch.uint8, device=device)
        self.work = torch.empty(wb + 256, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.state.device)
        sp = (self.state.data_ptr() + 255) & ~255
        wp = (self.work.data_ptr() + 255) & ~255
        self._check(self._L.mbt_bind(self._h, int(N), C.c_void_p(sp), sb, C.c_void_p(wp), wb,
                                     C.c_void_p(self.stream.cuda_stream)))
        self.N = int(N)

    def bind_static(self, N, device="cuda", stream=None):
        """mbt_bind_static: allocate only the particle state (a torch tensor)
        and bind it with the library's static workspace on the device."""
        sb, _ = self.query_bytes(N)
        self.state = torch.empty(sb + 256, dtype=torch.uint8, device=device)
        self.work = None
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.state.device)
        sp = (self.state.data_ptr() + 255) & ~255
        self._check(self._L.mbt_bind_static(self._h, int(N), C.c_void_p(sp), sb,
                                            C.c_void_p(self.stream.cuda_stream)))
        self.N = int(N)

    # ---- particles and state -------------------------------------------
    def init_gaussian(self, sigma_tau_s, sigma_delta, seed):
        self._check(self._L.mbt_init_gaussian(self._h, float(sigma_tau_s), float(sigma_delta),
                                              int(seed)))

    def set_particles(self, bunch, tau, delta):
        if isinstance(tau, torch.Tensor) and tau.is_cuda:
            t = tau.to(torch.float64).contiguous()
            d = delta.to(torch.float64).contiguous()
            assert t.numel() == self.N and d.numel() == self.N
            self._check(self._L.mbt_set_particles(self._h, int(bunch), C.c_void_p(t.data_ptr()),
                                                  C.c_void_p(d.data_ptr()), _abi.MBT_DEVICE))
            self.stream.synchronize()
            return
        t = np.ascontiguousarray(tau, dtype=np.float64)
        d = np.ascontiguousarray(delta, dtype=np.float64)
        assert t.size == self.N and d.size == self.N
        self._check(self._L.mbt_set_particles(self._h, int(bunch), C.c_void_p(t.ctypes.data),
                                              C.c_void_p(d.ctypes.data), _abi.MBT_HOST))

    def get_particles(self, bunch):
        t = np.empty(self.N)
        d = np.empty(self.N)
        self._check(self._L.mbt_get_particles(self._h, int(bunch), C.c_void_p(t.ctypes.data),
                                              C.c_void_p(d.ctypes.data), _abi.MBT_HOST))
        return t, d

    def get_state(self):
        turn, seed = C.c_int64(), C.c_uint64()
        ph = np.zeros(2 * max(1, self.n_lr))
        self._check(self._L.mbt_get_state(self._h, C.byref(turn), C.byref(seed),
                                          C.c_void_p(ph.ctypes.data)))
        return turn.value, seed.value, ph[:2 * self.n_lr].copy()

    def set_state(self, turn, seed, phasors=None):
        ph = None if phasors is None or len(phasors) == 0 else np.ascontiguousarray(phasors, np.float64)
        self._check(self._L.mbt_set_state(self._h, int(turn), int(seed),
                                          None if ph is None else C.c_void_p(ph.ctypes.data)))

    # ---- tracking and observables ---------------------------------------
    def track(self, nturns, profiles_stride=0, moments=True):
        """Track nturns; returns moments [nturns][M][4] (and profiles)."""
        mom = np.zeros((nturns, self.M, 4)) if moments else None
        counts = None
        if profiles_stride:
            rows = -(-nturns // profiles_stride)
            counts = np.zeros((rows, self.M, self.nbins), dtype=np.uint32)
        self._check(self._L.mbt_track(
            self._h, int(nturns), None if mom is None else C.c_void_p(mom.ctypes.data),
            None if counts is None else C.c_void_p(counts.ctypes.data), int(profiles_stride)))
        return (mom, counts) if profiles_stride else mom

    def profile(self):
        counts = np.zeros((self.M, self.nbins), dtype=np.uint32)
        self._check(self._L.mbt_profile(self._h, C.c_void_p(counts.ctypes.data)))
        return counts

    def wake_potential(self):
        V = np.zeros((self.M, self.nbins))
        self._check(self._L.mbt_wake_potential(self._h, C.c_void_p(V.ctypes.data)))
        return V

    WAKE_MODES = {"fp64": _abi.MBT_WAKE_FP64, "fp32": _abi.MBT_WAKE_FP32,
                  "bf16x2": _abi.MBT_WAKE_BF16X2, "bf16x3": _abi.MBT_WAKE_BF16X3}

    def set_wake_precision(self, mode):
        """Arithmetic of the short-range wake potential: "fp64" (default),
        "fp32", "bf16x2" or "bf16x3" (matrix cores)."""
        self._check(self._L.mbt_set_wake_precision(self._h, self.WAKE_MODES[mode]))

    def set_launch(self, nsub=0, push_grid=0):
        """Push launch shape (sub-histograms, persistent workgroups; 0: defaults)."""
        self._check(self._L.mbt_set_launch(self._h, int(nsub), int(push_grid)))

    def set_timing(self, every):
        self._check(self._L.mbt_set_timing(self._h, int(every)))

    def get_timing(self):
        """(push ms total, push launches timed, prep ms total, prep launches)."""
        a, b, c, d = C.c_double(), C.c_int64(), C.c_double(), C.c_int64()
        self._check(self._L.mbt_get_timing(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return a.value, b.value, c.value, d.value

    def wake_table(self):
        W = np.zeros(self.nbins)
        self._check(self._L.mbt_wake_table(self._h, C.c_void_p(W.ctypes.data)))
        return W


class Batch:
    """Several bound Trackers advanced together (mbt_batch_*): one launch of
    each kernel per turn covers every bunch of every job."""

    def __init__(self, trackers, stream=None, graph_turns=0, autotune=False):
        self._L = _abi.lib()
        self.trackers = list(trackers)
        n = len(self.trackers)
        self._jobs = (C.c_void_p * n)(*[t._h.value for t in self.trackers])
        wb = C.c_size_t()
        rc = self._L.mbt_batch_query_bytes(self._jobs, n, C.byref(wb))
        if rc:
            raise MbtError(rc, "mbt_batch_query_bytes")
        dev = self.trackers[0].state.device
        self.work = torch.empty(wb.value + 256, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        wp = (self.work.data_ptr() + 255) & ~255
        self._h = C.c_void_p()
        rc = self._L.mbt_batch_create(self._jobs, n, C.c_void_p(wp), wb.value,
                                      C.c_void_p(self.stream.cuda_stream), C.byref(self._h))
        if rc:
            raise MbtError(rc, "mbt_batch_create")
        self.configure(graph_turns, autotune)

    def close(self):
        """Destroy the batch (mbt_batch_destroy drains its stream first), then
        drop its table memory."""
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.mbt_batch_destroy(self._h)
            self._h = C.c_void_p()
        self.work = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc:
            raise MbtError(rc, self._L.mbt_batch_last_error(self._h).decode())

    def configure(self, graph_turns=0, autotune=False):
        self._check(self._L.mbt_batch_configure(self._h, int(graph_turns), int(bool(autotune))))

    def set_timing(self, every):
        """Bracket every `every`-th turn's launches with HIP events (eager
        launches while on; 0: off and totals cleared)."""
        self._check(self._L.mbt_batch_set_timing(self._h, int(every)))

    def get_timing(self):
        """(push ms total, push launches timed, between-turn ms total, its launches)."""
        a, b, c, d = C.c_double(), C.c_int64(), C.c_double(), C.c_int64()
        self._check(self._L.mbt_batch_get_timing(self._h, C.byref(a), C.byref(b), C.byref(c),
                                                 C.byref(d)))
        return a.value, b.value, c.value, d.value

    def launch_info(self):
        """[(long-range count, sub-histograms, workgroups)] per push group."""
        ng = C.c_int32()
        k = _abi.MBT_MAX_LONG_RANGE + 1
        a, b, c = (C.c_int32 * k)(), (C.c_int32 * k)(), (C.c_int32 * k)()
        self._check(self._L.mbt_batch_launch_info(self._h, C.byref(ng), a, b, c))
        return [(a[i], b[i], c[i]) for i in range(ng.value)]

    def track(self, nturns, profiles_stride=None, moments=True):
        """Track every job nturns; returns a list of moment arrays [nturns][M_j][4]
        (and a list of profile arrays when profiles_stride, a per-job list or
        one int, is given; a stride of 0 leaves that job's profiles off)."""
        n = len(self.trackers)
        moms = [np.zeros((nturns, t.M, 4)) for t in self.trackers] if moments else None
        strides = None
        if profiles_stride is not None:
            strides = (list(profiles_stride) if hasattr(profiles_stride, "__len__")
                       else [profiles_stride] * n)
        profs = None
        if strides is not None:
            profs = [np.zeros((-(-nturns // s), t.M, t.nbins), dtype=np.uint32) if s else None
                     for s, t in zip(strides, self.trackers)]
        out_p = (C.c_void_p * n)(*[m.ctypes.data for m in moms]) if moms else None
        cnt_p = (C.c_void_p * n)(*[(p.ctypes.data if p is not None else None) for p in profs]) \
            if profs else None
        st_p = (C.c_int32 * n)(*[int(s) for s in strides]) if strides else None
        self._check(self._L.mbt_batch_track(self._h, int(nturns), out_p, cnt_p, st_p))
        return (moms, profs) if strides is not None else moms
