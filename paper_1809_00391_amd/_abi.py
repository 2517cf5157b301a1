"""ctypes declarations of the C ABI in include/mbt.h (argument marshalling only).

Loads the in-tree libmbt.so.  There is no fallback: if the library is missing
the import of the tracker fails with an error that says how to build it.
"""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# MBT_LIBRARY may point at another build of the same library (A/B runs).
LIB_PATH = os.environ.get("MBT_LIBRARY") or os.path.join(_HERE, "libmbt.so")

MBT_OK = 0
MBT_EINVAL = -1
MBT_ESTATE = -2
MBT_ENOSPC = -3
MBT_EDEVICE = -4
MBT_ENUMERIC = -5
MBT_ENOMEM = -6
MBT_HOST = 0
MBT_DEVICE = 1
MBT_MAX_BINS = 4096
MBT_MAX_SHORT_RANGE = 16
MBT_MAX_LONG_RANGE = 4
MBT_WAKE_FP64 = 0
MBT_WAKE_FP32 = 1
MBT_WAKE_BF16X2 = 2
MBT_WAKE_BF16X3 = 3
MBT_STATIC_WORK_BYTES = 64 << 20


class Ring(C.Structure):
    _fields_ = [("energy_eV", C.c_double), ("f_rf_Hz", C.c_double), ("v_rf_V", C.c_double),
                ("alpha_c", C.c_double), ("u0_eV", C.c_double), ("tau_long_s", C.c_double),
                ("sigma_delta", C.c_double), ("harmonic", C.c_int32)]


class HC(C.Structure):
    _fields_ = [("n", C.c_int32), ("v_ratio", C.c_double), ("phase_n_rad", C.c_double)]


class Resonator(C.Structure):
    _fields_ = [("rs_ohm", C.c_double), ("q", C.c_double), ("fr_Hz", C.c_double)]


class Grid(C.Structure):
    _fields_ = [("nbins", C.c_int32), ("tau_min_s", C.c_double), ("tau_max_s", C.c_double)]


class ResistiveWall(C.Structure):
    _fields_ = [("radius_m", C.c_double), ("conductivity_S_m", C.c_double),
                ("length_m", C.c_double)]


class Transverse(C.Structure):
    _fields_ = [("tune", C.c_double), ("chromaticity", C.c_double), ("alpha", C.c_double),
                ("beta_m", C.c_double), ("disp_m", C.c_double), ("disp_prime", C.c_double),
                ("emittance_m", C.c_double), ("tau_damp_s", C.c_double)]


class TransverseRW(C.Structure):
    _fields_ = [("radius_m", C.c_double), ("conductivity_S_m", C.c_double),
                ("length_m", C.c_double), ("turns", C.c_int32)]


class TMoments(C.Structure):
    _fields_ = [("mean_x", C.c_double), ("mean_xp", C.c_double), ("rms_x", C.c_double),
                ("rms_xp", C.c_double)]


class Moments(C.Structure):
    _fields_ = [("mean_tau", C.c_double), ("mean_delta", C.c_double),
                ("rms_tau", C.c_double), ("rms_delta", C.c_double)]


_P = C.POINTER
_ctx = C.c_void_p
SIGNATURES = {
    "mbt_strerror": (C.c_char_p, [C.c_int]),
    "mbt_last_error": (C.c_char_p, [_ctx]),
    "mbt_create": (C.c_int, [_P(Ring), _P(_ctx)]),
    "mbt_destroy": (None, [_ctx]),
    "mbt_hc_flat_fraction": (C.c_int, [_P(Ring), C.c_int32, C.c_double, _P(HC)]),
    "mbt_set_harmonic_cavity": (C.c_int, [_ctx, _P(HC)]),
    "mbt_set_fill": (C.c_int, [_ctx, C.c_int32, _P(C.c_int32), _P(C.c_double), _P(C.c_int32)]),
    "mbt_set_short_range": (C.c_int, [_ctx, C.c_int32, _P(Resonator), _P(Grid)]),
    "mbt_set_long_range": (C.c_int, [_ctx, C.c_int32, _P(Resonator)]),
    "mbt_set_resistive_wall": (C.c_int, [_ctx, _P(ResistiveWall)]),
    "mbt_set_transverse": (C.c_int, [_ctx, _P(Transverse)]),
    "mbt_set_transverse_wake": (C.c_int, [_ctx, C.c_int32, _P(Resonator)]),
    "mbt_set_transverse_rw": (C.c_int, [_ctx, _P(TransverseRW)]),
    "mbt_init_transverse": (C.c_int, [_ctx, C.c_double, C.c_double]),
    "mbt_set_transverse_particles": (C.c_int, [_ctx, C.c_int32, C.c_void_p, C.c_void_p,
                                               C.c_int32]),
    "mbt_get_transverse_particles": (C.c_int, [_ctx, C.c_int32, C.c_void_p, C.c_void_p,
                                               C.c_int32]),
    "mbt_track2": (C.c_int, [_ctx, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "mbt_get_rw_history": (C.c_int, [_ctx, C.c_void_p]),
    "mbt_set_rw_history": (C.c_int, [_ctx, C.c_void_p]),
    "mbt_query_bytes": (C.c_int, [_ctx, C.c_int64, _P(C.c_size_t), _P(C.c_size_t)]),
    "mbt_bind": (C.c_int, [_ctx, C.c_int64, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t,
                           C.c_void_p]),
    "mbt_bind_static": (C.c_int, [_ctx, C.c_int64, C.c_void_p, C.c_size_t, C.c_void_p]),
    "mbt_init_gaussian": (C.c_int, [_ctx, C.c_double, C.c_double, C.c_uint64]),
    "mbt_set_particles": (C.c_int, [_ctx, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]),
    "mbt_get_particles": (C.c_int, [_ctx, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]),
    "mbt_track": (C.c_int, [_ctx, C.c_int64, C.c_void_p, C.c_void_p, C.c_int32]),
    "mbt_profile": (C.c_int, [_ctx, C.c_void_p]),
    "mbt_wake_potential": (C.c_int, [_ctx, C.c_void_p]),
    "mbt_wake_table": (C.c_int, [_ctx, C.c_void_p]),
    "mbt_get_state": (C.c_int, [_ctx, _P(C.c_int64), _P(C.c_uint64), C.c_void_p]),
    "mbt_set_state": (C.c_int, [_ctx, C.c_int64, C.c_uint64, C.c_void_p]),
    "mbt_set_timing": (C.c_int, [_ctx, C.c_int32]),
    "mbt_get_timing": (C.c_int, [_ctx, _P(C.c_double), _P(C.c_int64), _P(C.c_double),
                                 _P(C.c_int64)]),
    "mbt_set_launch": (C.c_int, [_ctx, C.c_int32, C.c_int32]),
    "mbt_set_wake_precision": (C.c_int, [_ctx, C.c_int32]),
    "mbt_batch_query_bytes": (C.c_int, [C.c_void_p, C.c_int32, _P(C.c_size_t)]),
    "mbt_batch_create": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                   _P(C.c_void_p)]),
    "mbt_batch_destroy": (None, [C.c_void_p]),
    "mbt_batch_last_error": (C.c_char_p, [C.c_void_p]),
    "mbt_batch_configure": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "mbt_batch_launch_info": (C.c_int, [C.c_void_p, _P(C.c_int32), C.c_void_p, C.c_void_p,
                                        C.c_void_p]),
    "mbt_batch_track": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mbt_batch_set_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "mbt_batch_get_timing": (C.c_int, [C.c_void_p, _P(C.c_double), _P(C.c_int64),
                                       _P(C.c_double), _P(C.c_int64)]),
    "mbt_philox4x32_10": (C.c_int, [C.c_int64, C.c_void_p, C.c_uint32, C.c_uint32, C.c_void_p,
                                    C.c_void_p]),
    "mbt_stream_copy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
}

_lib = None


class MissingLibraryError(ImportError):
    pass


def lib():
    """The loaded libmbt.so with prototypes set; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MissingLibraryError(
                f"{LIB_PATH} is not built; run `python paper_1809_00391_amd/build.py` "
                "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib
