"""The C-ABI library loads here (no GPU), exports every symbol include/mbt.h
declares, and rejects bad arguments and bad call order on the host before
any device work."""
import ctypes as C
import os
import re

import pytest

from paper_1809_00391_amd import _abi
from paper_1809_00391_amd import tracker as tr
from paper_1809_00391_amd import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(os.path.dirname(HERE), "include", "mbt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(mbt_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["mbt_create", "mbt_destroy", "mbt_set_fill", "mbt_set_short_range",
                 "mbt_set_long_range", "mbt_set_harmonic_cavity", "mbt_hc_flat_fraction",
                 "mbt_query_bytes", "mbt_bind", "mbt_init_gaussian", "mbt_set_particles",
                 "mbt_get_particles", "mbt_track", "mbt_get_state", "mbt_set_state",
                 "mbt_strerror", "mbt_last_error", "mbt_profile", "mbt_wake_potential",
                 "mbt_wake_table", "mbt_philox4x32_10"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    L = _abi.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
        assert n in _abi.SIGNATURES, f"{n} has no Python prototype"


def _ctx(ring=wl.RING_R480):
    L = _abi.lib()
    h = C.c_void_p()
    rc = L.mbt_create(C.byref(tr._ring(ring)), C.byref(h))
    return L, h, rc


def test_create_validation():
    bad = [dict(wl.RING_R480, energy_eV=-1.0), dict(wl.RING_R480, v_rf_V=0.4e6),
           dict(wl.RING_R480, alpha_c=0.0), dict(wl.RING_R480, harmonic=0),
           dict(wl.RING_R480, tau_long_s=0.0), dict(wl.RING_R480, sigma_delta=-1.0),
           dict(wl.RING_R480, f_rf_Hz=float("nan"))]
    for r in bad:
        L, h, rc = _ctx(r)
        assert rc == _abi.MBT_EINVAL and not h.value
    L, h, rc = _ctx()
    assert rc == 0 and h.value
    L.mbt_destroy(h)
    assert L.mbt_create(None, C.byref(C.c_void_p())) == _abi.MBT_EINVAL
    L.mbt_destroy(None)  # allowed


def test_call_order_and_argument_errors():
    L, h, rc = _ctx()
    sb, wb = C.c_size_t(), C.c_size_t()
    assert L.mbt_query_bytes(h, 100, C.byref(sb), C.byref(wb)) == _abi.MBT_ESTATE
    assert L.mbt_track(h, 10, None, None, 0) == _abi.MBT_ESTATE
    assert L.mbt_init_gaussian(h, 1e-11, 1e-3, 1) == _abi.MBT_ESTATE
    b = (C.c_int32 * 2)(0, 0)
    cur = (C.c_double * 2)(1e-3, 1e-3)
    assert L.mbt_set_fill(h, 2, b, cur, None) == _abi.MBT_EINVAL  # not increasing
    b2 = (C.c_int32 * 2)(0, 480)
    assert L.mbt_set_fill(h, 2, b2, cur, None) == _abi.MBT_EINVAL  # out of [0, h)
    b3 = (C.c_int32 * 2)(0, 5)
    neg = (C.c_double * 2)(1e-3, -1e-3)
    assert L.mbt_set_fill(h, 2, b3, neg, None) == _abi.MBT_EINVAL
    assert L.mbt_set_fill(h, 2, b3, cur, None) == 0
    g = _abi.Grid(0, -1e-11, 1e-11)
    res = (_abi.Resonator * 1)(_abi.Resonator(1e4, 1.0, 2e10))
    assert L.mbt_set_short_range(h, 1, res, C.byref(g)) == _abi.MBT_EINVAL
    g = _abi.Grid(64, 1e-11, -1e-11)
    assert L.mbt_set_short_range(h, 1, res, C.byref(g)) == _abi.MBT_EINVAL
    bad_q = (_abi.Resonator * 1)(_abi.Resonator(1e4, 0.5, 2e10))
    g = _abi.Grid(64, -1e-11, 1e-11)
    assert L.mbt_set_short_range(h, 1, bad_q, C.byref(g)) == _abi.MBT_EINVAL
    assert L.mbt_set_short_range(h, 1, res, C.byref(g)) == 0
    lr5 = (_abi.Resonator * 5)(*[_abi.Resonator(1e6, 2e4, 1.52e9)] * 5)
    assert L.mbt_set_long_range(h, 5, lr5) == _abi.MBT_EINVAL  # > MBT_MAX_LONG_RANGE
    assert L.mbt_set_long_range(h, 1, lr5) == 0
    assert L.mbt_query_bytes(h, 0, C.byref(sb), C.byref(wb)) == _abi.MBT_EINVAL
    assert L.mbt_query_bytes(h, 1000, C.byref(sb), C.byref(wb)) == 0
    assert sb.value >= 2 * 2 * 1000 * 8 and wb.value > 0
    # bind: null / misaligned pointers and undersized buffers fail before any device work
    assert L.mbt_bind(h, 1000, None, sb.value, None, wb.value, None) == _abi.MBT_EINVAL
    fake = C.c_void_p(1 << 20)
    assert L.mbt_bind(h, 1000, C.c_void_p((1 << 20) + 8), sb.value, fake, wb.value,
                      None) == _abi.MBT_EINVAL
    assert L.mbt_bind(h, 1000, fake, sb.value - 8, fake, wb.value, None) == _abi.MBT_ENOSPC
    assert b"need" in L.mbt_last_error(h)
    assert L.mbt_philox4x32_10(-1, None, 0, 0, None, None) == _abi.MBT_EINVAL
    L.mbt_destroy(h)


def test_static_bind_rejects_before_device_work():
    """mbt_bind_static checks its arguments and the job's workspace against
    MBT_STATIC_WORK_BYTES before touching the device."""
    L, h, rc = _ctx()
    fake = C.c_void_p(1 << 20)
    assert L.mbt_bind_static(h, 1000, fake, 1 << 30, None) == _abi.MBT_ESTATE  # no fill
    b = (C.c_int32 * 2)(0, 5)
    cur = (C.c_double * 2)(1e-3, 1e-3)
    assert L.mbt_set_fill(h, 2, b, cur, None) == 0
    sb, wb = C.c_size_t(), C.c_size_t()
    assert L.mbt_query_bytes(h, 1000, C.byref(sb), C.byref(wb)) == 0
    assert wb.value <= _abi.MBT_STATIC_WORK_BYTES
    assert L.mbt_bind_static(h, 1000, None, sb.value, None) == _abi.MBT_EINVAL
    assert L.mbt_bind_static(h, 1000, C.c_void_p((1 << 20) + 8), sb.value, None) == _abi.MBT_EINVAL
    assert L.mbt_bind_static(h, 1000, fake, sb.value - 8, None) == _abi.MBT_ENOSPC
    L.mbt_destroy(h)
    # a job whose tables, histograms and output rings exceed the static array
    big = 4000
    L, h, rc = _ctx(dict(wl.RING_R480, harmonic=big))
    bk = (C.c_int32 * big)(*range(big))
    cu = (C.c_double * big)(*([1e-3] * big))
    assert L.mbt_set_fill(h, big, bk, cu, None) == 0
    g = _abi.Grid(4096, -1e-10, 1e-10)
    res = (_abi.Resonator * 1)(_abi.Resonator(1e4, 1.0, 2e10))
    assert L.mbt_set_short_range(h, 1, res, C.byref(g)) == 0
    assert L.mbt_query_bytes(h, 1000, C.byref(sb), C.byref(wb)) == 0
    assert wb.value > _abi.MBT_STATIC_WORK_BYTES
    assert L.mbt_bind_static(h, 1000, fake, sb.value, None) == _abi.MBT_ENOSPC
    assert b"static workspace" in L.mbt_last_error(h)
    L.mbt_destroy(h)


def test_transverse_setters_validate_on_the_host():
    """The transverse plane's setters reject bad values and wrong call order,
    the plane doubles the state, and it excludes the matrix-core wakes."""
    L, h, rc = _ctx()
    T = _abi.Transverse
    good = T(18.2, 2.5, -0.7, 7.5, 0.12, -0.03, 1e-9, 8e-3)
    for bad in (T(18.2, 2.5, -0.7, 0.0, 0.12, -0.03, 1e-9, 8e-3),
                T(18.2, 2.5, -0.7, 7.5, 0.12, -0.03, -1e-9, 8e-3),
                T(18.2, 2.5, -0.7, 7.5, 0.12, -0.03, 1e-9, 0.0),
                T(float("nan"), 2.5, -0.7, 7.5, 0.12, -0.03, 1e-9, 8e-3)):
        assert L.mbt_set_transverse(h, C.byref(bad)) == _abi.MBT_EINVAL
    b = (C.c_int32 * 2)(0, 5)
    cur = (C.c_double * 2)(1e-3, 1e-3)
    assert L.mbt_set_fill(h, 2, b, cur, None) == 0
    sb0, wb0 = C.c_size_t(), C.c_size_t()
    assert L.mbt_query_bytes(h, 1000, C.byref(sb0), C.byref(wb0)) == 0
    assert L.mbt_set_transverse(h, C.byref(good)) == 0
    sb, wb = C.c_size_t(), C.c_size_t()
    assert L.mbt_query_bytes(h, 1000, C.byref(sb), C.byref(wb)) == 0
    assert sb.value == 2 * sb0.value and wb.value > wb0.value
    assert L.mbt_set_wake_precision(h, _abi.MBT_WAKE_BF16X2) == _abi.MBT_EINVAL
    assert L.mbt_set_wake_precision(h, _abi.MBT_WAKE_FP64) == 0
    bad_q = (_abi.Resonator * 1)(_abi.Resonator(1e6, 0.4, 1e10))
    assert L.mbt_set_transverse_wake(h, 1, bad_q) == _abi.MBT_EINVAL
    ok_r = (_abi.Resonator * 1)(_abi.Resonator(1e6, 1.0, 1e10))
    assert L.mbt_set_transverse_wake(h, 1, ok_r) == 0
    RW = _abi.TransverseRW
    for bad in (RW(0.01, 5.8e7, 288.0, 0), RW(0.01, 5.8e7, 288.0, 1025), RW(0.0, 5.8e7, 288.0, 4)):
        assert L.mbt_set_transverse_rw(h, C.byref(bad)) == _abi.MBT_EINVAL
    assert L.mbt_set_transverse_rw(h, C.byref(RW(0.01, 5.8e7, 288.0, 16))) == 0
    sb2, wb2 = C.c_size_t(), C.c_size_t()
    assert L.mbt_query_bytes(h, 1000, C.byref(sb2), C.byref(wb2)) == 0
    assert wb2.value >= wb.value + 16 * 2 * 8  # the wall's centroid history
    # calls that need a binding
    assert L.mbt_init_transverse(h, 1e-9, 0.0) == _abi.MBT_ESTATE
    assert L.mbt_get_rw_history(h, None) == _abi.MBT_ESTATE
    assert L.mbt_track2(h, 1, None, None, None, 0) == _abi.MBT_ESTATE
    assert L.mbt_set_transverse(h, None) == 0
    L.mbt_destroy(h)


def test_hc_flat_fraction_agrees_with_oracle():
    from oracle import ref
    for frac in (0.5, 0.9, 1.0):
        for ring in (wl.RING_R480, dict(wl.RING_R480, alpha_c=-6e-4)):
            a = tr.hc_flat_fraction(ring, 3, frac)
            b = ref.hc_flat_fraction(ring, 3, frac)
            assert a["v_ratio"] == pytest.approx(b["v_ratio"], rel=1e-15)
            assert a["phase_n_rad"] == pytest.approx(b["phase_n_rad"], rel=1e-15)
    with pytest.raises(tr.MbtError):
        tr.hc_flat_fraction(dict(wl.RING_R480, u0_eV=1.4e6), 3, 1.0)


def test_no_synchronous_phase_is_rejected():
    t = tr.Tracker(wl.RING_R480)
    with pytest.raises(tr.MbtError):
        t.set_harmonic_cavity({"n": 3, "v_ratio": 10.0, "phase_n_rad": -1.5})
    t.set_harmonic_cavity(tr.hc_flat_fraction(wl.RING_R480, 3, 0.9))


def test_stream_copy_argument_checks():
    """Rejected before anything is launched: sizes that are not a multiple of
    16, misaligned or overlapping ranges; a zero size is a no-op."""
    L = _abi.lib()
    assert L.mbt_stream_copy(None, None, 0, None) == 0
    assert L.mbt_stream_copy(0x1000, 0x9000, 24, None) == -1
    assert L.mbt_stream_copy(0x1000, 0x9000, -16, None) == -1
    assert L.mbt_stream_copy(0x1008, 0x9000, 16, None) == -1
    assert L.mbt_stream_copy(0x1000, 0x9004, 16, None) == -1
    assert L.mbt_stream_copy(0x1000, 0x1010, 32, None) == -1
    assert L.mbt_stream_copy(None, 0x9000, 16, None) == -1


def test_strerror():
    for code in (0, -1, -2, -3, -4, -5, -6, 7):
        assert isinstance(tr.strerror(code), str)


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "LIB_PATH", "/nonexistent/libmbt.so")
    with pytest.raises(_abi.MissingLibraryError):
        _abi.lib()


_ENOMEM_CHILD = r"""
import ctypes as C, resource, sys
sys.path.insert(0, sys.argv[1])
from paper_1809_00391_amd import _abi, tracker as tr
from paper_1809_00391_amd import workloads as wl
L = _abi.lib()
M = 65535
h = C.c_void_p()
assert L.mbt_create(C.byref(tr._ring(dict(wl.RING_R480, harmonic=M))), C.byref(h)) == 0
small = (C.c_int32 * 2)(0, 9)
cur = (C.c_double * M)(*([1e-3] * M))
assert L.mbt_set_fill(h, 2, small, cur, None) == 0
b = (C.c_int32 * M)(*range(M))
C.CDLL("libc.so.6").malloc_trim(0)
vm = [int(x.split()[1]) * 1024 for x in open("/proc/self/status") if x.startswith("VmSize:")][0]
soft, hard = resource.getrlimit(resource.RLIMIT_AS)
# no address space beyond what the process holds: the fill's three arrays
# (about 1 MB) cannot be allocated
resource.setrlimit(resource.RLIMIT_AS, (vm + 4096, hard))
rc = L.mbt_set_fill(h, M, b, cur, None)
resource.setrlimit(resource.RLIMIT_AS, (soft, hard))
msg = L.mbt_last_error(h).decode()
sb, wb = C.c_size_t(), C.c_size_t()
q = L.mbt_query_bytes(h, 1000, C.byref(sb), C.byref(wb))
rc2 = L.mbt_set_fill(h, M, b, cur, None)
L.mbt_destroy(h)
print(rc, q, sb.value, rc2, msg)
"""


def test_host_allocation_failure_returns_enomem():
    """A host allocation that fails inside an entry point comes back as
    MBT_ENOMEM with a message (no C++ exception leaves the library), and the
    context keeps its previous, consistent settings.  The failure is forced
    by capping the child process's address space at what it already holds."""
    import subprocess
    import sys
    root = os.path.dirname(HERE)
    out = subprocess.run([sys.executable, "-c", _ENOMEM_CHILD, root], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    rc, q, state_bytes, rc2, msg = out.stdout.split(maxsplit=4)
    assert int(rc) == _abi.MBT_ENOMEM
    assert "allocation" in msg
    # the two-bunch fill is still the one in force: 2 bunches x 2 rows x 1024 doubles
    assert int(q) == 0 and int(state_bytes) == 2 * 2 * 1024 * 8
    # once memory is there again the same call succeeds
    assert int(rc2) == 0
