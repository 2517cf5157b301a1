"""The allocation-free binding (mbt_bind_static): a job bound to the
library's static device workspace gives the same moments, profiles and
particles as the same job bound to caller memory with mbt_bind, on two
bindings in a row (the second with fewer particles and fewer bunches), and a
context whose static workspace was taken over by a later binding is refused.
Both forms run the same kernels, so the bar is bit-identity (stronger than
the oracle tolerances)."""
import numpy as np
import pytest

from paper_1809_00391_amd import tracker as tr
from paper_1809_00391_amd import workloads as wl

pytestmark = pytest.mark.gpu

CASE = wl.Workload(
    name="static workspace", ring=wl.RING_R480, buckets=(0, 3, 4, 9, 200),
    currents_A=(1e-3, 2.5e-3, 0.0, 1.5e-3, 4e-3), N=2 * 4096 + 77, turns=60, seed=7,
    sigma_tau0=20e-12, sigma_delta0=8.6e-4, short_range=(wl.BB,),
    grid=(200, -150e-12, 150e-12), long_range=(wl.HOM, (3e5, 5e3, 2.21e9)), hc_flat=(3, 0.9))


def configure(w):
    t = tr.Tracker(w.ring)
    t.set_harmonic_cavity(tr.hc_flat_fraction(w.ring, *w.hc_flat))
    t.set_fill(w.buckets, w.currents_A, w.streams)
    t.set_short_range(list(w.short_range), w.grid)
    t.set_long_range(list(w.long_range))
    return t


def run_pair(w, turns):
    print(f"[gpu case] static workspace M={w.M} N={w.N} turns={turns}", flush=True)
    a = configure(w)
    a.bind_static(w.N)
    b = configure(w)
    b.bind(w.N)
    for t in (a, b):
        t.init_gaussian(w.sigma_tau0, w.sigma_delta0, w.seed)
    ma, pa = a.track(turns, profiles_stride=7)
    mb, pb = b.track(turns, profiles_stride=7)
    assert np.array_equal(ma, mb)
    assert np.array_equal(pa, pb)
    # a second call continues from the device turn counter
    ma2 = a.track(turns // 2)
    mb2 = b.track(turns // 2)
    assert np.array_equal(ma2, mb2)
    assert np.array_equal(a.wake_potential(), b.wake_potential())
    assert a.get_state()[0] == b.get_state()[0] == turns + turns // 2
    assert np.array_equal(a.get_state()[2], b.get_state()[2])
    for k in range(w.M):
        ta, da = a.get_particles(k)
        tb, db = b.get_particles(k)
        assert np.array_equal(ta, tb) and np.array_equal(da, db)
    assert np.all(np.isfinite(ma))
    return a, b


def test_static_binding_matches_bound_workspace(cuda):
    a, b = run_pair(CASE, CASE.turns)
    a.close()
    b.close()
    # second binding in a row: fewer bunches and particles on the same array
    small = CASE.with_(buckets=(0, 7, 11), currents_A=(2e-3, 1e-3, 3e-3), N=3001, seed=9)
    a, b = run_pair(small, 40)
    a.close()
    b.close()


def test_static_workspace_taken_over(cuda):
    w = CASE.with_(N=1000, turns=10)
    print(f"[gpu case] static workspace takeover N={w.N}", flush=True)
    a = configure(w)
    a.bind_static(w.N)
    a.init_gaussian(w.sigma_tau0, w.sigma_delta0, w.seed)
    a.track(5)
    c = configure(w)
    c.bind_static(w.N)
    with pytest.raises(tr.MbtError) as e:
        a.track(5)
    assert e.value.code == -2  # MBT_ESTATE
    c.init_gaussian(w.sigma_tau0, w.sigma_delta0, w.seed)
    c.track(5)
    # rebinding gives the workspace back to a (and takes it from c)
    a.bind_static(w.N)
    a.init_gaussian(w.sigma_tau0, w.sigma_delta0, w.seed)
    m = a.track(5)
    assert np.all(np.isfinite(m))
    with pytest.raises(tr.MbtError):
        c.track(1)
    with pytest.raises(tr.MbtError):
        tr.Batch([a])
    a.close()
    c.close()
