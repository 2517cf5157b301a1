"""Batched tracking through the C ABI (mbt_batch_*): every job of a batch gives
bit for bit what it gives tracked alone, with graph replay and with the online
launch-shape tuner, and the launch shape of the push never changes a bit."""
import numpy as np
import pytest

from paper_1809_00391_amd import tracker as tr
from paper_1809_00391_amd import workloads as wl

from helpers import make_oracle, make_tracker, moment_excess

pytestmark = pytest.mark.gpu

# Jobs that differ in everything a batch has to keep apart: bunch count,
# particle count (ragged tiles), grid (none, 64 and 200 bins), long-range
# resonators (0, 1, 2: three push groups), harmonic cavity, seeds and fills.
JOBS = [
    wl.Workload(name="mb", ring=wl.RING_R480, buckets=(0, 3, 4, 9, 200),
                currents_A=(1e-3, 2.5e-3, 0.0, 1.5e-3, 4e-3), N=2 * 4096 + 77, turns=0, seed=7,
                sigma_tau0=20e-12, sigma_delta0=8.6e-4, short_range=(wl.BB,),
                grid=(200, -150e-12, 150e-12), long_range=(wl.HOM, (3e5, 5e3, 2.21e9)),
                hc_flat=(3, 0.9)),
    wl.C1.with_(N=5000, seed=11),
    wl.Workload(name="lr only", ring=wl.RING_R480, buckets=tuple(range(0, 480, 7)),
                currents_A=(1.2e-3,) * len(range(0, 480, 7)), N=300, turns=0, seed=12,
                sigma_tau0=12e-12, sigma_delta0=8.6e-4, long_range=(wl.HOM,)),
    wl.Workload(name="bb + hom", ring=wl.RING_R484, buckets=tuple(range(40)),
                currents_A=tuple(1e-3 * (1 + 0.3 * np.cos(b)) for b in range(40)), N=4096 + 1,
                turns=0, seed=13, sigma_tau0=10e-12, sigma_delta0=8.6e-4, short_range=(wl.BB,),
                grid=(64, -76e-12, 76e-12), long_range=(wl.HOM,)),
]
STRIDES = [5, 3, 0, 7]


def print_case(name, **kw):
    print(f"[gpu case] {name} {kw}", flush=True)


def _alone(w, turns, stride):
    g = make_tracker(w)
    if stride:
        m, p = g.track(turns, profiles_stride=stride)
    else:
        m, p = g.track(turns), None
    return m, p, [g.get_particles(b) for b in (0, w.M - 1)], g.get_state()


def _assert_same(res_a, res_b):
    (ma, pa, xa, sa), (mb, pb, xb, sb) = res_a, res_b
    assert np.array_equal(ma, mb)
    if pa is not None or pb is not None:
        assert np.array_equal(pa, pb)
    for (ta, da), (tb, db) in zip(xa, xb):
        assert np.array_equal(ta, tb) and np.array_equal(da, db)
    assert sa[0] == sb[0] and sa[1] == sb[1]
    assert np.array_equal(sa[2], sb[2])


@pytest.mark.parametrize("graph_turns,autotune", [(0, False), (8, False), (4, True)])
def test_batch_matches_jobs_alone(cuda, graph_turns, autotune):
    turns = 61  # with 8-turn graphs: 7 replays and an eager remainder
    print_case("batch vs alone", graph_turns=graph_turns, autotune=autotune, turns=turns)
    alone = [_alone(w, turns, s) for w, s in zip(JOBS, STRIDES)]
    gs = [make_tracker(w) for w in JOBS]
    b = tr.Batch(gs, graph_turns=graph_turns, autotune=autotune)
    # two calls: the second resumes from the device-side turn counters
    m1, p1 = b.track(40, profiles_stride=STRIDES)
    m2, p2 = b.track(turns - 40, profiles_stride=STRIDES)
    for j, (w, s) in enumerate(zip(JOBS, STRIDES)):
        mom = np.concatenate([m1[j], m2[j]])
        prof = None
        if s:
            # the second call's rows count from its own first turn
            rows1 = [r for r in range(0, 40, s)]
            rows2 = [40 + r for r in range(0, turns - 40, s)]
            want = {t: alone[j][1][t // s] for t in range(0, turns, s)}
            got = {t: p1[j][i] for i, t in enumerate(rows1)}
            got.update({t: p2[j][i] for i, t in enumerate(rows2)})
            for t in got:
                if t in want:
                    assert np.array_equal(got[t], want[t]), (j, t)
        res = (mom, prof, [gs[j].get_particles(bb) for bb in (0, w.M - 1)], gs[j].get_state())
        _assert_same(res, (alone[j][0], None, alone[j][2], alone[j][3]))
    if autotune:
        info = b.launch_info()
        assert [g[0] for g in info] == [0, 1, 2]
        print_case("tuned", info=info)
    b.close()


def test_graph_replays_match_eager(cuda):
    """Many replays of one captured graph, with host work and synchronisation
    between the calls, against the same turns launched one by one."""
    print_case("graph replays")
    eager = [make_tracker(w) for w in JOBS[:2]]
    graph = [make_tracker(w) for w in JOBS[:2]]
    be = tr.Batch(eager)
    bg = tr.Batch(graph, graph_turns=16)
    for call in range(4):
        me = be.track(32)
        mg = bg.track(32)
        for j in range(2):
            assert np.array_equal(me[j], mg[j]), (call, j)
        # host-side work between replays: read back particles, compare
        for te, tg in zip(eager, graph):
            xe, xg = te.get_particles(0), tg.get_particles(0)
            assert np.array_equal(xe[0], xg[0]) and np.array_equal(xe[1], xg[1])


def test_launch_shape_changes_no_bit(cuda):
    w = JOBS[0]
    print_case("launch shapes", N=w.N)
    ref = None
    for nsub, grid in [(0, 0), (1, 0), (2, 3), (8, 1), (4, 7)]:
        g = make_tracker(w)
        g.set_launch(nsub, grid)
        m = g.track(25)
        x = g.get_particles(3)
        if ref is None:
            ref = (m, x)
        else:
            assert np.array_equal(m, ref[0]), (nsub, grid)
            assert np.array_equal(x[0], ref[1][0]) and np.array_equal(x[1], ref[1][1])


def test_batch_job_against_oracle(cuda):
    """A job inside a mixed batch still meets the oracle bar (moments 1e-9)."""
    w = JOBS[3]
    print_case("batch vs oracle", M=w.M, N=w.N)
    o = make_oracle(w)
    mo = o.track(50)
    gs = [make_tracker(x) for x in JOBS]
    b = tr.Batch(gs, graph_turns=8)
    mg = b.track(50)[3]
    assert moment_excess(mg, mo) <= 1e-9


def test_output_rings_wrap_under_graphs(cuda):
    """More turns than the moment ring holds (1024 rows for small jobs) and
    more profile rows than the profile ring (64), in one call with graph
    replay and in several calls of uneven length: the rows that come back are
    those of the job tracked alone in one call."""
    w = wl.C1.with_(N=3000, seed=21)
    turns, stride = 2600, 13        # 2600 moment rows, 200 profile rows
    print_case("ring wrap", turns=turns, stride=stride)
    g = make_tracker(w)
    m_alone, p_alone = g.track(turns, profiles_stride=stride)
    gb = make_tracker(w)
    b = tr.Batch([gb], graph_turns=16)
    m1, p1 = b.track(turns, profiles_stride=[stride])
    assert np.array_equal(m1[0], m_alone)
    assert np.array_equal(p1[0], p_alone)
    # the same turns in calls of 999 + 1001 + 600 turns on a fresh job
    gc = make_tracker(w)
    bc = tr.Batch([gc], graph_turns=16)
    parts = [bc.track(n) for n in (999, 1001, 600)]
    assert np.array_equal(np.concatenate([p[0] for p in parts]), m_alone)


@pytest.mark.parametrize("graph_turns", [0, 8])
def test_mixed_arithmetic_batch(cuda, graph_turns):
    """One batch holding an FP64 job (its between-turn work in the prep), a
    BF16x2 and an FP32 job (theirs in the matrix-core wake kernel, no prep
    items) and a job without a grid (prep sums only): every job gives bit for
    bit what it gives tracked alone with the same arithmetic, profiles
    included, over two calls."""
    modes = ["fp64", "bf16x2", None, "fp32"]
    print_case("mixed arithmetic batch", graph_turns=graph_turns, modes=modes)
    turns1, turns2 = 23, 18

    def job(j):
        g = make_tracker(JOBS[j])
        if modes[j] not in (None, "fp64"):
            g.set_wake_precision(modes[j])
        return g

    alone = []
    for j, w in enumerate(JOBS):
        g = job(j)
        if STRIDES[j]:
            m1, p1 = g.track(turns1, profiles_stride=STRIDES[j])
            m2, p2 = g.track(turns2, profiles_stride=STRIDES[j])
        else:
            m1, p1 = g.track(turns1), None
            m2, p2 = g.track(turns2), None
        alone.append((m1, p1, m2, p2, g.get_particles(w.M - 1), g.get_state()))
    gs = [job(j) for j in range(len(JOBS))]
    b = tr.Batch(gs, graph_turns=graph_turns)
    r1 = b.track(turns1, profiles_stride=STRIDES)
    r2 = b.track(turns2, profiles_stride=STRIDES)
    for j, w in enumerate(JOBS):
        m1, p1, m2, p2, x, st = alone[j]
        assert np.array_equal(r1[0][j], m1) and np.array_equal(r2[0][j], m2), j
        if STRIDES[j]:
            assert np.array_equal(r1[1][j], p1) and np.array_equal(r2[1][j], p2), j
        xb = gs[j].get_particles(w.M - 1)
        assert np.array_equal(xb[0], x[0]) and np.array_equal(xb[1], x[1]), j
        sb = gs[j].get_state()
        assert sb[0] == st[0] and np.array_equal(sb[2], st[2]), j
    b.close()
