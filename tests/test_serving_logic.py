"""Host logic of the serving loop (admission by footprint in arrival order,
slices that end at job completions, retirement frees the budget), with the
GPU objects replaced by stand-ins that record what they were asked to do."""
import numpy as np

from paper_1809_00391_amd import serve


class FakeTracker:
    def __init__(self, w):
        self.w = w
        self.turn = 0
        self.closed = False

    def close(self):
        self.closed = True


class FakeBatch:
    log = []

    def __init__(self, trackers, graph_turns=0, autotune=False):
        self.trackers = trackers
        FakeBatch.log.append(("batch", tuple(t.w.name for t in trackers)))

    def track(self, n, moments=True):
        FakeBatch.log.append(("track", n, tuple(t.w.name for t in self.trackers)))
        out = []
        for t in self.trackers:
            m = np.zeros((n, t.w.M, 4))
            m[:, :, 0] = np.arange(t.turn, t.turn + n)[:, None]  # the turn index
            t.turn += n
            out.append(m)
        return out

    def close(self):
        pass


class W:
    def __init__(self, name, M, N, size):
        self.name, self.M, self.N, self.size = name, M, N, size


def test_admission_slices_and_retirement(monkeypatch):
    monkeypatch.setattr(serve, "make_job", lambda w, wake="fp64": FakeTracker(w))
    monkeypatch.setattr(serve, "footprint", lambda w: w.size)
    monkeypatch.setattr(serve.tr, "Batch", FakeBatch)
    monkeypatch.setattr(serve.torch.cuda, "synchronize", lambda: None)
    FakeBatch.log = []
    t = [0.0]

    def clock():
        t[0] += 0.01
        return t[0]

    reqs = [serve.Request(0, 0.0, W("a", 2, 10, 50), 30),
            serve.Request(1, 0.0, W("b", 1, 10, 40), 10),
            serve.Request(2, 0.0, W("c", 1, 10, 30), 25),   # must wait for memory
            serve.Request(3, 5.0, W("d", 1, 10, 10), 5)]    # arrives later
    srv = serve.Server(hbm_budget=100, quantum=12, clock=clock)
    res = srv.run(reqs)
    assert srv.peak_bytes <= 100
    # every job's rows are its own turns 0..turns-1, in order
    for r in reqs:
        m = res[r.job_id].moments
        assert m.shape[0] == r.turns
        assert np.array_equal(m[:, 0, 0], np.arange(r.turns))
    tracks = [e for e in FakeBatch.log if e[0] == "track"]
    # first slice stops at b's completion (10 < quantum), c is admitted only after
    assert tracks[0] == ("track", 10, ("a", "b"))
    assert "c" in tracks[1][2] and "b" not in tracks[1][2]
    assert all(e[1] <= 12 for e in tracks)
    assert res[3].admitted_s >= 5.0
    assert res[2].admitted_s >= res[1].done_s
