"""Serving with continuous batching (paper_1809_00391_amd.serve) on the GPU:
jobs arriving over time, admitted by HBM footprint, advanced together in
slices; every job's moments are bit for bit those of the job tracked alone."""
import numpy as np
import pytest

from paper_1809_00391_amd import serve
from paper_1809_00391_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _mix():
    jobs = []
    spec = [  # (arrival s, bunches, particles, turns, HOM fr)
        (0.00, 3, 5000, 45, 1.45e9), (0.00, 40, 1200, 30, 1.52e9), (0.00, 1, 20000, 61, 1.41e9),
        (0.05, 12, 4097, 23, 1.58e9), (0.20, 3, 777, 52, 1.50e9), (0.20, 1, 9000, 17, 1.55e9),
    ]
    for i, (t, M, N, turns, fr) in enumerate(spec):
        w = wl.Workload(name=f"job{i}", ring=wl.RING_R484, buckets=tuple(range(0, 3 * M, 3)),
                        currents_A=(0.5e-3 + 0.3e-3 * i,) * M, N=N, turns=turns, seed=100 + i,
                        sigma_tau0=10e-12, sigma_delta0=8.6e-4, short_range=(wl.BB,),
                        grid=(256, -76.15e-12, 76.15e-12), long_range=((1e6, 2e4, fr),))
        jobs.append(serve.Request(i, t, w, turns))
    return jobs


@pytest.mark.parametrize("wake", ["fp64", "bf16x2"])
def test_each_job_same_alone_and_in_mix(cuda, wake):
    reqs = _mix()
    sizes = sorted(serve.footprint(r.workload) for r in reqs)
    budget = sum(sizes[-3:])  # never all six at once: admission has to wait
    print(f"[gpu case] serving wake={wake} budget={budget}", flush=True)
    srv = serve.Server(hbm_budget=budget, quantum=16, graph_turns=4, autotune=True, wake=wake)
    res = srv.run(reqs)
    assert sorted(res) == list(range(len(reqs)))
    assert srv.peak_bytes <= budget
    assert srv.slices > len(reqs) and srv.batches_built >= 3
    for r in reqs:
        alone = serve.make_job(r.workload, wake).track(r.turns)
        got = res[r.job_id].moments
        assert got.shape == alone.shape
        assert np.array_equal(got, alone), r.job_id
        assert res[r.job_id].latency_s >= 0
    lat = serve.latency_percentiles(res)
    print(f"[serving] wake={wake} slices={srv.slices} batches={srv.batches_built} "
          f"p50={lat['p50']:.3f}s p99={lat['p99']:.3f}s", flush=True)


@pytest.mark.parametrize("wake,tol", [("fp64", 1e-9), ("bf16x2", 1e-4)])
def test_served_jobs_match_oracle(cuda, wake, tol):
    """Every job of a served mix (arrivals while others run, a budget that
    forces waiting, slices of 16 turns) against the FP64 oracle tracking the
    same job alone from the same seed: moments over its first 100 turns within
    1e-9 of the bunch scale with the FP64 wake, within 1e-4 with the BF16x2
    wake on the matrix cores (its element-wise error bound gives deviations of
    order 1e-5 of the rms over 100 turns)."""
    from helpers import make_oracle, moment_excess
    reqs = []
    for r in _mix():
        w = r.workload.with_(turns=100)
        reqs.append(serve.Request(r.job_id, r.arrival_s, w, 100))
    sizes = sorted(serve.footprint(r.workload) for r in reqs)
    budget = sum(sizes[-3:])
    print(f"[gpu case] served mix vs oracle, wake={wake}", flush=True)
    srv = serve.Server(hbm_budget=budget, quantum=16, graph_turns=4, autotune=False, wake=wake)
    res = srv.run(reqs)
    assert srv.batches_built >= 3
    worst = 0.0
    for r in reqs:
        o = make_oracle(r.workload)
        ref_m = o.track(r.turns)
        got = res[r.job_id].moments
        assert got.shape == ref_m.shape
        err = moment_excess(got, ref_m)
        worst = max(worst, err)
        assert err <= tol, (r.job_id, err)
    print(f"[serving vs oracle] wake={wake} worst moment deviation {worst:.2e} (bar {tol:g})",
          flush=True)
