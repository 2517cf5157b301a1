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
