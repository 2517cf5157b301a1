"""bench.py's output contract: one JSON line with the fields the measurement
needs (a miniature run on the GPU), and a clear refusal of more than one GPU
(on the CPU, before anything touches a device)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.gpu
def test_bench_json_line(cuda):
    print("[gpu case] bench contract (miniature run)", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "64",
                        "--warmup", "8", "--cpu-budget", "1", "--serve-scale", "0.002",
                        "--cache-resident-turns", "16", "--roofline-turns", "20",
                        "--table4-turns", "4", "--sustained-turns", "32", "--physics-turns", "8"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 64 and d["warmup"] == 8
    assert d["value"] > 0 and d["dtype"] == "f64" and "workload" in d["config"]
    assert "model" not in d["config"]
    # the headline is the full fill in the batched mixed-precision form, the
    # plain FP64 tracker beside it
    assert d["config"]["bunches"] == 484 and d["config"]["form"] == "batched_mixed"
    assert d["value"] == d["forms"]["batched_mixed"]["value"]
    assert d["forms"]["plain_fp64"]["value"] > 0 and d["batched_over_plain"] > 0
    assert d["sustained"]["turns"] == 32 and d["sustained"]["batched_over_plain"] > 0
    rl = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rl, k
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0
    assert abs(rl["frac"] - rl["achieved"] / rl["peak"]) < 1e-12
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and cb["sample"]
    assert cb["nproc"] >= 1 and "cpu_model" in cb
    assert rl["launches_timed"] >= 20
    assert d["cache_resident"]["value"] > 0
    assert d["serving"]["batched"]["p99_s"] >= d["serving"]["batched"]["p50_s"]
    assert len(d["paper_table4"]["rows"]) == 7
    pv = d["physics_variants"]
    for k in ("resistive_wall", "passive_hc", "transverse"):
        assert pv[k]["value"] > 0 and pv[k]["moments_finite"], k
        assert pv[k]["push"]["avg_launch_us"] > 0, k
    assert pv["transverse"]["push"]["bytes_per_particle_turn"] == 64
