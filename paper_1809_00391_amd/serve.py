"""Serving loop with continuous batching over the tracker's batch ABI.

Tracking requests (a workload each: ring, fill, wakes, particles, turns,
seed) arrive over time.  The loop keeps every admitted job's particle state,
phasors and tables resident in device memory and advances all admitted jobs
together, a slice of turns at a time, with one launch of each kernel per turn
covering every bunch of every job (mbt_batch_*).  Between slices it retires
finished jobs (freeing their memory) and admits waiting ones in arrival order
while their footprint (particle state and workspace from mbt_query_bytes; the
batch's own tables are a few bytes per tile and not counted) fits the HBM
budget.  A slice ends at the next job completion or after `quantum` turns,
whichever is first, so a job's moments are exactly those of tracking it alone:
each job keeps its own seed-keyed random streams and its own fixed reduction
layout, and a slice boundary is an ordinary resume from the device-side turn
counter.

Reports per job: arrival, admission and completion times (latency =
completion - arrival) and the moments [turns][M][4].
"""
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import tracker as tr

__all__ = ["Request", "Result", "Server"]


@dataclass
class Request:
    job_id: int
    arrival_s: float
    workload: object           # workloads.Workload
    turns: int


@dataclass
class Result:
    job_id: int
    arrival_s: float
    admitted_s: float = 0.0
    done_s: float = 0.0
    particle_turns: float = 0.0
    moments: list = field(default_factory=list)

    @property
    def latency_s(self):
        return self.done_s - self.arrival_s


def make_job(w, wake="fp64"):
    """A bound, initialised Tracker for workload w (allocates its memory)."""
    t = tr.Tracker(w.ring)
    if w.hc_flat is not None:
        t.set_harmonic_cavity(tr.hc_flat_fraction(w.ring, *w.hc_flat))
    t.set_fill(w.buckets, w.currents_A, w.streams)
    if w.grid is not None:
        t.set_short_range(list(w.short_range), w.grid)
    if w.long_range:
        t.set_long_range(list(w.long_range))
    if w.rw is not None:
        t.set_resistive_wall(w.rw)
    if wake != "fp64" and w.grid is not None:
        t.set_wake_precision(wake)
    t.bind(w.N)
    t.init_gaussian(w.sigma_tau0, w.sigma_delta0, w.seed)
    return t


def footprint(w):
    """Device bytes a job needs: particle state and workspace (mbt_query_bytes)."""
    t = tr.Tracker(w.ring)
    if w.hc_flat is not None:
        t.set_harmonic_cavity(tr.hc_flat_fraction(w.ring, *w.hc_flat))
    t.set_fill(w.buckets, w.currents_A, w.streams)
    if w.grid is not None:
        t.set_short_range(list(w.short_range), w.grid)
    if w.long_range:
        t.set_long_range(list(w.long_range))
    sb, wb = t.query_bytes(w.N)
    t.close()
    return sb + wb


class Server:
    """Continuous-batching request loop on one GPU.

    hbm_budget: device bytes the admitted jobs may hold together.
    quantum: most turns in one slice (admission and retirement happen between
    slices).  max_jobs: most jobs in one batch.  graph_turns, autotune: as in
    mbt_batch_configure (the tuner's choices are cached per shape, but every
    new batch composition is a new shape, so it is off by default).  wake:
    arithmetic of the short-range wake.  fill_particles: admit further jobs
    only while the admitted jobs hold fewer macro-particles than this (enough
    to fill the GPU); None admits whatever fits the budget.  With a fill
    target, large jobs run nearly in arrival order and small ones are
    batched together, which shortens the typical latency.
    """

    def __init__(self, hbm_budget, quantum=1000, max_jobs=64, graph_turns=16, autotune=False,
                 wake="fp64", fill_particles=None, clock=time.perf_counter):
        self.hbm_budget = int(hbm_budget)
        self.quantum = int(quantum)
        self.max_jobs = int(max_jobs)
        self.graph_turns = int(graph_turns)
        self.autotune = bool(autotune)
        self.wake = wake
        self.fill_particles = fill_particles
        self.clock = clock
        self.slices = 0
        self.batches_built = 0
        self.build_s = 0.0    # host time spent building batches (set-up, not tracking)
        self.peak_bytes = 0

    def run(self, requests, keep_moments=True):
        """Serve the requests (arrival times relative to the call); returns
        {job_id: Result} once every job has finished."""
        pending = deque(sorted(requests, key=lambda r: r.arrival_s))
        sizes = {}
        active = []          # [request, tracker, remaining turns, result]
        results = {}
        used = 0
        batch = None
        t0 = self.clock()
        while pending or active:
            now = self.clock() - t0
            # admission in arrival order while the footprint fits
            changed = False
            while pending and pending[0].arrival_s <= now and len(active) < self.max_jobs:
                if (self.fill_particles is not None and active and
                        sum(a[0].workload.M * a[0].workload.N for a in active) >= self.fill_particles):
                    break
                r = pending[0]
                if r.job_id not in sizes:
                    sizes[r.job_id] = footprint(r.workload)
                need = sizes[r.job_id]
                if need > self.hbm_budget:
                    raise ValueError(f"job {r.job_id} needs {need} bytes, more than the "
                                     f"budget {self.hbm_budget}")
                if used + need > self.hbm_budget:
                    break
                pending.popleft()
                res = Result(r.job_id, r.arrival_s, admitted_s=now)
                active.append([r, make_job(r.workload, self.wake), r.turns, res])
                used += need
                changed = True
            self.peak_bytes = max(self.peak_bytes, used)
            if not active:
                wait = pending[0].arrival_s - (self.clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
                continue
            if changed or batch is None:
                if batch is not None:
                    batch.close()
                tb = self.clock()
                batch = tr.Batch([a[1] for a in active], graph_turns=self.graph_turns,
                                 autotune=self.autotune)
                self.build_s += self.clock() - tb
                self.batches_built += 1
            n = min(self.quantum, min(a[2] for a in active))
            moms = batch.track(n, moments=keep_moments)
            self.slices += 1
            done_t = self.clock() - t0
            finished = []
            for j, a in enumerate(active):
                r, _, rem, res = a
                if keep_moments:
                    res.moments.append(moms[j])
                res.particle_turns += float(r.workload.M) * r.workload.N * n
                a[2] = rem - n
                if a[2] == 0:
                    res.done_s = done_t
                    if keep_moments:
                        res.moments = np.concatenate(res.moments)
                    results[r.job_id] = res
                    finished.append(j)
            if finished:
                batch.close()
                batch = None
                for j in reversed(finished):
                    r, trk, _, _ = active.pop(j)
                    trk.close()  # frees the job's state and workspace
                    used -= sizes[r.job_id]
                del trk, a  # no reference outlives the job's footprint
                torch.cuda.synchronize()
        if batch is not None:
            batch.close()
        return results


def latency_percentiles(results, q=(50, 99)):
    lat = np.array([r.latency_s for r in results.values()])
    return {f"p{p}": float(np.percentile(lat, p)) for p in q}
