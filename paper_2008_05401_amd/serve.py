"""Continuous-batching job server for CRBM-aided Monte Carlo sampling jobs.

A job asks for n_chains chains of an L x L Ising lattice at temperature T with
its own CRBM filters, run for n_sweeps propose+accept sweeps (the sweep of
include/crbm.h).  The server

* admits arriving jobs in FIFO order as soon as their HBM footprint (state,
  workspace, temperatures, filters) fits the budget next to the jobs already
  resident, and keeps every admitted job's chains resident on the GPU;
* splits jobs by lattice size into three lanes, each on its own stream
  (default priority), which overlap on the device.  A small job (L^2 below
  `medium_sites`) or a medium one (below `large_sites`) runs all its sweeps in
  one launch, shared with the jobs of its lane admitted in the same step.
  Large jobs advance together in blocks of `large_block` sweeps, a new block
  being issued when the previous one is done (at most `max_inflight` ahead), so
  a large job that arrives joins at the next block and the workgroups of large
  jobs free their compute units every few milliseconds.  A job thus waits
  behind launches of its own size class only: neither behind the block length
  of the largest lattices nor, for the smallest, behind a medium launch;
* within a launch the library orders the chains by descending lattice size,
  so the longest workgroups are dispatched first;
* puts a new job's filters and temperatures on the device through an idle
  admission stream, so that admitting a job never waits for launches already
  queued on the job streams;
* detects completion without blocking the GPU: after a job's last sweeps its
  per-chain records are copied on the device and an event is recorded; the
  host polls the event, then copies the small record buffer out and frees the
  job's memory.

Latency of a job = completion time - arrival time (queueing included).
Results do not depend on the mix, the stream or the block lengths: random
numbers are indexed by (seed, chain, sweep), so a job gives the same chains
alone and in any batch.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as C
from . import api, workloads


@dataclass
class JobResult:
    job_id: int
    arrival_s: float
    admit_s: float = 0.0
    done_s: float = 0.0
    stats: np.ndarray = None
    state: np.ndarray = None

    @property
    def latency_s(self):
        return self.done_s - self.arrival_s


@dataclass
class _Active:
    spec: workloads.Job
    job: api.Job
    res: JobResult
    footprint: int
    remaining: int
    event: torch.cuda.Event = None
    rec_dev: torch.Tensor = None


def job_filters(spec: workloads.Job, K: int = 8, Lw: int = 5, std: float = 0.05):
    return workloads.random_filters(K, 1, Lw, std, seed=spec.seed)


def footprint_bytes(spec: workloads.Job, K: int = 8, Lw: int = 5) -> int:
    """HBM bytes of a resident job: state, workspace (records), temperatures, filters."""
    n = spec.n_chains
    return n * spec.L * spec.L + 256 + n * C.STATS_DTYPE.itemsize + 512 + 8 * n + 4 * (K * Lw * Lw + K + 1)


@dataclass
class Server:
    budget_bytes: int = 16 << 30
    large_block: int = 4            # sweeps per launch of the large jobs
    medium_sites: int = 128 * 128   # L^2 >= medium_sites: medium lane
    large_sites: int = 256 * 256    # L^2 >= large_sites: large lane (blocks)
    max_inflight: int = 2           # large-job blocks issued ahead of the GPU
    K: int = 8
    Lw: int = 5
    keep_state: bool = False
    results: list = field(default_factory=list)

    def lane_of(self, L: int) -> int:
        """0: small, 1: medium (each a job's sweeps in one launch), 2: large (blocks)."""
        if L * L >= self.large_sites:
            return 2
        return 1 if L * L >= min(self.medium_sites, self.large_sites) else 0

    def _admit(self, sp, stream, now):
        # The filters and temperatures go to the device on an idle admission stream:
        # a host-to-device copy from pageable memory waits for its stream, and the
        # lane streams hold the running launches.  The job's stream then waits for
        # that stream before crbm_init.
        f = job_filters(sp, self.K, self.Lw)
        with torch.cuda.stream(self._s_admit):
            p = api.CRBMParams.from_filters(f)
            T = torch.full((sp.n_chains,), sp.T, dtype=torch.float64, device="cuda")
            ev = torch.cuda.Event()
            ev.record(self._s_admit)
        stream.wait_event(ev)
        with torch.cuda.stream(stream):
            job = api.Job(p, api.ISING, sp.L, T, seed=sp.seed, burnin=sp.n_sweeps // 10)
        res = JobResult(sp.job_id, sp.arrival_s, admit_s=now())
        return _Active(sp, job, res, footprint_bytes(sp, self.K, self.Lw), sp.n_sweeps)

    @staticmethod
    def _finish(jobs, stream, finishing):
        """Device-side copies of the records of jobs whose last sweeps are issued, and an event."""
        with torch.cuda.stream(stream):
            for a in jobs:
                a.rec_dev = a.job.stats_device()
            ev = torch.cuda.Event()
            ev.record(stream)
        for a in jobs:
            a.event = ev
            finishing.append(a)
        return ev

    def run(self, specs, time_scale: float = 1.0):
        """Serve `specs` (sorted by arrival); arrival times are seconds from the start,
        multiplied by time_scale."""
        specs = sorted(specs, key=lambda s: s.arrival_s)
        pending = list(specs)
        waiting = []            # arrived, not admitted
        large = []              # resident large jobs with sweeps left
        finishing = []          # last sweeps issued, waiting for their event
        inflight = []           # events of the large-job blocks issued
        used = 0
        streams = [torch.cuda.Stream() for _ in range(3)]
        self._s_admit = torch.cuda.Stream()
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        while pending or waiting or large or finishing:
            t = now()
            while pending and pending[0].arrival_s * time_scale <= t:
                sp = pending.pop(0)
                sp = workloads.Job(sp.job_id, sp.arrival_s * time_scale, sp.L, sp.T, sp.n_chains, sp.n_sweeps,
                                   sp.seed)
                waiting.append(sp)
            # FIFO admission under the HBM budget
            new = ([], [])
            while waiting:
                sp = waiting[0]
                fp = footprint_bytes(sp, self.K, self.Lw)
                if used + fp > self.budget_bytes and (large or finishing or new[0] or new[1]):
                    break
                waiting.pop(0)
                lane = self.lane_of(sp.L)
                a = self._admit(sp, streams[lane], now)
                used += fp
                (large if lane == 2 else new[lane]).append(a)
            # small and medium jobs: all their sweeps in one launch per lane and sweep count
            for lane in (0, 1):
                by_len = {}
                for a in new[lane]:
                    by_len.setdefault(a.remaining, []).append(a)
                for n_sw, group in by_len.items():
                    if n_sw > 0:
                        api.run_many([a.job for a in group], n_sw)
                    for a in group:
                        a.remaining = 0
                    self._finish(group, streams[lane], finishing)
            # large jobs: the next block when fewer than max_inflight are outstanding
            inflight = [ev for ev in inflight if not ev.query()]
            if large and len(inflight) < self.max_inflight:
                block = min(self.large_block, min(a.remaining for a in large))
                if block > 0:
                    api.run_many([a.job for a in large], block)
                for a in large:
                    a.remaining -= block
                ended = [a for a in large if a.remaining == 0]
                large = [a for a in large if a.remaining > 0]
                if ended:
                    inflight.append(self._finish(ended, streams[2], finishing))
                else:
                    with torch.cuda.stream(streams[2]):
                        ev = torch.cuda.Event()
                        ev.record(streams[2])
                    inflight.append(ev)
            # completions
            done = []
            for a in finishing:
                if a.event.query():
                    a.res.done_s = now()
                    st = np.frombuffer(a.rec_dev.cpu().numpy().tobytes(), dtype=C.STATS_DTYPE).copy()
                    a.res.stats = st
                    if self.keep_state:
                        a.res.state = a.job.state.cpu().numpy()
                    a.job.close()
                    used -= a.footprint
                    self.results.append(a.res)
                    done.append(a)
            if done:
                finishing = [a for a in finishing if a not in done]
            if not done and not new[0] and not new[1]:
                if finishing or inflight:
                    time.sleep(0.0001)
                elif pending and not waiting:
                    dt = pending[0].arrival_s * time_scale - now()
                    if dt > 0:
                        time.sleep(min(dt, 0.01))
        torch.cuda.synchronize()
        return self.results


def latency_summary(results, warmup_s: float = 0.0):
    lat = np.array([r.latency_s for r in results if r.arrival_s >= warmup_s])
    if lat.size == 0:
        return {"jobs": 0}
    return {"jobs": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p90_ms": float(np.percentile(lat, 90) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3)}


def run_plain(spec: workloads.Job, K: int = 8, Lw: int = 5, max_block: int = 10):
    """The plain form: the job's chains one at a time, one chain per launch."""
    f = job_filters(spec, K, Lw)
    p = api.CRBMParams.from_filters(f)
    states, recs = [], []
    for g in range(spec.n_chains):
        job = api.Job(p, api.ISING, spec.L, np.full(1, spec.T), seed=spec.seed, burnin=spec.n_sweeps // 10,
                      chain_offset=g)
        left = spec.n_sweeps
        while left:
            b = min(max_block, left)
            job.run(b)
            left -= b
        recs.append(job.stats())
        states.append(job.state)
        job.close()
    torch.cuda.synchronize()
    return torch.cat(states).cpu().numpy(), np.concatenate(recs)
