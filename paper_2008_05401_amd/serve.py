"""Continuous-batching job server for CRBM-aided Monte Carlo sampling jobs.

A job asks for n_chains chains of an L x L Ising lattice at temperature T with
its own CRBM filters, run for n_sweeps propose+accept sweeps (the sweep of
include/crbm.h).  The server

* admits arriving jobs in FIFO order as soon as their HBM footprint (state,
  workspace, temperatures, filters) fits the budget next to the jobs already
  resident;
* keeps every admitted job's chains resident on the GPU and advances all of
  them together: each scheduling step issues one `crbm_propose_accept_many`
  call (a handful of kernel launches shared by all jobs) for a block of
  sweeps no larger than any active job's remaining work, so jobs that arrive
  while others run join the next step;
* detects completion without blocking the GPU: after a job's last block its
  per-chain records are copied on the device and an event is recorded; the
  host polls the event, then copies the small record buffer out and frees the
  job's memory.

Latency of a job = completion time - arrival time (queueing included).
Results do not depend on the mix: random numbers are indexed by (seed, chain,
sweep), so a job gives the same chains alone and in any batch.
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
    max_block: int = 10
    max_inflight: int = 2
    K: int = 8
    Lw: int = 5
    keep_state: bool = False
    results: list = field(default_factory=list)

    def run(self, specs, time_scale: float = 1.0):
        """Serve `specs` (sorted by arrival); arrival times are seconds from the start."""
        specs = sorted(specs, key=lambda s: s.arrival_s)
        pending = list(specs)
        waiting = []            # arrived, not admitted
        active = []             # resident
        finishing = []          # last block issued, waiting for its event
        used = 0
        inflight = []
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        while pending or waiting or active or finishing:
            t = now()
            while pending and pending[0].arrival_s * time_scale <= t:
                waiting.append(pending.pop(0))
            # FIFO admission under the HBM budget
            while waiting:
                sp = waiting[0]
                fp = footprint_bytes(sp, self.K, self.Lw)
                if used + fp > self.budget_bytes and (active or finishing):
                    break
                waiting.pop(0)
                f = job_filters(sp, self.K, self.Lw)
                job = api.Job(api.CRBMParams.from_filters(f), api.ISING, sp.L, np.full(sp.n_chains, sp.T),
                              seed=sp.seed, burnin=sp.n_sweeps // 10)
                res = JobResult(sp.job_id, sp.arrival_s * time_scale, admit_s=now())
                active.append(_Active(sp, job, res, fp, sp.n_sweeps))
                used += fp
            if active:
                block = min(self.max_block, min(a.remaining for a in active))
                api.run_many([a.job for a in active], block)
                still, ended = [], []
                for a in active:
                    a.remaining -= block
                    if a.remaining == 0:
                        a.rec_dev = a.job.stats_device()  # device-side copy of the records
                        ended.append(a)
                    else:
                        still.append(a)
                ev = torch.cuda.Event()
                ev.record()  # after the sweeps and the record copies
                inflight.append(ev)
                for a in ended:
                    a.event = ev
                    finishing.append(a)
                active = still
                # bound the queue of work issued ahead of the GPU
                while len(inflight) > self.max_inflight:
                    inflight.pop(0).synchronize()
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
            if not active and not done:
                if finishing:
                    time.sleep(0.0002)
                elif pending and not waiting:
                    dt = pending[0].arrival_s * time_scale - now()
                    if dt > 0:
                        time.sleep(min(dt, 0.01))
        return self.results


def latency_summary(results, warmup_s: float = 0.0):
    lat = np.array([r.latency_s for r in results if r.arrival_s >= warmup_s])
    if lat.size == 0:
        return {"jobs": 0}
    return {"jobs": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
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
