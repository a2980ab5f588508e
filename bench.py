"""Benchmark of the CRBM-proposal + MH sweep on one MI355X.

Workload (batched Ising, the configuration the headline metric is quoted on):
L = 64 periodic square lattice, J = 1, CRBM with K = 8 hidden channels of 5x5
float32 filters ~ N(0, 0.05) (seed 0, biases 0), 4096 chains over 32
temperatures linspace(1.5, 3.5) (128 chains each), accumulators on (burn-in
10% of the timed sweeps).  One step = one propose+accept sweep of every chain
(steps 1-5 of the sweep: Gibbs proposal, F(x'), integer E(x'), MH test,
observables).  Steps are launched in blocks of `--block` sweeps per kernel
launch; the chains stay resident on the GPU between launches.

Printed: one JSON line with throughput (site-sweeps per second, every
completed propose+MH sweep counted, acceptance rate beside it), the roofline
of the sweep kernel measured with HIP events on its stream, and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# MI355X published peaks used for the roofline
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# LDS: 128 bytes per clock per CU, 256 CUs at 2.4 GHz
PEAK_LDS_TBS = 128 * 256 * 2.4e9 / 1e12

# HBM bytes of one sweep-kernel launch of this workload, from two rocprofv3 --pmc
# runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
# counter reads for a plain 256 MiB device-to-device copy (x2.0 and x1.0), per
# launch length.  The figures hold only for the kernel sources they were taken
# with (their SHA-256); after any change to them `traffic` is reported as null
# until re-measured.
KERNEL_SOURCES = ("paper_2008_05401_amd/csrc/sweep_ising_impl.h", "paper_2008_05401_amd/csrc/sweep_ising_launch.h",
                  "paper_2008_05401_amd/csrc/sweep_ising_k8l5.hip", "paper_2008_05401_amd/csrc/sweep_ising.h",
                  "paper_2008_05401_amd/csrc/device_common.h", "paper_2008_05401_amd/csrc/sweep_common.h")
MEASURED_TRAFFIC = {"sources_sha256": "eeb102db0e0d5894524de990dbe8ed293b7a8244d86d57d1dc44a1937f3375d3",
                    "chains": 4096, "L": 64, "fetch_scale": 2.0, "write_scale": 1.0,
                    # sweeps per launch -> (FETCH_SIZE KiB, WRITE_SIZE KiB) per dispatch, mean of two launches
                    "per_launch_kib": {20: (9415.3, 23265.5), 100: (9657.9, 24142.3)},
                    "source": "profiles/sweep_ising_L64_batched_hbm_counters.md"}

# VALU issue of the same kernel from SQ counters (SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU,
# GRBM_GUI_ACTIVE ...; two launches per length), reported while the kernel sources
# hash to the measured ones.  Issue slots: 256 CUs x 4 SIMDs x cycles / 4 (one wave64
# VALU instruction per four cycles per SIMD).
MEASURED_VALU = {"sources_sha256": "eeb102db0e0d5894524de990dbe8ed293b7a8244d86d57d1dc44a1937f3375d3",
                 "by_sweeps_per_launch": {
                     20: {"valu_issue_fraction": 1.0768, "valu_insts_per_site_sweep": 7.770,
                          "lanes_active": 0.9693, "lds_insts_per_site_sweep": 1.625,
                          "salu_insts_per_site_sweep": 1.419, "lds_bank_conflicts_per_access": 0.00116},
                     100: {"valu_issue_fraction": 1.0961, "valu_insts_per_site_sweep": 7.747,
                           "lanes_active": 0.9699, "lds_insts_per_site_sweep": 1.623,
                           "salu_insts_per_site_sweep": 1.406, "lds_bank_conflicts_per_access": 0.00099}},
                 "source": "profiles/sweep_ising_L64_batched_sq_counters.md"}


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic_bytes(chains, L, sweeps_per_launch):
    m = MEASURED_TRAFFIC
    if (chains, L) != (m["chains"], m["L"]) or kernel_sources_sha256() != m["sources_sha256"]:
        return None
    kib = m["per_launch_kib"].get(sweeps_per_launch)
    if kib is None:
        return None
    return 1024.0 * (kib[0] * m["fetch_scale"] + kib[1] * m["write_scale"])


def select_adds_per_site_sweep(K, C, Lw, gibbs_k=1):
    """Algorithmic work of one sweep per lattice site: the three correlation
    passes v->h and h->v' (gibbs_k times each) and v'->a' for F(x'), K*C*Lw^2
    taps each; the inputs are binary, so a tap is one FP32 select-add (counted
    as one flop)."""
    return float(K * C * Lw * Lw * (2 * gibbs_k + 1))


def lds_table_bytes_per_site_sweep(K, C, Lw, gibbs_k=1):
    """LDS bytes of the subset-sum/product table reads of one sweep per site:
    one float per (channel, filter row) in each of the hidden, visible and
    free-energy passes."""
    return 4.0 * K * C * Lw * (2 * gibbs_k + 1)


def gpu_warm(api, f, L, T, seconds, seed):
    """Bring the GPU to the clocks it holds under this kernel before the timed
    region: a throw-away job of the measured shape (another seed) runs 10-sweep
    launches for `seconds`, ending right before the measured job's warm-up
    sweeps (then its timed launches).  The
    batched workload runs 10^4 sweeps, seconds of continuous sweeps, while a
    run of --steps 20 lasts 4 ms: after even 50 ms of idle the first launches
    run at lower clocks (4.6-4.8 ms for 20 sweeps instead of 3.9).  The
    throw-away job uses another tile variant of the sweep kernel (2 rows per
    lane, 512 threads: the same chains, another kernel name), so a profile of
    the measured kernel sees only the measured job's launches.  Nothing of it
    is timed or reused."""
    import torch

    from paper_2008_05401_amd import autotune
    api.set_tuning(L, 8, 5, 2, 512)
    warm = api.Job(api.CRBMParams.from_filters(f), api.ISING, L, T, seed=seed)
    api.clear_tuning()
    autotune.apply()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        warm.run(10)
        torch.cuda.synchronize()
    warm.close()
    return time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(f, T, L, seed, seconds=8.0):
    """The FP64 oracle as it stands (never tuned), on the host's cores, on
    bounded samples of the measured workloads:
      - batched Ising (L=64, K=8 5x5): chains 0-255 with OpenMP over chains on
        all cores, chains 0-15 on one core;
      - Kitaev (K=8 3x3, C=3, T log-uniform in [0.005, 0.05]): N=36 (L=6, 256
        chains) and N=144 (L=12, 32 chains), all cores, MH steps per second;
      - gradient (B=1024, L=16, K=8 5x5, single-threaded): calls per second;
      - the small Ising configuration at its full size (L=8, 64 chains, 2000
        sweeps), wall time."""
    import oracle
    from paper_2008_05401_amd import workloads as WL
    oracle.build(force=False)
    all_threads = oracle.num_threads()
    m = oracle.CRBM(f.W, f.hbias, f.vbias)

    def sweeps_for(ch, secs):
        t0 = time.perf_counter()
        ch.run(1)
        one = time.perf_counter() - t0
        return max(1, int(secs / max(one, 1e-6)))

    def ising_rate(n, threads, secs):
        oracle.set_threads(threads)
        ch = oracle.Chains(m, oracle.ISING, L, T[:n], seed=seed)
        sw = sweeps_for(ch, secs)
        t0 = time.perf_counter()
        ch.run(sw)
        dt = time.perf_counter() - t0
        return n * L * L * sw / dt, sw, dt

    all_rate, all_sw, all_dt = ising_rate(256, all_threads, seconds)
    one_rate, one_sw, one_dt = ising_rate(16, 1, seconds * 0.6)
    oracle.set_threads(all_threads)
    fk = WL.random_filters(8, 3, 3, 0.1, seed=0)
    mk = oracle.CRBM(fk.W, fk.hbias, fk.vbias)
    kit = {}
    for Lk, n, tag in ((6, 256, "N36_L6"), (12, 32, "N144_L12")):
        ch = oracle.Chains(mk, oracle.KITAEV, Lk, WL.kitaev_temperatures(n), seed=0)
        t0 = time.perf_counter()
        ch.run(1)
        dt = time.perf_counter() - t0
        kit[tag] = {"mh_steps_per_s": n / dt, "chains": n, "sweeps": 1, "seconds": dt}
    fg = WL.alg1_init_filters(8, 5, seed=0)
    mg = oracle.CRBM(fg.W, fg.hbias, fg.vbias)
    xg = WL.random_states(1024, 1, 16, seed=1)
    gg = np.random.default_rng(2).standard_normal(1024)
    oracle.grad(mg, xg, gg)
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        oracle.grad(mg, xg, gg)
    grad_s = (time.perf_counter() - t0) / reps
    # the small configuration at its full size (L=8, 64 chains, 2000 sweeps) fits the oracle whole
    fs = WL_small_filters()
    chs = oracle.Chains(oracle.CRBM(fs.W, fs.hbias, fs.vbias), oracle.ISING, 8, np.full(64, 2.269), seed=0,
                        burnin=200)
    t1 = time.perf_counter()
    chs.run(2000)
    small_s = time.perf_counter() - t1
    return {
        "value": all_rate,
        "unit": "site-sweeps/s",
        "cores": all_threads,
        "kind": "oracle",
        "sample": f"batched Ising L=64 K=8 5x5: chains 0-255 (T=1.5 and 1.565), {all_sw} sweeps after 1 untimed "
                  f"sweep, FP64 C oracle with OpenMP over chains on {all_threads} threads, {all_dt:.1f} s",
        "single_core": {"value": one_rate, "unit": "site-sweeps/s", "cores": 1,
                        "sample": f"chains 0-15, {one_sw} sweeps, {one_dt:.1f} s"},
        "cpu_model": cpu_model(),
        "nproc": os.cpu_count(),
        "kitaev": kit,
        "grad_B1024_L16": {"calls_per_s": 1.0 / grad_s, "ms_per_call": grad_s * 1e3, "threads": 1},
        "small_config_full_size_s": small_s,
    }


def WL_small_filters():
    from paper_2008_05401_amd import workloads as WL
    return WL.random_filters(4, 1, 3, 0.1, seed=0)


def small_config(sweeps=2000, burnin=200):
    """The small Ising configuration at full size: L=8, K=4 3x3 filters ~ N(0, 0.1),
    T=2.269, 64 chains, 2000 sweeps with 200 of burn-in, in one launch;
    latency-bound, so the wall time of the whole run is the figure."""
    import torch

    from paper_2008_05401_amd import api
    job = api.Job(api.CRBMParams.from_filters(WL_small_filters()), api.ISING, 8, np.full(64, 2.269), seed=0,
                  burnin=burnin)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    job.run(sweeps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = job.stats()
    return {"wall_s": wall, "site_sweeps_per_s": 64 * 64 * sweeps / wall,
            "acceptance": float(st["n_acc"].sum() / st["sweeps"].sum())}


def served(n_jobs, rate, warmup_s, capacity, loads=(0.3, 0.6, 0.9), plain_jobs=3):
    """Served Ising jobs: Poisson arrivals at `rate` jobs/s, L uniform in
    {16,...,256}, T ~ U[1.8,2.8], 64-1024 chains (log-uniform), K=8 5x5 filters
    ~N(0,0.05) per job, 16 GiB budget.  The sweeps per job set the offered load:
    for each fraction of `capacity` (the batched throughput measured above),
    n_sweeps = load * capacity / (rate * mean(n_chains L^2)); p50/p90/p99 of
    completion - arrival over the jobs arriving after `warmup_s`, the jobs/s
    and site-sweeps/s achieved; each measured job is then run alone on the idle
    GPU, and the slowdown latency / alone time is summarised as well (job sizes
    n_chains L^2 span three decades, so raw p99/p50 is at least the spread of
    the alone times).  Beside it, the plain form (each chain alone, one
    launch per chain, jobs one after another) on a few jobs at the middle load."""
    import torch

    from paper_2008_05401_amd import serve, workloads as WL
    total = n_jobs + int(rate * warmup_s)
    base = WL.served_job_stream(total, rate_per_s=rate, n_sweeps=1, seed=0)
    mean_nl2 = float(np.mean([sp.n_chains * sp.L ** 2 for sp in base]))
    points = []
    for load in loads:
        n_sweeps = max(1, int(round(load * capacity / (rate * mean_nl2))))
        specs = WL.served_job_stream(total, rate_per_s=rate, n_sweeps=n_sweeps, seed=0)
        srv = serve.Server(budget_bytes=16 << 30)
        t0 = time.perf_counter()
        res = srv.run(specs)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        summ = serve.latency_summary(res, warmup_s=warmup_s)
        measured = [r for r in res if r.arrival_s >= warmup_s]
        span = max(r.done_s for r in measured) - min(r.arrival_s for r in measured)
        by_id = {sp.job_id: sp for sp in specs}
        site_sweeps = sum(by_id[r.job_id].n_chains * by_id[r.job_id].L ** 2 * n_sweeps for r in measured)
        small = [r.latency_s for r in measured if srv.lane_of(by_id[r.job_id].L) == 0]
        medium = [r.latency_s for r in measured if srv.lane_of(by_id[r.job_id].L) == 1]
        large = [r.latency_s for r in measured if srv.lane_of(by_id[r.job_id].L) == 2]
        # each measured job alone on the idle GPU (admission, set-up, sweeps, read-back):
        # its service floor; slowdown = latency / floor
        alone = {}
        for r in measured:
            sp = by_id[r.job_id]
            one = serve.Server(budget_bytes=16 << 30).run(
                [WL.Job(sp.job_id, 0.0, sp.L, sp.T, sp.n_chains, sp.n_sweeps, sp.seed)])
            alone[r.job_id] = one[0].latency_s
        floor = np.array([alone[r.job_id] for r in measured])
        slow = np.array([r.latency_s / alone[r.job_id] for r in measured])
        points.append({
            "offered_load": load, "sweeps_per_job": n_sweeps,
            "offered_site_sweeps_per_s": rate * mean_nl2 * n_sweeps,
            "jobs_measured": summ["jobs"], "p50_ms": summ["p50_ms"], "p90_ms": summ["p90_ms"],
            "p99_ms": summ["p99_ms"], "mean_ms": summ["mean_ms"], "p99_over_p50": summ["p99_ms"] / summ["p50_ms"],
            "jobs_per_s": summ["jobs"] / span, "site_sweeps_per_s": site_sweeps / span,
            "achieved_load": site_sweeps / span / capacity, "wall_s": wall,
            "small_jobs_p50_ms": float(np.percentile(small, 50) * 1e3) if small else None,
            "small_jobs_p99_ms": float(np.percentile(small, 99) * 1e3) if small else None,
            "medium_jobs_p50_ms": float(np.percentile(medium, 50) * 1e3) if medium else None,
            "medium_jobs_p99_ms": float(np.percentile(medium, 99) * 1e3) if medium else None,
            "large_jobs_p50_ms": float(np.percentile(large, 50) * 1e3) if large else None,
            "large_jobs_p99_ms": float(np.percentile(large, 99) * 1e3) if large else None,
            "alone_p50_ms": float(np.percentile(floor, 50) * 1e3), "alone_p99_ms": float(np.percentile(floor, 99) * 1e3),
            "alone_p99_over_p50": float(np.percentile(floor, 99) / np.percentile(floor, 50)),
            "slowdown_p50": float(np.percentile(slow, 50)), "slowdown_p90": float(np.percentile(slow, 90)),
            "slowdown_p99": float(np.percentile(slow, 99)), "slowdown_mean": float(slow.mean())})
    mid = points[len(points) // 2]["sweeps_per_job"]
    sample = WL.served_job_stream(total, rate_per_s=rate, n_sweeps=mid, seed=0)[-plain_jobs:]
    t1 = time.perf_counter()
    for sp in sample:
        serve.run_plain(sp)
    plain_t = (time.perf_counter() - t1) / len(sample)
    plain_ss = sum(sp.n_chains * sp.L ** 2 * mid for sp in sample) / (plain_t * len(sample))
    return {
        "workload": f"Poisson {rate:.0f} jobs/s, L in {{16,32,64,128,256}}, T~U[1.8,2.8], 64-1024 chains "
                    f"log-uniform, K=8 5x5 filters, 16 GiB budget; sweeps per job set the offered load as a "
                    f"fraction of the batched capacity {capacity:.3e} site-sweeps/s",
        "warmup_s": warmup_s, "mean_chains_x_sites": mean_nl2, "load_curve": points,
        "plain_one_chain_per_launch": {
            "sweeps_per_job": mid, "service_ms_per_job": plain_t * 1e3, "max_jobs_per_s": 1.0 / plain_t,
            "site_sweeps_per_s": plain_ss, "sample_jobs": len(sample),
            "note": "jobs run one after another; at the offered load the plain form's queue grows without bound "
                    "whenever max_jobs_per_s is below the arrival rate"},
    }


def _timed(fn, reps=1):
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def kitaev(sweeps6=20, sweeps12=2, sweeps_big=2, warm_s=0.2):
    """Kitaev honeycomb, J = (1,1,1), periodic, u on 3 L^2 bonds, CRBM K=8 3x3 ~ N(0,0.1):
    L=6 with 256 chains and L=12 with 128 chains, T log-uniform in [0.005, 0.05];
    also L=16 and L=24 (128 chains), where the eigen-step's M^T M no longer
    fits in LDS and sits in a per-chain global scratch.  Each job first runs
    launches of the timed length for `warm_s` seconds (the clocks of an idle
    GPU ramp over the first tens of milliseconds), then one timed launch."""
    import torch

    from paper_2008_05401_amd import api, workloads as WL
    out = {}
    for L, n, sw in ((6, 256, sweeps6), (12, 128, sweeps12), (16, 128, sweeps_big), (24, 128, sweeps_big)):
        f = WL.random_filters(8, 3, 3, 0.1, seed=0)
        job = api.Job(api.CRBMParams.from_filters(f), api.KITAEV, L, WL.kitaev_temperatures(n), seed=0)
        job.run(1)
        t_end = time.perf_counter() + warm_s
        while time.perf_counter() < t_end:
            job.run(sw)
            torch.cuda.synchronize()
        ms = _timed(lambda: job.run(sw)) / sw
        st = job.stats()
        N = L * L
        out[f"L{L}_chains{n}"] = {
            "ms_per_sweep": ms, "mh_steps_per_s": n / (ms * 1e-3),
            "eigen_flops_per_sweep": n * (4.0 / 3.0) * N ** 3,
            "acceptance": float(st["n_acc"].sum() / st["sweeps"].sum())}
    return out


def frbm(L=8, n=256, sweeps=10):
    """Sec. IV's comparison of proposals on the Kitaev eta model (C=1, L=8,
    256 chains, T log-uniform in [0.005, 0.05]): ms per sweep with the CRBM
    (K=8, 3x3 ~ N(0, 0.1)) and with fully connected RBMs of 64 and 128
    hidden units (W ~ N(0, 0.05)); the dense Gibbs passes run per chain from
    LDS inside the fused sweep."""
    from paper_2008_05401_amd import api, workloads as WL
    T = WL.kitaev_temperatures(n)
    cases = (("crbm_K8_3x3", api.CRBMParams.from_filters(WL.random_filters(8, 1, 3, 0.1, seed=0))),
             ("frbm_64_hidden", api.CRBMParams.from_filters(WL.random_frbm(64, 1, L, 0.05, seed=0), dense=True)),
             ("frbm_128_hidden", api.CRBMParams.from_filters(WL.random_frbm(128, 1, L, 0.05, seed=0), dense=True)))
    out = {}
    for name, p in cases:
        job = api.Job(p, api.KITAEV, L, T, seed=0)
        job.run(1)
        ms = _timed(lambda: job.run(sweeps)) / sweeps
        st = job.stats()
        out[name] = {"ms_per_sweep": ms, "mh_steps_per_s": n / (ms * 1e-3),
                     "acceptance": float(st["n_acc"].sum() / st["sweeps"].sum())}
        job.close()
    return out


def analytic_per_temperature(sweeps=1000, block=100):
    """The batched Ising shape (L=64, 4096 chains, 32 temperatures in
    [1.5, 3.5]) with the exact App. C kernel of each temperature (K=8, 5x5,
    zero-padded): one job of 128 chains per temperature, all 32 advanced in
    shared launches; acceptance is ~1 because the proposal is exact."""
    from paper_2008_05401_amd import api, workloads as WL
    import torch
    grid = np.linspace(1.5, 3.5, 32)
    jobs = [api.Job(api.CRBMParams.from_filters(WL.analytic_ising_filters(float(T), K=8, Lw=5)), api.ISING, 64,
                    np.full(128, T), seed=0, chain_offset=128 * q) for q, T in enumerate(grid)]
    api.run_many(jobs, block)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(sweeps // block):
        api.run_many(jobs, block)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    acc = sum(float(j.stats()["n_acc"].sum()) for j in jobs) / sum(float(j.stats()["sweeps"].sum()) for j in jobs)
    rech = sum(float(j.stats()["n_recheck"].sum()) for j in jobs)
    return {"site_sweeps_per_s": 4096 * 64 * 64 * sweeps / wall, "acceptance": acc, "sweeps": sweeps,
            "fp64_rechecks_per_site_sweep": rech / (4096 * 64 * 64 * (sweeps + block))}


def tempering(blocks=20, block_sweeps=5):
    """Parallel tempering with the exchange correction (App. B): the batched
    Ising config (4096 chains, L=64, K=8 5x5 ~ N(0,0.05), 32 rungs
    linspace(1.5, 3.5) x 128 ladders) with persistent CRBM replicas, one swap
    round after every block of sweeps; and Kitaev L=6 (K=8 3x3 ~ N(0,0.1),
    16 rungs geomspace(0.005, 0.05) x 16 ladders).  Reported: throughput of the
    whole cycle, swap acceptance, time of one swap round."""
    import torch

    from paper_2008_05401_amd import api, workloads as WL
    out = {}
    cases = (("ising_L64_4096", api.ISING, 64, WL.random_filters(8, 1, 5, 0.05, seed=0),
              WL.ising_temperatures_linspace(32, 1.5, 3.5, 4096), 128, block_sweeps, blocks),
             ("kitaev_L6_256", api.KITAEV, 6, WL.random_filters(8, 3, 3, 0.1, seed=0),
              np.repeat(np.geomspace(0.005, 0.05, 16), 16), 16, 1, 10))
    for name, target, L, f, T, nl, bs, nb in cases:
        job = api.Job(api.CRBMParams.from_filters(f), target, L, T, seed=0, replica=True)
        job.run(bs)
        job.tempering_swap(nl, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in range(nb):
            job.run(bs)
            job.tempering_swap(nl, 1 + b)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = job.stats()
        swap_ms = _timed(lambda: job.tempering_swap(nl, 10 ** 6), reps=1)
        n = len(T)
        rungs = n // nl
        pairs = sum(((rungs - (r % 2)) // 2) * nl for r in range(1, nb + 1))
        out[name] = {
            "chains": n, "ladders": nl, "rungs": rungs, "sweeps_per_swap_round": bs,
            "site_sweeps_per_s": n * L * L * bs * nb / wall if target == api.ISING else None,
            "mh_steps_per_s": n * bs * nb / wall,
            "exchange_acceptance": float(st["n_acc"].sum() / st["sweeps"].sum()),
            "swap_acceptance": float(st["n_swap"].sum() / 2 / max(1, pairs + ((rungs // 2) * nl))),
            "swap_round_ms": swap_ms}
    return out


def autocorrelation_times(sizes=(16, 32, 64, 128), chains=64, burn=1000, record=8000, max_lag=2000):
    """Integrated autocorrelation time of the energy (automatic window, c = 6)
    for the CRBM sampler with the exact Ising kernels of App. C (K=2, 2x2) at
    T = 2.2 and T = T_c, the temperatures of the Sec. III comparison: per L,
    `chains` independent chains, `burn` sweeps, then `record` sweeps kept in
    the device trace ring; mean and standard error of tau over the chains,
    and the time of one autocorrelation launch over all of them."""
    import math

    from paper_2008_05401_amd import api, workloads as WL
    out = {}
    tc = 2.0 / math.log(1.0 + math.sqrt(2.0))
    for tname, T in (("T2.2", 2.2), ("Tc", tc)):
        f = WL.analytic_ising_filters(T)
        for L in sizes:
            job = api.Job(api.CRBMParams.from_filters(f), api.ISING, L, np.full(chains, T), seed=L)
            for _ in range(burn // 100):
                job.run(100)
            job.record_trace(record)
            for _ in range(record // 100):
                job.run(100)
            ring, start, count = job.trace_ring()
            res = {}

            def go():
                res["r"] = api.autocorrelation(ring, max_lag, start=start)
            ms = _timed(go)
            cov, tau, win = (t.cpu().numpy() for t in res["r"])
            st = job.stats()
            ok = win > 0
            # pooled estimate: the chains are independent replicas at one temperature, so
            # their autocovariances are averaged before the window is chosen
            rho = cov.mean(0) / cov.mean(0)[0]
            tp, wp = 0.5, -1
            for t in range(1, max_lag + 1):
                tp += rho[t]
                if t >= 6.0 * tp:
                    wp = t
                    break
            out[f"{tname}_L{L}"] = {
                "tau_int_pooled": float(tp), "window_pooled": wp,
                "tau_int_mean": float(tau[ok].mean()) if ok.any() else None,
                "tau_int_sem": float(tau[ok].std(ddof=1) / np.sqrt(ok.sum())) if ok.sum() > 1 else None,
                "chains_with_window": int(ok.sum()), "chains": chains, "recorded_sweeps": count,
                "acceptance": float(st["n_acc"].sum() / st["sweeps"].sum()),
                "autocorr_kernel_ms": ms}
            job.close()
    return out


def training_and_transfer(epochs=100, lr=1e-3):
    """Gradient of F at B=1024 Ising states (L=16, T=2.3), an Alg. 1 training run
    (ADAM at the paper's learning rate 1e-3, batch 20, ub = 200), and sampling
    at L=128 with 2048 chains using the trained filters.  Reported: the loss of
    Eq. (loss) over x_phys U x_RBM (the quantity Alg. 1 minimises) for the
    initial and the trained parameters, on the final buffer, and over the
    physical states alone."""
    import torch

    from paper_2008_05401_amd import api, train
    L, T = 16, 2.3
    x, E, acc0 = train.exact_ising_samples(L, T, 1024, sweeps=1000, seed=0)
    f0 = train.workloads.alg1_init_filters(8, 5, seed=0)
    p0 = api.CRBMParams.from_filters(f0)
    g = torch.randn(1024, device="cuda", generator=torch.Generator(device="cuda").manual_seed(0))
    api.grad(p0, x, g)
    grad_ms = _timed(lambda: api.grad(p0, x, g), reps=20)
    fwd_ms = _timed(lambda: api.free_energy(p0, x), reps=20)
    z1 = torch.zeros(1, device="cuda")
    loss0 = train.full_loss(x, E, T, p0.W, p0.hbias, z1)
    t0 = time.perf_counter()
    r = train.train(x, E, T, epochs=epochs, batch=20, ub=200, lr=lr, seed=0, track=True)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    loss1 = train.full_loss(x, E, T, r.W, r.hbias, r.vbias)
    nlp = E.to(torch.float64) / T
    u0 = train.union_loss(r, x, nlp, p0.W, p0.hbias, z1)
    u1 = train.union_loss(r, x, nlp, r.W, r.hbias, r.vbias)
    h = r.history
    job = api.Job(api.CRBMParams(r.W, r.hbias, r.vbias), api.ISING, 128, np.full(2048, T), seed=1)
    job.run(5)
    sw = 20
    ms = _timed(lambda: job.run(sw))
    st = job.stats()
    return {
        "grad_ms_B1024_L16": grad_ms, "free_energy_ms_B1024_L16": fwd_ms,
        "exact_sample_acceptance": acc0, "train_epochs": epochs, "train_steps": r.steps, "train_s": train_s,
        "adam_lr": lr, "minibatch": 20, "replay_update": 200,
        "loss_phys_init": loss0, "loss_phys_trained": loss1,
        "loss_union_init": u0, "loss_union_trained": u1,
        "loss_union_by_epoch": [round(e["loss_tot_after"], 3) for e in h[::10]] + [round(h[-1]["loss_tot_after"], 3)],
        "epochs_lowering_their_loss": sum(e["loss_tot_after"] < e["loss_tot_before"] for e in h),
        "transfer_L128_chains2048_site_sweeps_per_s": 2048 * 128 * 128 * sw / (ms * 1e-3),
        "transfer_acceptance": float(st["n_acc"].sum() / st["sweeps"].sum())}


def kitaev_training_and_transfer(L=6, L_big=12, T=0.3):
    """Sec. IV: a Kitaev CRBM (K=8, C=3, 3x3) pre-trained on random gauge
    configurations at L=6, finished on samples it drew itself (persistent
    replicas; Alg. 1 with the replay buffer, the parameters of the epoch with
    the lowest loss kept), then used at L=12 (128 chains): exchange acceptance
    of the initial, pre-trained and trained filters with the refreshed replica."""
    import torch

    from paper_2008_05401_amd import api, train, workloads as WL
    t0 = time.perf_counter()
    pre, fin, x, acc_self, xr = train.kitaev_pretrain_and_train(L, T, n_random=4096, n_phys=512, pre_epochs=10,
                                                                epochs=10, sweeps=200, seed=0)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    f0 = WL.alg1_init_filters(8, 3, seed=0, C=3)
    nlp = train.kitaev_nlp(T)
    z8, z3 = torch.zeros(8, device="cuda"), torch.zeros(3, device="cuda")
    W0 = torch.tensor(f0.W, device="cuda")
    nx, nr = nlp(x), nlp(xr)
    out = {"L_train": L, "T": T, "train_s": train_s, "self_sample_acceptance": acc_self,
           "loss_random_states": {"initial": train.full_loss_nlp(xr, nr, W0, z8, z3),
                                  "pretrained": train.full_loss_nlp(xr, nr, pre.W, pre.hbias, pre.vbias)},
           "loss_self_samples": {"initial": train.full_loss_nlp(x, nx, W0, z8, z3),
                                 "pretrained": train.full_loss_nlp(x, nx, pre.W, pre.hbias, pre.vbias),
                                 "trained": train.full_loss_nlp(x, nx, fin.W, fin.hbias, fin.vbias)},
           # the quantity Alg. 1 minimises, over x_phys U x_RBM with the final buffer
           "loss_union": {"initial": train.union_loss(fin, x, nx, W0, z8, z3),
                          "pretrained": train.union_loss(fin, x, nx, pre.W, pre.hbias, pre.vbias),
                          "trained": train.union_loss(fin, x, nx, fin.W, fin.hbias, fin.vbias)},
           "fine_training_loss_by_epoch": [round(e["loss_tot_after"], 4) for e in fin.history],
           "fine_training_best_epoch": fin.best_epoch}
    for name, (W, hb, vb) in (("initial", (f0.W, f0.hbias, f0.vbias)), ("pretrained", (pre.W, pre.hbias, pre.vbias)),
                              ("trained", (fin.W, fin.hbias, fin.vbias))):
        job = api.Job(api.CRBMParams(W, hb, vb), api.KITAEV, L_big, np.full(128, T), seed=5)
        job.run(4)
        st = job.stats()
        out[f"acceptance_L{L_big}_{name}"] = float(st["n_acc"].sum() / st["sweeps"].sum())
        job.close()
    out["open_boundary"] = kitaev_open_boundary(pre, L_big, T)
    return out


def kitaev_open_boundary(periodic, L, T, n_edge=3):
    """Sec. IV.B at L=12, open columns: a locally connected CRBM (3 unshared
    filter banks per side) started from the periodic pre-trained CRBM,
    retrained on 256 samples it drew itself (40 exchange-corrected sweeps,
    6 epochs of Alg. 1); exchange acceptance with the refreshed replica (128
    chains, 4 sweeps) of the periodic CRBM, the initial and the retrained
    LCRBM, and the loss of Eq. (loss) on the samples."""
    import torch

    from paper_2008_05401_amd import api, train
    t0 = time.perf_counter()
    init, fin, x = train.kitaev_open_transfer(periodic, L, T, n_edge=n_edge, n_phys=256, sweeps=40, epochs=6)
    torch.cuda.synchronize()
    out = {"L": L, "T": T, "n_edge": n_edge, "retrain_s": time.perf_counter() - t0}
    nlp = train.kitaev_nlp(T, boundary=1)
    nx = nlp(x)
    out["loss_open_samples"] = {"initial": train.full_loss_nlp(x, nx, init.W, init.hbias, init.vbias),
                                "retrained": train.full_loss_nlp(x, nx, fin.W, fin.hbias, fin.vbias)}
    # the quantity Alg. 1 minimises: the loss over the samples and the final replay buffer
    out["loss_union"] = {"initial": train.union_loss(fin, x, nx, init.W, init.hbias, init.vbias),
                         "retrained": train.union_loss(fin, x, nx, fin.W, fin.hbias, fin.vbias),
                         "best_epoch": fin.best_epoch}
    cases = (("periodic_crbm", api.CRBMParams(periodic.W, periodic.hbias, periodic.vbias)),
             ("lcrbm_initial", api.CRBMParams(init.W, init.hbias, init.vbias)),
             ("lcrbm_retrained", api.CRBMParams(fin.W, fin.hbias, fin.vbias)))
    for name, p in cases:
        job = api.Job(p, api.KITAEV, L, np.full(128, T), seed=6, boundary=1)
        job.run(1)
        ms = _timed(lambda: job.run(3)) / 3
        st = job.stats()
        out[f"acceptance_{name}"] = float(st["n_acc"].sum() / st["sweeps"].sum())
        out[f"ms_per_sweep_{name}"] = ms
        job.close()
    return out


def graph_blocks(sweeps=2000, blocks=(1, 10), burnin=200):
    return [graph_block(sweeps, b, burnin) for b in blocks]


def graph_block(sweeps, block, burnin):
    """The small configuration advanced in short sweep blocks (launch-bound):
    eager launches against one HIP graph holding all the blocks; both jobs must
    end in identical states and records."""
    import torch

    from paper_2008_05401_amd import api
    p = api.CRBMParams.from_filters(WL_small_filters())
    mk = lambda: api.Job(p, api.ISING, 8, np.full(64, 2.269), seed=0, burnin=burnin)  # noqa: E731
    eager, graphed = mk(), mk()
    g = api.SweepGraph([graphed], sweeps // block, block)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(sweeps // block):
        eager.run(block)
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0
    t0 = time.perf_counter()
    g.launch()
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    same = bool(torch.equal(eager.state, graphed.state)) and eager.stats().tobytes() == graphed.stats().tobytes()
    g.close()
    return {"sweeps": sweeps, "sweeps_per_block": block, "launches": sweeps // block,
            "eager_wall_s": t_eager, "graph_wall_s": t_graph, "identical": same}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--block", type=int, default=100, help="sweeps per kernel launch")
    ap.add_argument("--chains", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-served", action="store_true", help="skip the served-jobs measurement")
    ap.add_argument("--no-extra", action="store_true", help="skip the Kitaev and training measurements")
    ap.add_argument("--served-jobs", type=int, default=1000)
    ap.add_argument("--served-rate", type=float, default=200.0)
    ap.add_argument("--served-warmup", type=float, default=2.0)
    ap.add_argument("--only-kitaev", action="store_true",
                    help="run only the Kitaev sweep measurements (for profiling) and print them")
    ap.add_argument("--gpu-warm-ms", type=float, default=400.0,
                    help="run a throw-away job this long right before the timed steps (clocks of the sweep kernel)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this size first (scale for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); chains are independent, so the "
              f"path shards across GPUs without communication; this benchmark measures one GPU only.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2008_05401_amd import api, workloads as WL

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.only_kitaev:
        print(json.dumps({"kitaev": kitaev()}), flush=True)
        return
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    L, K, C, Lw = 64, 8, 1, 5
    n = args.chains
    seed = 0
    f = WL.random_filters(K, C, Lw, 0.05, seed=seed)
    T = WL.ising_temperatures_linspace(32, 1.5, 3.5, n)
    burnin = args.warmup + args.steps // 10
    job = api.Job(api.CRBMParams.from_filters(f), api.ISING, L, T, seed=seed, burnin=burnin)

    def run(total):
        done = 0
        while done < total:
            b = min(args.block, total - done)
            job.run(b)
            done += b

    # clocks first, then the measured job's own warm-up sweeps, so that its state is the
    # last data the GPU touched before the timed launches
    warm_s = gpu_warm(api, f, L, T, args.gpu_warm_ms * 1e-3, seed + 12345) if args.gpu_warm_ms > 0 else 0.0
    run(args.warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    launches = []
    t0 = time.perf_counter()
    done = 0
    while done < args.steps:
        b = min(args.block, args.steps - done)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        job.run(b)
        e1.record(stream)
        launches.append((b, e0, e1))
        done += b
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = job.stats()

    # per-launch kernel time from HIP events on the launch stream; the roofline is taken
    # over the launches of the most common length (all of them unless the last is short)
    lengths = [b for b, _, _ in launches]
    sweeps_per_launch = max(set(lengths), key=lengths.count)
    durs = [e0.elapsed_time(e1) * 1e-3 for (b, e0, e1) in launches if b == sweeps_per_launch]
    avg_launch_s = float(np.mean(durs))
    ops_site = select_adds_per_site_sweep(K, C, Lw)
    achieved = ops_site * n * L * L * sweeps_per_launch / avg_launch_s / 1e12
    # state read and written once (int8 per site) plus the per-chain records read and written
    algo_bytes = 2.0 * n * L * L + 2.0 * n * 160

    site_sweeps = n * L * L * args.steps
    value = site_sweeps / wall
    acc = float(st["n_acc"].sum() / max(1, st["sweeps"].sum()))
    valu = None
    if kernel_sources_sha256() == MEASURED_VALU["sources_sha256"] and (n, L) == (4096, 64):
        v = MEASURED_VALU["by_sweeps_per_launch"].get(sweeps_per_launch)
        if v is not None:
            valu = dict(v, sweeps_per_launch=sweeps_per_launch, source=MEASURED_VALU["source"])
    out = {
        "metric": "MH-accepted CRBM sweeps·sites/sec on 1 GPU",
        "value": value,
        "unit": "site-sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched Ising L=64, 4096 chains x 32 temperatures in [1.5,3.5], CRBM K=8 5x5 "
                               "filters ~N(0,0.05), CRBM-Gibbs+MH sweep with E/M/C accumulators",
                   "L": L, "chains": n, "K": K, "Lw": Lw, "sweeps_per_launch": sweeps_per_launch,
                   "launches_timed": len(launches), "gibbs_k": 1, "seed": seed,
                   "gpu_warm_s": warm_s},
        "acceptance": acc,
        "fp64_rechecks_per_site_sweep": float(st["n_recheck"].sum()) / (n * L * L * (args.steps + args.warmup)),
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_VECTOR_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
            "traffic": measured_traffic_bytes(n, L, sweeps_per_launch),
            "traffic_unit": "HBM bytes per launch",
            "algorithmic_bytes_per_launch": algo_bytes,
            "kernel_avg_ms": avg_launch_s * 1e3,
            "sweeps_per_launch": sweeps_per_launch,
            "algorithmic_ops_per_site_sweep": ops_site,
            "op": "FP32 select-add on a binary input, one flop each (3 passes x K C Lw^2 taps)",
            "hbm_algorithmic_GBps": algo_bytes / avg_launch_s / 1e9,
            "hbm_frac": algo_bytes / avg_launch_s / 1e9 / PEAK_HBM_GBS,
            "valu_issue_frac": valu["valu_issue_fraction"] if valu else None,
        },
    }
    lds_tbs = lds_table_bytes_per_site_sweep(K, C, Lw) * n * L * L * sweeps_per_launch / avg_launch_s / 1e12
    out["lds"] = {"table_bytes_per_site_sweep": lds_table_bytes_per_site_sweep(K, C, Lw), "achieved": lds_tbs,
                  "peak": PEAK_LDS_TBS, "unit": "TB/s", "frac": lds_tbs / PEAK_LDS_TBS}
    # the binding resource: VALU issue slots (one wave64 instruction per 4 cycles per SIMD)
    out["valu_issue"] = valu
    if not args.no_extra:
        # the timed sweeps start from a random state, so "acceptance" above is a
        # transient at short runs; the same chains after a long burn-in give the
        # steady-state rate of the batched workload
        burn, over = 3000, 1000
        run(burn)
        s0 = job.stats()
        run(over)
        s1 = job.stats()
        out["acceptance_steady"] = {"value": float((s1["n_acc"].sum() - s0["n_acc"].sum()) / (n * over)),
                                    "after_sweeps": args.warmup + args.steps + burn, "over_sweeps": over}
        out["kitaev"] = kitaev()
        out["autocorrelation"] = autocorrelation_times()
        out["frbm"] = frbm()
        out["analytic_per_temperature"] = analytic_per_temperature()
        out["small_config"] = small_config()
        out["small_config_graph_blocks"] = graph_blocks()
        out["tempering"] = tempering()
        out["training"] = training_and_transfer()
        out["kitaev_training"] = kitaev_training_and_transfer()
    if not args.no_served:
        del job
        out["served"] = served(args.served_jobs, args.served_rate, args.served_warmup, capacity=value)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(f, T, L, seed, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
