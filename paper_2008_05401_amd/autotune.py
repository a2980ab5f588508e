"""Autotuner of the bit-packed Ising sweep's tile shape.

For a lattice shape (L, K, Lw) it times every candidate (rows per lane block,
threads per workgroup) on a synthetic batch with HIP events and keeps the
fastest; the choices are stored as JSON (`tuning.json` next to this file) and
handed to the library with `crbm_set_tuning` when `api` is imported.

Tile shapes change only the speed: random numbers are indexed by (unit, sweep,
chain), so every candidate produces bit-identical chains (the parity tests
check this).

    python -m paper_2008_05401_amd.autotune --shape 64,8,5 --shape 128,8,5 --out tuning.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning.json")
ROWS = (1, 2, 4)
THREADS = (64, 256, 512, 1024)


def candidates(L: int):
    out = []
    for rows in ROWS:
        if 4 * rows > L:
            continue
        blocks = L * L // (4 * rows)
        for nt in THREADS:
            if nt > 64 and blocks < nt // 2:
                continue  # mostly idle lanes
            out.append((rows, nt))
    return out


def time_candidate(L, K, Lw, rows, nt, n_chains, sweeps, reps=3, seed=0, warm_s=0.2):
    import torch

    from . import api, workloads
    _lib.crbm_set_tuning(L, K, Lw, rows, nt)
    f = workloads.random_filters(K, 1, Lw, 0.05, seed=seed)
    T = np.linspace(1.5, 3.5, n_chains)
    job = api.Job(api.CRBMParams.from_filters(f), api.ISING, L, T, seed=seed)
    # run the candidate until the GPU holds its clocks under it (a cold start or a
    # few milliseconds of idle cost 10-20% on the first launches), then time it
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < warm_s:
        job.run(sweeps)
        torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        job.run(sweeps)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    job.close()
    return float(np.median(times))


def tune_shape(L, K, Lw, n_chains=None, sweeps=20, verbose=True):
    if n_chains is None:
        n_chains = 4096 if L <= 64 else (1024 if L == 128 else 256)
    best = None
    results = []
    for rows, nt in candidates(L):
        ms = time_candidate(L, K, Lw, rows, nt, n_chains, sweeps)
        rate = n_chains * L * L * sweeps / (ms * 1e-3)
        results.append({"rows": rows, "threads": nt, "ms": ms, "site_sweeps_per_s": rate})
        if verbose:
            print(f"L={L} K={K} Lw={Lw} rows={rows} threads={nt}: {ms:.3f} ms  {rate:.3e} site-sweeps/s",
                  flush=True)
        if best is None or ms < best["ms"]:
            best = results[-1]
    _lib.crbm_clear_tuning()
    return best, results


def apply(path: str = DEFAULT_CACHE) -> int:
    """Load tile choices from `path` into the library; returns the number applied."""
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        data = json.load(f)
    n = 0
    for key, v in data.get("shapes", {}).items():
        L, K, Lw = (int(x) for x in key.split(","))
        _lib.crbm_set_tuning(L, K, Lw, int(v["rows"]), int(v["threads"]))
        n += 1
    return n


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--shape", action="append", required=True, help="L,K,Lw")
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--sweeps", type=int, default=20)
    args = ap.parse_args()
    data = {"device": "gfx950", "created": time.strftime("%Y-%m-%d %H:%M:%S"), "shapes": {}}
    if os.path.exists(args.out):
        with open(args.out) as f:
            data["shapes"].update(json.load(f).get("shapes", {}))
    for sh in args.shape:
        L, K, Lw = (int(x) for x in sh.split(","))
        best, results = tune_shape(L, K, Lw, sweeps=args.sweeps)
        data["shapes"][f"{L},{K},{Lw}"] = {"rows": best["rows"], "threads": best["threads"], "ms": best["ms"],
                                          "site_sweeps_per_s": best["site_sweeps_per_s"], "candidates": results}
    with open(args.out, "w") as f:
        json.dump(data, f, indent=1)
    print(json.dumps({k: (v["rows"], v["threads"]) for k, v in data["shapes"].items()}))


if __name__ == "__main__":
    main()
