"""Seeded synthetic inputs for the CRBM sampler (filters, temperature grids,
job streams).

This module creates input DATA only; it holds none of the sampler's
arithmetic, so both the GPU path and the CPU oracle can be fed from it.

* random filters: ``numpy.random.default_rng(seed).normal(0, std, (K, C, Lw, Lw))``
  as float32, biases zero (the workloads of the benchmark configurations);
* the exact Ising -> CRBM kernels of App. C (analytical solution): two 2x2
  kernels [[W,0],[W,0]] and [[W,W],[0,0]], hidden bias -W, visible bias -2W,
  with W = +-W_min(beta) and W_min = log(2 e^{2 beta}(sqrt(e^{4 beta}-1)+e^{2 beta})-1);
  optionally zero-padded into a larger (K, Lw) shape, which adds a constant
  to F and leaves the distribution unchanged;
* the initialisation of Alg. 1 ("Train the RBM"): W ~ N(0, 2/(K Lw^2)), biases 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Filters:
    W: np.ndarray      # float32 [K][C][Lw][Lw], or [banks][K][C][Lw][Lw] for a locally connected CRBM
    hbias: np.ndarray  # float32 [K], or [banks][K]
    vbias: np.ndarray  # float32 [C]

    @property
    def K(self):
        return self.W.shape[-4]

    @property
    def C(self):
        return self.W.shape[-3]

    @property
    def Lw(self):
        return self.W.shape[-1]

    @property
    def banks(self):
        return 1 if self.W.ndim == 4 else self.W.shape[0]


def random_filters(K: int, C: int, Lw: int, std: float, seed: int = 0) -> Filters:
    rng = np.random.default_rng(seed)
    W = rng.normal(0.0, std, (K, C, Lw, Lw)).astype(np.float32)
    return Filters(W, np.zeros(K, np.float32), np.zeros(C, np.float32))


def random_filters_with_bias(K: int, C: int, Lw: int, std: float, bias_std: float, seed: int = 0) -> Filters:
    rng = np.random.default_rng(seed)
    W = rng.normal(0.0, std, (K, C, Lw, Lw)).astype(np.float32)
    hb = rng.normal(0.0, bias_std, K).astype(np.float32)
    vb = rng.normal(0.0, bias_std, C).astype(np.float32)
    return Filters(W, hb, vb)


def alg1_init_filters(K: int, Lw: int, seed: int = 0, C: int = 1) -> Filters:
    """Initial parameters of Alg. 1: W ~ N(m=0, sigma=2/(K Lw^2)), biases 0."""
    return random_filters(K, C, Lw, 2.0 / (K * Lw * Lw), seed)


def w_min(beta: float) -> float:
    """Smallest |W| of the exact Ising kernels of App. C (= 2 arccosh(e^{2 beta}))."""
    e2 = math.exp(2.0 * beta)
    return math.log(2.0 * e2 * (math.sqrt(e2 * e2 - 1.0) + e2) - 1.0)


def analytic_ising_filters(T: float, sign: int = +1, K: int = 2, Lw: int = 2) -> Filters:
    """Exact Ising kernels of App. C at temperature T, zero-padded to (K, Lw)."""
    assert K >= 2 and Lw >= 2
    W = sign * w_min(1.0 / T)
    f = np.zeros((K, 1, Lw, Lw), np.float32)
    f[0, 0, 0, 0] = W
    f[0, 0, 1, 0] = W
    f[1, 0, 0, 0] = W
    f[1, 0, 0, 1] = W
    hb = np.zeros(K, np.float32)
    hb[:2] = -W
    vb = np.array([-2.0 * W], np.float32)
    return Filters(f, hb, vb)


def ising_temperatures_linspace(n_temps: int, lo: float, hi: float, n_chains: int) -> np.ndarray:
    """Temperatures of the batched Ising workload: linspace(lo, hi, n_temps);
    chain g gets T[g // (n_chains // n_temps)]."""
    grid = np.linspace(lo, hi, n_temps)
    per = n_chains // n_temps
    assert per * n_temps == n_chains
    return np.repeat(grid, per).astype(np.float64)


def kitaev_temperatures(n_chains: int, lo: float = 0.005, hi: float = 0.05) -> np.ndarray:
    """Log-uniform grid T_g = lo (hi/lo)^{g/(n-1)}, g = 0..n-1."""
    g = np.arange(n_chains, dtype=np.float64)
    return lo * (hi / lo) ** (g / max(n_chains - 1, 1))


@dataclass
class Job:
    job_id: int
    arrival_s: float
    L: int
    T: float
    n_chains: int
    n_sweeps: int
    seed: int


def served_job_stream(n_jobs: int, rate_per_s: float = 200.0, n_sweeps: int = 20, seed: int = 0,
                      sizes=(16, 32, 64, 128, 256), t_lo: float = 1.8, t_hi: float = 2.8,
                      chains_lo: int = 64, chains_hi: int = 1024):
    """Poisson arrivals (exponential gaps), L uniform over `sizes`, T uniform,
    chain count log-uniform in [chains_lo, chains_hi]; job id doubles as seed."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, n_jobs)
    arr = np.cumsum(gaps)
    Ls = rng.choice(np.asarray(sizes), n_jobs)
    Ts = rng.uniform(t_lo, t_hi, n_jobs)
    nc = np.rint(np.exp(rng.uniform(math.log(chains_lo), math.log(chains_hi), n_jobs))).astype(int)
    return [Job(i, float(arr[i]), int(Ls[i]), float(Ts[i]), int(nc[i]), n_sweeps, i) for i in range(n_jobs)]


def random_states(n: int, C: int, L: int, seed: int = 0, p_up: float = 0.5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.where(rng.random((n, C, L, L)) < p_up, 1, -1).astype(np.int8)


def ar1_series(n: int, length: int, phi: float, seed: int = 0) -> np.ndarray:
    """n stationary AR(1) series x_{i+1} = phi x_i + e_i, e ~ N(0, 1), started
    from the stationary law N(0, 1/(1-phi^2)); [n, length] float64.  Its
    integrated autocorrelation time is (1+phi) / (2 (1-phi))."""
    rng = np.random.default_rng(seed)
    e = rng.standard_normal((n, length))
    x = np.empty((n, length))
    x[:, 0] = e[:, 0] / math.sqrt(1.0 - phi * phi)
    for i in range(1, length):
        x[:, i] = phi * x[:, i - 1] + e[:, i]
    return x


def lcrbm_from_crbm(f: Filters, n_edge: int, edge_std: float = 0.0, seed: int = 0) -> Filters:
    """Filter banks of a locally connected CRBM started from a periodic CRBM
    (Sec. IV.B starts the open-boundary machine from the periodic one): bank 0
    and the 2 n_edge edge banks are copies of f, the edge banks plus
    N(0, edge_std) noise."""
    assert f.W.ndim == 4
    nb = 1 + 2 * n_edge
    rng = np.random.default_rng(seed)
    W = np.repeat(f.W[None], nb, 0).astype(np.float32)
    hb = np.repeat(f.hbias.reshape(1, -1), nb, 0).astype(np.float32)
    if edge_std > 0 and n_edge > 0:
        W[1:] += rng.normal(0.0, edge_std, W[1:].shape).astype(np.float32)
        hb[1:] += rng.normal(0.0, edge_std, hb[1:].shape).astype(np.float32)
    return Filters(W, hb, f.vbias.copy())


def random_frbm(K: int, C: int, L: int, std: float, bias_std: float = 0.0, seed: int = 0) -> Filters:
    """A fully connected RBM on an L x L lattice of C channels: W[K][C][L][L]
    ~ N(0, std), hbias[K] and vbias[C][L][L] ~ N(0, bias_std)."""
    rng = np.random.default_rng(seed)
    W = rng.normal(0.0, std, (K, C, L, L)).astype(np.float32)
    hb = rng.normal(0.0, bias_std, K).astype(np.float32) if bias_std > 0 else np.zeros(K, np.float32)
    vb = rng.normal(0.0, bias_std, (C, L, L)).astype(np.float32) if bias_std > 0 else np.zeros((C, L, L), np.float32)
    return Filters(W, hb, vb)
