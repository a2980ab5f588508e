"""Exact finite-lattice results for the periodic 2D Ising model, computed from
first principles (brute-force enumeration, row transfer matrix), used to pin
the oracle's sampler.  Nothing here calls the oracle.

E(s) = -sum_<ij> s_i s_j (J = 1, each bond of the periodic L x L lattice once),
P(s) ~ exp(-beta E(s)).  E takes the values -2L^2 + 2 n, n = number of
unsatisfied bonds.
"""
from __future__ import annotations

import numpy as np


def all_states(L: int) -> np.ndarray:
    n = L * L
    idx = np.arange(2 ** n, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(n)[None, :]) & 1
    return (2 * bits - 1).astype(np.int8).reshape(-1, L, L)


def energies_bruteforce(states: np.ndarray) -> np.ndarray:
    s = states.astype(np.int64)
    return -(s * np.roll(s, -1, axis=-1)).sum(axis=(-1, -2)) - (s * np.roll(s, -1, axis=-2)).sum(axis=(-1, -2))


def dos_bruteforce(L: int) -> np.ndarray:
    E = energies_bruteforce(all_states(L))
    n = (E + 2 * L * L) // 2
    return np.bincount(n, minlength=2 * L * L + 1).astype(np.float64)


def dos_transfer(L: int) -> np.ndarray:
    """Density of states g[n] (n unsatisfied bonds) by a row transfer matrix
    that carries the energy histogram, summed over the first row."""
    R = 2 ** L
    rows = ((np.arange(R)[:, None] >> np.arange(L)[None, :]) & 1) * 2 - 1
    u_row = ((rows != np.roll(rows, -1, axis=1)).sum(1))            # unsatisfied bonds within a row
    u_pair = (rows[:, None, :] != rows[None, :, :]).sum(2)           # between consecutive rows
    nmax = 2 * L * L
    step = u_pair + u_row[None, :]                                    # [r, r'] added when r' follows r
    masks = [(step == d).astype(np.float64) for d in range(2 * L + 1)]
    g = np.zeros(nmax + 1)
    for r0 in range(R):
        dp = np.zeros((R, nmax + 1))
        dp[r0, u_row[r0]] = 1.0
        for _ in range(L - 1):
            new = np.zeros_like(dp)
            for d, Md in enumerate(masks):
                if d == 0:
                    new += Md.T @ dp
                else:
                    new[:, d:] += Md.T @ dp[:, :-d]
            dp = new
        for r in range(R):
            d = u_pair[r, r0]
            if d == 0:
                g += dp[r]
            else:
                g[d:] += dp[r, :-d]
    return g


def thermo(g: np.ndarray, L: int, T: float):
    """Exact <E>, <E^2> and C = beta^2 (<E^2> - <E>^2) / L^2."""
    beta = 1.0 / T
    E = -2.0 * L * L + 2.0 * np.arange(g.shape[0])
    w = np.log(np.maximum(g, 1e-300)) - beta * E
    w[g == 0] = -np.inf
    w -= w.max()
    p = np.exp(w)
    p /= p.sum()
    e1 = float((p * E).sum())
    e2 = float((p * E * E).sum())
    return e1, e2, beta * beta * (e2 - e1 * e1) / (L * L)


def boltzmann_weights(states: np.ndarray, T: float) -> np.ndarray:
    E = energies_bruteforce(states).astype(np.float64)
    w = -E / T
    w -= w.max()
    p = np.exp(w)
    return p / p.sum()


def chi2_pvalue(obs: np.ndarray, expected_prob: np.ndarray, min_expected: float = 5.0):
    """Pearson chi-square of counts against probabilities; bins with small
    expectation are pooled into one.  Returns (chi2, dof, p-value)."""
    from scipy import stats
    n = obs.sum()
    exp = expected_prob * n
    big = exp >= min_expected
    o = list(obs[big])
    e = list(exp[big])
    if (~big).any():
        o.append(obs[~big].sum())
        e.append(exp[~big].sum())
    o = np.asarray(o, np.float64)
    e = np.asarray(e, np.float64)
    chi2 = float(((o - e) ** 2 / e).sum())
    dof = len(o) - 1
    return chi2, dof, float(stats.chi2.sf(chi2, dof))


def state_index(states: np.ndarray) -> np.ndarray:
    """Index of +-1 states in the ordering of all_states()."""
    b = (states.reshape(states.shape[0], -1) > 0).astype(np.int64)
    return (b << np.arange(b.shape[1])[None, :]).sum(1)


__all__ = ["all_states", "energies_bruteforce", "dos_bruteforce", "dos_transfer", "thermo",
           "boltzmann_weights", "chi2_pvalue", "state_index"]
