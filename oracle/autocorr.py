"""Integrated autocorrelation time of a Monte Carlo observable series: the
sampler diagnostic by which Sec. III (Ising) and Sec. IV (Kitaev) compare the
CRBM sampler with Metropolis.

TEST INFRASTRUCTURE ONLY (same callers as the rest of this package).

The paper does not state its estimator.  The reading used here is the
standard one for Markov-chain output (Sokal's automatic windowing):
  C(t)   = 1/(N - t) sum_{i < N - t} (x_i - m)(x_{i+t} - m),  m = mean of x
  rho(t) = C(t) / C(0)
  tau(W) = 1/2 + sum_{t=1..W} rho(t)
  W      = the smallest W >= 1 with W >= c * tau(W)  (c = 6 by default)
With no qualifying W up to max_lag (or C(0) = 0) the window is reported as -1
and tau is the sum up to max_lag.  Plain FP64; one dot product per lag.
"""
from __future__ import annotations

import numpy as np


def autocovariance(x, max_lag: int) -> np.ndarray:
    """C(t), t = 0..max_lag, of the 1-D series x (definition above)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    assert 0 <= max_lag < n
    y = x - x.mean()
    out = np.empty(max_lag + 1)
    for t in range(max_lag + 1):
        out[t] = np.dot(y[: n - t], y[t:]) / (n - t)
    return out


def tau_from_autocovariance(c, c_window: float = 6.0):
    """(tau, W) from C(0..max_lag) by automatic windowing."""
    c = np.asarray(c, dtype=np.float64)
    tau = 0.5
    if not c[0] > 0.0:
        return tau, -1
    for t in range(1, c.shape[0]):
        tau += c[t] / c[0]
        if t >= c_window * tau:
            return tau, t
    return tau, -1


def integrated_time(x, max_lag: int, c_window: float = 6.0):
    """(C, tau, W) of the series x."""
    c = autocovariance(x, max_lag)
    tau, w = tau_from_autocovariance(c, c_window)
    return c, tau, w
