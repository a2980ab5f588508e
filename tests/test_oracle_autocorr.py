"""Pins of the oracle's autocorrelation-time estimator against values fixed
by the mathematics: a hand-worked series, exactly periodic series, an
independent library route (numpy.correlate) and the closed form of the AR(1)
process, tau = (1 + phi) / (2 (1 - phi)).  Also pins the oracle's per-sweep
energy log against an energy recomputed from the chain's state."""
import os

import numpy as np
import pytest

from oracle import autocorr as AC
from paper_2008_05401_amd import workloads as WL

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "autocov_tiny.txt")


def test_hand_worked_series():
    rows = np.loadtxt(GOLD)
    c = AC.autocovariance([1.0, 2.0, 4.0], 2)
    for lag, num, den in rows:
        assert c[int(lag)] == pytest.approx(num / den, rel=1e-15, abs=1e-15)


@pytest.mark.parametrize("offset", [0.0, 5.0, -1234.5])
def test_alternating_series_exact(offset):
    # x_i = offset + (-1)^i, even N: mean = offset, C(t) = (-1)^t exactly for every lag
    n = 40
    x = offset + (-1.0) ** np.arange(n)
    c = AC.autocovariance(x, n - 1)
    np.testing.assert_allclose(c, (-1.0) ** np.arange(n), rtol=0, atol=1e-12)
    tau, w = AC.tau_from_autocovariance(c)
    # tau(1) = 1/2 - 1 = -1/2 and 1 >= 6 * (-1/2): the window closes at W = 1
    assert w == 1 and tau == pytest.approx(-0.5)


def test_constant_series_has_no_window():
    c, tau, w = AC.integrated_time(np.full(17, 3.25), 5)
    assert np.all(c == 0.0) and tau == 0.5 and w == -1


def test_period_three_series():
    # x = (a, b, c) repeated: C(t) depends only on t mod 3 at lags where the
    # overlap is whole periods of the pattern: C(3k) = pattern variance
    pat = np.array([1.0, -2.0, 4.0])
    x = np.tile(pat, 30)
    c = AC.autocovariance(x, 60)
    var = ((pat - pat.mean()) ** 2).mean()
    for t in range(0, 61, 3):
        assert c[t] == pytest.approx(var, rel=1e-12)


def test_matches_library_correlation():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(777) * 3 + 1
    y = x - x.mean()
    full = np.correlate(y, y, mode="full")[len(y) - 1:]
    ref = full / (len(y) - np.arange(len(y)))
    np.testing.assert_allclose(AC.autocovariance(x, 400), ref[:401], rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("phi", [0.0, 0.5, 0.9])
def test_ar1_closed_form(phi):
    x = WL.ar1_series(1, 400_000, phi, seed=int(phi * 10) + 1)[0]
    c, tau, w = AC.integrated_time(x, 400)
    exact = (1 + phi) / (2 * (1 - phi))
    assert w > 0
    # Sokal's variance estimate of the windowed estimator, 2 (2W + 1) / N tau^2
    sigma = exact * np.sqrt(2 * (2 * w + 1) / x.shape[0])
    assert abs(tau - exact) < 5 * sigma + exact * phi ** w / (1 - phi), (tau, exact, sigma)
    rho = c / c[0]
    for t in range(1, 6):
        assert abs(rho[t] - phi ** t) < 0.01


def test_energy_log_matches_state_energy(orc):
    # the energy recorded after each sweep is the Ising energy of the state the chain holds
    f = WL.random_filters_with_bias(4, 1, 3, 0.3, 0.1, seed=3)
    ch = orc.Chains(orc.CRBM(f.W, f.hbias, f.vbias), orc.ISING, 6, np.full(5, 2.5), seed=2)
    logs = []
    for _ in range(12):
        ch.run(1, log_energy=True)
        s = ch.state[:, 0].astype(np.int64)
        E = -(s * np.roll(s, -1, -1)).sum((-1, -2)) - (s * np.roll(s, -1, -2)).sum((-1, -2))
        assert np.array_equal(ch.energy_log[:, 0], E.astype(np.float64))
        logs.append(ch.energy_log[:, 0])
    # one call over several sweeps logs the same energies
    ch2 = orc.Chains(orc.CRBM(f.W, f.hbias, f.vbias), orc.ISING, 6, np.full(5, 2.5), seed=2)
    ch2.run(12, log_energy=True)
    assert np.array_equal(ch2.energy_log, np.stack(logs, 1))


def test_energy_log_kitaev_is_fermion_energy(orc):
    f = WL.random_filters(4, 3, 2, 0.1, seed=1)
    ch = orc.Chains(orc.CRBM(f.W, f.hbias, f.vbias), orc.KITAEV, 3, WL.kitaev_temperatures(3), seed=4)
    for _ in range(3):
        ch.run(1, log_energy=True)
        np.testing.assert_array_equal(ch.energy_log[:, 0], ch.rec["Ef"])
