"""The guarded Kitaev MH decision (Sec. IV, F(eta); App. B, Eq. (acceptance)).

The fast eigen-step squares M (eigenvalues of M^T M), so the cached S carries
a rigorous bound S_bound (the Householder backward error times the largest
slope of log 2cosh(beta sqrt(lambda) / 2) in lambda); an MH decision with
|log r - log u| inside the sum of the bounds is taken again from singular
values of M by one-sided Jacobi.  Checked here:
  - the bound holds against LAPACK's SVD of the oracle's matrix (random gauge
    fields, L = 6, 12, 24, T = 0.005 and 0.05) and is not vacuous at L = 6;
  - with the band forced open (mh_band_min huge) every decision goes through
    the Jacobi route, and trajectories still match the oracle bit for bit;
  - trajectories at the benchmarked sizes and the lowest temperatures:
    L = 24 (16 chains x 2 sweeps, T in [0.005, 0.05]) and L = 12 (128 chains
    x 10 sweeps), states and decisions bit-exact, no oracle ties.
The oracle computes S by one-sided Jacobi too (its own code), in the order of
the paper's formula."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2008_05401_amd import workloads as WL  # noqa: E402


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_05401_amd import api as A
    return A


def S_of(eps, T):
    x = 0.5 * eps / T
    return float(np.sum(np.abs(x) + np.log1p(np.exp(-2 * np.abs(x)))))


@pytest.mark.parametrize("L,C", [(5, 1), (6, 3), (8, 3), (9, 1), (12, 3), (24, 1)])
def test_bound_holds_against_lapack(orc, api, L, C):
    T = np.array([0.005, 0.05, 0.005, 0.05])
    u = WL.random_states(4, C, L, seed=100 + L)
    u[0] = 1  # flux-free: zero modes when 3 | L
    f = WL.random_filters(4, C, 3, 0.1, seed=0)
    job = api.Job(api.CRBMParams.from_filters(f), api.KITAEV, L, T, state=u)
    st = job.stats()
    for g in range(4):
        eps = np.linalg.svd(orc.kitaev_matrix(u[g]), compute_uv=False)
        Sref = S_of(eps, T[g])
        err = abs(st["S"][g] - Sref)
        # LAPACK's own error (|eps| ~ 6, beta <= 200) is ~1e-12 relative
        assert err <= st["S_bound"][g] + 1e-11 * abs(Sref), (g, err, st["S_bound"][g])
        assert 0 < st["S_bound"][g] < np.inf
    if L == 6:
        # small lattices: the bound is far inside the 1e-6 tie band
        assert st["S_bound"].max() < 1e-6


@pytest.mark.parametrize("L,n,sweeps,C", [(6, 32, 6, 3), (12, 8, 2, 3), (16, 2, 1, 1)])
def test_forced_jacobi_route_matches_oracle(orc, api, L, n, sweeps, C):
    f = WL.random_filters_with_bias(8, C, 3, 0.1, 0.05, seed=L)
    T = WL.kitaev_temperatures(n)
    job = api.Job(api.CRBMParams.from_filters(f), api.KITAEV, L, T, seed=5, mh_band_min=1e300)
    ch = orc.Chains(orc.CRBM(f.W, f.hbias, f.vbias), orc.KITAEV, L, T, seed=5)
    job.run(sweeps)
    ch.run(sweeps)
    st = job.stats()
    assert np.array_equal(job.state.cpu().numpy(), ch.state)
    assert np.array_equal(st["n_acc"], ch.rec["n_acc"])
    # every MH decision was re-taken on the Jacobi route (Gibbs re-checks may add more)
    assert np.all(st["n_recheck"] >= sweeps)
    # the cached S is then the Jacobi one: it agrees with the oracle's Jacobi closely
    np.testing.assert_allclose(st["S"], ch.rec["S"], rtol=1e-11, atol=1e-9)
    assert np.all(st["S_bound"] == 0.0)
    for name in ("Ef", "Cf", "kE", "kCf"):
        np.testing.assert_allclose(st[name], ch.rec[name], rtol=1e-9, atol=1e-9, err_msg=name)
    assert ch.ties[0] == 0 and ch.ties[1] == 0


def test_forced_exact_route_ising(orc, api):
    # the bit-packed Ising kernel with every MH decision on FP64 free energies
    f = WL.random_filters_with_bias(8, 1, 5, 0.05, 0.05, seed=21)
    T = np.linspace(1.5, 3.5, 16)
    job = api.Job(api.CRBMParams.from_filters(f), api.ISING, 32, T, seed=7, burnin=2, mh_band_min=1e300)
    ch = orc.Chains(orc.CRBM(f.W, f.hbias, f.vbias), orc.ISING, 32, T, seed=7, burnin=2)
    job.run(12)
    ch.run(12)
    st = job.stats()
    assert np.array_equal(job.state.cpu().numpy(), ch.state)
    for name in ("n_acc", "E", "sumE", "sumE2", "sumM", "sumAbsM", "sumM2"):
        assert np.array_equal(st[name], ch.rec[name]), name
    assert np.all(st["n_recheck"] >= 12)
    assert np.all(st["F_bound"] == 0.0)
    np.testing.assert_allclose(st["F"], ch.rec["F"], rtol=1e-12)
    assert ch.ties[0] == 0 and ch.ties[1] == 0


def _trajectory(orc, api, L, n, sweeps, seed, C=3):
    f = WL.random_filters(8, C, 3, 0.1, seed=0)
    T = WL.kitaev_temperatures(n)
    job = api.Job(api.CRBMParams.from_filters(f), api.KITAEV, L, T, seed=seed)
    ch = orc.Chains(orc.CRBM(f.W, f.hbias, f.vbias), orc.KITAEV, L, T, seed=seed)
    job.run(sweeps)
    ch.run(sweeps)
    st = job.stats()
    assert np.array_equal(job.state.cpu().numpy(), ch.state)
    assert np.array_equal(st["n_acc"], ch.rec["n_acc"])
    for name in ("S", "Ef", "Cf", "kE", "kE2", "kCf"):
        np.testing.assert_allclose(st[name], ch.rec[name], rtol=1e-8, atol=1e-8, err_msg=name)
    np.testing.assert_allclose(st["F"], ch.rec["F"], rtol=1e-9)
    assert ch.ties[0] == 0 and ch.ties[1] == 0
    # the fast S stays within its bound of the oracle's Jacobi S
    fast = st["S_bound"] > 0
    assert np.all(np.abs(st["S"] - ch.rec["S"])[fast] <= st["S_bound"][fast] + 1e-10 * np.abs(ch.rec["S"][fast]))
    return st


def test_trajectory_L24_low_temperature(orc, api):
    st = _trajectory(orc, api, 24, 16, 2, seed=8)
    assert st["S_bound"].max() < 1e-2


def test_trajectory_L12_128_chains_10_sweeps(orc, api):
    st = _trajectory(orc, api, 12, 128, 10, seed=9)
    assert 0 < st["n_acc"].sum() < 128 * 10
