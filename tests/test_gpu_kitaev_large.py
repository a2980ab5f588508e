"""Kitaev jobs beyond L = 12 (the eigen-step's M^T M then lives in a per-chain
global scratch, stored in full): S, E_f, C_f of the initial states against
closed forms (Bloch's theorem for the flux-free sector, periodic and open
columns) and against the oracle's matrix with LAPACK's SVD (numpy) for random
gauge fields, 1e-10 relative; one sweep of whole trajectories against the
oracle at L = 13 and 16 (states and decisions bit-exact, sums 1e-8)."""
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


def weights_of(eps, T):
    x = 0.5 * eps / T
    S = np.sum(np.abs(x) + np.log1p(np.exp(-2 * np.abs(x))))
    Ef = -np.sum(0.5 * eps * np.tanh(x))
    Cf = np.sum(x * x / np.cosh(x) ** 2)
    return S, Ef, Cf


def bloch_periodic(L, J):
    q = 2 * np.pi * np.arange(L) / L
    q1, q2 = np.meshgrid(q, q, indexing="ij")
    return (2 * np.abs(J[2] + J[0] * np.exp(1j * q1) + J[1] * np.exp(1j * q2))).ravel()


def bloch_open(L, J):
    S = np.eye(L, k=1)
    out = [np.linalg.svd((2 * J[2] + 2 * J[1] * np.exp(1j * q)) * np.eye(L) + 2 * J[0] * S, compute_uv=False)
           for q in 2 * np.pi * np.arange(L) / L]
    return np.concatenate(out)


def _job_stats(api, state, T, boundary=0, J=(1.0, 1.0, 1.0)):
    C, L = state.shape[1], state.shape[-1]
    f = WL.random_filters(4, C, 3, 0.1, seed=0)
    job = api.Job(api.CRBMParams.from_filters(f), api.KITAEV, L, T, state=state, J=J, boundary=boundary)
    return job.stats()


@pytest.mark.parametrize("L", [13, 16, 24])
@pytest.mark.parametrize("boundary", [0, 1])
def test_flux_free_closed_form(api, L, boundary):
    J = (1.0, 0.9, 1.1)
    T = np.array([0.02, 0.3])
    u = np.ones((2, 3, L, L), np.int8)
    st = _job_stats(api, u, T, boundary, J)
    eps = bloch_open(L, J) if boundary else bloch_periodic(L, J)
    for g in range(2):
        S, Ef, Cf = weights_of(eps, T[g])
        assert st["S"][g] == pytest.approx(S, rel=1e-10)
        assert st["Ef"][g] == pytest.approx(Ef, rel=1e-10)
        assert st["Cf"][g] == pytest.approx(Cf, rel=1e-8, abs=1e-9)


@pytest.mark.parametrize("L,C,boundary", [(13, 3, 0), (16, 1, 1), (16, 3, 0), (24, 1, 0), (24, 3, 1)])
def test_random_gauge_against_lapack(orc, api, L, C, boundary):
    T = np.array([0.01, 0.05, 0.4])
    u = WL.random_states(3, C, L, seed=L + C)
    st = _job_stats(api, u, T, boundary)
    for g in range(3):
        M = orc.kitaev_matrix(u[g], open_cols=bool(boundary))
        eps = np.linalg.svd(M, compute_uv=False)
        S, Ef, Cf = weights_of(eps, T[g])
        assert st["S"][g] == pytest.approx(S, rel=1e-10)
        assert st["Ef"][g] == pytest.approx(Ef, rel=1e-10)


@pytest.mark.parametrize("L,C,boundary", [(13, 3, 0), (16, 1, 1)])
def test_trajectory_against_oracle(orc, api, L, C, boundary):
    f = WL.random_filters_with_bias(6, C, 3, 0.1, 0.05, seed=L)
    T = WL.kitaev_temperatures(3)
    mo = orc.CRBM(f.W, f.hbias, f.vbias)
    job = api.Job(api.CRBMParams.from_filters(f), api.KITAEV, L, T, seed=3, boundary=boundary)
    ch = orc.Chains(mo, orc.KITAEV, L, T, seed=3, boundary=boundary)
    job.run(1)
    ch.run(1)
    assert np.array_equal(job.state.cpu().numpy(), ch.state)
    st = job.stats()
    assert np.array_equal(st["n_acc"], ch.rec["n_acc"])
    for name in ("S", "Ef", "Cf", "kE", "kCf"):
        np.testing.assert_allclose(st[name], ch.rec[name], rtol=1e-8, atol=1e-8, err_msg=name)
    np.testing.assert_allclose(st["F"], ch.rec["F"], rtol=1e-9)
    assert ch.ties[0] == 0 and ch.ties[1] == 0


def test_large_tempering_uses_stored_spectra(orc, api):
    # temperature swaps recompute S from the stored singular values of each chain
    L = 16
    f = WL.random_filters(4, 1, 3, 0.1, seed=1)
    T = np.array([0.02, 0.03, 0.05, 0.08])
    job = api.Job(api.CRBMParams.from_filters(f), api.KITAEV, L, T, seed=2, replica=True)
    job.run(1)
    for r in range(4):
        job.tempering_swap(1, r)
    st = job.stats()
    x = job.state.cpu().numpy()
    for g in range(4):
        eps = np.linalg.svd(orc.kitaev_matrix(x[g]), compute_uv=False)
        S, Ef, _ = weights_of(eps, T[g])
        assert st["S"][g] == pytest.approx(S, rel=1e-10)
        assert st["Ef"][g] == pytest.approx(Ef, rel=1e-10)
