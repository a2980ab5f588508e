"""GPU parity of the exchange-correction cycle (persistent CRBM replica) and of
the temperature swaps, through the C ABI, against the FP64 oracle.

Bars: states (physical and replica), accept decisions, swap decisions,
integer sums and swap counts bit-exact; F within its rigorous float32 bound
(bit-packed Ising path) and 1e-9 relative otherwise; Kitaev S, Ef, Cf and
their sums to 1e-8 relative.  Oracle tie counters must be zero."""
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


def _compare(job, ch, target):
    st = job.stats()
    r = ch.rec
    assert np.array_equal(job.state.cpu().numpy(), ch.state)
    if ch.rbm is not None:
        assert np.array_equal(job.rbm_state.cpu().numpy(), ch.rbm)
    for name in ("sweeps", "n_acc", "n_meas", "n_swap"):
        assert np.array_equal(st[name], r[name]), name
    if target == 0:
        for name in ("E", "sumE", "sumE2", "sumM", "sumAbsM", "sumM2"):
            assert np.array_equal(st[name], r[name]), name
    else:
        for name in ("S", "Ef", "Cf", "kE", "kE2", "kCf"):
            np.testing.assert_allclose(st[name], r[name], rtol=1e-8, atol=1e-8, err_msg=name)
    tol = st["F_bound"] + 1e-9 * (1.0 + np.abs(r["F"]))
    assert np.all(np.abs(st["F"] - r["F"]) <= tol), np.abs(st["F"] - r["F"]).max()
    assert not ch.ties.any(), ch.ties
    return st


def _pair(orc, api, f, target, L, T, seed, replica=True, gibbs_k=1, burnin=0, state=None, rbm_state=None,
          chain_offset=0):
    job = api.Job(api.CRBMParams.from_filters(f), target, L, T, seed=seed, gibbs_k=gibbs_k, burnin=burnin,
                  state=state, rbm_state=rbm_state, replica=replica, chain_offset=chain_offset)
    ch = orc.Chains(orc.CRBM(f.W, f.hbias, f.vbias), target, L, T, seed=seed, gibbs_k=gibbs_k, burnin=burnin,
                    state=state, rbm_state=rbm_state, replica=replica, g0=chain_offset)
    return job, ch


@pytest.mark.parametrize("L,K,Lw,gk", [(16, 8, 5, 1), (32, 8, 5, 2), (64, 8, 5, 1), (8, 4, 3, 1), (5, 3, 2, 2),
                                       (6, 4, 3, 1)])
def test_replica_trajectory_ising(orc, api, L, K, Lw, gk):
    # L in {8, 16, 32, 64}: bit-packed kernel; L = 5, 6: byte-lattice kernel
    f = WL.random_filters_with_bias(K, 1, Lw, 0.5 / Lw, 0.1, seed=L + K)
    T = np.linspace(1.5, 3.5, 12)
    job, ch = _pair(orc, api, f, 0, L, T, seed=L * 3 + 1, gibbs_k=gk, burnin=2)
    for b in (3, 5):
        job.run(b)
        ch.run(b)
    st = _compare(job, ch, 0)
    assert st["n_acc"].sum() > 0
    # the replica is not simply the physical state
    assert not np.array_equal(job.rbm_state.cpu().numpy(), job.state.cpu().numpy())


def test_replica_exact_kernel_recheck_path(orc, api):
    # acceptance ~ 1 with the App. C kernel: the exchange decides inside the float32 band often
    T = 2.269
    f = WL.analytic_ising_filters(T, K=8, Lw=5)
    job, ch = _pair(orc, api, f, 0, 16, np.full(8, T), seed=4)
    job.run(10)
    ch.run(10)
    st = _compare(job, ch, 0)
    assert st["n_acc"].sum() / st["sweeps"].sum() > 0.9


def test_replica_given_states(orc, api):
    f = WL.random_filters_with_bias(4, 1, 3, 0.3, 0.1, seed=9)
    s0 = WL.random_states(6, 1, 16, seed=4)
    y0 = WL.random_states(6, 1, 16, seed=5)
    job, ch = _pair(orc, api, f, 0, 16, np.full(6, 2.0), seed=3, state=s0, rbm_state=y0, chain_offset=77)
    job.run(7)
    ch.run(7)
    _compare(job, ch, 0)


@pytest.mark.parametrize("C,L", [(3, 3), (3, 6), (1, 6)])
def test_replica_kitaev(orc, api, C, L):
    f = WL.random_filters_with_bias(8, C, 3, 0.1, 0.05, seed=C + L)
    T = WL.kitaev_temperatures(8)
    job, ch = _pair(orc, api, f, 1, L, T, seed=2, burnin=1)
    job.run(5)
    ch.run(5)
    _compare(job, ch, 1)


@pytest.mark.parametrize("L,replica", [(32, True), (16, False), (6, True)])
def test_tempering_ising(orc, api, L, replica):
    n_ladders, rungs = 8, 5
    f = WL.random_filters_with_bias(8 if L >= 8 else 4, 1, 5 if L >= 8 else 3, 0.06, 0.05, seed=L)
    T = np.repeat(np.linspace(1.8, 3.2, rungs), n_ladders)
    job, ch = _pair(orc, api, f, 0, L, T, seed=11, replica=replica, burnin=2)
    for rnd in range(6):
        job.run(2)
        ch.run(2)
        job.tempering_swap(n_ladders, rnd)
        ch.tempering_swap(n_ladders, rnd)
    st = _compare(job, ch, 0)
    assert st["n_swap"].sum() > 0


@pytest.mark.parametrize("C,L", [(3, 3), (3, 6)])
def test_tempering_kitaev(orc, api, C, L):
    n_ladders, rungs = 4, 4
    f = WL.random_filters_with_bias(8, C, 3, 0.1, 0.05, seed=5)
    T = np.repeat(np.geomspace(0.02, 0.2, rungs), n_ladders)
    job, ch = _pair(orc, api, f, 1, L, T, seed=13)
    for rnd in range(4):
        job.run(1)
        ch.run(1)
        job.tempering_swap(n_ladders, rnd)
        ch.tempering_swap(n_ladders, rnd)
    st = _compare(job, ch, 1)
    assert st["n_swap"].sum() > 0
    # cached S of the swapped states equals a fresh evaluation at the slot's temperature
    S = api.kitaev_weight(job.state, T).cpu().numpy()
    np.testing.assert_allclose(st["S"], S, rtol=1e-10)


def test_tempering_swap_validation(api):
    f = WL.random_filters(4, 1, 3, 0.1)
    job = api.Job(api.CRBMParams.from_filters(f), 0, 8, np.full(6, 2.0), seed=1)
    with pytest.raises(api.C.CRBMError):
        job.tempering_swap(4, 0)   # 4 does not divide 6
    with pytest.raises(api.C.CRBMError):
        job.tempering_swap(3, -1)
    job.tempering_swap(6, 1)       # one rung: no pairs, a no-op
    assert job.stats()["n_swap"].sum() == 0
    g = api.Job(api.CRBMParams.from_filters(f), 2, 8, np.full(2, 2.0), seed=1)
    with pytest.raises(api.C.CRBMError):
        g.tempering_swap(1, 0)
    with pytest.raises(api.C.CRBMError):
        api.Job(api.CRBMParams.from_filters(f), 2, 8, np.full(2, 2.0), seed=1, replica=True)
