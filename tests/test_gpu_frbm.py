"""GPU parity of the fully connected RBM (the FRBM of the Sec. IV
comparison) through the C ABI against the FP64 oracle: free energy (1e-12),
gradient (1e-5 of the largest component), trajectories with an FRBM proposal
(states, decisions, integer sums bit-exact; Kitaev sums 1e-8), and the
equivalence of a CRBM with its structured dense expansion on the GPU."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from grad_bar import R_SIG64, assert_grad_close, grad_abs  # noqa: E402
from paper_2008_05401_amd import workloads as WL  # noqa: E402
from test_oracle_frbm import dense_from_filters  # noqa: E402


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_05401_amd import api as A
    return A


def _both(orc, api, f):
    return orc.FRBM(f.W, f.hbias, f.vbias), api.CRBMParams.from_filters(f, dense=True)


@pytest.mark.parametrize("K,C,L", [(64, 1, 8), (128, 1, 8), (16, 3, 4), (7, 1, 5), (256, 1, 4), (3, 3, 1)])
def test_free_energy_parity(orc, api, K, C, L):
    f = WL.random_frbm(K, C, L, 0.2, 0.1, seed=K + L)
    mo, mg = _both(orc, api, f)
    x = WL.random_states(11, C, L, seed=L)
    np.testing.assert_allclose(api.free_energy(mg, torch.from_numpy(x).cuda()).cpu().numpy(), orc.free_energy(mo, x),
                               rtol=1e-12, atol=1e-10)


def test_crbm_equals_structured_frbm_on_gpu(api):
    L = 6
    f = WL.random_filters_with_bias(3, 1, 3, 0.4, 0.2, seed=1)
    g = dense_from_filters(f, L)
    x = torch.from_numpy(WL.random_states(16, 1, L, seed=2)).cuda()
    Fc = api.free_energy(api.CRBMParams.from_filters(f), x)
    Fd = api.free_energy(api.CRBMParams.from_filters(g, dense=True), x)
    torch.testing.assert_close(Fd, Fc, rtol=1e-12, atol=1e-11)


@pytest.mark.parametrize("K,C,L,B", [(64, 1, 8, 32), (16, 3, 4, 7), (5, 1, 3, 1)])
def test_grad_parity(orc, api, K, C, L, B):
    f = WL.random_frbm(K, C, L, 0.3, 0.2, seed=3)
    mo, mg = _both(orc, api, f)
    x = WL.random_states(B, C, L, seed=4)
    g = np.random.default_rng(5).standard_normal(B).astype(np.float32)
    ref = orc.grad(mo, x, g.astype(np.float64))
    got = api.grad(mg, torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda())
    A = grad_abs(orc, mo, x, g)
    for a, rr, aa in zip(got, ref, A):
        # the dense RBM keeps its K sigma values in FP64
        assert_grad_close(a.cpu().numpy(), rr, aa, R_SIG64)


def test_autograd_dense(api):
    f = WL.random_frbm(32, 1, 6, 0.2, 0.1, seed=6)
    W = torch.from_numpy(f.W).cuda().requires_grad_()
    hb = torch.from_numpy(f.hbias).cuda().requires_grad_()
    vb = torch.from_numpy(f.vbias).cuda().requires_grad_()
    x = torch.from_numpy(WL.random_states(5, 1, 6, seed=7)).cuda()
    api.crbm_free_energy_fn(x, W, hb, vb, None, True).sum().backward()
    dW, dhb, dvb = api.grad(api.CRBMParams(W.detach(), hb.detach(), vb.detach(), dense=True), x,
                            torch.ones(5, device="cuda"))
    assert torch.equal(W.grad, dW) and torch.equal(hb.grad, dhb) and torch.equal(vb.grad, dvb.reshape(vb.shape))


def _compare(gpu, ora, target):
    for name in ("sweeps", "n_acc", "n_meas"):
        assert np.array_equal(gpu[name], ora[name]), name
    if target != 1:
        for name in ("E", "sumE", "sumE2", "sumM", "sumAbsM", "sumM2"):
            assert np.array_equal(gpu[name], ora[name]), name
    else:
        for name in ("S", "Ef", "Cf", "kE", "kE2", "kCf"):
            np.testing.assert_allclose(gpu[name], ora[name], rtol=1e-8, atol=1e-8, err_msg=name)
    np.testing.assert_allclose(gpu["F"], ora["F"], rtol=1e-9, atol=1e-9)


def _run_pair(orc, api, f, target, L, T, seed, blocks, gibbs_k=1, burnin=0, replica=False):
    mo, mg = _both(orc, api, f)
    job = api.Job(mg, target, L, T, seed=seed, gibbs_k=gibbs_k, burnin=burnin, replica=replica)
    ch = orc.Chains(mo, target, L, T, seed=seed, gibbs_k=gibbs_k, burnin=burnin, replica=replica)
    torch.cuda.synchronize()
    _compare(job.stats(), ch.rec, target)
    for b in blocks:
        job.run(b)
        ch.run(b)
    assert np.array_equal(job.state.cpu().numpy(), ch.state)
    if replica:
        assert np.array_equal(job.rbm_state.cpu().numpy(), ch.rbm)
    st = job.stats()
    _compare(st, ch.rec, target)
    assert ch.ties[0] == 0 and ch.ties[1] == 0
    return job, ch


@pytest.mark.parametrize("K,L,gk", [(64, 8, 1), (13, 5, 2), (256, 4, 1)])
def test_ising_trajectory_with_frbm(orc, api, K, L, gk):
    f = WL.random_frbm(K, 1, L, 0.1, 0.1, seed=K)
    _run_pair(orc, api, f, 0, L, np.linspace(1.8, 3.0, 10), seed=K, blocks=(6, 14), gibbs_k=gk, burnin=3)


@pytest.mark.parametrize("K,C,L", [(64, 1, 8), (128, 1, 8), (48, 3, 4)])
def test_kitaev_trajectory_with_frbm(orc, api, K, C, L):
    f = WL.random_frbm(K, C, L, 0.05, 0.05, seed=K + C)
    _run_pair(orc, api, f, 1, L, WL.kitaev_temperatures(8), seed=2, blocks=(2, 3), burnin=1)


def test_kitaev_frbm_replica_and_tempering(orc, api):
    f = WL.random_frbm(64, 1, 8, 0.05, 0.05, seed=9)
    T = np.repeat(np.geomspace(0.01, 0.1, 3), 2)
    job, ch = _run_pair(orc, api, f, 1, 8, T, seed=4, blocks=(2,), replica=True)
    for r in range(3):
        job.tempering_swap(2, r)
        ch.tempering_swap(2, r)
        job.run(1)
        ch.run(1)
    assert np.array_equal(job.state.cpu().numpy(), ch.state)
    _compare(job.stats(), ch.rec, 1)
    assert np.array_equal(job.stats()["n_swap"], ch.rec["n_swap"])
