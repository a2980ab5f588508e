"""GPU parity of the open-boundary path (Sec. IV.B) through the C ABI: the
locally connected CRBM (filter banks, windows that stop at the column edge)
and the open-column Ising and Kitaev targets, against the FP64 oracle.

Bars as in the periodic parity tests: states, decisions and integer sums
bit-exact; F within 1e-12 relative (stand-alone FP64 kernel) or the cached
F within 1e-9; Kitaev S 1e-10 relative and chain sums 1e-8; gradients per element within the bar of tests/grad_bar.py (formerly 1e-5 of
the largest component.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from grad_bar import R_SIG32, R_SIG64, assert_grad_close, grad_abs, sigma_is_fp64  # noqa: E402
from paper_2008_05401_amd import workloads as WL  # noqa: E402


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_05401_amd import api as A
    return A


def rand_lcrbm(K, C, Lw, n_edge, seed, std=0.3, bias=0.2):
    f = WL.random_filters_with_bias(K, C, Lw, std, bias, seed=seed)
    return WL.lcrbm_from_crbm(f, n_edge, edge_std=std, seed=seed + 100)


def _both(orc, api, f, open_cols=None):
    return (orc.CRBM(f.W, f.hbias, f.vbias, open_cols=open_cols),
            api.CRBMParams.from_filters(f, open_cols=open_cols))


@pytest.mark.parametrize("K,C,Lw,L,ne,open_cols", [
    (4, 1, 3, 8, 1, None), (8, 1, 5, 16, 3, None), (2, 3, 2, 5, 2, None), (3, 1, 3, 7, 0, True),
    (4, 1, 3, 6, 3, None), (3, 3, 3, 6, 1, False), (8, 1, 5, 64, 3, None)])
def test_free_energy_parity(orc, api, K, C, Lw, L, ne, open_cols):
    f = rand_lcrbm(K, C, Lw, ne, seed=K + L)
    mo, mg = _both(orc, api, f, open_cols)
    x = WL.random_states(9, C, L, seed=L)
    Fo = orc.free_energy(mo, x)
    Fg = api.free_energy(mg, torch.from_numpy(x).cuda()).cpu().numpy()
    np.testing.assert_allclose(Fg, Fo, rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("L", [1, 2, 3, 8, 17, 64])
def test_open_ising_energy_parity(orc, api, L):
    x = WL.random_states(21, 1, L, seed=L)
    x[0] = 1
    Eo = orc.target(orc.ISING, x, boundary=1)
    Eg = api.ising_energy(torch.from_numpy(x).cuda(), boundary=1).cpu().numpy()
    assert np.array_equal(Eg.astype(np.int64), Eo)


@pytest.mark.parametrize("C,L", [(3, 1), (3, 2), (1, 3), (3, 4), (1, 6), (3, 9), (3, 12)])
def test_open_kitaev_weight_parity(orc, api, C, L):
    B = 5
    x = WL.random_states(B, C, L, seed=L + C)
    x[0] = 1
    T = np.geomspace(0.005, 0.5, B)
    J = (1.0, 0.9, 1.1)
    So = orc.target(orc.KITAEV, x, T=T, J=J, boundary=1)
    Sg = api.kitaev_weight(torch.from_numpy(x).cuda(), T, J, boundary=1).cpu().numpy()
    np.testing.assert_allclose(Sg, So, rtol=1e-10, atol=1e-8)


@pytest.mark.parametrize("K,C,Lw,L,ne,B", [(4, 1, 3, 8, 1, 16), (2, 3, 2, 6, 3, 5), (8, 1, 5, 16, 3, 64)])
def test_grad_parity(orc, api, K, C, Lw, L, ne, B):
    f = rand_lcrbm(K, C, Lw, ne, seed=1)
    mo, mg = _both(orc, api, f)
    x = WL.random_states(B, C, L, seed=2)
    g = np.random.default_rng(3).standard_normal(B).astype(np.float32)
    ref = orc.grad(mo, x, g.astype(np.float64))
    got = api.grad(mg, torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda())
    A = grad_abs(orc, mo, x, g)
    r = R_SIG64 if sigma_is_fp64(K, C, Lw, L, 1 + 2 * ne) else R_SIG32
    for a, rr, aa in zip(got, ref, A):
        a = a.cpu().numpy()
        assert a.shape == rr.shape
        assert_grad_close(a, rr, aa, r)


def test_autograd_function_with_banks(api):
    f = rand_lcrbm(4, 1, 3, 2, seed=4)
    W = torch.from_numpy(f.W).cuda().requires_grad_()
    hb = torch.from_numpy(f.hbias).cuda().requires_grad_()
    vb = torch.from_numpy(f.vbias).cuda().requires_grad_()
    x = torch.from_numpy(WL.random_states(6, 1, 8, seed=5)).cuda()
    F = api.crbm_free_energy_fn(x, W, hb, vb)
    F.sum().backward()
    dW, dhb, dvb = api.grad(api.CRBMParams(W.detach(), hb.detach(), vb.detach()), x, torch.ones(6, device="cuda"))
    assert torch.equal(W.grad, dW) and torch.equal(hb.grad, dhb) and torch.equal(vb.grad, dvb)


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


def _run_pair(orc, api, f, target, L, T, seed, sweeps, boundary, open_cols=None, gibbs_k=1, burnin=0,
              replica=False, blocks=None):
    mo, mg = _both(orc, api, f, open_cols)
    job = api.Job(mg, target, L, T, seed=seed, gibbs_k=gibbs_k, burnin=burnin, boundary=boundary, replica=replica)
    ch = orc.Chains(mo, target, L, T, seed=seed, gibbs_k=gibbs_k, burnin=burnin, boundary=boundary,
                    replica=replica)
    torch.cuda.synchronize()
    assert np.array_equal(job.state.cpu().numpy(), ch.state)
    _compare(job.stats(), ch.rec, target)
    for b in (blocks or (sweeps,)):
        job.run(b)
        ch.run(b)
    assert np.array_equal(job.state.cpu().numpy(), ch.state)
    if replica:
        assert np.array_equal(job.rbm_state.cpu().numpy(), ch.rbm)
    st = job.stats()
    _compare(st, ch.rec, target)
    assert ch.ties[0] == 0 and ch.ties[1] == 0
    return job, ch, st


@pytest.mark.parametrize("L,K,Lw,ne", [(8, 4, 3, 1), (16, 8, 5, 3), (5, 2, 2, 2), (12, 4, 3, 0)])
def test_open_ising_trajectory_with_lcrbm(orc, api, L, K, Lw, ne):
    f = rand_lcrbm(K, 1, Lw, ne, seed=L)
    _run_pair(orc, api, f, 0, L, np.linspace(1.5, 3.5, 12), seed=L, sweeps=30, boundary=1,
              open_cols=True, burnin=5, blocks=(7, 23))


def test_open_target_with_periodic_crbm(orc, api):
    # an open-boundary target with the plain periodic CRBM still samples it exactly
    # (MH corrects the proposal); the bit-packed kernel must not take this job
    f = WL.random_filters_with_bias(8, 1, 5, 0.05, 0.05, seed=3)
    _run_pair(orc, api, f, 0, 16, np.full(16, 2.3), seed=2, sweeps=20, boundary=1)


def test_lcrbm_proposal_on_periodic_target(orc, api):
    f = rand_lcrbm(4, 1, 3, 2, seed=5)
    _run_pair(orc, api, f, 0, 8, np.full(10, 2.2), seed=3, sweeps=25, boundary=0)


@pytest.mark.parametrize("C,L,ne", [(1, 6, 3), (3, 6, 1), (1, 4, 2), (3, 3, 1), (3, 5, 2), (1, 7, 3), (3, 8, 1)])
def test_open_kitaev_trajectory(orc, api, C, L, ne):
    f = rand_lcrbm(6, C, 3 if L >= 3 else 2, ne, seed=C, std=0.1, bias=0.05)
    _run_pair(orc, api, f, 1, L, WL.kitaev_temperatures(12), seed=7, sweeps=6, boundary=1, burnin=1)


def test_open_kitaev_l12_trajectory(orc, api):
    f = rand_lcrbm(8, 1, 3, 3, seed=0, std=0.1, bias=0.0)
    _run_pair(orc, api, f, 1, 12, WL.kitaev_temperatures(4), seed=1, sweeps=2, boundary=1)


def test_open_kitaev_replica_and_tempering(orc, api):
    L, C = 6, 1
    f = rand_lcrbm(6, C, 3, 3, seed=9, std=0.1, bias=0.05)
    T = np.repeat(np.geomspace(0.01, 0.1, 4), 3)
    job, ch, _ = _run_pair(orc, api, f, 1, L, T, seed=4, sweeps=3, boundary=1, replica=True)
    for r in range(4):
        job.tempering_swap(3, r)
        ch.tempering_swap(3, r)
        job.run(2)
        ch.run(2)
    assert np.array_equal(job.state.cpu().numpy(), ch.state)
    assert np.array_equal(job.rbm_state.cpu().numpy(), ch.rbm)
    st = job.stats()
    _compare(st, ch.rec, 1)
    assert np.array_equal(st["n_swap"], ch.rec["n_swap"])
    assert ch.ties[2] == 0


def test_open_trace(orc, api):
    f = rand_lcrbm(4, 1, 3, 1, seed=2)
    mo, mg = _both(orc, api, f)
    T = np.full(6, 2.4)
    job = api.Job(mg, 0, 8, T, seed=5, boundary=1)
    ch = orc.Chains(mo, 0, 8, T, seed=5, boundary=1)
    job.record_trace(32)
    job.run(10)
    ch.run(10, log_energy=True)
    assert np.array_equal(job.trace().cpu().numpy(), ch.energy_log)
