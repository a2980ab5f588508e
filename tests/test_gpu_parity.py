"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.

Bars (stated per test): integer energies, states and accept decisions are
bit-exact; floating-point values agree to 1e-5 relative or better; gradients
per element within the bar of tests/grad_bar.py.  The
oracle's tie counters must be zero for bitwise comparisons to be meaningful
(a decision within 1e-6 of its threshold may legitimately differ).
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


def _o_crbm(orc, f):
    return orc.CRBM(f.W, f.hbias, f.vbias)


def _p(api, f):
    return api.CRBMParams.from_filters(f)


def _compare_records(gpu, ora, target, f_rtol=1e-9):
    for name in ("sweeps", "n_acc", "n_meas"):
        assert np.array_equal(gpu[name], ora[name]), name
    if target == 0:
        for name in ("E", "sumE", "sumE2", "sumM", "sumAbsM", "sumM2"):
            assert np.array_equal(gpu[name], ora[name]), name
    else:
        for name in ("S", "Ef", "Cf", "kE", "kE2", "kCf"):
            np.testing.assert_allclose(gpu[name], ora[name], rtol=1e-8, atol=1e-8, err_msg=name)
    # F: FP64 on the generic path; on the bit-packed Ising path a float32-term sum whose
    # rigorous error bound is kept in F_bound; both far inside the 1e-5 relative bar
    tol = gpu["F_bound"] + f_rtol * (1.0 + np.abs(ora["F"]))
    assert np.all(np.abs(gpu["F"] - ora["F"]) <= tol), np.abs(gpu["F"] - ora["F"]).max()
    assert np.all(np.abs(gpu["F"] - ora["F"]) <= 1e-5 * np.abs(ora["F"]) + 1e-9)


# ----------------------------------------------------------------- stand-alone ops
@pytest.mark.parametrize("K,C,Lw,L", [(4, 1, 3, 8), (8, 1, 5, 64), (2, 3, 2, 5), (8, 3, 3, 6), (3, 1, 1, 7),
                                      (8, 1, 5, 256)])
def test_free_energy_parity(orc, api, K, C, Lw, L):
    f = WL.random_filters_with_bias(K, C, Lw, 0.3, 0.2, seed=K + L)
    B = 3 if L == 256 else 17
    x = WL.random_states(B, C, L, seed=L)
    Fo = orc.free_energy(_o_crbm(orc, f), x)
    Fg = api.free_energy(_p(api, f), torch.from_numpy(x).cuda()).cpu().numpy()
    np.testing.assert_allclose(Fg, Fo, rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("L", [1, 2, 3, 8, 17, 64, 256])
def test_ising_energy_parity(orc, api, L):
    x = WL.random_states(33, 1, L, seed=L)
    x[0] = 1
    Eo = orc.target(orc.ISING, x)
    Eg = api.ising_energy(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.array_equal(Eg.astype(np.int64), Eo)


@pytest.mark.parametrize("C,L", [(3, 1), (3, 2), (3, 3), (1, 4), (1, 5), (3, 6), (3, 7), (1, 8), (3, 9), (3, 12),
                                 (1, 12)])
def test_kitaev_weight_parity(orc, api, C, L):
    B = 6
    x = WL.random_states(B, C, L, seed=L + C)
    x[0] = 1
    T = np.geomspace(0.005, 0.5, B)
    J = (1.0, 0.9, 1.1)
    So = orc.target(orc.KITAEV, x, T=T, J=J)
    Sg = api.kitaev_weight(torch.from_numpy(x).cuda(), T, J).cpu().numpy()
    np.testing.assert_allclose(Sg, So, rtol=1e-10, atol=1e-8)


@pytest.mark.parametrize("K,C,Lw,L,B", [(8, 1, 5, 16, 64), (2, 3, 3, 5, 7), (4, 1, 3, 8, 1), (8, 1, 5, 16, 1024)])
def test_grad_parity(orc, api, K, C, Lw, L, B):
    f = WL.random_filters_with_bias(K, C, Lw, 0.2, 0.3, seed=1)
    x = WL.random_states(B, C, L, seed=2)
    g = np.random.default_rng(3).standard_normal(B).astype(np.float32)
    m = _o_crbm(orc, f)
    dWo, dhbo, dvbo = orc.grad(m, x, g.astype(np.float64))
    dWg, dhbg, dvbg = api.grad(_p(api, f), torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda())
    A = grad_abs(orc, m, x, g)
    r = R_SIG64 if sigma_is_fp64(K, C, Lw, L) else R_SIG32
    for got, ref, a in zip((dWg, dhbg, dvbg), (dWo, dhbo, dvbo), A):
        assert_grad_close(got.cpu().numpy(), ref, a, r)


def test_grad_parity_float32_sigma(orc, api):
    # K L^2 doubles beyond LDS (K=8, L=64): sigma is kept as float32
    K, C, Lw, L, B = 8, 1, 5, 64, 24
    assert not sigma_is_fp64(K, C, Lw, L)
    f = WL.random_filters_with_bias(K, C, Lw, 0.2, 0.3, seed=4)
    x = WL.random_states(B, C, L, seed=5)
    g = np.random.default_rng(6).standard_normal(B).astype(np.float32)
    m = _o_crbm(orc, f)
    ref = orc.grad(m, x, g.astype(np.float64))
    got = api.grad(_p(api, f), torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda())
    A = grad_abs(orc, m, x, g)
    for a, rr, aa in zip(got, ref, A):
        assert_grad_close(a.cpu().numpy(), rr, aa, R_SIG32)


def test_grad_empty_batch(api):
    f = WL.random_filters(4, 1, 3, 0.1)
    x = torch.zeros((0, 1, 8, 8), dtype=torch.int8, device="cuda")
    dW, dhb, dvb = api.grad(_p(api, f), x, torch.zeros(0, device="cuda"))
    assert float(dW.abs().sum()) == 0.0 and float(dhb.abs().sum()) == 0.0 and float(dvb.abs().sum()) == 0.0


# ----------------------------------------------------------------- chains
def _run_pair(orc, api, f, target, L, T, seed, sweeps, gibbs_k=1, burnin=0, J=(1.0, 1.0, 1.0), blocks=(None,),
              state=None, chain_offset=0):
    n = len(T)
    job = api.Job(_p(api, f), target, L, T, seed=seed, gibbs_k=gibbs_k, burnin=burnin, J=J, state=state,
                  chain_offset=chain_offset)
    ch = orc.Chains(_o_crbm(orc, f), target, L, T, seed=seed, gibbs_k=gibbs_k, burnin=burnin, J=J, state=state,
                    g0=chain_offset)
    if state is None:
        torch.cuda.synchronize()
        assert np.array_equal(job.state.cpu().numpy(), ch.state), "initial states differ"
    init = job.stats()
    _compare_records(init, ch.rec, target)
    done = 0
    for b in blocks:
        nb = sweeps - done if b is None else b
        job.run(nb)
        ch.run(nb)
        done += nb
    st = job.stats()
    assert np.array_equal(job.state.cpu().numpy(), ch.state)
    _compare_records(st, ch.rec, target)
    assert ch.ties[1] == 0 and ch.ties[0] == 0
    assert n == st.shape[0]
    return job, ch, st


def test_ising_small_config_trajectory(orc, api):
    # L=8, K=4 filters 3x3 ~ N(0, 0.1), T=2.269, 64 chains (shortened run)
    f = WL.random_filters(4, 1, 3, 0.1, seed=0)
    _run_pair(orc, api, f, 0, 8, np.full(64, 2.269), seed=0, sweeps=200, burnin=20)


def test_ising_exact_kernel_high_acceptance(orc, api):
    T = 2.269
    f = WL.analytic_ising_filters(T, K=8, Lw=5)
    job, ch, st = _run_pair(orc, api, f, 0, 16, np.full(32, T), seed=5, sweeps=60, burnin=10, blocks=(7, 23, None))
    assert st["n_acc"].sum() / st["sweeps"].sum() > 0.95


def test_ising_batched_shape_with_bias(orc, api):
    f = WL.random_filters_with_bias(8, 1, 5, 0.05, 0.05, seed=2)
    T = WL.ising_temperatures_linspace(8, 1.5, 3.5, 64)
    _run_pair(orc, api, f, 0, 64, T, seed=11, sweeps=6, burnin=2)


@pytest.mark.parametrize("L,K,Lw,gk", [(3, 2, 3, 2), (5, 3, 2, 1), (12, 4, 5, 3), (1, 1, 1, 1), (2, 2, 2, 2)])
def test_ising_ragged_shapes(orc, api, L, K, Lw, gk):
    f = WL.random_filters_with_bias(K, 1, Lw, 0.5, 0.3, seed=L)
    _run_pair(orc, api, f, 0, L, np.linspace(1.0, 4.0, 9), seed=L, sweeps=40, gibbs_k=gk, burnin=5)


def test_ising_given_state_and_offset(orc, api):
    f = WL.random_filters_with_bias(4, 1, 3, 0.3, 0.1, seed=9)
    s0 = WL.random_states(10, 1, 8, seed=4)
    _run_pair(orc, api, f, 0, 8, np.full(10, 2.0), seed=3, sweeps=25, state=s0, chain_offset=1000)


@pytest.mark.parametrize("C,L", [(3, 6), (1, 6), (3, 3), (3, 2), (1, 4), (3, 5), (1, 7), (3, 8)])
def test_kitaev_trajectory(orc, api, C, L):
    f = WL.random_filters_with_bias(8, C, 3 if L >= 3 else 2, 0.1, 0.05, seed=C)
    T = WL.kitaev_temperatures(16)
    _run_pair(orc, api, f, 1, L, T, seed=7, sweeps=6, burnin=1)


def test_kitaev_l12_trajectory(orc, api):
    f = WL.random_filters(8, 3, 3, 0.1, seed=0)
    T = WL.kitaev_temperatures(4)
    _run_pair(orc, api, f, 1, 12, T, seed=1, sweeps=2)


@pytest.mark.parametrize("C,L", [(3, 9), (1, 10), (3, 11)])
def test_kitaev_block_path_trajectory(orc, api, C, L):
    """L = 9..11: the packed-LDS eigen-step of 512-thread workgroups at the
    other slot counts of its rank-2 update."""
    f = WL.random_filters(8, C, 3, 0.1, seed=L)
    T = WL.kitaev_temperatures(4)
    _run_pair(orc, api, f, 1, L, T, seed=2, sweeps=2)


def test_many_jobs_equal_alone(orc, api):
    fa = WL.random_filters(4, 1, 3, 0.2, seed=1)
    fb = WL.random_filters(8, 1, 5, 0.05, seed=2)
    fk = WL.random_filters(8, 3, 3, 0.1, seed=3)
    mk = lambda: [api.Job(_p(api, fa), 0, 8, np.full(5, 2.2), seed=1),  # noqa: E731
                  api.Job(_p(api, fb), 0, 16, np.full(7, 2.5), seed=2, chain_offset=40),
                  api.Job(_p(api, fk), 1, 4, np.full(3, 0.05), seed=3)]
    alone = mk()
    for j in alone:
        j.run(9)
    mixed = mk()
    api.run_many(mixed, 4)
    api.run_many(mixed, 5)
    for a, m in zip(alone, mixed):
        assert np.array_equal(a.state.cpu().numpy(), m.state.cpu().numpy())
        sa, sm = a.stats(), m.stats()
        for name in ("sweeps", "n_acc", "E", "sumE", "sumM"):
            assert np.array_equal(sa[name], sm[name])
        np.testing.assert_allclose(sa["F"], sm["F"], rtol=1e-12)
        np.testing.assert_allclose(sa["S"], sm["S"], rtol=1e-12)


def test_invalid_arguments_raise(api):
    from paper_2008_05401_amd import _lib
    f = WL.random_filters(4, 1, 3, 0.1)
    with pytest.raises(_lib.CRBMError):
        api.Job(_p(api, f), 0, 2, np.full(2, 2.0))           # Lw > L
    f3 = WL.random_filters(4, 3, 3, 0.1)
    with pytest.raises(_lib.CRBMError):
        api.Job(_p(api, f3), 0, 8, np.full(2, 2.0))          # Ising with C=3
    with pytest.raises(_lib.CRBMError):
        api.Job(_p(api, f3), 1, 25, np.full(2, 0.1))         # Kitaev jobs stop at L = 24
