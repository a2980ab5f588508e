"""GPU parity of the bit-packed Ising path (L in {8, 16} or a multiple of 32,
Lw <= 6) against the FP64 oracle: final states, accept counts and integer
accumulators bit-exact, F to 1e-9 relative (the GPU value is the float32-term
sum when no re-check happened, bounded by its own error bound)."""
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


def check_chains(orc, job, ch, f_atol):
    st = job.stats()
    assert np.array_equal(job.state.cpu().numpy(), ch.state)
    for name in ("sweeps", "n_acc", "n_meas", "E", "sumE", "sumE2", "sumM", "sumAbsM", "sumM2"):
        assert np.array_equal(st[name], ch.rec[name]), name
    # F of the current state: float32-term sum within its rigorous bound (F_bound)
    # (FP64 sums in a different order agree to ~1e-13 relative)
    bound = st["F_bound"]
    tol = bound + f_atol + 1e-11 * np.abs(ch.rec["F"])
    assert np.all(np.abs(st["F"] - ch.rec["F"]) <= tol), np.abs(st["F"] - ch.rec["F"]).max()
    assert ch.ties[0] == 0 and ch.ties[1] == 0
    return st


def run_pair(orc, api, f, L, T, seed, sweeps, gibbs_k=1, burnin=0, blocks=None, chain_offset=0):
    job = api.Job(api.CRBMParams.from_filters(f), api.ISING, L, T, seed=seed, gibbs_k=gibbs_k, burnin=burnin,
                  chain_offset=chain_offset)
    ch = orc.Chains(orc.CRBM(f.W, f.hbias, f.vbias), orc.ISING, L, T, seed=seed, gibbs_k=gibbs_k, burnin=burnin,
                    g0=chain_offset)
    for b in (blocks or [sweeps]):
        job.run(b)
        ch.run(b)
    return job, ch


def test_small_config_full(orc, api):
    # L=8, K=4 3x3 filters ~ N(0, 0.1), T=2.269, 64 chains x 2000 sweeps, burn-in 10%
    f = WL.random_filters(4, 1, 3, 0.1, seed=0)
    job, ch = run_pair(orc, api, f, 8, np.full(64, 2.269), seed=0, sweeps=2000, burnin=200,
                       blocks=[500, 500, 1000])
    check_chains(orc, job, ch, 1e-9)


@pytest.mark.parametrize("L,K,Lw,gk,n,sweeps", [
    (16, 8, 5, 1, 32, 30), (32, 8, 5, 1, 16, 10), (32, 4, 1, 1, 8, 20), (32, 2, 6, 2, 8, 10),
    (32, 3, 2, 1, 8, 12), (32, 5, 4, 3, 4, 6), (64, 8, 5, 2, 8, 4), (128, 8, 5, 1, 4, 2), (256, 8, 5, 1, 2, 2),
    (16, 1, 3, 1, 64, 40), (8, 8, 6, 2, 16, 25),
])
def test_shapes(orc, api, L, K, Lw, gk, n, sweeps):
    f = WL.random_filters_with_bias(K, 1, Lw, 0.3 / Lw, 0.1, seed=L + K + Lw)
    T = np.linspace(1.2, 4.0, n)
    job, ch = run_pair(orc, api, f, L, T, seed=L * 7 + Lw, sweeps=sweeps, gibbs_k=gk, burnin=1)
    check_chains(orc, job, ch, 1e-9)


@pytest.mark.parametrize("L", [16, 64])
def test_exact_kernel_mh_recheck_path(orc, api, L):
    # acceptance ~ 1: |log r - log u| is often inside the float32 band, so the
    # FP64 re-evaluation of both free energies decides
    T = 2.269
    f = WL.analytic_ising_filters(T, K=8, Lw=5)
    job, ch = run_pair(orc, api, f, L, np.full(16, T), seed=3, sweeps=24, burnin=4, blocks=[10, 14])
    st = check_chains(orc, job, ch, 1e-9)
    assert st["n_acc"].sum() / st["sweeps"].sum() > 0.9
    assert st["n_recheck"].sum() > 0


def test_batched_config_sampled_chains(orc, api):
    # full-size batched Ising launch (4096 chains, L=64, K=8 5x5 ~ N(0,0.05)); the oracle
    # recomputes a sample of chains one by one from their chain index
    L, n = 64, 4096
    f = WL.random_filters(8, 1, 5, 0.05, seed=0)
    T = WL.ising_temperatures_linspace(32, 1.5, 3.5, n)
    job = api.Job(api.CRBMParams.from_filters(f), api.ISING, L, T, seed=0, burnin=1)
    job.run(3)
    st = job.stats()
    state = job.state.cpu().numpy()
    m = orc.CRBM(f.W, f.hbias, f.vbias)
    for g in (0, 1, 777, 2048, 4095):
        ch = orc.Chains(m, orc.ISING, L, T[g:g + 1], seed=0, burnin=1, g0=g)
        ch.run(3)
        assert np.array_equal(state[g], ch.state[0])
        for name in ("n_acc", "E", "sumE", "sumM2"):
            assert st[name][g] == ch.rec[name][0]


def test_timed_launch_parity(orc, api):
    # the launch bench.py times: 4096 chains, L=64, K=8 5x5 filters ~ N(0, 0.05) (seed 0),
    # 32 temperatures, tuned tile shape, burn-in = warm-up + steps // 10 (driver: 5 + 2);
    # 5 warm-up sweeps, one 100-sweep launch (it crosses the 64-sweep refill of the MH
    # uniforms) and one 20-sweep launch.  Two chains of every temperature block
    # (g = 128 t and 128 t + 127) are recomputed one by one by the oracle.
    from concurrent.futures import ThreadPoolExecutor
    L, n, burnin = 64, 4096, 7
    f = WL.random_filters(8, 1, 5, 0.05, seed=0)
    T = WL.ising_temperatures_linspace(32, 1.5, 3.5, n)
    job = api.Job(api.CRBMParams.from_filters(f), api.ISING, L, T, seed=0, burnin=burnin)
    blocks = (5, 100, 20)
    for b in blocks:
        job.run(b)
    st = job.stats()
    state = job.state.cpu().numpy()
    m = orc.CRBM(f.W, f.hbias, f.vbias)
    picks = [g for t in range(32) for g in (128 * t, 128 * t + 127)]

    def one(g):
        ch = orc.Chains(m, orc.ISING, L, T[g:g + 1], seed=0, burnin=burnin, g0=g)
        for b in blocks:
            ch.run(b)
        return g, ch

    with ThreadPoolExecutor(max_workers=8) as ex:
        done = list(ex.map(one, picks))
    for g, ch in done:
        assert np.array_equal(state[g], ch.state[0]), g
        for name in ("sweeps", "n_acc", "n_meas", "E", "sumE", "sumE2", "sumM", "sumAbsM", "sumM2"):
            assert st[name][g] == ch.rec[name][0], (g, name)
        assert abs(st["F"][g] - ch.rec["F"][0]) <= st["F_bound"][g] + 1e-9 + 1e-11 * abs(ch.rec["F"][0]), g
        assert ch.ties[0] == 0 and ch.ties[1] == 0, g
    # the first sweeps out of the random start accept some proposals
    assert st["n_acc"][picks].sum() > 0


def test_resume_is_bitwise(api):
    f = WL.random_filters(8, 1, 5, 0.05, seed=1)
    T = np.linspace(1.5, 3.5, 32)
    a = api.Job(api.CRBMParams.from_filters(f), api.ISING, 32, T, seed=9, burnin=3)
    a.run(12)
    b = api.Job(api.CRBMParams.from_filters(f), api.ISING, 32, T, seed=9, burnin=3)
    b.run(5)
    # checkpoint: state + records; restore into a fresh job and continue
    saved_state = b.state.clone()
    saved_rec = b.stats_device().clone()
    c = api.Job(api.CRBMParams.from_filters(f), api.ISING, 32, T, seed=9, burnin=3, state=saved_state)
    ws = c.workspace
    base = (ws.data_ptr() + 255) // 256 * 256 - ws.data_ptr()
    ws[base + 256: base + 256 + saved_rec.numel()].copy_(saved_rec)
    c.run(7)
    assert np.array_equal(a.state.cpu().numpy(), c.state.cpu().numpy())
    sa, sc = a.stats(), c.stats()
    for name in ("sweeps", "n_acc", "sumE", "sumE2", "sumM", "E"):
        assert np.array_equal(sa[name], sc[name])


def _filter_sums(f):
    """S_k = |h_b| + sum |W_k| per channel and S_v = |b| + sum |W| (C = 1)."""
    Sk = np.abs(f.hbias.astype(np.float64)) + np.abs(f.W.astype(np.float64)).reshape(f.W.shape[0], -1).sum(1)
    Sv = abs(float(f.vbias[0])) + float(np.abs(f.W.astype(np.float64)).sum())
    return Sk, Sv


@pytest.mark.parametrize("case", ["product_near_limit", "additive_large_filters", "additive_one_channel"])
def test_table_modes(orc, api, case):
    # The kernel evaluates e^{-a} as products of tabulated exponentials while every
    # partial product stays inside float32 range (S_k, S_v < 80, sum_k S_k + K < 80),
    # and as exp2 of tabulated sums otherwise; both must reproduce the oracle.
    rng = np.random.default_rng(11)
    if case == "product_near_limit":
        K, Lw = 2, 5
        W = (rng.choice([-1.0, 1.0], (K, 1, Lw, Lw)) * 1.42).astype(np.float32)
        f = WL.Filters(W, np.array([0.3, -0.2], np.float32), np.array([0.1], np.float32))
        Sk, Sv = _filter_sums(f)
        assert Sk.max() < 80 and Sv < 80 and Sk.sum() + K < 80 and Sv > 70
    elif case == "additive_large_filters":
        K, Lw = 8, 5
        f = WL.random_filters_with_bias(K, 1, Lw, 1.0, 0.5, seed=5)
        Sk, Sv = _filter_sums(f)
        assert Sk.sum() + K > 80
    else:
        K, Lw = 1, 3
        W = (rng.choice([-1.0, 1.0], (K, 1, Lw, Lw)) * 9.5).astype(np.float32)
        f = WL.Filters(W, np.array([0.4], np.float32), np.array([-0.3], np.float32))
        Sk, Sv = _filter_sums(f)
        assert Sk.max() > 80
    T = np.linspace(1.2, 4.0, 8)
    job, ch = run_pair(orc, api, f, 32, T, seed=21, sweeps=12, burnin=2, blocks=[5, 7])
    check_chains(orc, job, ch, 1e-9)


@pytest.mark.parametrize("L", [32, 64])
def test_tile_shapes_give_identical_chains(orc, api, L):
    # every (rows, threads) tile choice yields the same chains (doubles as a race check)
    from paper_2008_05401_amd import autotune
    f = WL.random_filters_with_bias(8, 1, 5, 0.06, 0.05, seed=4)
    T = np.linspace(1.8, 3.0, 12)
    ref = None
    try:
        for rows, nt in autotune.candidates(L):
            api.set_tuning(L, 8, 5, rows, nt)
            job = api.Job(api.CRBMParams.from_filters(f), api.ISING, L, T, seed=13, burnin=2)
            job.run(5)
            job.run(4)
            st = job.stats()
            got = (job.state.cpu().numpy(), st)
            if ref is None:
                ref = got
                ch = orc.Chains(orc.CRBM(f.W, f.hbias, f.vbias), orc.ISING, L, T, seed=13, burnin=2)
                ch.run(9)
                assert np.array_equal(ref[0], ch.state)
            else:
                assert np.array_equal(got[0], ref[0]), (rows, nt)
                for name in ("n_acc", "E", "sumE", "sumE2", "sumM", "sumAbsM", "sumM2"):
                    assert np.array_equal(st[name], ref[1][name]), (rows, nt, name)
                # F: float32 terms grouped per lane block, so equal only within the two bounds
                tol = st["F_bound"] + ref[1]["F_bound"] + 1e-11 * np.abs(st["F"])
                assert np.all(np.abs(st["F"] - ref[1]["F"]) <= tol), (rows, nt)
    finally:
        api.clear_tuning()
        autotune.apply()


@pytest.mark.parametrize("L,K,Lw", [(16, 8, 5), (5, 3, 2), (64, 8, 5)])
def test_gibbs_only_target(orc, api, L, K, Lw):
    f = WL.random_filters_with_bias(K, 1, Lw, 0.3, 0.2, seed=L)
    T = np.full(8, 2.0)
    job = api.Job(api.CRBMParams.from_filters(f), api.GIBBS, L, T, seed=21, burnin=1)
    ch = orc.Chains(orc.CRBM(f.W, f.hbias, f.vbias), orc.GIBBS, L, T, seed=21, burnin=1)
    job.run(7)
    ch.run(7)
    st = job.stats()
    assert np.array_equal(job.state.cpu().numpy(), ch.state)
    assert np.all(st["n_acc"] == 7)
    for name in ("E", "sumE", "sumM2"):
        assert np.array_equal(st[name], ch.rec[name])


def test_transfer_shape_sampled_chains(orc, api):
    # the transfer-sampling launch (L=128, 2048 chains) with the exact kernel zero-padded to
    # K=8 5x5 (acceptance ~1, so the FP64 MH re-check path runs); sampled chains recomputed
    # one by one by the oracle from their chain index
    L, n, T = 128, 2048, 2.3
    f = WL.analytic_ising_filters(T, K=8, Lw=5)
    job = api.Job(api.CRBMParams.from_filters(f), api.ISING, L, np.full(n, T), seed=1)
    job.run(4)
    st = job.stats()
    state = job.state.cpu().numpy()
    assert st["n_acc"].sum() > 0.9 * n * 4
    m = orc.CRBM(f.W, f.hbias, f.vbias)
    for g in (0, 1023, 2047):
        ch = orc.Chains(m, orc.ISING, L, np.full(1, T), seed=1, g0=g)
        ch.run(4)
        assert ch.ties[0] == 0 and ch.ties[1] == 0
        assert np.array_equal(state[g], ch.state[0])
        for name in ("n_acc", "E", "sumE", "sumM2"):
            assert st[name][g] == ch.rec[name][0]
        assert abs(st["F"][g] - ch.rec["F"][0]) <= st["F_bound"][g] + 1e-9 * abs(ch.rec["F"][0])
