"""Serving: every job's chains are identical whether it runs alone, in the
continuous-batching server next to other jobs (small and medium jobs in one
launch each on their streams, large jobs in blocks on a third), or in the plain one-chain-per-launch
form; admission respects the HBM budget."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2008_05401_amd import workloads as WL  # noqa: E402


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_05401_amd import api, serve
    return api, serve


def _specs():
    rng = np.random.default_rng(3)
    out = []
    for i in range(10):
        out.append(WL.Job(job_id=i, arrival_s=0.002 * i, L=int(rng.choice([8, 16, 32, 64])),
                          T=float(rng.uniform(1.8, 2.8)), n_chains=int(rng.integers(1, 24)),
                          n_sweeps=int(rng.integers(5, 23)), seed=100 + i))
    return out


def _alone(api, serve, sp):
    f = serve.job_filters(sp)
    job = api.Job(api.CRBMParams.from_filters(f), api.ISING, sp.L, np.full(sp.n_chains, sp.T), seed=sp.seed,
                  burnin=sp.n_sweeps // 10)
    job.run(sp.n_sweeps)
    return job.state.cpu().numpy(), job.stats()


@pytest.mark.parametrize("budget", [16 << 30, 1])
def test_served_results_equal_alone(mods, budget):
    api, serve = mods
    specs = _specs()
    # L = 16 is medium and L >= 32 large here, so every lane (the one-launch
    # small and medium paths, the blocked large path) serves part of the stream
    srv = serve.Server(budget_bytes=budget, large_block=4, medium_sites=16 * 16, large_sites=32 * 32,
                       keep_state=True)
    assert {srv.lane_of(sp.L) for sp in specs} == {0, 1, 2}
    res = {r.job_id: r for r in srv.run(specs)}
    assert sorted(res) == [s.job_id for s in specs]
    for sp in specs:
        st, rec = _alone(api, serve, sp)
        r = res[sp.job_id]
        assert np.array_equal(r.state, st), sp
        for name in ("sweeps", "n_acc", "n_meas", "E", "sumE", "sumE2", "sumM", "sumAbsM", "sumM2"):
            assert np.array_equal(r.stats[name], rec[name]), (sp, name)
        np.testing.assert_allclose(r.stats["F"], rec["F"], rtol=1e-12)
        assert r.latency_s >= 0 and r.admit_s >= r.arrival_s - 1e-9
    if budget == 1:
        # one job resident at a time: admissions follow completions in FIFO order
        order = sorted(res.values(), key=lambda r: r.admit_s)
        assert [r.job_id for r in order] == [s.job_id for s in specs]
        for a, b in zip(order, order[1:]):
            assert b.admit_s >= a.done_s - 1e-3


def test_plain_form_equals_batched(mods):
    api, serve = mods
    sp = WL.Job(job_id=7, arrival_s=0.0, L=16, T=2.2, n_chains=5, n_sweeps=9, seed=77)
    st_plain, rec_plain = serve.run_plain(sp, max_block=4)
    st, rec = _alone(api, serve, sp)
    assert np.array_equal(st_plain, st)
    for name in ("n_acc", "sumE", "sumM2"):
        assert np.array_equal(rec_plain[name], rec[name])


def test_served_matches_oracle(mods, orc):
    api, serve = mods
    sp = WL.Job(job_id=3, arrival_s=0.0, L=8, T=2.0, n_chains=6, n_sweeps=15, seed=33)
    srv = serve.Server(large_block=4, large_sites=8 * 8, keep_state=True)
    r = srv.run([sp])[0]
    f = serve.job_filters(sp)
    ch = orc.Chains(orc.CRBM(f.W, f.hbias, f.vbias), orc.ISING, sp.L, np.full(sp.n_chains, sp.T), seed=sp.seed,
                    burnin=sp.n_sweeps // 10)
    ch.run(sp.n_sweeps)
    assert np.array_equal(r.state, ch.state)
    for name in ("n_acc", "E", "sumE", "sumM"):
        assert np.array_equal(r.stats[name], ch.rec[name])
