"""HIP-graph sweep blocks (crbm_graph_create / crbm_graph_launch) through the
C ABI: every replay of a captured graph must leave the jobs exactly where the
same eager calls leave them, with eager work, synchronisations and other
stream-ordered calls (tempering swaps, trace changes, eager sweeps) between
the replays.  Bars: states, records and traces bit-exact against the eager
path (same kernels, same random streams); one case against the FP64 oracle
with the bars of the periodic parity tests.
"""
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


def _eager_noise():
    # unrelated eager work and a synchronisation between replays
    a = torch.randn(4096, device="cuda")
    torch.cuda.synchronize()
    return float((a * a).sum())


def _same(a, b, trace=False):
    torch.cuda.synchronize()
    assert torch.equal(a.state, b.state)
    if a.rbm_state is not None:
        assert torch.equal(a.rbm_state, b.rbm_state)
    sa, sb = a.stats(), b.stats()
    assert sa.tobytes() == sb.tobytes()
    assert a.sweeps == b.sweeps
    if trace:
        assert torch.equal(a.trace(), b.trace())


def test_graph_replays_equal_eager_fast_kernel(api):
    T = 2.269
    f = WL.analytic_ising_filters(T, K=8, Lw=5)
    p = api.CRBMParams.from_filters(f)
    mk = lambda: api.Job(p, api.ISING, 16, np.full(32, T), seed=4, burnin=3)  # noqa: E731
    eager, graphed = mk(), mk()
    g = api.SweepGraph([graphed], n_blocks=3, sweeps_per_block=5)
    _same(eager, graphed)                     # capture ran nothing
    for r in range(4):
        g.launch()
        for _ in range(3):
            eager.run(5)
        _eager_noise()
        _same(eager, graphed)
        if r == 1:                            # eager sweeps between replays
            eager.run(7)
            graphed.run(7)
            _same(eager, graphed)
    assert graphed.sweeps == 4 * 15 + 7
    g.close()


def test_graph_mixed_jobs_with_trace(api):
    fa = WL.random_filters_with_bias(4, 1, 3, 0.2, 0.1, seed=1)
    fb = WL.random_filters(8, 1, 5, 0.05, seed=2)
    fk = WL.random_filters(8, 3, 3, 0.1, seed=3)
    ff = WL.random_frbm(6, 1, 8, 0.1, seed=4)

    def mk():
        return [api.Job(api.CRBMParams.from_filters(fa), api.ISING, 8, np.full(5, 2.2), seed=1),
                api.Job(api.CRBMParams.from_filters(fb), api.ISING, 16, np.full(7, 2.5), seed=2, chain_offset=40),
                api.Job(api.CRBMParams.from_filters(fk), api.KITAEV, 4, np.full(3, 0.05), seed=3),
                # beyond L = 12 the eigen-step works in the job's global scratch
                api.Job(api.CRBMParams.from_filters(fk), api.KITAEV, 13, np.full(2, 0.1), seed=6),
                api.Job(api.CRBMParams.from_filters(ff, dense=True), api.ISING, 8, np.full(4, 2.0), seed=5,
                        boundary=1)]
    eager, graphed = mk(), mk()
    for a, b in zip(eager, graphed):
        a.record_trace(16)
        b.record_trace(16)
    g = api.SweepGraph(graphed, n_blocks=2, sweeps_per_block=3)
    for r in range(3):
        g.launch()
        api.run_many(eager, 3)
        api.run_many(eager, 3)
        _eager_noise()
        for a, b in zip(eager, graphed):
            _same(a, b, trace=True)
        if r == 0:                            # a new trace buffer is picked up by later replays
            for a, b in zip(eager, graphed):
                a.record_trace(8)
                b.record_trace(8)


def test_graph_with_tempering_between_replays(api):
    f = WL.random_filters_with_bias(4, 1, 3, 0.3, 0.1, seed=6)
    T = np.repeat(np.linspace(2.0, 2.6, 4), 2)
    mk = lambda: api.Job(api.CRBMParams.from_filters(f), api.ISING, 8, T, seed=8, replica=True)  # noqa: E731
    eager, graphed = mk(), mk()
    g = api.SweepGraph([graphed], n_blocks=1, sweeps_per_block=4)
    for r in range(4):
        g.launch()
        eager.run(4)
        graphed.tempering_swap(2, r)
        eager.tempering_swap(2, r)
        _eager_noise()
        _same(eager, graphed)


def test_graph_against_oracle(orc, api):
    f = WL.random_filters(4, 1, 3, 0.1, seed=0)
    T = np.full(16, 2.269)
    job = api.Job(api.CRBMParams.from_filters(f), api.ISING, 8, T, seed=0, burnin=5)
    ch = orc.Chains(orc.CRBM(f.W, f.hbias, f.vbias), orc.ISING, 8, T, seed=0, burnin=5)
    g = api.SweepGraph([job], n_blocks=4, sweeps_per_block=5)
    for _ in range(3):
        g.launch()
        ch.run(20)
        _eager_noise()
        assert np.array_equal(job.state.cpu().numpy(), ch.state)
        st = job.stats()
        for name in ("sweeps", "n_acc", "n_meas", "E", "sumE", "sumE2", "sumM", "sumAbsM", "sumM2"):
            assert np.array_equal(st[name], ch.rec[name]), name
        tol = st["F_bound"] + 1e-9 * (1.0 + np.abs(ch.rec["F"]))
        assert np.all(np.abs(st["F"] - ch.rec["F"]) <= tol)
    assert ch.ties[0] == 0 and ch.ties[1] == 0


def test_graph_argument_errors(api):
    from paper_2008_05401_amd import _lib
    f = WL.random_filters(4, 1, 3, 0.1)
    a = api.Job(api.CRBMParams.from_filters(f), api.ISING, 8, np.full(2, 2.0), seed=0)
    with pytest.raises(_lib.CRBMError):
        api.SweepGraph([a, a], 1, 1)              # listed twice
    with pytest.raises(_lib.CRBMError):
        api.SweepGraph([a], 0, 1)                 # no block
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = api.Job(api.CRBMParams.from_filters(f), api.ISING, 8, np.full(2, 2.0), seed=0, stream=s)
    with pytest.raises(_lib.CRBMError):
        api.SweepGraph([a, b], 1, 1)              # two streams
    g = api.SweepGraph([b], 2, 3)
    g.launch()
    s.synchronize()
    assert b.sweeps == 6
    b.close()
    with pytest.raises(RuntimeError):
        g.launch()
    g.close()
