"""GPU parity of the sampler diagnostics: the per-sweep energy trace written
by the sweep kernels (bit-exact integer energies for Ising, 1e-8 relative for
the Kitaev fermion energy) and the autocovariance / integrated
autocorrelation-time kernel against the oracle (1e-10 relative on C(t) and
tau, identical windows)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import autocorr as AC  # noqa: E402
from paper_2008_05401_amd import workloads as WL  # noqa: E402


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_05401_amd import api as A
    return A


def _pair(orc, api, f, target, L, T, seed, **kw):
    job = api.Job(api.CRBMParams.from_filters(f), target, L, T, seed=seed, **kw)
    ch = orc.Chains(orc.CRBM(f.W, f.hbias, f.vbias), target, L, T, seed=seed, **kw)
    return job, ch


@pytest.mark.parametrize("L,K,Lw,n,ring,blocks", [
    (16, 8, 5, 12, 64, (10, 30)),      # bit-packed Ising kernel, no wrap
    (16, 8, 5, 12, 7, (5, 9, 13)),     # ring wraps several times
    (64, 8, 5, 40, 11, (6,)),          # batched lattice size
    (5, 3, 2, 9, 4, (3, 10)),          # generic kernel, ragged L
])
def test_ising_trace_bit_exact(orc, api, L, K, Lw, n, ring, blocks):
    f = WL.random_filters_with_bias(K, 1, Lw, 0.1, 0.05, seed=L)
    T = np.linspace(1.8, 3.0, n)
    job, ch = _pair(orc, api, f, 0, L, T, seed=L + 1)
    job.run(3)  # sweeps before recording starts are not in the trace
    ch.run(3)
    job.record_trace(ring)
    logs = []
    for b in blocks:
        job.run(b)
        ch.run(b, log_energy=True)
        logs.append(ch.energy_log)
    ref = np.concatenate(logs, 1)[:, -ring:]
    got = job.trace().cpu().numpy()
    assert ch.ties[0] == 0 and ch.ties[1] == 0
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)
    # the stored energies are those of the final state
    assert np.array_equal(got[:, -1], job.stats()["E"].astype(np.float64))


def test_trace_off_leaves_buffer(orc, api):
    f = WL.random_filters(4, 1, 3, 0.1, seed=0)
    job = api.Job(api.CRBMParams.from_filters(f), 0, 8, np.full(4, 2.3), seed=0)
    job.record_trace(8)
    job.run(4)
    ring = job._trace
    before = ring.clone()
    job.record_trace(0)
    job.run(5)
    torch.cuda.synchronize()
    assert torch.equal(ring, before)


@pytest.mark.parametrize("C,L", [(3, 4), (1, 6)])
def test_kitaev_trace(orc, api, C, L):
    f = WL.random_filters_with_bias(6, C, 2, 0.1, 0.05, seed=C)
    T = WL.kitaev_temperatures(6)
    job, ch = _pair(orc, api, f, 1, L, T, seed=3)
    job.record_trace(16)
    job.run(5)
    ch.run(5, log_energy=True)
    np.testing.assert_allclose(job.trace().cpu().numpy(), ch.energy_log, rtol=1e-8, atol=1e-10)


def test_gibbs_only_three_channel_trace(orc, api):
    f = WL.random_filters_with_bias(4, 3, 2, 0.2, 0.1, seed=9)
    job, ch = _pair(orc, api, f, 2, 5, np.full(6, 2.0), seed=8)
    job.record_trace(9)
    job.run(6)
    ch.run(6, log_energy=True)
    assert np.array_equal(job.trace().cpu().numpy(), ch.energy_log)


@pytest.mark.parametrize("n,length,max_lag,start,phi", [
    (5, 1000, 200, 0, 0.7),
    (3, 257, 256, 100, 0.3),     # max_lag = len - 1, rotated start
    (1, 1, 0, 0, 0.0),           # single sample
    (2, 8176, 300, 8175, 0.95),  # longest series, start at the last slot
    (300, 64, 20, 5, 0.5),       # many series
])
def test_autocorr_parity(api, n, length, max_lag, start, phi):
    x = WL.ar1_series(n, length, phi, seed=length) + 2.5
    g = torch.from_numpy(x).cuda()
    c, tau, win = api.autocorrelation(g, max_lag, start=start)
    c, tau, win = c.cpu().numpy(), tau.cpu().numpy(), win.cpu().numpy()
    for i in range(n):
        xi = np.roll(x[i], -start)
        cr, tr, wr = AC.integrated_time(xi, max_lag)
        scale = abs(cr[0]) + 1e-300
        np.testing.assert_allclose(c[i], cr, rtol=0, atol=1e-10 * scale + 1e-300)
        assert win[i] == wr
        assert tau[i] == pytest.approx(tr, rel=1e-10, abs=1e-12)


def test_autocorr_sokal_window_constant(api):
    x = WL.ar1_series(4, 2000, 0.8, seed=1)
    g = torch.from_numpy(x).cuda()
    for cw in (3.0, 6.0, 10.0):
        _, tau, win = api.autocorrelation(g, 400, c_window=cw)
        for i in range(4):
            _, tr, wr = AC.integrated_time(x[i], 400, cw)
            assert int(win[i]) == wr and float(tau[i]) == pytest.approx(tr, rel=1e-10)


def test_autocorr_of_chain_trace(orc, api):
    # the trace ring feeds the autocorrelation kernel directly (rotated start)
    f = WL.analytic_ising_filters(2.269, K=8, Lw=5)
    job = api.Job(api.CRBMParams.from_filters(f), 0, 16, np.full(8, 2.269), seed=4)
    job.record_trace(100)
    job.run(130)
    ring, start, count = job.trace_ring()
    assert count == 100
    c, tau, win = api.autocorrelation(ring, 30, start=start)
    ordered = job.trace().cpu().numpy()
    for i in range(8):
        cr, tr, wr = AC.integrated_time(ordered[i], 30)
        np.testing.assert_allclose(c[i].cpu().numpy(), cr, rtol=1e-10, atol=1e-9)
        assert int(win[i]) == wr
