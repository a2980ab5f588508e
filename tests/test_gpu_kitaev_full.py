"""Kitaev parity at the benchmarked sizes, every chain against the oracle:
L=6 with 256 chains (u on the 3 L^2 bonds, K=8 3x3 filters ~ N(0, 0.1),
T log-uniform in [0.005, 0.05]) and L=12 with 128 chains, in the launch
configuration bench.py times.  States and decisions bit-exact, S, E_f, C_f
and their sums 1e-8 relative, F 1e-9."""
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


@pytest.mark.parametrize("L,n,sweeps", [(6, 256, 5), (12, 128, 2)])
def test_kitaev_full_size(orc, api, L, n, sweeps):
    f = WL.random_filters(8, 3, 3, 0.1, seed=0)
    T = WL.kitaev_temperatures(n)
    job = api.Job(api.CRBMParams.from_filters(f), api.KITAEV, L, T, seed=0)
    ch = orc.Chains(orc.CRBM(f.W, f.hbias, f.vbias), orc.KITAEV, L, T, seed=0)
    job.run(sweeps)
    ch.run(sweeps)
    assert np.array_equal(job.state.cpu().numpy(), ch.state)
    st = job.stats()
    assert np.array_equal(st["n_acc"], ch.rec["n_acc"])
    for name in ("S", "Ef", "Cf", "kE", "kE2", "kCf"):
        np.testing.assert_allclose(st[name], ch.rec[name], rtol=1e-8, atol=1e-8, err_msg=name)
    np.testing.assert_allclose(st["F"], ch.rec["F"], rtol=1e-9)
    assert ch.ties[0] == 0 and ch.ties[1] == 0
    assert 0 < st["n_acc"].sum() < n * sweeps
