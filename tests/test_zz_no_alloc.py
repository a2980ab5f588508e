"""crbm_grad_static, the gradient entry point that allocates nothing (its
partial gradients live in the library's static per-GPU scratch), called
through the C ABI against crbm_grad (the same kernels with a caller
workspace) and the oracle: two calls in a row, the second with a smaller
batch, and the size limit."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from grad_bar import R_SIG64, assert_grad_close, grad_abs, sigma_is_fp64  # noqa: E402
from paper_2008_05401_amd import workloads as WL  # noqa: E402


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_05401_amd import api as A
    return A


def test_grad_static_matches_grad_twice(orc, api):
    # the training shape (K=8 5x5, L=16): B=1024, then a smaller batch that
    # leaves the first call's partial sums beyond it in the scratch
    K, C, Lw, L = 8, 1, 5, 16
    f = WL.random_filters_with_bias(K, C, Lw, 0.2, 0.3, seed=11)
    p = api.CRBMParams.from_filters(f)
    m = orc.CRBM(f.W, f.hbias, f.vbias)
    assert sigma_is_fp64(K, C, Lw, L)
    for B, seed in ((1024, 12), (300, 13)):
        x = WL.random_states(B, C, L, seed=seed)
        g = np.random.default_rng(seed).standard_normal(B).astype(np.float32)
        xt, gt = torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda()
        got = api.grad_static(p, xt, gt)
        ref_gpu = api.grad(p, xt, gt)
        for a, b in zip(got, ref_gpu):
            assert torch.equal(a, b)
        ref = orc.grad(m, x, g.astype(np.float64))
        A = grad_abs(orc, m, x, g)
        for a, r, aa in zip(got, ref, A):
            assert_grad_close(a.cpu().numpy(), r, aa, R_SIG64)


def test_grad_static_size_limit(api):
    from paper_2008_05401_amd import _lib
    f = WL.random_filters(8, 1, 5, 0.05, seed=0)
    p = api.CRBMParams.from_filters(f)
    # 6000 samples x 209 parameters x 8 bytes > 8 MiB
    x = torch.ones((6000, 1, 16, 16), dtype=torch.int8, device="cuda")
    with pytest.raises(_lib.CRBMError) as ei:
        api.grad_static(p, x, torch.ones(6000, device="cuda"))
    assert ei.value.status == _lib.CRBM_EBUDGET
    # the largest batch that fits still runs and matches crbm_grad
    B = (8 << 20) // (209 * 8)
    xb = torch.from_numpy(WL.random_states(B, 1, 16, seed=3)).cuda()
    gb = torch.from_numpy(np.random.default_rng(4).standard_normal(B).astype(np.float32)).cuda()
    for a, b in zip(api.grad_static(p, xb, gb), api.grad(p, xb, gb)):
        assert torch.equal(a, b)
