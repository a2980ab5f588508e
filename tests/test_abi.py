"""CPU-side checks of the C ABI: the library loads, exports every function that
include/crbm.h declares, and its host-side validation rejects bad arguments
with the documented status codes before any device work."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2008_05401_amd import _lib
    try:
        return _lib, _lib.load()
    except ImportError as e:  # pragma: no cover - build() runs before the suite
        pytest.fail(str(e))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"CRBM_API\s+[\w\s\*]+?\b(\w+)\s*\(", src)
    return names


def test_every_declared_symbol_is_exported(lib):
    _lib, L = lib
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) >= set(_lib.EXPORTS)


def test_version(lib):
    _lib, _ = lib
    assert "gfx950" in _lib.crbm_version()


def _params(K=4, C=1, Lw=3, ptr=0x1000, open_cols=0, n_edge=0, dense=0):
    from paper_2008_05401_amd import _lib
    return _lib.crbm_params(K, C, Lw, ptr, ptr, ptr, open_cols, n_edge, dense)


def _desc(target=0, L=8, n=4, gk=1, rbm=None, boundary=0):
    from paper_2008_05401_amd import _lib
    return _lib.crbm_batch_desc(target=target, L=L, n_chains=n, gibbs_k=gk, burnin_sweeps=0, init_state=1,
                                chain_offset=0, boundary=boundary, seed=0, J=(ct.c_double * 3)(1, 1, 1), T=0x1000,
                                state=0x1000, rbm_state=rbm, workspace=0x1000, workspace_bytes=1 << 20)


def test_workspace_size_validation(lib):
    _lib, _ = lib
    assert _lib.crbm_workspace_size(_params(), _desc()) >= 4 * 160
    assert _lib.crbm_workspace_size(_params(Lw=9), _desc()) == 0          # Lw > 8
    assert _lib.crbm_workspace_size(_params(Lw=5), _desc(L=4)) == 0       # Lw > L
    assert _lib.crbm_workspace_size(_params(C=3), _desc(target=0)) == 0   # Ising needs C = 1
    assert _lib.crbm_workspace_size(_params(C=2), _desc()) == 0
    assert _lib.crbm_workspace_size(_params(K=65), _desc()) == 0
    assert _lib.crbm_workspace_size(_params(), _desc(n=0)) == 0
    assert _lib.crbm_workspace_size(_params(), _desc(gk=0)) == 0
    assert _lib.crbm_workspace_size(_params(), _desc(L=257)) == 0
    assert _lib.crbm_workspace_size(_params(C=3), _desc(target=1, L=25)) == 0
    # beyond L = 12 the Kitaev eigen-step keeps an N x N FP64 matrix per chain in the workspace
    assert _lib.crbm_workspace_size(_params(C=3), _desc(target=1, L=16)) >= 4 * 256 * 256 * 8
    assert _lib.crbm_workspace_size(_params(), _desc(target=2, rbm=0x1000)) == 0  # replica needs a target
    assert _lib.crbm_workspace_size(_params(C=3), _desc(target=2)) > 0            # Gibbs-only chains, C = 3
    assert _lib.crbm_workspace_size(_params(), _desc(rbm=0x1000)) > 0
    # locally connected CRBM and open boundaries
    assert _lib.crbm_workspace_size(_params(open_cols=1, n_edge=3), _desc(L=6, boundary=1)) > 0
    assert _lib.crbm_workspace_size(_params(open_cols=1, n_edge=3), _desc(L=5)) == 0   # 2 n_edge > L
    assert _lib.crbm_workspace_size(_params(n_edge=5), _desc(L=16)) == 0               # n_edge > 4
    assert _lib.crbm_workspace_size(_params(open_cols=2), _desc()) == 0
    assert _lib.crbm_workspace_size(_params(), _desc(boundary=2)) == 0
    assert _lib.crbm_workspace_size(_params(C=3, n_edge=1, open_cols=1), _desc(target=1, L=6, boundary=1)) > 0
    # fully connected RBM: K up to 256, built for the job's L, no banks
    assert _lib.crbm_workspace_size(_params(K=128, Lw=8, dense=1), _desc(target=1, L=8)) > 0
    assert _lib.crbm_workspace_size(_params(K=257, Lw=8, dense=1), _desc(L=8)) == 0
    assert _lib.crbm_workspace_size(_params(K=64, Lw=6, dense=1), _desc(L=8)) == 0            # Lw != L
    assert _lib.crbm_workspace_size(_params(K=64, Lw=8, dense=1, n_edge=1), _desc(L=8)) == 0
    assert _lib.crbm_workspace_size(_params(K=64, Lw=8, dense=2), _desc(L=8)) == 0
    assert _lib.crbm_workspace_size(_params(K=256, C=3, Lw=12, dense=1), _desc(target=1, L=12)) == 0  # LDS
    assert _lib.crbm_grad_workspace_size(_params(K=64, Lw=8, dense=1), 10) >= 10 * (64 * 64 + 64 + 64) * 8
    # Kitaev keeps the singular values of every chain: 4 chains x 36 doubles more
    kit = _lib.crbm_workspace_size(_params(C=3), _desc(target=1, L=6))
    assert kit >= _lib.crbm_workspace_size(_params(), _desc(L=6)) + 4 * 36 * 8


def test_init_rejects_before_device_work(lib):
    _lib, L = lib
    ctx = ct.c_void_p()
    st = L.crbm_init(ct.byref(ctx), ct.byref(_params(Lw=5)), ct.byref(_desc(L=4)), None)
    assert st == _lib.CRBM_EINVAL and ctx.value is None
    assert "Lw" in _lib.crbm_last_error()
    d = _desc()
    d.workspace_bytes = 16
    st = L.crbm_init(ct.byref(ctx), ct.byref(_params()), ct.byref(d), None)
    assert st == _lib.CRBM_EBUDGET
    st = L.crbm_init(ct.byref(ctx), ct.byref(_params(C=3)), ct.byref(_desc(target=1, L=25)), None)
    assert st == _lib.CRBM_EUNSUPPORTED
    st = L.crbm_init(ct.byref(ctx), ct.byref(_params(C=3)), ct.byref(_desc(target=1, L=16)), None)
    assert st == _lib.CRBM_EBUDGET   # 1 MiB of workspace is short of the L=16 eigen-step scratch


def test_other_entry_points_validate(lib):
    _lib, L = lib
    p = _params()
    assert L.crbm_free_energy(ct.byref(p), None, -1, 8, None, None) == _lib.CRBM_EINVAL
    assert L.crbm_free_energy(ct.byref(p), None, 0, 8, None, None) == _lib.CRBM_OK   # empty batch
    J = (ct.c_double * 3)(1, 1, 1)
    assert L.target_energy(0, None, 1, 3, 8, 0, J, None, None, None, None) == _lib.CRBM_EINVAL
    assert L.target_energy(7, None, 1, 1, 8, 0, J, None, None, None, None) == _lib.CRBM_EINVAL
    assert L.target_energy(1, None, 1, 3, 13, 0, J, None, None, None, None) == _lib.CRBM_EUNSUPPORTED
    assert L.target_energy(0, None, 1, 1, 8, 2, J, None, None, None, None) == _lib.CRBM_EINVAL   # boundary
    assert L.crbm_grad_workspace_size(ct.byref(p), 10) >= 10 * (36 + 4 + 1) * 8
    assert L.crbm_grad(ct.byref(p), None, 1, 8, None, 0x1000, 0x1000, 0x1000, None, 0, None) == _lib.CRBM_EINVAL
    assert L.crbm_grad(ct.byref(p), 0x1000, 1, 8, 0x1000, 0x1000, 0x1000, 0x1000, None, 0, None) == _lib.CRBM_EBUDGET
    assert L.crbm_propose_accept(None, 1) == _lib.CRBM_EINVAL
    assert L.crbm_propose_accept_many(None, 1, 1) == _lib.CRBM_EINVAL
    g = ct.c_void_p(0x1000)
    assert L.crbm_graph_create(ct.byref(g), None, 1, 1, 1) == _lib.CRBM_EINVAL and g.value is None
    assert L.crbm_graph_create(None, None, 1, 1, 1) == _lib.CRBM_EINVAL
    jobs = (ct.c_void_p * 1)(None)
    assert L.crbm_graph_create(ct.byref(g), jobs, 0, 1, 1) == _lib.CRBM_EINVAL        # no job
    assert L.crbm_graph_create(ct.byref(g), jobs, 1, 1, 1) == _lib.CRBM_EINVAL        # NULL job
    assert L.crbm_graph_create(ct.byref(g), jobs, 1, 0, 1) == _lib.CRBM_EINVAL        # no block
    assert L.crbm_graph_launch(None) == _lib.CRBM_EINVAL
    assert L.crbm_graph_destroy(None) == _lib.CRBM_OK
    assert L.crbm_tempering_swap(None, 1, 0) == _lib.CRBM_EINVAL
    assert L.crbm_set_trace(None, 0x1000, 4) == _lib.CRBM_EINVAL
    ac = L.crbm_autocorr
    assert ac(0x1000, 1, 8177, 0, 3, 6.0, 0x1000, None, None, None) == _lib.CRBM_EINVAL   # longest series 8176
    assert ac(0x1000, 1, 0, 0, 0, 6.0, 0x1000, None, None, None) == _lib.CRBM_EINVAL      # empty series
    assert ac(0x1000, 1, 8, 0, 8, 6.0, 0x1000, None, None, None) == _lib.CRBM_EINVAL      # max_lag >= len
    assert ac(0x1000, 1, 8, -1, 3, 6.0, 0x1000, None, None, None) == _lib.CRBM_EINVAL     # negative start
    assert ac(0x1000, 1, 8, 0, 3, 0.0, 0x1000, None, None, None) == _lib.CRBM_EINVAL      # window constant
    assert ac(0x1000, 1, 8, 0, 3, 6.0, 0x1000, 0x1000, None, None) == _lib.CRBM_EINVAL    # tau without window
    assert ac(None, 1, 8, 0, 3, 6.0, 0x1000, None, None, None) == _lib.CRBM_EINVAL
    assert ac(None, 0, 8, 0, 3, 6.0, None, None, None, None) == _lib.CRBM_OK              # no series


def test_stats_record_layout(lib):
    _lib, _ = lib
    assert _lib.STATS_DTYPE.itemsize == 160
    assert np.dtype(_lib.STATS_DTYPE).names[:4] == ("sweeps", "n_acc", "n_meas", "n_recheck")
    assert _lib.STATS_DTYPE.fields["F_bound"][1] == 136 and _lib.STATS_DTYPE.fields["n_swap"][1] == 144


def test_grad_static_rejects_oversize_before_device_work(lib):
    # 6000 samples x (8*25 + 8 + 1) parameters x 8 bytes exceed the 8 MiB static scratch:
    # rejected on the host, no device call is made (this runs without a GPU)
    _lib, _ = lib
    with pytest.raises(_lib.CRBMError) as ei:
        _lib.crbm_grad_static(_params(K=8, Lw=5), 0x1000, 6000, 16, 0x1000, 0x1000, 0x1000, 0x1000, None)
    assert ei.value.status == _lib.CRBM_EBUDGET
    assert "static scratch" in _lib.crbm_last_error()
    with pytest.raises(_lib.CRBMError) as ei:
        _lib.crbm_grad_static(_params(K=8, Lw=5), 0x1000, -1, 16, 0x1000, 0x1000, 0x1000, 0x1000, None)
    assert ei.value.status == _lib.CRBM_EINVAL
