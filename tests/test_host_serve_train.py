"""Host-side logic of the job server and of Alg. 1 (no GPU): lane assignment
by lattice size, the HBM footprint used for admission, and argument checks of
the training loop."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2008_05401_amd import serve, train, workloads as WL  # noqa: E402


def test_lanes_by_lattice_size():
    s = serve.Server()
    assert [s.lane_of(L) for L in (8, 16, 32, 64, 128, 256)] == [0, 0, 0, 0, 1, 2]
    s = serve.Server(medium_sites=16 * 16, large_sites=32 * 32)
    assert [s.lane_of(L) for L in (8, 16, 32, 64)] == [0, 1, 2, 2]
    # a medium threshold above the large one collapses the medium lane
    s = serve.Server(medium_sites=64 * 64, large_sites=32 * 32)
    assert [s.lane_of(L) for L in (16, 32, 64)] == [0, 2, 2]


def test_footprint_counts_state_records_and_parameters():
    sp = WL.Job(job_id=0, arrival_s=0.0, L=64, T=2.0, n_chains=100, n_sweeps=10, seed=0)
    fp = serve.footprint_bytes(sp, K=8, Lw=5)
    # int8 state, 256 B job descriptor, per-chain records, temperatures, filters
    expect = 100 * 64 * 64 + 256 + 100 * 160 + 512 + 8 * 100 + 4 * (8 * 25 + 8 + 1)
    assert fp == expect
    sp2 = WL.Job(job_id=1, arrival_s=0.0, L=64, T=2.0, n_chains=200, n_sweeps=10, seed=1)
    assert serve.footprint_bytes(sp2) > fp


def test_alg1_rejects_empty_buffer_update():
    x = torch.from_numpy(WL.random_states(4, 1, 4, seed=0))
    with pytest.raises(ValueError):
        train.train_crbm(x, torch.zeros(4, dtype=torch.float64), None, 2.0, K=2, Lw=3, epochs=1, ub=0)
