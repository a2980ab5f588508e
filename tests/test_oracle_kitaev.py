"""Pins of the oracle's Kitaev gauge-field weight (Sec. IV).

* flux-free closed form: for u = +1 the hopping block is translation
  invariant and its singular values are 2|J_z + J_x e^{i q1} + J_y e^{i q2}|,
  q = 2 pi m / L (Bloch's theorem); zero modes exist iff 3 divides L;
* gauge invariance: flipping the three bonds of one site leaves the spectrum
  unchanged (it is a sign change of one row or column of M);
* normalisation: at high temperature S - N log 2 -> (beta^2/8) sum eps^2 =
  (beta^2/2) L^2 (J_x^2+J_y^2+J_z^2), which equals beta^2 Tr(H^2)/(2 dim)
  of the spin Hamiltonian; checked against an explicit spin-operator trace
  on the L=2 cluster built from the same bond list;
* the one-sided Jacobi solver against LAPACK's SVD (numpy);
* exact enumeration at L=2 (4096 gauge configurations): chains started from
  exact samples keep the distribution P(u) ~ exp(S(u)).
"""
import itertools
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import exact_ising as X  # noqa: E402

from paper_2008_05401_amd import workloads as WL  # noqa: E402


def bloch_spectrum(L, J):
    q = 2 * np.pi * np.arange(L) / L
    q1, q2 = np.meshgrid(q, q, indexing="ij")
    return np.sort((2 * np.abs(J[2] + J[0] * np.exp(1j * q1) + J[1] * np.exp(1j * q2))).ravel())


@pytest.mark.parametrize("L", [3, 4, 5, 6])
@pytest.mark.parametrize("J", [(1.0, 1.0, 1.0), (0.7, 1.1, 1.3)])
def test_flux_free_spectrum(orc, L, J):
    u = np.ones((3, L, L), np.int8)
    _, eps, _, _ = orc.kitaev_S(u, 0.5, J)
    assert np.allclose(np.sort(eps), bloch_spectrum(L, J), atol=1e-12)
    # the z-bond-only field with u_x = u_y = +1 gives the same matrix
    M3 = orc.kitaev_matrix(u, J)
    M1 = orc.kitaev_matrix(np.ones((1, L, L), np.int8), J)
    assert np.array_equal(M3, M1)


@pytest.mark.parametrize("L,nzero", [(3, 2), (4, 0), (6, 2), (9, 2)])
def test_zero_modes(orc, L, nzero):
    _, eps, _, _ = orc.kitaev_S(np.ones((3, L, L), np.int8), 0.5)
    assert (eps < 1e-10).sum() == nzero


def _flip_site(u, L, black, i, j):
    v = u.copy()
    if black:   # bonds of b(i,j): x, y, z of cell (i,j)
        v[0, i, j] *= -1
        v[1, i, j] *= -1
        v[2, i, j] *= -1
    else:       # bonds of w(i,j): z of (i,j), x of (i,j-1), y of (i-1,j)
        v[2, i, j] *= -1
        v[0, i, (j - 1) % L] *= -1
        v[1, (i - 1) % L, j] *= -1
    return v


def test_gauge_invariance(orc):
    L = 5
    rng = np.random.default_rng(0)
    u = np.where(rng.random((3, L, L)) < 0.5, 1, -1).astype(np.int8)
    S0, e0, _, _ = orc.kitaev_S(u, 0.3)
    for black in (True, False):
        for (i, j) in [(0, 0), (2, 3), (4, 4)]:
            S1, e1, _, _ = orc.kitaev_S(_flip_site(u, L, black, i, j), 0.3)
            assert np.allclose(np.sort(e0), np.sort(e1), atol=1e-12)
            assert abs(S0 - S1) < 1e-10 * abs(S0)


@pytest.mark.parametrize("L", [2, 4, 6])
def test_high_temperature_normalisation(orc, L):
    J = (0.7, 1.1, 1.3)
    rng = np.random.default_rng(L)
    beta = 1e-3
    for _ in range(3):
        u = np.where(rng.random((3, L, L)) < 0.5, 1, -1).astype(np.int8)
        S, eps, _, _ = orc.kitaev_S(u, 1.0 / beta, J)
        lead = 0.5 * beta * beta * L * L * sum(j * j for j in J)
        assert abs((S - L * L * np.log(2.0)) / lead - 1.0) < 1e-4


def test_spin_side_trace_matches(orc):
    # Tr(H^2)/dim of H = -sum_alpha J_alpha sum_<ij>_alpha s^a_i s^a_j over the same bond list;
    # its beta^2 coefficient must match the Majorana side's (1/8) sum eps^2 per configuration.
    L = 2
    J = (0.7, 1.1, 1.3)
    nsite = 2 * L * L
    sx = np.array([[0, 1], [1, 0]], complex)
    sy = np.array([[0, -1j], [1j, 0]])
    sz = np.array([[1, 0], [0, -1]], complex)
    P = {0: sx, 1: sy, 2: sz}

    def op(site, m):
        out = np.array([[1.0 + 0j]])
        for s in range(nsite):
            out = np.kron(out, m if s == site else np.eye(2))
        return out

    b = lambda i, j: 2 * ((i % L) * L + (j % L))      # noqa: E731
    w = lambda i, j: 2 * ((i % L) * L + (j % L)) + 1  # noqa: E731
    H = np.zeros((2 ** nsite, 2 ** nsite), complex)
    for i, j in itertools.product(range(L), range(L)):
        for alpha, (bi, bj) in ((2, (i, j)), (0, (i, j + 1)), (1, (i + 1, j))):
            H -= J[alpha] * op(b(i, j), P[alpha]) @ op(w(bi, bj), P[alpha])
    tr = np.trace(H @ H).real / 2 ** nsite
    _, eps, _, _ = orc.kitaev_S(np.ones((3, L, L), np.int8), 1.0, J)
    assert abs(tr - (eps ** 2).sum() / 4) < 1e-10
    assert abs(tr - L * L * sum(j * j for j in J)) < 1e-10


@pytest.mark.parametrize("L", [2, 3, 4, 5, 6])
def test_jacobi_against_lapack(orc, L):
    rng = np.random.default_rng(L)
    for _ in range(3):
        u = np.where(rng.random((3, L, L)) < 0.5, 1, -1).astype(np.int8)
        M = orc.kitaev_matrix(u, (1.0, 0.8, 1.2))
        sv, _ = orc.singular_values(M)
        ref = np.linalg.svd(M, compute_uv=False)
        assert np.allclose(np.sort(sv), np.sort(ref), rtol=0, atol=1e-13 * ref.max())
    A = rng.standard_normal((20, 20))
    sv, _ = orc.singular_values(A)
    assert np.allclose(np.sort(sv), np.sort(np.linalg.svd(A, compute_uv=False)), atol=1e-12)


def test_fermion_energy_and_fluctuation_are_derivatives(orc):
    # E_f = -dS/dbeta and C_f = beta^2 d^2S/dbeta^2 (central differences)
    L = 4
    rng = np.random.default_rng(3)
    u = np.where(rng.random((3, L, L)) < 0.5, 1, -1).astype(np.int8)
    T = 0.4
    beta = 1 / T
    h = 1e-4
    S0, _, Ef, Cf = orc.kitaev_S(u, T)
    Sp = orc.kitaev_S(u, 1 / (beta + h))[0]
    Sm = orc.kitaev_S(u, 1 / (beta - h))[0]
    assert abs(-(Sp - Sm) / (2 * h) - Ef) < 1e-6 * abs(Ef)
    assert abs(beta * beta * (Sp - 2 * S0 + Sm) / h ** 2 - Cf) < 1e-4 * abs(Cf)


def test_kitaev_sampler_keeps_exact_distribution(orc):
    L, T = 2, 0.6
    nb = 3 * L * L
    idx = np.arange(2 ** nb)
    U = (2 * ((idx[:, None] >> np.arange(nb)) & 1) - 1).astype(np.int8).reshape(-1, 3, L, L)
    S = orc.target(orc.KITAEV, U, T=np.full(len(U), T))
    p = np.exp(S - S.max())
    p /= p.sum()
    n = 30000
    rng = np.random.default_rng(5)
    s0 = U[rng.choice(len(p), size=n, p=p)].copy()
    f = WL.random_filters_with_bias(2, 3, 2, 0.4, 0.2, seed=6)
    m = orc.CRBM(f.W, f.hbias, f.vbias)
    ch = orc.Chains(m, orc.KITAEV, L, np.full(n, T), seed=4, state=s0)
    ch.run(8)
    b = (ch.state.reshape(n, -1) > 0).astype(np.int64)
    counts = np.bincount((b << np.arange(nb)).sum(1), minlength=2 ** nb).astype(np.float64)
    chi2, dof, pv = X.chi2_pvalue(counts, p)
    assert pv > 1e-4, (chi2, dof)
    acc = ch.rec["n_acc"].sum() / ch.rec["sweeps"].sum()
    assert acc > 0.05
    # cached S of the final states equals a fresh evaluation
    S_fin = orc.target(orc.KITAEV, ch.state[:64], T=np.full(64, T))
    assert np.allclose(ch.rec["S"][:64], S_fin, atol=1e-12)
