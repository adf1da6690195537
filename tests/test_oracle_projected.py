"""Pins of the oracle's projector-cut factorization (Section 5.2, eqs.
approxlong2, fullfactpi, Bpions).

* Completeness: with the projector spanning every site that D_dGamma* reads
  (unit vectors on the slice below the cut, and on slice 0 when the time
  direction wraps), the projected correlator equals the factorized one of
  eq. approxlong summed over every source of a slice, computed point source
  by point source with the (separately pinned) factorized propagator.  This
  checks the gamma5-hermiticity rewriting of eq. Bpions, the Gram matrices and
  the trace of eq. fullfactpi in one go.
* Orthonormalisation: Q has orthonormal columns and X = Q R with R upper
  triangular and positive real diagonal (the property that makes Q unique).
* Inverse iteration converges to an invariant subspace of D_Omega^{-1}.
"""
import numpy as np
import pytest

import inputs
import oracle

L8 = (8, 2, 2, 2)


def _unit_vectors(L, slices):
    V = int(np.prod(L))
    V3 = V // L[0]
    sites = [t * V3 + k for t in slices for k in range(V3)]
    phi = np.zeros((12 * len(sites), V, 4, 3), complex)
    for m, s in enumerate(sites):
        for c in range(12):
            phi[12 * m + c, s, c // 3, c % 3] = 1.0
    return phi


@pytest.mark.parametrize("bc", [oracle.OPEN, True])
def test_complete_projector_reproduces_the_factorized_correlator(bc):
    L = L8
    kappa = 0.13
    U = inputs.random_links(L, 1601701, 0.4)
    C = oracle.clover_term(U, L, 1.2)
    V = int(np.prod(L))
    V3 = V // L[0]
    xcut, delta = 4, 2
    bar = ((0, 0, 0, 0), (xcut + delta, 2, 2, 2))
    star = ((xcut, 0, 0, 0), L)
    slices = [xcut - 1] if bc == oracle.OPEN else [0, xcut - 1]
    phi = _unit_vectors(L, slices)
    Cp, G, Gt = oracle.projected_pion(U, L, kappa, phi, bar, star, C=C, antiperiodic=bc)
    ref = np.zeros((L[0], L[0]))
    for x0 in range(bar[1][0]):
        for k in range(V3):
            x = (x0,) + tuple(np.unravel_index(k, L[1:]))
            sf, _ = oracle.factorized_propagator(U, L, kappa, inputs.point_source(L, x), bar, star, C=C,
                                                 antiperiodic=bc)
            ref[:, x0] += oracle.pion_connected(sf, L)
    sc = np.abs(ref).max()
    assert sc > 0
    assert np.abs(Cp - ref).max() < 1e-10 * sc
    # zero outside the two time ranges
    assert not Cp[:xcut, :].any() and not Cp[:, xcut + delta:].any()
    # Gram matrices are Hermitian, positive semi-definite per slice
    for Gm in (G, Gt):
        assert np.abs(Gm - np.conj(Gm.transpose(0, 2, 1))).max() < 1e-13 * np.abs(Gm).max()
        assert min(np.linalg.eigvalsh(g).min() for g in Gm) > -1e-12 * np.abs(Gm).max()


def test_orthonormal_q_is_the_positive_diagonal_qr_factor():
    rng = np.random.default_rng(1601702)
    V = 32
    X = rng.normal(size=(7, V, 4, 3)) + 1j * rng.normal(size=(7, V, 4, 3))
    Q = oracle.orthonormal_q(X)
    M = Q.reshape(7, -1)
    assert np.abs(np.conj(M) @ M.T - np.eye(7)).max() < 1e-13
    R = np.conj(M) @ X.reshape(7, -1).T            # R_ij = q_i^dag x_j
    assert np.abs(np.tril(R, -1)).max() < 1e-12
    assert np.all(np.abs(np.diag(R).imag) < 1e-12) and np.all(np.diag(R).real > 0)
    assert np.abs(M.T @ R - X.reshape(7, -1).T).max() < 1e-12


def test_inverse_iteration_converges_to_an_invariant_subspace():
    L = (8, 2, 2, 2)
    kappa = 0.13
    U = inputs.random_links(L, 1601703, 0.4)
    lo, hi = (2, 0, 0, 0), (6, 2, 2, 2)
    V = int(np.prod(L))
    start = inputs.gaussian(1601704, 0, (6, V, 4, 3)) + 1j * inputs.gaussian(1601704, 1, (6, V, 4, 3))
    res = []
    for niter in (1, 10, 40):
        Q = oracle.inverse_iteration(U, L, kappa, start, niter, lo=lo, hi=hi)
        W, _, _ = oracle.solve(U, L, kappa, Q, lo=lo, hi=hi)      # D^{-1} Q
        Qm, Wm = Q.reshape(6, -1), W.reshape(6, -1)
        P = Wm - (Wm @ np.conj(Qm).T) @ Qm                     # part of D^{-1} Q outside span(Q)
        res.append(np.linalg.norm(P) / np.linalg.norm(Wm))
        assert np.abs(Q[:, ~oracle.domain_mask(L, lo, hi)]).max() < 1e-14
    assert res[0] > res[1] > res[2] and res[2] < 5e-3 * res[0], res


@pytest.mark.parametrize("bc", [oracle.OPEN, True])
def test_incomplete_projector_matches_dense_approxlong2(bc):
    """eq. approxlong2 written with dense blocks, S~ = -D_*^{-1} D_d P D_bar^{-1}
    with P = sum_i phi_i phi_i^dag for 10 random orthonormal vectors around the
    cut, against the Gram-matrix form of eq. fullfactpi (this catches a missing
    gamma5 of eq. Bpions, which a complete projector cannot see)."""
    from tests import _dense
    from tests.test_oracle_factorized import _dense_operator
    L = L8
    kappa = 0.13
    U = inputs.random_links(L, 1601705, 0.4)
    C = oracle.clover_term(U, L, 0.9)
    V = int(np.prod(L))
    V3 = V // L[0]
    xcut, delta = 4, 2
    bar = ((0, 0, 0, 0), (xcut + delta, 2, 2, 2))
    star = ((xcut, 0, 0, 0), L)
    om = ((xcut - delta, 0, 0, 0), (xcut + delta, 2, 2, 2))
    m = oracle.domain_mask(L, *om)
    raw = inputs.gaussian(1601706, 0, (10, V, 4, 3)) + 1j * inputs.gaussian(1601706, 1, (10, V, 4, 3))
    phi = oracle.orthonormal_q(raw * m[None, :, None, None])
    Cp, _, _ = oracle.projected_pion(U, L, kappa, phi, bar, star, C=C, antiperiodic=bc)
    D = _dense_operator(U, L, kappa, bc, C)
    ib = _dense.domain_indices(L, *bar)
    i_s = _dense.domain_indices(L, *star)
    ic = np.setdiff1d(np.arange(12 * V), i_s)
    Dbar = np.zeros_like(D)
    Dbar[np.ix_(ib, ib)] = np.linalg.inv(D[np.ix_(ib, ib)])
    Dst = np.zeros_like(D)
    Dst[np.ix_(i_s, i_s)] = np.linalg.inv(D[np.ix_(i_s, i_s)])
    Dd = np.zeros_like(D)
    Dd[np.ix_(i_s, ic)] = D[np.ix_(i_s, ic)]
    Phi = phi.reshape(10, -1).T
    S = -Dst @ Dd @ (Phi @ np.conj(Phi).T) @ Dbar
    blocks = S.reshape(V, 12, V, 12)
    w = np.einsum("yaxb,yaxb->yx", blocks, np.conj(blocks)).real      # tr{S S^dag} per (y, x)
    ref = -w.reshape(L[0], V3, L[0], V3).sum(axis=(1, 3)) / V3
    assert np.abs(Cp - ref).max() < 1e-10 * np.abs(ref).max()
