"""Pins of the oracle's nucleon with the projector cut (Section 5.2, eq.
W0tbary), against the Wick contraction W_N1 - W_N2 (eq. baryfact) that the
nucleon pins fix by brute-force enumeration:

* a complete projector on the sites D_dGamma* reads: the colourless-spinor
  form equals the point-source factorized nucleon (eq. approxlong) summed
  over every source of each slice;
* an incomplete random projector: it equals W_N1 - W_N2 of the projected
  propagator S(y,x) = -sum_i eta_i(y) xi_i(x)^T (eq. approxlong2) with xi_i^T =
  phi_i^dag D_Gammabar^{-1} and eta_i taken from dense block inverses.
Together they fix the index orders of the two terms, the overall sign and the
gamma5-hermiticity step that gives xi from a solve with gamma5 phi.  Written
out, the substitution gives +sum B^T P_- B for both terms (the three minus
signs of S and the reordering of eps cancel); the printed eq. W0tbary carries
-gamma5 P_- instead, which the random-projector pin shows to be a different
number.
"""
import numpy as np
import pytest

import inputs
import oracle
from tests import _dense
from tests.test_oracle_factorized import _dense_operator

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


def _nucleon_of_sources(L, columns_of_x, slices):
    """C(y0, x0) = (1/L^3) sum over sources x in slice x0 of sum_y (W_N1 - W_N2)(y, x)."""
    V3 = int(np.prod(L[1:]))
    out = np.zeros((L[0], L[0]), complex)
    for x0 in slices:
        for k in range(V3):
            out[:, x0] += oracle.nucleon(columns_of_x(x0 * V3 + k), L)
    return out / V3


def test_complete_projector_equals_the_point_source_factorized_nucleon():
    """Open time boundaries (96 vectors; with a wrap the projector needs two
    slices and the N^3 spinors get large; the wrap face is covered by the
    random-projector pin)."""
    bc = oracle.OPEN
    L = L8
    kappa = 0.13
    U = inputs.random_links(L, 1601401, 0.4)
    C = oracle.clover_term(U, L, 1.2)
    xcut, delta = 4, 2
    bar = ((0, 0, 0, 0), (xcut + delta,) + L[1:])
    star = ((xcut, 0, 0, 0), L)
    phi = _unit_vectors(L, [xcut - 1] if bc == oracle.OPEN else [0, xcut - 1])
    got, _, _ = oracle.projected_nucleon(U, L, kappa, phi, bar, star, C=C, antiperiodic=bc)

    def cols(site):
        x = np.unravel_index(site, L)
        sf, _ = oracle.factorized_propagator(U, L, kappa, inputs.point_source(L, x), bar, star, C=C,
                                             antiperiodic=bc)
        return sf

    ref = _nucleon_of_sources(L, cols, range(xcut + delta))
    ys, xs = slice(xcut, L[0]), slice(0, xcut + delta)
    scale = np.abs(ref[ys, xs]).max()
    assert scale > 0
    assert np.abs(got[ys, xs] - ref[ys, xs]).max() < 1e-10 * scale
    assert np.abs(got[:xcut]).max() == 0 and np.abs(got[:, xcut + delta:]).max() == 0


@pytest.mark.parametrize("bc", [oracle.OPEN, True])
def test_random_projector_equals_the_dense_projected_propagator_contraction(bc):
    L = L8
    kappa = 0.13
    rng = np.random.default_rng(1601402)
    U = inputs.random_links(L, 1601403, 0.4)
    V = int(np.prod(L))
    V3 = V // L[0]
    xcut, delta = 4, 2
    bar = ((0, 0, 0, 0), (xcut + delta,) + L[1:])
    star = ((xcut, 0, 0, 0), L)
    # 5 orthonormal vectors supported on the slices D_dGamma* reads (with a wrap also slice 0)
    n = 5
    raw = np.zeros((n, V, 4, 3), complex)
    for t in ([xcut - 1] if bc == oracle.OPEN else [0, xcut - 1]):
        raw[:, t * V3:(t + 1) * V3] = rng.normal(size=(n, V3, 4, 3)) + 1j * rng.normal(size=(n, V3, 4, 3))
    q, _ = np.linalg.qr(raw.reshape(n, -1).T)
    phi = q.T.reshape(n, V, 4, 3)
    got, Bx, By = oracle.projected_nucleon(U, L, kappa, phi, bar, star, antiperiodic=bc)

    D = _dense_operator(U, L, kappa, bc)
    ib = _dense.domain_indices(L, *bar)
    i_s = _dense.domain_indices(L, *star)
    ic = np.setdiff1d(np.arange(12 * V), i_s)
    Ph = phi.reshape(n, 12 * V)
    Dbar_inv = np.zeros((12 * V, 12 * V), complex)
    Dbar_inv[np.ix_(ib, ib)] = np.linalg.inv(D[np.ix_(ib, ib)])
    XiT = Ph.conj() @ Dbar_inv                          # rows xi_i^T = phi_i^dag D_Gammabar^{-1}
    Eta = np.zeros((n, 12 * V), complex)
    Eta[:, i_s] = np.linalg.solve(D[np.ix_(i_s, i_s)], D[np.ix_(i_s, ic)] @ Ph[:, ic].T).T

    def cols(site):
        # S(y, x)[alpha a, beta b] = -sum_i eta_i(y)_{alpha a} xi_i(x)_{beta b}; column 3 beta + b
        S = -Eta.T @ XiT[:, 12 * site:12 * site + 12]   # [12V, 12]
        return S.T.reshape(12, V, 4, 3)

    ref = _nucleon_of_sources(L, cols, range(xcut + delta))
    ys, xs = slice(xcut, L[0]), slice(0, xcut + delta)
    scale = np.abs(ref[ys, xs]).max()
    assert scale > 0
    assert np.abs(got[ys, xs] - ref[ys, xs]).max() < 1e-10 * scale
    # the printed form, -sum B^T g5 P_- B, is not this contraction
    G = oracle.gamma5() @ oracle.P_minus()
    lit = -(np.einsum("xjikr,rq,yijkq->yx", Bx, G, By) - np.einsum("xkijr,rq,yijkq->yx", Bx, G, By)) / V3
    assert np.abs(lit[ys, xs] - ref[ys, xs]).max() > 0.1 * scale


def test_colourless_spinor_is_antisymmetric_in_colour_and_bilinear():
    """B[s_i, s_j, s_k] with s_i = s_j of a single colour vanishes (eps), and
    B is linear in each argument."""
    rng = np.random.default_rng(1601404)
    L = (2, 2, 2, 2)
    V = 16
    s = rng.normal(size=(3, V, 4, 3)) + 1j * rng.normal(size=(3, V, 4, 3))
    one = s.copy()
    one[:, :, :, 1:] = 0
    B1 = oracle.colourless_spinors(one, L)
    assert np.abs(B1).max() == 0
    B = oracle.colourless_spinors(s, L)
    s2 = s.copy()
    s2[0] *= 2.5
    B2 = oracle.colourless_spinors(s2, L)
    assert np.allclose(B2[:, 0, 1:, 1:], 2.5 * B[:, 0, 1:, 1:]) and np.allclose(B2[:, 1:, 0, 1:], 2.5 * B[:, 1:, 0, 1:])
