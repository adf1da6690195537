"""Pins of the oracle's stochastic trace estimator with the hopping parameter
expansion (Section 6, eq. HPEtr and the estimator after it).

With every unit vector of the domain as a source the estimator is an exact
trace, so it must reproduce sum_x tr{gamma5 D_Gamma^{-1}(x,x)} per time slice
from a dense inverse of the domain block for every p the identity allows
(p <= 8 Wilson, p <= 2 with the clover term) and must miss it for the first p
beyond (a random field has non-zero loops of that length).  With Gaussian
sources it must equal sum_i eta_i^dag X eta_i for the dense matrix
X = (1 - 2 kappa D_Gamma)^p D_Gamma^{-1} gamma5.
"""
import numpy as np
import pytest

import inputs
import oracle
from tests import _dense

L6 = (6, 2, 2, 2)
LO, HI = (1, 0, 0, 0), (5, 2, 2, 2)


def _dense_domain(U, L, kappa, C, lo, hi):
    V = int(np.prod(L))
    D = _dense.wilson_dirac(U, L, kappa)
    if C is not None:
        for s in range(V):
            D[12 * s:12 * s + 12, 12 * s:12 * s + 12] += C[s]
    idx = _dense.domain_indices(L, lo, hi)
    return D, idx


def _exact_slices(U, L, kappa, C, lo, hi):
    D, idx = _dense_domain(U, L, kappa, C, lo, hi)
    Dinv = np.linalg.inv(D[np.ix_(idx, idx)])
    G5 = np.kron(np.diag([1, 1, -1, -1]), np.eye(3))
    V3 = int(np.prod(L[1:]))
    out = np.zeros(L[0], complex)
    sites = idx[::12] // 12
    for k, s in enumerate(sites):
        out[s // V3] += np.trace(G5 @ Dinv[12 * k:12 * k + 12, 12 * k:12 * k + 12])
    return out


def _unit_sources(L, lo, hi):
    V = int(np.prod(L))
    m = oracle.domain_mask(L, lo, hi)
    sites = np.nonzero(m)[0]
    eta = np.zeros((12 * len(sites), V, 4, 3), complex)
    for k, s in enumerate(sites):
        for c in range(12):
            eta[12 * k + c, s, c // 3, c % 3] = 1.0
    return eta


@pytest.mark.parametrize("csw,pmax", [(0.0, 8), (1.5, 2)])
def test_unit_sources_give_the_exact_trace_for_allowed_p(csw, pmax):
    L = L6
    kappa = 0.12
    U = inputs.random_links(L, 1601401, eps=1.0)
    C = oracle.clover_term(U, L, csw) if csw else None
    exact = _exact_slices(U, L, kappa, C, LO, HI)
    assert np.abs(exact).max() > 1e-6
    eta = _unit_sources(L, LO, HI)
    n = eta.shape[0]
    for p in sorted({0, 1, pmax // 2, pmax}):
        est = oracle.hpe_trace(U, L, kappa, eta, p, C=C, lo=LO, hi=HI) * n
        assert np.abs(est - exact).max() < 1e-10 * np.abs(exact).max(), p
    # one order beyond the allowed range the identity fails on a random field
    est = oracle.hpe_trace(U, L, kappa, eta, pmax + 1, C=C, lo=LO, hi=HI) * n
    assert np.abs(est - exact).max() > 1e-6 * np.abs(exact).max()


@pytest.mark.parametrize("p", [0, 2])
def test_gaussian_sources_match_the_dense_quadratic_form(p):
    L = L6
    kappa = 0.125
    U = inputs.random_links(L, 1601402, eps=0.5)
    C = oracle.clover_term(U, L, 1.0)
    V = int(np.prod(L))
    D, idx = _dense_domain(U, L, kappa, C, LO, HI)
    Dg = np.zeros_like(D)
    Dg[np.ix_(idx, idx)] = D[np.ix_(idx, idx)]           # D_Gamma, zero outside
    Dinv = np.zeros_like(D)
    Dinv[np.ix_(idx, idx)] = np.linalg.inv(D[np.ix_(idx, idx)])
    G5 = np.kron(np.eye(V), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    H = np.eye(12 * V) - 2 * kappa * Dg
    X = np.linalg.matrix_power(H, p) @ Dinv @ G5
    n = 5
    eta = (inputs.gaussian(1601403, 0, (n, V, 4, 3)) + 1j * inputs.gaussian(1601403, 1, (n, V, 4, 3))) / np.sqrt(2)
    e = eta.reshape(n, 12 * V)
    w = np.einsum("ni,ij,nj->ni", np.conj(e), X, e).reshape(n, L[0], -1, 12).sum(axis=(2, 3))
    ref = w.sum(axis=0) / n
    est = oracle.hpe_trace(U, L, kappa, eta, p, C=C, lo=LO, hi=HI)
    assert np.abs(est - ref).max() < 1e-10 * np.abs(ref).max()
