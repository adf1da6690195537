"""Pins of the oracle's multi-slab factorized propagator (Section 4, steps
1-3, eqs. stp2, dec1, fctpr).

* eq. fctpr written with dense blocks of an independently assembled D:
  S^(f) = (-1)^(l-m) A_l B_{l,l-1} ... A_{m+1} B_{m+1,m} C, with A_i the
  inverse of the block D[Omega*_i, Omega*_i], B_{i,i-1} the block
  D[Lambda_i, Lambda_{i-1}] (eq. fact1) and C the inverse of
  D[Omega_{m+2}, Omega_{m+2}];
* exactness of iterated eq. Scmpt2: with open time boundaries, when every
  domain runs to the end of the lattice (and the first is the whole lattice)
  the chain is the exact propagator;
* with two domains it is the two-domain factorization (eq. approxlong);
* its error shrinks as the slab thickness grows (eq. errorfact).
"""
import numpy as np
import pytest

import inputs
import oracle
from tests import _dense
from tests.test_oracle_factorized import _columns, _dense_operator, _src_cols


def _block(L, t0, t1):
    return ((t0, 0, 0, 0), (t1,) + tuple(L[1:]))


def _chain_domains(L, delta, m, l):
    """Omega_{m+2} = Lambda_{m-1..m+1}, then Omega*_i = Lambda_i u Lambda_{i+1}, i = m+1..l."""
    doms = [_block(L, (m - 1) * delta, (m + 2) * delta)]
    doms += [_block(L, i * delta, min((i + 2) * delta, L[0])) for i in range(m + 1, l + 1)]
    return doms


@pytest.mark.parametrize("bc", [oracle.OPEN, True])
@pytest.mark.parametrize("csw", [0.0, 1.1])
def test_chain_equals_the_dense_block_product_of_eq_fctpr(bc, csw):
    L = (12, 2, 2, 2)
    delta, m, l = 2, 1, 4
    kappa = 0.13
    U = inputs.random_links(L, 1601301, 0.4)
    V = int(np.prod(L))
    Cl = oracle.clover_term(U, L, csw) if csw else None
    D = _dense_operator(U, L, kappa, bc, Cl)
    idx = lambda t0, t1: _dense.domain_indices(L, *_block(L, t0, t1))
    x = (m * delta + 1, 1, 0, 1)
    E = np.zeros((12 * V, 12))
    E[_src_cols(L, x), np.arange(12)] = 1
    iw = idx((m - 1) * delta, (m + 2) * delta)
    psi = np.zeros((12 * V, 12), complex)
    psi[iw] = np.linalg.solve(D[np.ix_(iw, iw)], E[iw])
    for i in range(m + 1, l + 1):
        ia = idx(i * delta, (i + 2) * delta)
        ii, ip = idx(i * delta, (i + 1) * delta), idx((i - 1) * delta, i * delta)
        hop = np.zeros((12 * V, 12), complex)
        hop[ii] = D[np.ix_(ii, ip)] @ psi[ip]                   # B_{i,i-1} psi
        psi = np.zeros((12 * V, 12), complex)
        psi[ia] = -np.linalg.solve(D[np.ix_(ia, ia)], hop[ia])  # -A_i B_{i,i-1} psi
    got = oracle.factorized_chain(U, L, kappa, inputs.point_source(L, x), _chain_domains(L, delta, m, l),
                                  C=Cl, antiperiodic=bc)
    assert len(got) == l - m + 1
    ref = _columns(psi, V)
    assert np.abs(got[-1] - ref).max() < 1e-11 * np.abs(ref).max()


def test_domains_running_to_the_end_give_the_exact_propagator():
    """Open time boundaries (with a wrap, the later domains would also need
    the propagator on slice 0, which the previous domain does not hold)."""
    bc = oracle.OPEN
    L = (10, 2, 2, 2)
    kappa = 0.13
    U = inputs.random_links(L, 1601302, 0.4)
    V = int(np.prod(L))
    C = oracle.clover_term(U, L, 0.9)
    Dinv = np.linalg.inv(_dense_operator(U, L, kappa, bc, C))
    x = (1, 0, 1, 0)
    doms = [_block(L, 0, L[0])] + [_block(L, t, L[0]) for t in (3, 5, 8)]
    got = oracle.factorized_chain(U, L, kappa, inputs.point_source(L, x), doms, C=C, antiperiodic=bc)
    S = _columns(Dinv[:, _src_cols(L, x)], V)
    for (lo, hi), psi in zip(doms, got):
        mk = oracle.domain_mask(L, lo, hi)
        assert np.abs(psi[:, mk] - S[:, mk]).max() < 1e-11 * np.abs(S).max()
        assert not psi[:, ~mk].any()


def test_two_domains_are_the_two_domain_factorization():
    L = (8, 2, 2, 2)
    U = inputs.random_links(L, 1601303, 0.4)
    b = inputs.point_source(L, (1, 0, 0, 1))
    bar, star = _block(L, 0, 6), _block(L, 4, 8)
    chain = oracle.factorized_chain(U, L, 0.13, b, [bar, star], antiperiodic=oracle.OPEN)
    sf, psi = oracle.factorized_propagator(U, L, 0.13, b, bar, star, antiperiodic=oracle.OPEN)
    # the same steps (the oracle's threaded reductions may round differently run to run)
    assert np.abs(chain[0] - psi).max() < 1e-14 * np.abs(psi).max()
    assert np.abs(chain[1] - sf).max() < 1e-13 * np.abs(sf).max()


def test_error_shrinks_with_the_slab_thickness():
    L = (24, 2, 2, 2)
    kappa = 0.11
    U = inputs.random_links(L, 1601304, 0.3)
    V = int(np.prod(L))
    Dinv = np.linalg.inv(_dense_operator(U, L, kappa, oracle.OPEN))
    x = (4, 0, 0, 0)
    S = _columns(Dinv[:, _src_cols(L, x)], V)
    ysl = (20, 24)
    mk = oracle.domain_mask(L, *_block(L, *ysl))
    err = []
    for delta in (2, 3, 4):
        m, l = x[0] // delta, ysl[0] // delta       # source slab, sink slab
        got = oracle.factorized_chain(U, L, kappa, inputs.point_source(L, x), _chain_domains(L, delta, m, l),
                                      antiperiodic=oracle.OPEN)
        err.append(np.linalg.norm(got[-1][:, mk] - S[:, mk]) / np.linalg.norm(S[:, mk]))
    assert err[0] > err[1] > err[2], err
    assert err[2] < 0.1 * err[0], err
