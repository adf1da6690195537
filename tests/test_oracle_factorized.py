"""Pins of the oracle's two-domain factorization and connected pion contraction.

The factorized propagator S^(f) = -D_{Gamma*}^{-1} D_{dGamma*} D_{Gammabar}^{-1}
(Section 5.2, eq. approxlong) is checked against dense block algebra of a
matrix assembled independently from the difference operators of Appendix A:
it is the exact off-diagonal block of D^{-1} (eq. Scmpt2) when Gammabar is the
whole lattice, it is the stated product of dense blocks for a smaller
Gammabar, and its distance to the exact propagator falls exponentially with
the overlap thickness Delta (eq. errorfact).  The pion contraction is pinned by
the free-field propagator in momentum space and by the gamma5 form of the Wick
contraction computed from the other off-diagonal block.  Open boundary
conditions in time are pinned by embedding the lattice in a longer one.
"""
import numpy as np
import pytest

import inputs
import oracle
from tests import _dense
from tests.test_oracle_operator import _free_momentum_propagator

L8 = (8, 2, 2, 2)
ORIGIN = (0, 0, 0, 0)


def _dense_operator(U, L, kappa, bc, C=None):
    """Dense D on the lattice L.  Open time boundaries: the block [0,T) of the
    periodic operator on a lattice twice as long in time, whose first T slices
    carry U (Dirichlet restriction, eq. blkdec, keeps the site-diagonal part)."""
    V = int(np.prod(L))
    if bc == oracle.OPEN:
        Lb = (2 * L[0],) + tuple(L[1:])
        Ub = np.concatenate([U, inputs.random_links(L, 1601990, 0.3)])
        D = _dense.wilson_dirac(Ub, Lb, kappa, antiperiodic=False)[:12 * V, :12 * V]
    else:
        D = _dense.wilson_dirac(U, L, kappa, antiperiodic=bool(bc))
    if C is not None:
        for s in range(V):
            D[12 * s:12 * s + 12, 12 * s:12 * s + 12] += C[s]
    return D


def _columns(vec12, V):
    """[12V, 12] matrix of point-source columns -> [12, V, 4, 3] propagator array."""
    return vec12.T.reshape(12, V, 4, 3)


def _src_cols(L, x):
    s = inputs.site_index(L, x)
    return np.arange(12 * s, 12 * s + 12)


def test_open_time_boundary_matches_embedded_dirichlet_block(rng):
    L = (6, 2, 2, 2)
    kappa = 0.13
    U = inputs.random_links(L, 1601201, 0.4)
    V = int(np.prod(L))
    D = _dense_operator(U, L, kappa, oracle.OPEN)
    psi = rng.normal(size=(2, V, 4, 3)) + 1j * rng.normal(size=(2, V, 4, 3))
    out = oracle.apply_D(U, L, kappa, psi, antiperiodic=oracle.OPEN)
    ref = (D @ psi.reshape(2, -1).T).T.reshape(out.shape)
    assert np.abs(out - ref).max() < 1e-13
    # and it differs from both periodic and antiperiodic (the wrap hops are gone)
    for bc in (True, False):
        assert np.abs(oracle.apply_D(U, L, kappa, psi, antiperiodic=bc) - out).max() > 0.1


@pytest.mark.parametrize("bc", [True, oracle.OPEN])
@pytest.mark.parametrize("csw", [0.0, 1.2])
def test_factorized_is_exact_when_gammabar_is_the_lattice(bc, csw):
    """Bottom-left block of eq. Scmpt2: for x outside Gamma* and y in Gamma*,
    S(y,x) = -D_{Gamma*}^{-1} D_{dGamma*} S(.,x) exactly."""
    L = L8
    kappa = 0.13
    U = inputs.random_links(L, 1601202, 0.4)
    V = int(np.prod(L))
    C = oracle.clover_term(U, L, csw) if csw else None
    Dinv = np.linalg.inv(_dense_operator(U, L, kappa, bc, C))
    x = (1, 1, 0, 1)
    star = ((4, 0, 0, 0), L)
    b = inputs.point_source(L, x)
    sf, psi = oracle.factorized_propagator(U, L, kappa, b, (ORIGIN, L), star, C=C, antiperiodic=bc)
    S = _columns(Dinv[:, _src_cols(L, x)], V)
    m = oracle.domain_mask(L, *star)
    assert np.abs(psi - S).max() < 1e-11 * np.abs(S).max()
    assert np.abs(sf[:, m] - S[:, m]).max() < 1e-11 * np.abs(S[:, m]).max()
    assert not sf[:, ~m].any()


@pytest.mark.parametrize("bc", [True, oracle.OPEN])
def test_factorized_equals_dense_block_product(bc):
    """eq. approxlong for Gammabar smaller than the lattice, written with
    dense blocks: D_{dGamma*} is the block D[Gamma*, complement of Gamma*]."""
    L = L8
    kappa = 0.13
    U = inputs.random_links(L, 1601203, 0.4)
    V = int(np.prod(L))
    D = _dense_operator(U, L, kappa, bc)
    bar = (ORIGIN, (6, 2, 2, 2))
    star = ((4, 0, 0, 0), L)
    ib = _dense.domain_indices(L, *bar)
    i_s = _dense.domain_indices(L, *star)
    ic = np.setdiff1d(np.arange(12 * V), i_s)
    x = (1, 0, 1, 1)
    E = np.zeros((12 * V, 12))
    E[_src_cols(L, x), np.arange(12)] = 1
    psi = np.zeros((12 * V, 12), complex)
    psi[ib] = np.linalg.solve(D[np.ix_(ib, ib)], E[ib])
    bstar = -D[np.ix_(i_s, ic)] @ psi[ic]
    sf = np.zeros((12 * V, 12), complex)
    sf[i_s] = np.linalg.solve(D[np.ix_(i_s, i_s)], bstar)
    got, gpsi = oracle.factorized_propagator(U, L, kappa, inputs.point_source(L, x), bar, star, antiperiodic=bc)
    ref = _columns(sf, V)
    assert np.abs(gpsi - _columns(psi, V)).max() < 1e-11 * np.abs(psi).max()
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()
    # D_{dGamma*} reaches Gamma* only through its faces: the cut at t=4, and with
    # a periodic or antiperiodic time direction also the wrap at t=7
    bs = -oracle.apply_boundary(U, L, gpsi, *star, antiperiodic=bc)
    slices = sorted({t for t in range(L[0]) if np.abs(bs.reshape(12, L[0], -1)[:, t]).max() > 0})
    assert slices == ([4] if bc == oracle.OPEN else [4, 7])


def test_factorization_error_falls_exponentially_with_delta():
    """eq. errorfact: ||S - S^(f)|| on Gamma* decays like exp(-M Delta)."""
    L = (20, 2, 2, 2)
    kappa = 0.11
    U = inputs.random_links(L, 1601204, 0.3)
    V = int(np.prod(L))
    Dinv = np.linalg.inv(_dense_operator(U, L, kappa, oracle.OPEN))
    x = (3, 0, 0, 0)
    star = ((8, 0, 0, 0), L)
    m = oracle.domain_mask(L, *star)
    S = _columns(Dinv[:, _src_cols(L, x)], V)
    b = inputs.point_source(L, x)
    err = []
    for delta in range(1, 9):
        sf, _ = oracle.factorized_propagator(U, L, kappa, b, (ORIGIN, (8 + delta, 2, 2, 2)), star,
                                             antiperiodic=oracle.OPEN)
        err.append(np.linalg.norm(sf[:, m] - S[:, m]) / np.linalg.norm(S[:, m]))
    err = np.array(err)
    assert np.all(np.diff(err) < 0), err
    rate = np.log(err[:-1] / err[1:])          # per slice of Delta
    assert rate.min() > 0.5, rate
    assert err[-1] < 1e-3 * err[0]


def test_pion_contraction_free_field_closed_form():
    """C_Pc(y0) = -(1/L^3) sum_y tr{S S^dag} with the free momentum-space
    propagator (trivial colour: a factor 3)."""
    L = (8, 4, 2, 2)
    kappa = 0.12
    V = int(np.prod(L))
    U = inputs.unit_links(L)
    b = inputs.point_source(L, ORIGIN)
    x, _, res = oracle.solve(U, L, kappa, b, tol=1e-13)
    assert res.max() < 1e-13
    Sx = _free_momentum_propagator(L, kappa, _dense.gammas())          # [y, alpha, beta]
    w = 3 * np.einsum("yab,yab->y", Sx, Sx.conj()).real
    ref = -w.reshape(L[0], -1).sum(axis=1) / (V // L[0])
    got = oracle.pion_connected(x, L)
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()
    assert np.all(got < 0)


def test_pion_contraction_equals_gamma5_wick_form():
    """W_Pc(y,x) = tr{g5 S(y,x) g5 S(x,y)} (eq. pipi) equals tr{S S^dag}
    (eq. W0pc) by gamma5-hermiticity; S(x,y) is read from the other
    off-diagonal block of a dense inverse."""
    L = L8
    kappa = 0.13
    U = inputs.random_links(L, 1601205, 0.4)
    V = int(np.prod(L))
    C = oracle.clover_term(U, L, 1.0)
    Dinv = np.linalg.inv(_dense_operator(U, L, kappa, True, C))
    x = (2, 1, 0, 1)
    sx = inputs.site_index(L, x)
    g = _dense.gammas()
    G5 = np.kron(g[0] @ g[1] @ g[2] @ g[3], np.eye(3))
    W = np.array([np.trace(G5 @ Dinv[12 * y:12 * y + 12, 12 * sx:12 * sx + 12] @ G5
                           @ Dinv[12 * sx:12 * sx + 12, 12 * y:12 * y + 12]) for y in range(V)])
    assert np.abs(W.imag).max() < 1e-12 * np.abs(W).max()
    ref = -W.real.reshape(L[0], -1).sum(axis=1) / (V // L[0])
    sol = _columns(Dinv[:, _src_cols(L, x)], V)
    assert np.abs(oracle.pion_connected(sol, L) - ref).max() < 1e-12 * np.abs(ref).max()
    # series bookkeeping of eq. seriespi: the differences telescope and the rest closes it
    lv = np.stack([0.5 * sol, 0.9 * sol, sol])
    Cs, diffs, rest = oracle.contract_pion(lv, L, full=1.1 * sol)
    assert np.allclose(diffs.sum(axis=0), Cs[-1]) and np.allclose(Cs[-1] + rest, 1.21 * Cs[-1])


@pytest.mark.parametrize("bc", [True, oracle.OPEN])
def test_site_by_site_operator_and_boundary_agree_with_whole_field(rng, bc):
    """The site-by-site forms used on large lattices give the whole-field values."""
    L = (8, 4, 2, 4)
    kappa = 0.13
    U = inputs.random_links(L, 1601206, 0.4)
    V = int(np.prod(L))
    C = oracle.clover_term(U, L, 1.3)
    psi = rng.normal(size=(3, V, 4, 3)) + 1j * rng.normal(size=(3, V, 4, 3))
    sites = rng.choice(V, size=40, replace=False)
    lo, hi = (2, 0, 0, 2), (6, 4, 2, 4)
    full = oracle.apply_D(U, L, kappa, psi, C=C, antiperiodic=bc, lo=lo, hi=hi)
    assert np.array_equal(oracle.apply_D_sites(U, L, kappa, psi, sites, csw=1.3, antiperiodic=bc, lo=lo, hi=hi),
                          full[:, sites])
    bd = oracle.apply_boundary(U, L, psi, lo, hi, antiperiodic=bc)
    got = oracle.apply_boundary_sites(U, L, psi, sites, lo, hi, antiperiodic=bc)
    assert np.abs(got - bd[:, sites]).max() < 1e-13 * np.abs(bd).max()
