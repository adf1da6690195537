"""Dense-inverse pin of the disconnected pseudoscalar trace and its f/r1/r2 split.

Section 3, eqs. sing, W0, rall0, rall: with two non-overlapping thick time
slices Gamma_0 (holding x) and Gamma_0* (holding y),

    W^(f)  = tr{g5 D_G0^-1(x,x)} tr{g5 D_G0*^-1(y,y)}
    W^(r1) = tr{g5 K_x(x,x)} tr{g5 D_G0*^-1(y,y)} + (Gamma_0, x) <-> (Gamma_0*, y)
    W^(r2) = tr{g5 K_x(x,x)} tr{g5 K_y(y,y)}

with K_x = D_G0^-1 D_dG0 D^-1 D_dG0* D_G0^-1, whose middle D^-1 is the
(Gamma_0*, Gamma_0*) block of the inverse of the whole operator.  Every
expected value here is built from the dense Wilson-Dirac matrix of
``tests/_dense.py`` (assembled from the difference operators of App. A): the
domain operators are its diagonal blocks (eq. blkdec), the boundary operators
its off-diagonal blocks, the inverses are LAPACK's.  The oracle reaches the
same numbers a different way (point-source solves on each domain and on the
lattice, r-kernels as [S - S^(0)](x,x) by eq. bella), so a trace without g5,
a transposed or wrong-sign boundary term or a wrong 1/L^3 (eq. sing, L^3 the
spatial volume) cannot pass.  The test plants those mistakes and checks that
they fail.
"""
import numpy as np
import pytest

import inputs
import oracle
from tests import _dense

L = (6, 2, 2, 2)
KAPPA = 0.12
XS = (1, 1, 0, 1)     # in Gamma_0 = t in [0, 3)
YS = (4, 0, 1, 1)     # in Gamma_0* = t in [3, 6)
G0 = ((0, 0, 0, 0), (3, 2, 2, 2))
G0S = ((3, 0, 0, 0), (6, 2, 2, 2))


def _g5_site_trace(M, L, site):
    """tr_{spin,colour}{g5 M(site,site)} of a 12V x 12V dense matrix; the
    chiral g5 is diag(1,1,-1,-1) in spin (gamma_0 gamma_1 gamma_2 gamma_3)."""
    g = _dense.gammas()
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    blk = M[12 * site:12 * site + 12, 12 * site:12 * site + 12]
    return np.trace(np.kron(g5, np.eye(3)) @ blk)


def _embed(Minv_dom, idx, V):
    full = np.zeros((12 * V, 12 * V), complex)
    full[np.ix_(idx, idx)] = Minv_dom
    return full


@pytest.fixture(scope="module")
def dense_case():
    U = inputs.random_links(L, 16010307)
    V = int(np.prod(L))
    D = _dense.wilson_dirac(U, L, KAPPA)
    Dinv = np.linalg.inv(D)
    ia = _dense.domain_indices(L, *G0)
    ib = _dense.domain_indices(L, *G0S)
    Ainv = np.linalg.inv(D[np.ix_(ia, ia)])          # D_Gamma0^-1
    Binv = np.linalg.inv(D[np.ix_(ib, ib)])          # D_Gamma0*^-1
    # eq. rall0 kernels written with the blocks of D (Gamma_0 and Gamma_0*
    # cover the lattice, so the boundary operators are the off-diagonal blocks)
    Kx = Ainv @ D[np.ix_(ia, ib)] @ Dinv[np.ix_(ib, ib)] @ D[np.ix_(ib, ia)] @ Ainv
    Ky = Binv @ D[np.ix_(ib, ia)] @ Dinv[np.ix_(ia, ia)] @ D[np.ix_(ia, ib)] @ Binv
    sx, sy = inputs.site_index(L, XS), inputs.site_index(L, YS)
    tr = dict(
        x0=_g5_site_trace(_embed(Ainv, ia, V), L, sx),
        y0=_g5_site_trace(_embed(Binv, ib, V), L, sy),
        kx=_g5_site_trace(_embed(Kx, ia, V), L, sx),
        ky=_g5_site_trace(_embed(Ky, ib, V), L, sy),
        xfull=_g5_site_trace(Dinv, L, sx),
        yfull=_g5_site_trace(Dinv, L, sy),
        # the trace without g5, to show the pin can tell them apart
        x0_nog5=np.trace(_embed(Ainv, ia, V)[12 * sx:12 * sx + 12, 12 * sx:12 * sx + 12]),
    )
    # oracle side: point-source columns on the domain and on the lattice
    bx = inputs.point_source(L, XS)
    by = inputs.point_source(L, YS)
    full = ((0, 0, 0, 0), L)
    px = [oracle.solve(U, L, KAPPA, bx, lo=lo, hi=hi, tol=1e-13)[0] for lo, hi in (G0, full)]
    py = [oracle.solve(U, L, KAPPA, by, lo=lo, hi=hi, tol=1e-13)[0] for lo, hi in (G0S, full)]
    return U, sx, sy, tr, px, py


def test_dense_traces_are_distinct(dense_case):
    """The g5 trace differs from the plain trace and the r-kernels are not
    small here, so the comparisons below can see each mistake."""
    _, _, _, tr, _, _ = dense_case
    assert abs(tr["x0"] - tr["x0_nog5"]) > 1e-2 * abs(tr["x0_nog5"])
    assert abs(tr["kx"]) > 1e-4 * abs(tr["x0"]) and abs(tr["ky"]) > 1e-4 * abs(tr["y0"])
    # eq. bella: the r-kernel is the difference of the full and the domain trace
    assert abs(tr["xfull"] - tr["x0"] - tr["kx"]) < 1e-11 * abs(tr["xfull"])
    assert abs(tr["yfull"] - tr["y0"] - tr["ky"]) < 1e-11 * abs(tr["yfull"])


def test_pp_trace_equals_dense_g5_trace(dense_case):
    """pp_trace on one domain and on the whole lattice against tr{g5 D^-1(x,x)}."""
    _, sx, sy, tr, px, py = dense_case
    assert abs(oracle.pp_trace(px[0], sx) - tr["x0"]) < 1e-10 * abs(tr["x0"])
    assert abs(oracle.pp_trace(py[0], sy) - tr["y0"]) < 1e-10 * abs(tr["y0"])
    assert abs(oracle.pp_trace(px[1], sx) - tr["xfull"]) < 1e-10 * abs(tr["xfull"])
    assert abs(oracle.pp_trace(py[1], sy) - tr["yfull"]) < 1e-10 * abs(tr["yfull"])


def _expected(tr, L3):
    f = tr["x0"] * tr["y0"]
    r1 = tr["kx"] * tr["y0"] + tr["x0"] * tr["ky"]
    r2 = tr["kx"] * tr["ky"]
    full = tr["xfull"] * tr["yfull"]
    return np.array([f, r1, r2, full]) / L3


def _agrees(out, exp):
    return bool(np.all(np.abs(out - exp) < 1e-9 * np.abs(exp).max()))


def _contract(px, py, sx, sy, L3):
    tx, _ = oracle.series(px)
    ty, _ = oracle.series(py)
    return oracle.contract_pp_disconnected(tx, ty, sx, sy, L3)


def _level0(px, py, sx, sy, L3):
    return _contract(px, py, sx, sy, L3)[0]


def test_disconnected_pieces_equal_dense_blocks(dense_case):
    _, sx, sy, tr, px, py = dense_case
    L3 = L[1] * L[2] * L[3]
    out = _contract(px, py, sx, sy, L3)
    assert _agrees(out[0], _expected(tr, L3))
    # last level: the domain is the lattice, the rest vanishes
    assert abs(out[1, 0] - out[1, 3]) < 1e-12 * abs(out[1, 3])


def test_planted_mistakes_fail(dense_case, monkeypatch):
    """A trace without g5 and a normalisation other than 1/L^3 must fail."""
    _, sx, sy, tr, px, py = dense_case
    L3 = L[1] * L[2] * L[3]
    exp = _expected(tr, L3)
    # wrong normalisation: 1/V (the four-volume) instead of the spatial 1/L^3
    assert not _agrees(_level0(px, py, sx, sy, int(np.prod(L))), exp)
    # g5 dropped from the trace
    good = oracle.pp_trace

    def no_g5(sol, x_site):
        return np.trace(oracle.prop_matrix(sol, x_site))

    monkeypatch.setattr(oracle, "pp_trace", no_g5)
    assert not _agrees(_level0(px, py, sx, sy, L3), exp)
    monkeypatch.setattr(oracle, "pp_trace", good)
    assert _agrees(_level0(px, py, sx, sy, L3), exp)
