"""Pins of the FP64 oracle's operator, domain restriction and solver.

Each test checks the oracle against something other than its own formulas:
closed forms (free-field propagators in momentum space), an independent dense
assembly from the difference operators of Appendix A, exact identities
(gamma5-hermiticity eq. g5h, gauge covariance, the hopping-parameter trace
identity eq. HPEtr, the block-inverse identity eq. bella / eq. Scmpt) and a
hand-computed clover term.
"""
import numpy as np
import pytest

import inputs
import oracle
from tests import _dense

L44 = (4, 4, 4, 4)


def _rand_spinor(rng, L, n=1):
    V = int(np.prod(L))
    return rng.normal(size=(n, V, 4, 3)) + 1j * rng.normal(size=(n, V, 4, 3))


def _g5(psi):
    out = psi.copy()
    out[..., 2:, :] *= -1
    return out


# ------------------------------------------------------------ gamma algebra
def test_gamma_algebra_and_charge_conjugation():
    g = [oracle.gamma(m) for m in range(4)]
    gd = _dense.gammas()
    for m in range(4):
        assert np.array_equal(g[m], gd[m])                       # basis from Pauli matrices
        assert np.allclose(g[m], g[m].conj().T)                  # Hermitian
        for n in range(4):
            assert np.allclose(g[m] @ g[n] + g[n] @ g[m], 2 * (m == n) * np.eye(4))
    g5 = oracle.gamma5()
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))
    C = oracle.charge_conjugation()
    Ci = np.linalg.inv(C)
    for m in range(4):
        assert np.allclose(C @ g[m] @ Ci, -g[m].T)
    Cg5 = C @ g5
    assert np.allclose(Cg5, -Cg5.T)
    Pm = oracle.P_minus()
    assert np.allclose(Pm @ Pm, Pm)


# --------------------------------------------------------------- free field
def _free_momentum_propagator(L, kappa, g):
    """S(x, 0) = (1/V) sum_p e^{ipx} [m(p) - i gamma.sin p] / [m(p)^2 + sum sin^2 p]."""
    V = int(np.prod(L))
    m0 = 1 / (2 * kappa) - 4
    ps = [(2 * np.arange(L[0]) + 1) * np.pi / L[0]] + [2 * np.pi * np.arange(n) / n for n in L[1:]]
    P = np.meshgrid(*ps, indexing="ij")
    X = np.meshgrid(*[np.arange(n) for n in L], indexing="ij")
    S = np.zeros(tuple(L) + (4, 4), complex)
    for idx in np.ndindex(*L):
        p = [P[m][idx] for m in range(4)]
        mp = m0 + sum(1 - np.cos(q) for q in p)
        num = mp * np.eye(4) - 1j * sum(g[m] * np.sin(p[m]) for m in range(4))
        den = mp ** 2 + sum(np.sin(q) ** 2 for q in p)
        ph = np.exp(1j * sum(p[m] * X[m] for m in range(4)))
        S += ph[..., None, None] * (num / den)
    return (S / V).reshape(V, 4, 4)


def test_free_field_full_lattice_matches_momentum_space():
    L = (8, 4, 4, 4)
    kappa = 0.12
    U = inputs.unit_links(L)
    b = inputs.point_source(L, (0, 0, 0, 0))
    x, it, res = oracle.solve(U, L, kappa, b, tol=1e-13)
    assert res.max() < 1e-13
    V = int(np.prod(L))
    S_or = x.reshape(4, 3, V, 4, 3)[:, 0, :, :, 0].transpose(1, 2, 0)   # [y, alpha, beta]
    S_ex = _free_momentum_propagator(L, kappa, _dense.gammas())
    assert np.abs(S_or - S_ex).max() < 1e-12
    # colour is diagonal and trivial for U = 1
    assert np.abs(x.reshape(4, 3, V, 4, 3)[:, 0, :, :, 1]).max() < 1e-14


def test_free_field_dirichlet_slab_matches_spatial_fourier_solution():
    """U = 1 on a time slab [t0,t1): spatial Fourier modes decouple and each
    leaves a block-tridiagonal matrix in time with diagonal
    (m0+1) + sum_k (1 - cos p_k + i gamma_k sin p_k) and couplings -P_- (t -> t+1),
    -P_+ (t -> t-1), both dropped at the slab ends (Dirichlet)."""
    L = (8, 4, 4, 4)
    t0, t1 = 2, 6
    kappa = 0.125
    m0 = 1 / (2 * kappa) - 4
    g = _dense.gammas()
    Pm = 0.5 * (np.eye(4) - g[0])
    Pp = 0.5 * (np.eye(4) + g[0])
    ts = 3
    U = inputs.unit_links(L)
    b = inputs.point_source(L, (ts, 0, 0, 0))
    x, it, res = oracle.solve(U, L, kappa, b, lo=(t0, 0, 0, 0), hi=(t1, 4, 4, 4), tol=1e-13)
    V = int(np.prod(L))
    S_or = x.reshape(4, 3, V, 4, 3)[:, 0, :, :, 0].transpose(1, 2, 0).reshape(L + (4, 4))
    nt = t1 - t0
    V3 = L[1] * L[2] * L[3]
    S_ex = np.zeros(L + (4, 4), complex)
    X = np.meshgrid(*[np.arange(n) for n in L[1:]], indexing="ij")
    for n in np.ndindex(*L[1:]):
        p = [2 * np.pi * n[k] / L[k + 1] for k in range(3)]
        diag = (m0 + 1) * np.eye(4) + sum((1 - np.cos(p[k])) * np.eye(4) + 1j * np.sin(p[k]) * g[k + 1]
                                          for k in range(3))
        M = np.zeros((4 * nt, 4 * nt), complex)
        for t in range(nt):
            M[4 * t:4 * t + 4, 4 * t:4 * t + 4] = diag
            if t + 1 < nt:
                M[4 * t:4 * t + 4, 4 * t + 4:4 * t + 8] = -Pm
                M[4 * t + 4:4 * t + 8, 4 * t:4 * t + 4] = -Pp
        Minv = np.linalg.inv(M)
        ph = np.exp(1j * sum(p[k] * X[k] for k in range(3)))
        for t in range(nt):
            blk = Minv[4 * t:4 * t + 4, 4 * (ts - t0):4 * (ts - t0) + 4]
            S_ex[t0 + t] += ph[..., None, None] * blk / V3
    assert np.abs(S_or - S_ex).max() < 1e-12
    outside = np.r_[0:t0, t1:L[0]]
    assert np.abs(S_or[outside]).max() == 0.0


# ------------------------------------------------------ dense construction
@pytest.fixture(scope="module")
def tiny():
    L = (4, 2, 2, 2)
    U = inputs.random_links(L, 1601001)
    return L, U


def test_stencil_equals_dense_assembly_from_difference_operators(tiny, rng):
    L, U = tiny
    kappa = 0.12
    D = _dense.wilson_dirac(U, L, kappa)
    psi = _rand_spinor(rng, L, 3)
    out = oracle.apply_D(U, L, kappa, psi)
    ref = (D @ psi.reshape(3, -1).T).T.reshape(psi.shape)
    assert np.abs(out - ref).max() < 1e-13 * np.abs(ref).max()
    # periodic time as well
    Dp = _dense.wilson_dirac(U, L, kappa, antiperiodic=False)
    outp = oracle.apply_D(U, L, kappa, psi, antiperiodic=False)
    assert np.abs(outp - (Dp @ psi.reshape(3, -1).T).T.reshape(psi.shape)).max() < 1e-12


def test_domain_operator_is_the_diagonal_block(tiny, rng):
    """eq. blkdec: D_Gamma acts like D on Gamma with every term that touches the
    exterior boundary set to zero, i.e. it is the Gamma-Gamma block of D."""
    L, U = tiny
    kappa = 0.13
    D = _dense.wilson_dirac(U, L, kappa)
    lo, hi = (1, 0, 0, 0), (3, 2, 2, 2)
    idx = _dense.domain_indices(L, lo, hi)
    V = int(np.prod(L))
    psi = _rand_spinor(rng, L, 2)
    mask = oracle.domain_mask(L, lo, hi)
    psi_g = psi * mask[None, :, None, None]
    out = oracle.apply_D(U, L, kappa, psi_g, lo=lo, hi=hi).reshape(2, -1)
    ref = np.zeros((2, 12 * V), complex)
    ref[:, idx] = (D[np.ix_(idx, idx)] @ psi_g.reshape(2, -1)[:, idx].T).T
    assert np.abs(out - ref).max() < 1e-13 * np.abs(ref).max()


def test_gamma5_hermiticity_full_and_domain(rng):
    """eq. g5h (and its block form eq. g5Hermite): <phi, D psi> = <g5 D g5 phi, psi>."""
    L = (4, 4, 4, 4)
    U = inputs.random_links(L, 3)
    C = oracle.clover_term(U, L, 1.769)
    for lo, hi, CC in [(None, None, None), ((1, 0, 0, 0), (3, 4, 4, 4), None), (None, None, C),
                       ((0, 1, 0, 0), (4, 3, 4, 4), C)]:
        mask = oracle.domain_mask(L, lo, hi)[None, :, None, None]
        phi = _rand_spinor(rng, L) * mask
        psi = _rand_spinor(rng, L) * mask
        lhs = np.vdot(phi, oracle.apply_D(U, L, 0.134, psi, C=CC, lo=lo, hi=hi))
        rhs = np.vdot(_g5(oracle.apply_D(U, L, 0.134, _g5(phi), C=CC, lo=lo, hi=hi)), psi)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _random_su3(rng, n):
    Z = rng.normal(size=(n, 3, 3)) + 1j * rng.normal(size=(n, 3, 3))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=1, axis2=2)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    return Q / det[:, None, None] ** (1 / 3)


def _gauge_transform(U, L, Om):
    V = int(np.prod(L))
    Up = np.empty_like(U)
    for s, x in enumerate(np.ndindex(*L)):
        for mu in range(4):
            y = list(x)
            y[mu] = (y[mu] + 1) % L[mu]
            sy = inputs.site_index(L, y)
            Up[s, mu] = Om[s] @ U[s, mu] @ Om[sy].conj().T
    return Up


def test_gauge_covariance_with_clover(rng):
    L = (4, 4, 2, 2)
    U = inputs.random_links(L, 5)
    V = int(np.prod(L))
    Om = _random_su3(rng, V)
    Up = _gauge_transform(U, L, Om)
    psi = _rand_spinor(rng, L, 2)
    C = oracle.clover_term(U, L, 1.769)
    Cp = oracle.clover_term(Up, L, 1.769)
    lo, hi = (1, 0, 0, 0), (4, 4, 2, 2)
    out = oracle.apply_D(U, L, 0.13, psi, C=C, lo=lo, hi=hi)
    psi_p = np.einsum("sab,rsib->rsia", Om, psi)
    out_p = oracle.apply_D(Up, L, 0.13, psi_p, C=Cp, lo=lo, hi=hi)
    assert np.abs(out_p - np.einsum("sab,rsib->rsia", Om, out)).max() < 1e-12


# ------------------------------------------------------------------ clover
def test_clover_basic_properties():
    L = (4, 4, 4, 4)
    U = inputs.random_links(L, 9)
    C = oracle.clover_term(U, L, 1.769)
    assert np.abs(C - C.conj().transpose(0, 2, 1)).max() < 1e-14           # Hermitian
    G5 = np.kron(np.diag([1, 1, -1, -1]), np.eye(3))
    assert np.abs(G5 @ C - C @ G5).max() < 1e-14                            # chiral blocks
    assert np.abs(oracle.clover_term(U, L, 0.0)).max() == 0.0               # c_sw = 0: Wilson
    assert np.abs(oracle.clover_term(inputs.unit_links(L), L, 1.769)).max() == 0.0
    assert np.abs(C).max() > 0.01


def test_clover_single_link_hand_computed():
    """Only U_0(x0) = W = diag(e^{i th}, e^{-i th}, 1) differs from 1.

    In the (0,nu) plane, the plaquette with lower corner x0 gives leaf W at its
    four corners and the one with lower corner x0 - nu gives W^dag.  So at
    x0 + nu: Fhat_{0 nu} = (W - W^dag)/8 = (i sin th / 4) diag(1,-1,0), and the
    clover term there is c_sw (i/4) * 2 sigma_{0 nu} Fhat_{0 nu}
    = -(c_sw sin th / 8) sigma_{0 nu} (x) diag(1,-1,0), sigma_{0 nu} = i g0 g_nu.
    At x0 and x0 + 0 the two plaquettes cancel."""
    L = (4, 4, 4, 4)
    th = 0.7
    csw = 1.3
    U = inputs.unit_links(L)
    x0 = (1, 2, 1, 3)
    s0 = inputs.site_index(L, x0)
    U[s0, 0] = np.diag([np.exp(1j * th), np.exp(-1j * th), 1.0])
    C = oracle.clover_term(U, L, csw)
    g = _dense.gammas()
    dcol = np.diag([1.0, -1.0, 0.0])
    for nu in (1, 2, 3):
        x = list(x0)
        x[nu] = (x[nu] + 1) % 4
        sig = 1j * g[0] @ g[nu]
        expect = -(csw * np.sin(th) / 8) * np.kron(sig, dcol)
        assert np.abs(C[inputs.site_index(L, x)] - expect).max() < 1e-15
        x = list(x0)
        x[nu] = (x[nu] - 1) % 4
        assert np.abs(C[inputs.site_index(L, x)] + expect).max() < 1e-15
    assert np.abs(C[s0]).max() < 1e-15
    x = list(x0)
    x[0] += 1
    assert np.abs(C[inputs.site_index(L, x)]).max() < 1e-15
    nonzero = np.nonzero(np.abs(C).reshape(C.shape[0], -1).max(axis=1) > 0)[0]
    assert len(nonzero) == 12          # 3 planes x 4 sites (x0 +- nu, x0 + 0 +- nu)


# ---------------------------------------------------------- normalisation
def test_hopping_parameter_trace_identity():
    """eq. HPEtr: tr{g5 D^{-1}} = kappa^p tr{g5 D_hop^p D^{-1}} for p <= 8 (Wilson),
    with 2 kappa D = 1 - kappa D_hop; exact with a dense inverse on 4^4."""
    L = L44
    kappa = 0.12
    U = inputs.random_links(L, 1601001, eps=1.0)
    V = int(np.prod(L))
    D = _dense.wilson_dirac(U, L, kappa)
    Dinv = np.linalg.inv(D)
    # gamma5 is diagonal in the (site, spin, colour) basis: tr{g5 X} = sum_i g5_i X_ii
    g5 = np.tile(np.repeat([1.0, 1.0, -1.0, -1.0], 3), V)
    lhs = np.sum(g5 * np.diagonal(Dinv))
    # D_hop applied with the oracle to the columns of D^{-1}
    cols = Dinv.T.reshape(12 * V, V, 4, 3)
    Y = cols
    for p in range(1, 9):
        Y = oracle.apply_hop(U, L, Y)
        rhs = kappa ** p * np.sum(g5 * np.diagonal(Y.reshape(12 * V, 12 * V)))
        assert abs(rhs - lhs) < 1e-10 * abs(lhs), p
    # p = 9 is no longer exact on a random field
    Y = oracle.apply_hop(U, L, Y)
    r9 = kappa ** 9 * np.sum(g5 * np.diagonal(Y.reshape(12 * V, 12 * V)))
    assert abs(r9 - lhs) > 1e-6 * abs(lhs)
    # normalisation of D: D = (1 - kappa D_hop) / (2 kappa) exactly
    psi = np.random.default_rng(0).normal(size=(1, V, 4, 3)) + 0j
    assert np.abs(oracle.apply_D(U, L, kappa, psi)
                  - (psi - kappa * oracle.apply_hop(U, L, psi)) / (2 * kappa)).max() < 1e-13


# ------------------------------------------------------------------ solver
@pytest.mark.slow
def test_solve_matches_dense_lu_on_4_4():
    """4^4 lattice, U = exp(i 0.3 H), kappa = 0.12, antiperiodic time: BiCGstab
    columns vs a dense LU solve of the 3072 x 3072 matrix."""
    L = L44
    kappa = 0.12
    U = inputs.random_links(L, 1601001)
    D = _dense.wilson_dirac(U, L, kappa)
    b = inputs.point_source(L, (0, 0, 0, 0))
    x, it, res = oracle.solve(U, L, kappa, b, tol=1e-13)
    assert res.max() <= 1e-13
    ref = np.linalg.solve(D, b.reshape(12, -1).T).T.reshape(b.shape)
    assert np.abs(x - ref).max() < 1e-11 * np.abs(ref).max()


def test_domain_solve_and_block_inverse_identity():
    """eq. bella: for x, y in Gamma,
    S(y,x) = S^(i)(y,x) + sum_{w1,w2} S^(i)(y,w1) [D_dG D^{-1} D_dG*](w1,w2) S^(i)(w2,x)
    with S^(i) = D_Gamma^{-1} from the oracle's domain solve, D^{-1} from its full
    solve and the boundary blocks taken from the independent dense matrix."""
    L = (4, 2, 2, 2)
    U = inputs.random_links(L, 77)
    kappa = 0.125
    lo, hi = (1, 0, 0, 0), (3, 2, 2, 2)
    V = int(np.prod(L))
    D = _dense.wilson_dirac(U, L, kappa)
    g = _dense.domain_indices(L, lo, hi)
    gs = np.setdiff1d(np.arange(12 * V), g)
    # oracle: full inverse and domain inverse, all columns
    E = np.eye(12 * V).reshape(12 * V, V, 4, 3)
    Sfull, _, r1 = oracle.solve(U, L, kappa, E, tol=1e-13)
    Sdom, _, r2 = oracle.solve(U, L, kappa, E[g], lo=lo, hi=hi, tol=1e-13)
    assert r1.max() < 1e-12 and r2.max() < 1e-12
    Sfull = Sfull.reshape(12 * V, 12 * V).T
    Sdom = Sdom.reshape(len(g), 12 * V).T[g]                   # D_Gamma^{-1} on Gamma
    # the domain inverse is the inverse of the diagonal block of the dense matrix
    assert np.abs(Sdom @ D[np.ix_(g, g)] - np.eye(len(g))).max() < 1e-11
    rhs = Sdom + Sdom @ D[np.ix_(g, gs)] @ Sfull[np.ix_(gs, gs)] @ D[np.ix_(gs, g)] @ Sdom
    assert np.abs(Sfull[np.ix_(g, g)] - rhs).max() < 1e-11
    assert np.abs(Sfull[np.ix_(g, g)] - Sdom).max() > 1e-4    # the correction is not trivial


def test_full_domain_equals_global_solve_and_series_telescopes():
    L = (16, 4, 4, 4)
    U = inputs.random_links(L, 12)
    C = oracle.clover_term(U, L, 1.769)
    kappa = 0.12
    ts = 8
    b = inputs.point_source(L, (ts, 1, 0, 2))
    doms = [((6, 0, 0, 0), (11, 4, 4, 4)), ((4, 0, 0, 0), (13, 4, 4, 4)), ((0, 0, 0, 0), L)]
    props = [oracle.solve(U, L, kappa, b, C=C, lo=lo, hi=hi, tol=1e-13)[0] for lo, hi in doms]
    xg, _, _ = oracle.solve(U, L, kappa, b, C=C, tol=1e-13)
    terms, total = oracle.series(props)
    assert np.abs(total - xg).max() < 1e-11 * np.abs(xg).max()
    assert np.abs(terms.sum(axis=0) - xg).max() < 1e-11 * np.abs(xg).max()
    # terms vanish outside their domain
    for i, (lo, hi) in enumerate(doms):
        m = ~oracle.domain_mask(L, lo, hi)
        if m.any():
            assert np.abs(props[i][:, m]).max() == 0.0
    # eq. error, qualitative: with x, y on the source slice, |S - S^(i)| falls
    # as the distance to the domain boundary grows
    V3 = 64
    sl = slice(ts * V3, (ts + 1) * V3)
    e0 = np.linalg.norm((xg - props[0])[:, sl])
    e1 = np.linalg.norm((xg - props[1])[:, sl])
    assert e1 < 0.8 * e0
