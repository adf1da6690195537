"""FP64 CPU oracle: plain definitions of everything the GPU path computes.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke`` and the
benchmark's CPU-baseline leg may import this package.  The product library in
``paper_1601_04587_amd`` never imports or links it, and shares no code with it.

Contents and the passages they follow:
  * ``apply_D``, ``apply_hop``, ``clover_term``, ``solve``  (oracle.c):
      Wilson-Dirac operator (Appendix A, eq. wdo), normalisation
      2 kappa D = 1 - kappa D_hop (Section 6), Sheikholeslami-Wohlert term
      (O(a) improvement, footnotes of Sections 4 and 6), Dirichlet restriction
      D_Gamma (Section 2, eq. blkdec), S^(i) = D_Gamma_i^{-1} (eq. diric).
  * ``series``: telescoping expansion S = S^(0) + [S^(1)-S^(0)] + ...
      (Section 1, eq. Dseries).
  * ``pp_trace``/``contract_pp_disconnected``: tr{gamma5 D_Gamma^{-1}(x,x)} and
      the split W = W^(f) + W^(r1) (+ swap) + W^(r2) (Section 3, eqs. W0, rall0,
      rall, with eq. bella identifying the r-kernels with [S - S^(0)](x,x)),
      normalised by 1/L^3 (eq. sing).
  * ``nucleon``: W_N1 - W_N2 (Section 5.2, eq. baryfact) summed over the sink
      time slice (eq. baryN), with C = i gamma0 gamma2 and P_- = (1-gamma0)/2.
  * ``apply_boundary``: D_{dGamma}, the block of D that couples the sites
      outside a domain to the sites inside it (Section 2, eq. blkdec; Appendix
      A, eq. Scmpt2).  Its entries are those of D itself, so a backward time
      hop into the domain carries -P_+ U_0(x-0)^dag and a forward one -P_-
      U_0(x), with the 1/2 of eq. wdo and the minus sign that the block formula
      eq. fact3 leaves out.
  * ``factorized_propagator``: S^(f) = -D_{Gamma*}^{-1} D_{dGamma*}
      D_{Gammabar}^{-1} (Section 5.2, eq. approxlong), the bottom-left block of
      eq. Scmpt2 with the exact Schur-complement inverse replaced by the
      propagator of the larger domain Gammabar.
  * ``factorized_chain``: the multi-slab product of Section 4 (steps 1-3,
      eqs. stp2, dec1, fctpr): psi_0 = D_{Omega_{m+2}}^{-1} b, then for each
      thick slab Omega*_i = Lambda_i u Lambda_{i+1} in turn
      psi_i = -D_{Omega*_i}^{-1} D_{Lambda_{i,i-1}} psi_{i-1}; the last one is
      S^(f) b on Omega*_l.  D_{Lambda_{i,i-1}} is the block of D itself (the
      same reading of eq. fact3 as for D_{dGamma}).
  * ``pion_connected``/``contract_pion``: C_Pc(y0) = -(1/L^3) sum tr{S S^dag}
      (eqs. pipi, W0pc) and its expansion in the overlap thickness Delta
      (eqs. decpi, seriespi, with the rest W^(r) = W - W^(f) of eq. W0pc2).

  * ``hop_power``/``hpe_trace``: the stochastic estimator of the
      disconnected trace sum_x tr{gamma5 D_Gamma^{-1}(x,x)} per time slice
      with the hopping parameter expansion (Section 6, eq. HPEtr and the
      estimator that follows it):
      (1/n) sum_i sum_x eta_i^dag(x) [(kappa D_hop)^p D_Gamma^{-1} gamma5 eta_i](x),
      with kappa D_hop = 1 - 2 kappa D (so that the clover term, when present,
      sits in the site-diagonal part of D_hop).  The identity holds for p <= 8
      with the Wilson operator and p <= 2 with the clover term (the trace of
      gamma5 (1 - A)^2 does not vanish).

  * ``inverse_iteration``/``gram_slices``/``projected_pion``: the
      projector-cut factorization (Section 5.2, eqs. approxlong2, fullfactpi,
      Bpions): basis vectors from inverse iterations of D on a domain, each
      iterate orthonormalised (Q of the QR factorisation with positive real
      diagonal R), per-slice Gram matrices of chi = D_Gammabar^{-1} gamma5 phi
      and eta = D_Gamma*^{-1} D_dGamma* phi, and C(y0, x0) =
      -(1/L^3) Re Tr(Gt(y0) G(x0)).

  * ``colourless_spinors``/``projected_nucleon``: the nucleon with the
      projector cut (Section 5.2, eq. W0tbary): colourless spinors
      B[s_i, s_j, s_k; x] of xi_i^T = phi_i^dag D_Gammabar^{-1} and of
      eta_i = D_Gamma*^{-1} D_dGamma* phi_i, summed per time slice, contracted
      with g5 P_- for W_N1 and W_N2.

  * ``level1_update``: quenched updates of a time slab with the spatial links
      of its first slice fixed (the level-1 updates of Section 3.1): Wilson
      plaquette action, Cabibbo-Marinari heatbath (Kennedy-Pendleton SU(2)
      sampler) plus SU(2) over-relaxation, Philox4x32-10 random numbers keyed
      by link and sweep (oracle.c states the exact mapping).

  * ``two_level``: the two-level estimator (Section 3.1): for every level-0
      field the level-1 means of the two factors, each over the updates of its
      own region, then the level-0 mean of their product; the remaining
      pieces grouped in bins of n1 and treated as n0 independent measurements
      (the averaging of the numerical part of Section 6).

Parity unpinned: the clover term's convention against the paper, which
mentions the O(a) improvement without writing the term; it is pinned to the
Sheikholeslami-Wohlert definition stated in oracle.c (single-link closed form,
hermiticity, gauge covariance), not to a formula of the paper.

Time boundary conditions: ``antiperiodic`` is True (antiperiodic), False
(periodic) or ``OPEN`` (hops across the time boundary dropped, the set-up
Sections 2 and 5.2 assume).

Array conventions (complex128):
  links U[site, mu, 3, 3]; spinors / propagator columns psi[rhs, site, 4, 3];
  a point-source propagator has rhs = 3*beta + b, so S(y,x)[alpha a, beta b] =
  psi[3*beta+b, y, alpha, a].
"""
import ctypes
import os
import subprocess

import numpy as np

OPEN = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=False):
    """Compile oracle.c into liboracle.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O2", "-fcx-limited-range", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", "-o", _LIB + ".tmp", _SRC, "-lm"])
        os.replace(_LIB + ".tmp", _LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i4 = ctypes.POINTER(ctypes.c_int)
        d = ctypes.c_double
        i = ctypes.c_int
        lib.oracle_gamma.argtypes = [i, P]
        lib.oracle_field_strength.argtypes = [i4, P, i, i, P]
        lib.oracle_clover_term.argtypes = [i4, P, d, P]
        lib.oracle_apply_D.argtypes = [i4, P, P, d, i, i4, i4, i, P, P]
        lib.oracle_apply_hop.argtypes = [i4, P, i, i4, i4, i, P, P]
        lib.oracle_apply_D_sites.argtypes = [i4, P, d, d, i, i4, i4, i, ctypes.c_long, P, P, P]
        u32 = ctypes.c_uint32
        lib.oracle_philox.argtypes = [P, P, P]
        lib.oracle_kp_sample.argtypes = [d, ctypes.c_uint64, ctypes.c_long, P]
        lib.oracle_level1_update.argtypes = [i4, d, ctypes.c_uint64, u32, i, i, i, i, P]
        lib.oracle_plaquette.argtypes = [i4, P]
        lib.oracle_plaquette.restype = d
        lib.oracle_solve.argtypes = [i4, P, P, d, i, i4, i4, i, P, P, d, i, P, P]
        lib.oracle_solve.restype = i
        _lib = lib
    return _lib


def _i4(v):
    return (ctypes.c_int * 4)(*[int(a) for a in v])


def _c(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _domain(L, lo, hi):
    lo = (0, 0, 0, 0) if lo is None else tuple(lo)
    hi = tuple(L) if hi is None else tuple(hi)
    return _i4(lo), _i4(hi)


# ----------------------------------------------------------------- algebra
def gamma(mu):
    """gamma_mu, mu = 0..3, in the chiral basis used throughout."""
    out = np.zeros((4, 4), dtype=np.complex128)
    _load().oracle_gamma(mu, out.ctypes.data)
    return out


def gamma5():
    return gamma(0) @ gamma(1) @ gamma(2) @ gamma(3)


def charge_conjugation():
    """C = i gamma0 gamma2 (Section 5.2)."""
    return 1j * gamma(0) @ gamma(2)


def P_minus():
    return 0.5 * (np.eye(4) - gamma(0))


# ---------------------------------------------------------------- operator
def field_strength(U, L, mu, nu):
    F = np.empty((int(np.prod(L)), 3, 3), dtype=np.complex128)
    _load().oracle_field_strength(_i4(L), _c(U).ctypes.data, mu, nu, F.ctypes.data)
    return F


def clover_term(U, L, csw):
    """Per-site 12x12 matrix c_sw (i/4) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}, index spin*3+colour."""
    C = np.empty((int(np.prod(L)), 12, 12), dtype=np.complex128)
    _load().oracle_clover_term(_i4(L), _c(U).ctypes.data, float(csw), C.ctypes.data)
    return C


def apply_D(U, L, kappa, psi, C=None, antiperiodic=True, lo=None, hi=None):
    """D_Gamma psi for psi[nrhs, V, 4, 3] (Gamma = [lo,hi), default the full lattice)."""
    U = _c(U)
    psi = _c(psi)
    squeeze = psi.ndim == 3
    if squeeze:
        psi = psi[None]
    out = np.empty_like(psi)
    Cp = None if C is None else _c(C).ctypes.data
    clo, chi = _domain(L, lo, hi)
    _load().oracle_apply_D(_i4(L), U.ctypes.data, Cp, float(kappa), int(antiperiodic), clo, chi,
                           psi.shape[0], psi.ctypes.data, out.ctypes.data)
    return out[0] if squeeze else out


def apply_D_sites(U, L, kappa, psi, sites, csw=0.0, antiperiodic=True, lo=None, hi=None):
    """(D_Gamma psi)(x) at the listed sites only: [nrhs, len(sites), 4, 3].

    The clover term (csw != 0) is built at those sites only, so a check on a
    large lattice needs no [V, 12, 12] array."""
    U = _c(U)
    psi = _c(psi)
    if psi.ndim == 3:
        psi = psi[None]
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((psi.shape[0], len(sites), 4, 3), dtype=np.complex128)
    clo, chi = _domain(L, lo, hi)
    _load().oracle_apply_D_sites(_i4(L), U.ctypes.data, float(csw), float(kappa), int(antiperiodic), clo, chi,
                                 psi.shape[0], len(sites), sites.ctypes.data, psi.ctypes.data, out.ctypes.data)
    return out


def apply_hop(U, L, psi, antiperiodic=True, lo=None, hi=None):
    """D_hop psi, the hopping term with 2 kappa D = 1 - kappa D_hop (Wilson)."""
    U = _c(U)
    psi = _c(psi)
    squeeze = psi.ndim == 3
    if squeeze:
        psi = psi[None]
    out = np.empty_like(psi)
    clo, chi = _domain(L, lo, hi)
    _load().oracle_apply_hop(_i4(L), U.ctypes.data, int(antiperiodic), clo, chi, psi.shape[0],
                             psi.ctypes.data, out.ctypes.data)
    return out[0] if squeeze else out


def solve(U, L, kappa, b, C=None, antiperiodic=True, lo=None, hi=None, tol=1e-13, maxiter=20000):
    """x = D_Gamma^{-1} b (zero outside Gamma) by BiCGstab; returns (x, iters, rel_residuals)."""
    U = _c(U)
    b = _c(b)
    squeeze = b.ndim == 3
    if squeeze:
        b = b[None]
    x = np.zeros_like(b)
    n = b.shape[0]
    iters = np.zeros(n, dtype=np.int32)
    res = np.zeros(n, dtype=np.float64)
    Cp = None if C is None else _c(C).ctypes.data
    clo, chi = _domain(L, lo, hi)
    _load().oracle_solve(_i4(L), U.ctypes.data, Cp, float(kappa), int(antiperiodic), clo, chi, n,
                         b.ctypes.data, x.ctypes.data, float(tol), int(maxiter), iters.ctypes.data,
                         res.ctypes.data)
    if squeeze:
        return x[0], iters, res
    return x, iters, res


def residual(U, L, kappa, b, x, C=None, antiperiodic=True, lo=None, hi=None):
    """Per-rhs ||P_Gamma b - D_Gamma x|| / ||P_Gamma b|| (x restricted to Gamma first)."""
    b = _c(b)
    x = _c(x)
    mask = domain_mask(L, lo, hi)
    bm = b * mask[None, :, None, None]
    xm = x * mask[None, :, None, None]
    r = bm - apply_D(U, L, kappa, xm, C=C, antiperiodic=antiperiodic, lo=lo, hi=hi)
    num = np.sqrt(np.sum(np.abs(r) ** 2, axis=(1, 2, 3)))
    den = np.sqrt(np.sum(np.abs(bm) ** 2, axis=(1, 2, 3)))
    return num / den


def domain_mask(L, lo=None, hi=None):
    lo = (0, 0, 0, 0) if lo is None else lo
    hi = tuple(L) if hi is None else hi
    t, x1, x2, x3 = np.meshgrid(*[np.arange(n) for n in L], indexing="ij")
    m = np.ones(L, dtype=bool)
    for c, a, b in zip((t, x1, x2, x3), lo, hi):
        m &= (c >= a) & (c < b)
    return m.reshape(-1)


# ------------------------------------------------------------------ series
def series(props):
    """Terms of eq. Dseries from the nested-domain propagators S^(0..n-1).

    Returns (terms, total): terms[0] = S^(0), terms[i] = S^(i) - S^(i-1),
    total = S^(n-1) (each S^(i) already zero outside Gamma_i)."""
    props = [np.asarray(p) for p in props]
    terms = [props[0].copy()] + [props[i] - props[i - 1] for i in range(1, len(props))]
    return np.stack(terms), props[-1].copy()


def cumulative(terms):
    """S^(i) = sum_{j<=i} terms[j]."""
    return np.cumsum(np.asarray(terms), axis=0)


# ----------------------------------------------------------- contractions
def prop_matrix(sol, site):
    """12x12 matrix S(y,x)[alpha a, beta b] at sink `site` from 12 point-source columns."""
    sol = np.asarray(sol)
    return sol[:, site, :, :].reshape(12, 12).T


def pp_trace(sol, x_site):
    """tr_{spin,colour}{gamma5 S(x,x)} (Section 3, eq. W0)."""
    S = prop_matrix(sol, x_site)
    G5 = np.kron(gamma5(), np.eye(3))
    return np.trace(G5 @ S)


def contract_pp_disconnected(terms_x, terms_y, x_site, y_site, L3):
    """Disconnected pseudoscalar pieces per level (Section 3, eqs. deco1, W0, rall0, rall).

    terms_x: series terms of the propagator from x (levels: nested domains
    around x, the last one the full lattice); terms_y the same for y.  For
    level i the domain propagators are S^(i) = sum_{j<=i} terms[j] and the full
    propagator is the sum of all terms; by eq. bella the r-kernels equal
    [S - S^(i)](x,x).  Returns out[level] = (f, r1, r2, full) each divided
    by L^3 (eq. sing; for point sources the spatial sums collapse).
    """
    cx = cumulative(terms_x)
    cy = cumulative(terms_y)
    n = cx.shape[0]
    tx = np.array([pp_trace(cx[i], x_site) for i in range(n)])
    ty = np.array([pp_trace(cy[i], y_site) for i in range(n)])
    out = np.zeros((n, 4), dtype=np.complex128)
    for i in range(n):
        dx = tx[-1] - tx[i]
        dy = ty[-1] - ty[i]
        out[i, 0] = tx[i] * ty[i]
        out[i, 1] = dx * ty[i] + tx[i] * dy
        out[i, 2] = dx * dy
        out[i, 3] = tx[-1] * ty[-1]
    return out / L3


def _eps():
    e = np.zeros((3, 3, 3))
    for a, b, c, s in [(0, 1, 2, 1), (1, 2, 0, 1), (2, 0, 1, 1), (0, 2, 1, -1), (2, 1, 0, -1), (1, 0, 2, -1)]:
        e[a, b, c] = s
    return e


def nucleon_W(Sarr):
    """W_N1 - W_N2 (eq. baryfact) per sink site; Sarr as in ``nucleon_W_parts``."""
    W1, W2 = nucleon_W_parts(Sarr)
    return W1 - W2


def nucleon_W_parts(Sarr):
    """W_N1 and W_N2 (eq. baryfact) per sink site.

    Sarr[y, alpha, a, beta, b] = S^{ab}_{alpha beta}(y, x) with S_u = S_d = S.
      W_N1 = eps^{abc} eps^{feg} tr[S^{ag T} C g5 S^{bf} C g5] tr[S^{ce} P_-]
      W_N2 = eps^{abc} eps^{feg} tr[S^{ag T} C g5 S^{be} P_- S^{cf} C g5]
    (traces and transposes over spin only).
    """
    eps = _eps()
    Cg5 = charge_conjugation() @ gamma5()
    Pm = P_minus()
    # tr[X^T M Y M] = X_{rs} M_{rk} Y_{kl} M_{ls}
    T1 = np.einsum("yrasg,rk,ykblf,ls->yagbf", Sarr, Cg5, Sarr, Cg5, optimize=True)
    T2 = np.einsum("yacbe,ba->yce", Sarr, Pm, optimize=True)
    W1 = np.einsum("abc,feg,yagbf,yce->y", eps, eps, T1, T2, optimize=True)
    W2 = _w2(eps, Sarr, Cg5, Pm)
    return W1, W2


def _w2(eps, Sarr, Cg5, Pm):
    # X = S^{ag}, Y = S^{be}, Z = S^{cf}:  X_{rs} (Cg5)_{rk} Y_{kl} (P_-)_{lm} Z_{mn} (Cg5)_{ns}
    XM = np.einsum("yrasg,rk->yaskg", Sarr, Cg5, optimize=True)      # (X^T Cg5)_{sk}
    YP = np.einsum("ykble,lm->ykbme", Sarr, Pm, optimize=True)       # (Y P_-)_{km}
    ZM = np.einsum("ymcnf,ns->ymcsf", Sarr, Cg5, optimize=True)      # (Z Cg5)_{ms}
    XMY = np.einsum("yaskg,ykbme->yasmgbe", XM, YP, optimize=True)   # (X^T Cg5 Y P_-)_{sm}
    tr = np.einsum("yasmgbe,ymcsf->yagbecf", XMY, ZM, optimize=True)
    return np.einsum("abc,feg,yagbecf->y", eps, eps, tr, optimize=True)


def nucleon(sol, L, t_range=None):
    """C_N(y0) = sum_{y in slice y0} (W_N1 - W_N2)(y, x) for every y0 (eq. baryN).

    sol: the 12 point-source columns [12, V, 4, 3] of one propagator."""
    L = tuple(L)
    V = int(np.prod(L))
    V3 = V // L[0]
    sol = np.asarray(sol)
    # Sarr[y, alpha, a, beta, b] = sol[3 beta + b, y, alpha, a]
    Sarr = sol.reshape(4, 3, V, 4, 3).transpose(2, 3, 4, 0, 1)
    out = np.zeros(L[0], dtype=np.complex128)
    ts = range(L[0]) if t_range is None else t_range
    for t in ts:
        out[t] = nucleon_W(np.ascontiguousarray(Sarr[t * V3:(t + 1) * V3])).sum()
    return out


def contract_nucleon(terms, L):
    """C^(i)_N(y0) for each level's cumulative propagator, and the series differences.

    Returns (levels, diffs): levels[i] = C_N[S^(i)], diffs[0] = levels[0],
    diffs[i] = levels[i] - levels[i-1] (eq. seriesN)."""
    cum = cumulative(terms)
    levels = np.stack([nucleon(cum[i], L) for i in range(cum.shape[0])])
    diffs = np.concatenate([levels[:1], np.diff(levels, axis=0)], axis=0)
    return levels, diffs


# ------------------------------------------------- two-domain factorization
def apply_boundary(U, L, psi, lo, hi, antiperiodic=True):
    """D_{dGamma} psi for Gamma = [lo,hi): rows in Gamma, columns outside it.

    By definition the block P_Gamma D (1 - P_Gamma) of the full operator
    (eq. blkdec; the bottom-left block of eq. Scmpt2 when Gamma is the second
    block).  Only hops cross a domain boundary, so kappa and the clover term
    do not enter: D is applied with an arbitrary kappa to psi with its
    components inside Gamma cleared, and the diagonal part then vanishes on the
    rows that are kept."""
    psi = _c(psi)
    m = domain_mask(L, lo, hi)
    outside = psi * (~m)[..., :, None, None]
    return apply_D(U, L, 0.125, outside, antiperiodic=antiperiodic) * m[..., :, None, None]


def apply_boundary_sites(U, L, psi, sites, lo, hi, antiperiodic=True):
    """(D_{dGamma} psi)(x) at listed sites x: on a row of Gamma the full operator
    is D_Gamma plus the couplings from outside, so the boundary block is the
    difference of the two there (zero for sites outside Gamma)."""
    full = apply_D_sites(U, L, 0.125, psi, sites, antiperiodic=antiperiodic)
    dom = apply_D_sites(U, L, 0.125, psi, sites, antiperiodic=antiperiodic, lo=lo, hi=hi)
    m = domain_mask(L, lo, hi)[np.asarray(sites)]
    return (full - dom) * m[None, :, None, None]


def factorized_propagator(U, L, kappa, b, bar, star, C=None, antiperiodic=True, tol=1e-13):
    """S^(f) b = -D_{Gamma*}^{-1} D_{dGamma*} D_{Gammabar}^{-1} b (Section 5.2, eq. approxlong).

    bar = (lo, hi) of Gammabar (it holds the source), star = (lo, hi) of
    Gamma*.  Returns (S^(f) b, D_{Gammabar}^{-1} b); the first is zero outside
    Gamma*, the second outside Gammabar."""
    psi, _, _ = solve(U, L, kappa, b, C=C, antiperiodic=antiperiodic, lo=bar[0], hi=bar[1], tol=tol)
    bstar = -apply_boundary(U, L, psi, star[0], star[1], antiperiodic)
    sf, _, _ = solve(U, L, kappa, bstar, C=C, antiperiodic=antiperiodic, lo=star[0], hi=star[1], tol=tol)
    return sf, psi


def factorized_chain(U, L, kappa, b, doms, C=None, antiperiodic=True, tol=1e-13):
    """Multi-slab factorized propagator (Section 4, eq. fctpr) applied to b.

    doms = [(lo, hi) of Omega_{m+2}, then of Omega*_{m+1}, ..., Omega*_l]:
    psi_0 = D_{doms[0]}^{-1} b and psi_k = -D_{doms[k]}^{-1} D_{d doms[k]} psi_{k-1},
    where D_{d doms[k]} keeps the entries of D from outside doms[k] into it
    (of which only the hop out of the previous slab's last time slice meets
    psi_{k-1}).  Returns the list [psi_0, ..., psi_{n-1}]."""
    psi, _, _ = solve(U, L, kappa, b, C=C, antiperiodic=antiperiodic, lo=doms[0][0], hi=doms[0][1], tol=tol)
    out = [psi]
    for lo, hi in doms[1:]:
        rhs = -apply_boundary(U, L, out[-1], lo, hi, antiperiodic)
        psi, _, _ = solve(U, L, kappa, rhs, C=C, antiperiodic=antiperiodic, lo=lo, hi=hi, tol=tol)
        out.append(psi)
    return out


def pion_W(sol):
    """W_Pc(y, x) = tr{S(y,x) S(y,x)^dag} at every sink y (eq. W0pc), from 12 point-source columns."""
    sol = np.asarray(sol)
    V = sol.shape[1]
    # S[y][alpha a, beta b] = sol[3 beta + b, y, alpha, a]
    S = sol.reshape(12, V, 12).transpose(1, 2, 0)
    SS = np.matmul(S, np.conj(S).transpose(0, 2, 1))
    return np.trace(SS, axis1=1, axis2=2).real


def pion_connected(sol, L):
    """C_Pc(y0) = -(1/L^3) sum_{y in slice y0} W_Pc(y, x) for every y0 (eq. pipi).

    With a point source the sum over the source's spatial position reduces to
    that one point, as for the disconnected pieces."""
    L = tuple(L)
    V3 = int(np.prod(L[1:]))
    W = pion_W(sol)
    return -W.reshape(L[0], V3).sum(axis=1) / V3


def contract_pion(levels, L, full=None):
    """The connected pion correlator of each factorized level, the series of
    eq. seriespi and its rest (eqs. decpi, W0pc2).

    levels: [n, 12, V, 4, 3] factorized propagators S^(f) for a growing overlap
    Delta; full: the propagator S on the whole lattice, or None.  Returns
    (C, diffs, rest): C[i] = C^(i)_Pc, diffs[0] = C[0], diffs[i] = C[i] - C[i-1],
    rest = C_Pc[S] - C[n-1] (None without ``full``)."""
    C = np.stack([pion_connected(levels[i], L) for i in range(len(levels))])
    diffs = np.concatenate([C[:1], np.diff(C, axis=0)], axis=0)
    rest = None if full is None else pion_connected(full, L) - C[-1]
    return C, diffs, rest


# ------------------------------------------- stochastic traces with the HPE
def hop_power(U, L, kappa, psi, p, C=None, antiperiodic=True, lo=None, hi=None):
    """(kappa D_hop)^p psi with kappa D_hop = 1 - 2 kappa D_Gamma (Section 6)."""
    psi = _c(psi)
    for _ in range(p):
        psi = psi - 2.0 * kappa * apply_D(U, L, kappa, psi, C=C, antiperiodic=antiperiodic, lo=lo, hi=hi)
    return psi


def apply_gamma5(psi):
    """gamma5 on the spin index of psi[..., 4, 3]."""
    return np.einsum("ab,...bc->...ac", gamma5(), _c(psi))


def hpe_trace(U, L, kappa, eta, p, C=None, antiperiodic=True, lo=None, hi=None, tol=1e-13):
    """Per time slice t: (1/n) sum_i sum_{x in slice t} eta_i^dag(x) [(kappa D_hop)^p D_Gamma^{-1} gamma5 eta_i](x)
    (Section 6, eq. HPEtr and the stochastic estimator after it).

    eta: [n, V, 4, 3] sources (Gaussian noise; unit vectors give the exact
    trace).  Only the part of each source on Gamma enters the solve; the
    contraction runs over the whole slice.  Returns a complex array [T]."""
    L = tuple(L)
    eta = _c(eta)
    V3 = int(np.prod(L[1:]))
    x, _, _ = solve(U, L, kappa, apply_gamma5(eta), C=C, antiperiodic=antiperiodic, lo=lo, hi=hi, tol=tol)
    phi = hop_power(U, L, kappa, x, p, C=C, antiperiodic=antiperiodic, lo=lo, hi=hi)
    w = np.einsum("nsac,nsac->s", np.conj(eta), phi)
    return w.reshape(L[0], V3).sum(axis=1) / eta.shape[0]


# ------------------------------------------------ projector-cut factorization
def orthonormal_q(X):
    """Q of X = Q R with R upper triangular and real positive diagonal (columns
    of X are the fields: X[n, V, 4, 3]); numpy's QR, phases fixed."""
    n = X.shape[0]
    M = _c(X).reshape(n, -1).T
    Q, R = np.linalg.qr(M)
    d = np.diag(R)
    Q = Q * (np.abs(d) / d)[None, :]
    return Q.T.reshape(X.shape)


def inverse_iteration(U, L, kappa, start, niter, C=None, antiperiodic=True, lo=None, hi=None, tol=1e-13):
    """v <- orth(D_Gamma^{-1} v), niter times, from start[n, V, 4, 3]
    (Section 5.2: basis vectors by inverse iteration on a domain)."""
    v = _c(start)
    for _ in range(niter):
        x, _, _ = solve(U, L, kappa, v, C=C, antiperiodic=antiperiodic, lo=lo, hi=hi, tol=tol)
        v = orthonormal_q(x)
    return v


def gram_slices(X, L):
    """G[t]_ij = sum_{x in slice t} X_i(x)^dag X_j(x) for fields X[n, V, 4, 3]."""
    L = tuple(L)
    X = _c(X)
    n = X.shape[0]
    Y = X.reshape(n, L[0], -1)
    return np.einsum("itk,jtk->tij", np.conj(Y), Y)


def projected_pion(U, L, kappa, phi, bar, star, C=None, antiperiodic=True, tol=1e-13):
    """-(1/L^3) Re Tr(Gt(y0) G(x0)) [T, T] with G from chi = D_Gammabar^{-1} gamma5 phi
    and Gt from eta = D_Gamma*^{-1} D_dGamma* phi (eqs. approxlong2, fullfactpi, Bpions).
    Returns (C, G, Gt)."""
    L = tuple(L)
    chi, _, _ = solve(U, L, kappa, apply_gamma5(phi), C=C, antiperiodic=antiperiodic, lo=bar[0], hi=bar[1], tol=tol)
    eta, _, _ = solve(U, L, kappa, apply_boundary(U, L, phi, star[0], star[1], antiperiodic), C=C,
                      antiperiodic=antiperiodic, lo=star[0], hi=star[1], tol=tol)
    G = gram_slices(chi, L)
    Gt = gram_slices(eta, L)
    V3 = int(np.prod(L[1:]))
    Cm = -np.einsum("yij,xji->yx", Gt, G).real / V3
    return Cm, G, Gt


def colourless_spinors(s, L):
    """Slice sums of the colourless spinors of eq. W0tbary for every index triple:
    out[t, i, j, k, alpha] = sum_{x in slice t} eps^{abc} (s_i^a(x)^T C g5 s_j^b(x)) s_k^c_alpha(x),
    s[n, V, 4, 3] (the spinor index transposed, not conjugated)."""
    L = tuple(L)
    V3 = int(np.prod(L[1:]))
    s = np.asarray(s).reshape(s.shape[0], L[0], V3, 4, 3)
    Cg5 = charge_conjugation() @ gamma5()
    d = np.einsum("itxra,rq,jtxqb->tijxab", s, Cg5, s, optimize=True)         # diquark, colours a, b
    e = np.einsum("abc,tijxab->tijxc", _eps(), d, optimize=True)
    return np.einsum("tijxc,ktxgc->tijkg", e, s, optimize=True)


def projected_nucleon(U, L, kappa, phi, bar, star, C=None, antiperiodic=True, tol=1e-13):
    """C_N(y0, x0) = (1/L^3) sum_{x,y} (W_N1 - W_N2) with every propagator replaced by
    the projected factorized one of eq. approxlong2, S(y,x) = -sum_i eta_i(y) xi_i(x)^T,
    written with the colourless spinors of eq. W0tbary.  Substituting S into
    eq. baryfact (three minus signs, and eps^{feg} reordered to eps^{fge}) gives
      W_N1 = sum_ijk B[xi_j, xi_i, xi_k; x]^T P_- B[eta_i, eta_j, eta_k; y],
      W_N2 = sum_ijk B[xi_k, xi_i, xi_j; x]^T P_- B[eta_i, eta_j, eta_k; y]
    (the index orders of eq. W0tbary; its printed prefactor -g5 P_- is read as P_-),
    xi_i^T = phi_i^dag D_Gammabar^{-1}, i.e. xi_i = conj(g5 D_Gammabar^{-1} g5 phi_i) by
    gamma5-hermiticity (eq. g5h), and eta_i = D_Gamma*^{-1} D_dGamma* phi_i.
    Returns (C [T, T] indexed [y0, x0], slice-summed spinors of xi, of eta)."""
    L = tuple(L)
    chi, _, _ = solve(U, L, kappa, apply_gamma5(phi), C=C, antiperiodic=antiperiodic, lo=bar[0], hi=bar[1], tol=tol)
    eta, _, _ = solve(U, L, kappa, apply_boundary(U, L, phi, star[0], star[1], antiperiodic), C=C,
                      antiperiodic=antiperiodic, lo=star[0], hi=star[1], tol=tol)
    xi = np.conj(apply_gamma5(chi))
    Bx = colourless_spinors(xi, L)
    By = colourless_spinors(eta, L)
    G = P_minus()
    V3 = int(np.prod(L[1:]))
    W1 = np.einsum("xjikr,rq,yijkq->yx", Bx, G, By, optimize=True)
    W2 = np.einsum("xkijr,rq,yijkq->yx", Bx, G, By, optimize=True)
    return (W1 - W2) / V3, Bx, By


# ------------------------------------------------------- level-1 updates
def philox(ctr, key):
    """Philox4x32-10 of a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().oracle_philox(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def kp_sample(alpha, seed, n):
    """n draws of the Kennedy-Pendleton sampler (density ~ sqrt(1-x^2) exp(alpha x))."""
    out = np.empty(int(n))
    _load().oracle_kp_sample(float(alpha), int(seed), int(n), out.ctypes.data)
    return out


def level1_update(U, L, beta, seed, update_id, t0, t1, nsweeps=1, n_or=0):
    """A copy of U after nsweeps level-1 sweeps of the slab [t0, t1) (random
    stream 3 + update_id)."""
    out = _c(U).copy()
    _load().oracle_level1_update(_i4(L), float(beta), int(seed), int(3 + update_id), int(t0), int(t1),
                                 int(nsweeps), int(n_or), out.ctypes.data)
    return out


def plaquette(U, L):
    """Average of Re tr U_P / 3 over all plaquettes."""
    return _load().oracle_plaquette(_i4(L), _c(U).ctypes.data)


def two_level(a, b, rest=None):
    """Two-level estimator of <F_A F_B> from level-1 measurements.

    a: [n0, n1, nc, ma] measurements of a factor that depends on the links of
    region A only, made on the n1 level-1 updates of A for each of the n0
    level-0 fields; b: [n0, n1, nc, mb] the same for region B (its own n1
    updates).  For level-0 field i the level-1 means [a]_i, [b]_i are taken
    separately (Section 3.1) and multiplied, contracting the index c:
    P_i[x, y] = sum_c [a]_i[c, x] [b]_i[c, y].  Returns (mean over i of P_i,
    its standard error over the n0 values), and for rest [n0, n1, k] the mean
    and standard error of the n0 bin means (bins of the n1 measurements of one
    level-0 field).  Standard errors are 0 when n0 = 1.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n0 = a.shape[0]
    ma = a.mean(axis=1)                       # [n0, nc, ma]: level-1 means of region A
    mb = b.mean(axis=1)                       # [n0, nc, mb]: level-1 means of region B
    P = np.einsum("icx,icy->ixy", ma, mb)     # product of the means for each level-0 field
    est = P.mean(axis=0)
    err = P.std(axis=0, ddof=1) / np.sqrt(n0) if n0 > 1 else np.zeros_like(est)
    if rest is None:
        return est, err
    bins = np.asarray(rest, dtype=np.float64).mean(axis=1)   # [n0, k]
    est_r = bins.mean(axis=0)
    err_r = bins.std(axis=0, ddof=1) / np.sqrt(n0) if n0 > 1 else np.zeros_like(est_r)
    return est, err, est_r, err_r
