"""Pins of the oracle's series and Wick contractions.

* nucleon: W_N1 - W_N2 of eq. baryfact against a brute-force fermionic Wick
  enumeration of tr[<N(y) Nbar(x)> P_-] built directly from the interpolators
  of Section 5.2 (generic pairing of Grassmann fields with permutation signs);
* disconnected pseudoscalar: reality of tr{g5 S(x,x)} (gamma5-hermiticity,
  eq. g5h), f + r1 + r2 = full (eq. deco1), gauge invariance.
"""
import itertools

import numpy as np
import pytest

import inputs
import oracle
from tests import _dense


def _perm_sign(p):
    p = list(p)
    s = 1
    for i in range(len(p)):
        for j in range(i + 1, len(p)):
            if p[i] > p[j]:
                s = -s
    return s


def _wick(fields, props):
    """<f_0 f_1 ... f_{n-1}> for Grassmann fields f = (flavour, is_bar, spin, colour).

    Sums over every complete pairing of each psi with a psibar of the same
    flavour; each pairing contributes sign * prod S_flavour[psi, psibar], with the
    sign of the permutation that brings each psi next to (left of) its partner,
    since <psi_A psibar_B> = S_AB."""
    psis = [i for i, f in enumerate(fields) if not f[1]]
    bars = [i for i, f in enumerate(fields) if f[1]]
    total = 0.0
    for perm in itertools.permutations(bars):
        if any(fields[i][0] != fields[j][0] for i, j in zip(psis, perm)):
            continue
        order = []
        for i, j in zip(psis, perm):
            order += [i, j]
        val = _perm_sign(order)
        for i, j in zip(psis, perm):
            fl, _, a, ca = fields[i]
            _, _, b, cb = fields[j]
            val = val * props[fl][a, ca, b, cb]
        total += val
    return total


def _eps_terms():
    for a, b, c in itertools.permutations(range(3)):
        yield (a, b, c), _perm_sign((a, b, c))


def brute_force_nucleon(Su, Sd):
    """tr[<N(y) Nbar(x)> P_-] with N = eps^{abc} [u^{aT} C g5 d^b] d^c and
    Nbar = eps^{feg} dbar^e [dbar^f C g5 ubar^{gT}] (Section 5.2), C = i g0 g2."""
    g = _dense.gammas()
    C = 1j * g[0] @ g[2]
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    Cg5 = C @ g5
    Pm = 0.5 * (np.eye(4) - g[0])
    props = {"u": Su, "d": Sd}
    total = 0.0
    nz = [(i, j) for i in range(4) for j in range(4) if abs(Cg5[i, j]) > 0]
    for (a, b, c), sabc in _eps_terms():
        for (f, e, gg), sfeg in _eps_terms():
            for al in range(4):
                for be in range(4):
                    if Pm[be, al] == 0:
                        continue
                    for ga, de in nz:
                        for rh, si in nz:
                            fields = [("u", False, ga, a), ("d", False, de, b), ("d", False, al, c),
                                      ("d", True, be, e), ("d", True, rh, f), ("u", True, si, gg)]
                            coef = sabc * sfeg * Cg5[ga, de] * Cg5[rh, si] * Pm[be, al]
                            total += coef * _wick(fields, props)
    return total


def test_nucleon_contraction_matches_brute_force_wick(rng):
    S = rng.normal(size=(4, 3, 4, 3)) + 1j * rng.normal(size=(4, 3, 4, 3))
    W = oracle.nucleon_W(S[None])[0]
    B = brute_force_nucleon(S, S)
    assert abs(W - B) < 1e-12 * abs(B)
    assert abs(B) > 1e-3


def test_nucleon_pin_is_sensitive_to_sign_and_pieces(rng):
    """Plausible mistakes (relative sign of the two contractions, a dropped
    contraction) must not agree with the brute-force result."""
    S = rng.normal(size=(4, 3, 4, 3)) + 1j * rng.normal(size=(4, 3, 4, 3))
    B = brute_force_nucleon(S, S)
    W1, W2 = oracle.nucleon_W_parts(S[None])
    for wrong in (W1 + W2, W1, -W2):
        assert abs(wrong[0] - B) > 1e-3 * abs(B)


@pytest.fixture(scope="module")
def solved():
    L = (8, 4, 4, 4)
    U = inputs.heatbath(L, 6.0, 21, 30)
    kappa, csw = 0.13, 1.769
    C = oracle.clover_term(U, L, csw)
    xs = (2, 1, 2, 3)
    b = inputs.point_source(L, xs)
    doms = [((0, 0, 0, 0), (4, 4, 4, 4)), ((0, 0, 0, 0), L)]
    props = [oracle.solve(U, L, kappa, b, C=C, lo=lo, hi=hi, tol=1e-12)[0] for lo, hi in doms]
    return L, U, kappa, csw, xs, props


def test_pp_trace_is_real_and_decomposition_adds_up(solved):
    L, U, kappa, csw, xs, props = solved
    s = inputs.site_index(L, xs)
    for p in props:
        t = oracle.pp_trace(p, s)
        assert abs(t.imag) < 1e-10 * abs(t.real)
    terms, _ = oracle.series(props)
    out = oracle.contract_pp_disconnected(terms, terms, s, s, 64)
    for lev in range(out.shape[0]):
        f, r1, r2, full = out[lev]
        assert abs(f + r1 + r2 - full) < 1e-13 * abs(full)
    # at the last level (full lattice) the rest vanishes
    assert abs(out[-1, 1]) < 1e-14 and abs(out[-1, 2]) < 1e-14


def _gauge_transform(U, L, Om):
    Up = np.empty_like(U)
    for s, x in enumerate(np.ndindex(*L)):
        for mu in range(4):
            y = list(x)
            y[mu] = (y[mu] + 1) % L[mu]
            Up[s, mu] = Om[s] @ U[s, mu] @ Om[inputs.site_index(L, y)].conj().T
    return Up


def test_contractions_are_gauge_invariant(solved, rng):
    L, U, kappa, csw, xs, props = solved
    V = int(np.prod(L))
    Z = rng.normal(size=(V, 3, 3)) + 1j * rng.normal(size=(V, 3, 3))
    Om, _ = np.linalg.qr(Z)
    Om = Om / np.linalg.det(Om)[:, None, None] ** (1 / 3)
    Up = _gauge_transform(U, L, Om)
    Cp = oracle.clover_term(Up, L, csw)
    s = inputs.site_index(L, xs)
    # S'(y,x) = Om(y) S(y,x) Om(x)^dag solves the transformed equation with the
    # same point source; traces and the eps-eps contractions cannot see Om
    b = inputs.point_source(L, xs)
    lo, hi = (0, 0, 0, 0), (4, 4, 4, 4)
    xq, _, _ = oracle.solve(Up, L, kappa, b, C=Cp, lo=lo, hi=hi, tol=1e-12)
    assert np.abs(xq - props[0]).max() > 1e-3                 # the propagator itself changes
    t0 = oracle.pp_trace(props[0], s)
    t1 = oracle.pp_trace(xq, s)
    assert abs(t0 - t1) < 1e-9 * abs(t0)
    n0 = oracle.nucleon(props[0], L, t_range=[1, 2, 3])
    n1 = oracle.nucleon(xq, L, t_range=[1, 2, 3])
    assert np.abs(n0 - n1).max() < 1e-9 * np.abs(n0).max()


def test_nucleon_series_differences(solved):
    L, U, kappa, csw, xs, props = solved
    terms, _ = oracle.series(props)
    levels, diffs = oracle.contract_nucleon(terms, L)
    assert np.abs(diffs.sum(axis=0) - levels[-1]).max() < 1e-13 * np.abs(levels[-1]).max()
    # the domain propagator vanishes outside Gamma_0, and so does C^(0)
    assert np.abs(levels[0][4:]).max() == 0.0
