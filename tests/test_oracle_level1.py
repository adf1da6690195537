"""Pins of the oracle's level-1 gauge updates (Section 3.1: the links of a
time slab are updated with the spatial links of its first slice fixed).

* Philox4x32-10 against the published known-answer vectors.
* The Kennedy-Pendleton sampler against the exact moments of its target
  density sqrt(1 - x^2) exp(alpha x) (first moment I_2(alpha)/I_1(alpha),
  second by quadrature).
* Heatbath + over-relaxation from a cold start reach the known average
  plaquette of the SU(3) Wilson action at beta = 6.0 (0.5937 in large volume).
* Updated links stay in SU(3); links outside the slab and the frozen spatial
  links of its first slice are untouched; the update depends on no link
  outside the slices [t0, t1] (bitwise).
* An independent implementation of the same conventions (the input
  generator's level-1 update) gives the same links.
"""
import os

import numpy as np
import pytest
from scipy import integrate, special

import inputs
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    for r in rows:
        v = [int(h, 16) for h in r]
        assert [int(o) for o in oracle.philox(v[0:4], v[4:6])] == v[6:10]


@pytest.mark.parametrize("alpha", [0.5, 3.0, 12.0])
def test_kennedy_pendleton_moments(alpha):
    n = 200000
    x = oracle.kp_sample(alpha, 1601951, n)
    assert np.all(np.abs(x) <= 1.0)
    m1 = special.iv(2, alpha) / special.iv(1, alpha)
    w = lambda t: np.sqrt(1 - t * t) * np.exp(alpha * (t - 1))
    z = integrate.quad(w, -1, 1)[0]
    m2 = integrate.quad(lambda t: t * t * w(t), -1, 1)[0] / z
    s = x.std() / np.sqrt(n)
    assert abs(x.mean() - m1) < 5 * s, (x.mean(), m1, s)
    assert abs((x * x).mean() - m2) < 5 * (x * x).std() / np.sqrt(n)


@pytest.mark.slow
def test_heatbath_reaches_the_beta6_plaquette():
    L = (8, 8, 8, 8)
    U = inputs.unit_links(L)                           # cold start
    V3 = int(np.prod(L[1:]))
    for sweep in range(40):
        U = oracle.level1_update(U, L, 6.0, 1601953, sweep, 0, L[0], nsweeps=1, n_or=2)
        # move the frozen first slice around: shift the field by one slice in time
        U = np.roll(U.reshape(L[0], V3, 4, 3, 3), 1, axis=0).reshape(U.shape)
    p = oracle.plaquette(U, L)
    assert 0.590 < p < 0.598, p


def test_slab_update_is_unitary_local_and_keeps_its_frozen_links():
    L = (8, 4, 4, 4)
    V3 = 64
    U = inputs.random_links(L, 1601954, eps=0.8)
    t0, t1 = 2, 6
    new = oracle.level1_update(U, L, 6.0, 1601955, 7, t0, t1, nsweeps=2, n_or=2)
    Un = new.reshape(L[0], V3, 4, 3, 3)
    Uo = U.reshape(L[0], V3, 4, 3, 3)
    # outside the slab and the frozen spatial links of slice t0: unchanged
    assert np.array_equal(Un[:t0], Uo[:t0]) and np.array_equal(Un[t1:], Uo[t1:])
    assert np.array_equal(Un[t0, :, 1:], Uo[t0, :, 1:])
    # everything else moved and stays in SU(3)
    moved = Un[t0:t1].reshape(-1, 4, 3, 3)
    assert np.abs(Un[t0 + 1:t1] - Uo[t0 + 1:t1]).max() > 0.1
    M = moved.reshape(-1, 3, 3)
    assert np.abs(np.einsum("nji,njk->nik", np.conj(M), M) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(M) - 1).max() < 1e-13
    # locality: links outside the slices [t0, t1] do not matter, nor the time links of slice t1
    W = inputs.random_links(L, 1601956, eps=0.8).reshape(L[0], V3, 4, 3, 3)
    Uw = Uo.copy()
    Uw[:t0] = W[:t0]
    Uw[t1 + 1:] = W[t1 + 1:]
    Uw[t1, :, 0] = W[t1, :, 0]
    new2 = oracle.level1_update(Uw.reshape(U.shape), L, 6.0, 1601955, 7, t0, t1, nsweeps=2, n_or=2)
    assert np.array_equal(new2.reshape(L[0], V3, 4, 3, 3)[t0:t1], Un[t0:t1])


def test_agrees_with_the_input_generators_level1_update():
    L = (8, 4, 4, 4)
    U = inputs.random_links(L, 1601957, eps=0.8)
    a = oracle.level1_update(U, L, 6.0, 1601958, 3, 2, 6, nsweeps=1, n_or=1)
    b = inputs.level1_update(U, L, 6.0, 1601958, 3, 2, 6, nsweeps=1, n_or=1)
    assert np.abs(a - b).max() < 1e-13
