"""Seeded input generators: Philox known answers, SU(3) properties, heatbath equilibrium."""
import os

import numpy as np
import pytest

import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(h, 16) for h in r]
        out = inputs.philox4x32_10(v[0:4], v[4:6])
        assert [int(o) for o in out] == v[6:10]


def test_random_links_are_su3():
    L = (4, 4, 4, 4)
    U = inputs.random_links(L, 1601001).reshape(-1, 3, 3)
    eye = np.einsum("sij,skj->sik", U, U.conj())
    assert np.abs(eye - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13
    # exp(i 0.3 H) with unit-variance H stays close to, but away from, the identity
    d = np.abs(U - np.eye(3)).mean()
    assert 0.05 < d < 0.5


def test_generators_are_seeded_and_deterministic():
    L = (4, 4, 4, 4)
    a = inputs.random_links(L, 7)
    b = inputs.random_links(L, 7)
    c = inputs.random_links(L, 8)
    assert np.array_equal(a, b)
    assert not np.allclose(a, c)
    g1 = inputs.gaussian(3, 1, (5, 7))
    g2 = inputs.gaussian(3, 1, (5, 7))
    assert np.array_equal(g1, g2)


def test_heatbath_plaquette_at_beta6():
    # The average plaquette of quenched SU(3) at beta=6.0 is 0.5937 in large
    # volume (a standard literature value of the Wilson gauge action); an 8^4
    # lattice sits a few 1e-3 above it.
    L = (8, 8, 8, 8)
    U = inputs.heatbath(L, 6.0, 11, 120)
    p = inputs.plaquette(U, L)
    assert 0.590 < p < 0.600
    V = U.reshape(-1, 3, 3)
    assert np.abs(np.einsum("sij,skj->sik", V, V.conj()) - np.eye(3)).max() < 1e-12
    # beta -> 0 (strong coupling): plaquette near 0
    L = (4, 4, 4, 4)
    U0 = inputs.heatbath(L, 0.01, 11, 5)
    assert abs(inputs.plaquette(U0, L)) < 0.05


def test_level1_update_touches_only_its_slab_and_keeps_frozen_links():
    L = (8, 4, 4, 4)
    U = inputs.heatbath(L, 6.0, 5, 20)
    t0, t1 = 2, 6
    U2 = inputs.level1_update(U, L, 6.0, 99, 0, t0, t1, nsweeps=1)
    V3 = 4 * 4 * 4
    t = np.arange(U.shape[0]) // V3
    outside = (t < t0) | (t >= t1)
    assert np.array_equal(U2[outside], U[outside])
    first = t == t0
    assert np.array_equal(U2[first, 1:], U[first, 1:])      # frozen spatial links
    assert not np.allclose(U2[first, 0], U[first, 0])       # temporal links on t0 update
    inner = (t > t0) & (t < t1)
    assert not np.allclose(U2[inner], U[inner])


def test_tile_is_periodic_replication():
    Ls = (4, 2, 2, 2)
    L = (8, 4, 4, 4)
    Us = inputs.random_links(Ls, 3)
    U = inputs.tile(Us, Ls, L)
    for x in [(0, 0, 0, 0), (5, 3, 1, 2), (7, 2, 3, 3)]:
        y = tuple(a % b for a, b in zip(x, Ls))
        assert np.array_equal(U[inputs.site_index(L, x)], Us[inputs.site_index(Ls, y)])


def test_point_source():
    L = (4, 4, 4, 4)
    b = inputs.point_source(L, (1, 2, 3, 0))
    s = inputs.site_index(L, (1, 2, 3, 0))
    assert b.shape == (12, 256, 4, 3)
    assert np.array_equal(b[:, s].reshape(12, 12), np.eye(12))
    assert np.count_nonzero(b) == 12
