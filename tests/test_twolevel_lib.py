"""The library's two-level estimator (host code, no GPU needed) against the
oracle's on the same synthetic measurements, with the argument checks."""
import numpy as np
import pytest

import oracle

ddml = pytest.importorskip("paper_1601_04587_amd.ddml")


@pytest.mark.parametrize("n0,n1,nc,ma,mb,k", [(1, 1, 1, 1, 1, 0), (7, 5, 2, 3, 4, 6), (40, 16, 1, 32, 32, 3)])
def test_matches_the_oracle(n0, n1, nc, ma, mb, k):
    rng = np.random.default_rng(160140 + n0)
    a = rng.normal(size=(n0, n1, nc, ma))
    b = 2 + rng.normal(size=(n0, n1, nc, mb))
    rest = rng.normal(size=(n0, n1, k)) if k else None
    got = ddml.two_level_average(a, b, rest)
    ref = oracle.two_level(a, b, rest)
    assert len(got) == len(ref)
    for g, r in zip(got, ref):
        assert g.shape == r.shape
        assert np.abs(g - r).max() <= 1e-12 * max(1.0, np.abs(r).max())


def test_bad_sizes_are_rejected():
    lib = ddml.load()
    x = np.zeros(8)
    p = x.ctypes.data
    assert lib.ddml_two_level_average(0, 1, 1, 1, 1, p, p, 0, None, p, p, p, p) == ddml.EINVAL
    assert lib.ddml_two_level_average(1, 1, 1, 1, 1, None, p, 0, None, p, p, p, p) == ddml.EINVAL
    assert lib.ddml_two_level_average(1, 1, 1, 1, 1, p, p, 2, None, p, p, p, p) == ddml.EINVAL
    with pytest.raises(ValueError):
        ddml.two_level_average(np.zeros((2, 3, 1, 1)), np.zeros((2, 4, 1, 1)))
