"""Pins of the oracle's two-level estimator (Section 3.1, and the averaging of
the numerical part of Section 6).

The estimator is fixed by what it must do statistically, checked on synthetic
measurements whose distribution is known:
* the two level-1 averages are taken independently, so only the set of each
  region's updates matters, not how they are paired (a same-update pairing
  fails this);
* it is unbiased for the product of the two conditional means, and its error
  over level-0 fields falls like 1/sqrt(n1) when the level-0 fluctuations
  vanish (a product taken before the averages does not fall);
* the other pieces are binned per level-0 field: perfectly correlated
  measurements inside a bin give the error of n0, not n0 n1, measurements;
  independent ones give the plain sqrt(n0 n1) law.
"""
import numpy as np

import oracle


def _model(rng, n0, n1, nc=1, ma=3, mb=2, sig0=0.3, sig1=1.0):
    """a = alpha_i + noise, b = beta_i + noise with per-level-0 means."""
    alpha = 1.0 + sig0 * rng.normal(size=(n0, 1, nc, ma))
    beta = 2.0 + sig0 * rng.normal(size=(n0, 1, nc, mb))
    a = alpha + sig1 * rng.normal(size=(n0, n1, nc, ma))
    b = beta + sig1 * rng.normal(size=(n0, n1, nc, mb))
    return a, b, alpha[:, 0], beta[:, 0]


def test_only_each_regions_set_of_updates_matters():
    rng = np.random.default_rng(160131)
    a, b, _, _ = _model(rng, 6, 5, nc=2)
    est, err = oracle.two_level(a, b)
    pa = np.stack([rng.permutation(5) for _ in range(6)])
    pb = np.stack([rng.permutation(5) for _ in range(6)])
    a2 = np.take_along_axis(a, pa[:, :, None, None], axis=1)
    b2 = np.take_along_axis(b, pb[:, :, None, None], axis=1)
    est2, err2 = oracle.two_level(a2, b2)
    assert np.abs(est2 - est).max() < 1e-13 and np.abs(err2 - err).max() < 1e-13
    # a same-update pairing (the mean over j of a_ij b_ij) is not invariant
    same = np.einsum("ijcx,ijcy->ixy", a, b).mean(axis=0) / 5
    same2 = np.einsum("ijcx,ijcy->ixy", a2, b2).mean(axis=0) / 5
    assert np.abs(same2 - same).max() > 1e-3


def test_unbiased_for_the_product_of_conditional_means():
    rng = np.random.default_rng(160132)
    n0, n1 = 40, 1000
    a, b, alpha, beta = _model(rng, n0, n1)
    est, err = oracle.two_level(a, b)
    target = np.einsum("icx,icy->xy", alpha, beta) / n0
    # spread of [a][b] around alpha beta: (alpha^2 + beta^2) / n1 per level-0 field
    sd = np.sqrt((alpha[:, 0, :, None] ** 2 + beta[:, 0, None, :] ** 2).sum(axis=0) / n1) / n0
    assert np.all(np.abs(est - target) < 5 * sd), (est - target) / sd


def test_error_falls_like_one_over_sqrt_n1_without_level0_fluctuations():
    rng = np.random.default_rng(160133)
    n0 = 400
    errs = []
    for n1 in (25, 100, 400):
        a, b, _, _ = _model(rng, n0, n1, sig0=0.0)
        errs.append(oracle.two_level(a, b)[1])
    errs = np.array(errs)
    ratio = errs[1:] / errs[:-1]
    assert np.all(np.abs(ratio - 0.5) < 0.1), ratio
    # closed form at n1 = 400: sd of [a][b] is sqrt((1 + 4) / n1), over sqrt(n0)
    assert np.all(np.abs(errs[2] / (np.sqrt(5 / 400) / np.sqrt(n0)) - 1) < 0.15)


def test_rest_is_binned_per_level0_field():
    rng = np.random.default_rng(160134)
    n0, n1 = 300, 16
    a, b, _, _ = _model(rng, n0, n1)
    gamma = rng.normal(size=(n0, 1, 2))
    rest = np.repeat(gamma, n1, axis=1)                # identical inside a bin
    _, _, est_r, err_r = oracle.two_level(a, b, rest)
    assert np.abs(est_r - gamma.mean(axis=(0, 1))).max() < 1e-13
    assert np.all(np.abs(err_r * np.sqrt(n0) - 1) < 0.15)     # the error of n0 measurements of unit spread
    iid = rng.normal(size=(n0, n1, 2))
    _, _, _, err_iid = oracle.two_level(a, b, iid)
    assert np.all(np.abs(err_iid * np.sqrt(n0 * n1) - 1) < 0.15)


def test_single_level0_field_has_no_error_and_n1_one_is_the_plain_product():
    rng = np.random.default_rng(160135)
    a, b, _, _ = _model(rng, 1, 7)
    est, err, est_r, err_r = oracle.two_level(a, b, rng.normal(size=(1, 7, 3)))
    assert not err.any() and not err_r.any()
    a1 = rng.normal(size=(4, 1, 1, 2))
    b1 = rng.normal(size=(4, 1, 1, 2))
    est1, _ = oracle.two_level(a1, b1)
    assert np.abs(est1 - sum(np.outer(a1[i, 0, 0], b1[i, 0, 0]) for i in range(4)) / 4).max() < 1e-15
