"""Pins for the oracle's cone projections (CPU only).

A projection p = Pi_K(x) onto a closed convex cone is characterised by
p in K, p - x in K^*, <p, p - x> = 0 (Moreau, Sect. 3.2, e-moreau); these
conditions are checked with membership tests that do not call the
projection.  Closed forms, reductions to simpler cones and a brute-force
distance search pin the rest.
"""

import math

import numpy as np
import pytest

from oracle import cones as K


RNG = np.random.default_rng(1234)


def test_nonneg_closed_form():
    x = np.array([-2.0, 0.0, 3.5, -1e-300])
    assert np.array_equal(K.proj_nonneg(x), np.array([0.0, 0.0, 3.5, 0.0]))


@pytest.mark.parametrize("x,expected", [
    ([5.0, 3.0, 4.0], [5.0, 3.0, 4.0]),          # inside
    ([-5.0, 3.0, 4.0], [0.0, 0.0, 0.0]),         # inside the polar
    ([1.0, 3.0, 4.0], [3.0, 1.8, 2.4]),          # ((1+5)/2)(1, (3,4)/5)
    ([0.0, 0.0, 2.0], [1.0, 0.0, 1.0]),
])
def test_soc_closed_form_values(x, expected):
    np.testing.assert_allclose(K.proj_soc(np.array(x)), expected, rtol=0, atol=1e-15)


def test_soc_size_one_is_nonneg():
    for t in [-3.0, -0.0, 0.0, 2.5]:
        np.testing.assert_array_equal(K.proj_soc(np.array([t])), K.proj_nonneg(np.array([t])))


def _soc_member(p, tol):
    return np.linalg.norm(p[1:]) <= p[0] + tol


@pytest.mark.parametrize("k", [2, 3, 7, 50])
def test_soc_moreau(k):
    for _ in range(200):
        x = RNG.standard_normal(k) * RNG.choice([0.01, 1.0, 100.0])
        p = K.proj_soc(x)
        tol = 1e-13 * (1 + np.linalg.norm(x))
        assert _soc_member(p, tol)
        assert _soc_member(p - x, tol)            # self-dual
        assert abs(p @ (p - x)) <= 1e-12 * (1 + x @ x)


def test_svec_isometry():
    for d in [1, 2, 5, 9]:
        X = RNG.standard_normal((d, d))
        X = X + X.T
        Y = RNG.standard_normal((d, d))
        Y = Y + Y.T
        assert abs(K.svec(X) @ K.svec(Y) - np.trace(X @ Y)) <= 1e-12 * (1 + abs(np.trace(X @ Y)))
        np.testing.assert_allclose(K.smat(K.svec(X), d), X, atol=1e-14)


def test_svec_layout_by_hand():
    # lower triangle, column-major, off-diagonals x sqrt 2
    X = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 5.0], [3.0, 5.0, 6.0]])
    r2 = math.sqrt(2.0)
    np.testing.assert_allclose(K.svec(X), [1.0, 2 * r2, 3 * r2, 4.0, 5 * r2, 6.0])


def test_psd_reductions():
    # 1x1 is the nonnegative cone
    for t in [-2.0, 0.0, 3.0]:
        np.testing.assert_allclose(K.proj_psd(np.array([t]), 1), [max(t, 0.0)])
    # diagonal matrices project by clamping the diagonal
    d = 6
    diag = RNG.standard_normal(d)
    np.testing.assert_allclose(K.smat(K.proj_psd(K.svec(np.diag(diag)), d), d),
                               np.diag(np.maximum(diag, 0)), atol=1e-14)


def test_psd_2x2_closed_form():
    # [[a, b], [b, c]]: eigenvalues (a+c)/2 +- sqrt(((a-c)/2)^2 + b^2)
    a, b, c = 1.0, 2.0, -3.0
    mid, rad = (a + c) / 2, math.sqrt(((a - c) / 2) ** 2 + b * b)
    lam = mid + rad
    vec = np.array([b, lam - a])
    vec /= np.linalg.norm(vec)
    expected = lam * np.outer(vec, vec)
    got = K.smat(K.proj_psd(K.svec(np.array([[a, b], [b, c]])), 2), 2)
    np.testing.assert_allclose(got, expected, atol=1e-14)


@pytest.mark.parametrize("d", [2, 4, 8, 13])
def test_psd_moreau(d):
    L = d * (d + 1) // 2
    for _ in range(20):
        x = RNG.standard_normal(L)
        p = K.proj_psd(x, d)
        q = p - x
        tol = 1e-12 * (1 + np.linalg.norm(x))
        assert np.linalg.eigvalsh(K.smat(p, d)).min() >= -tol
        assert np.linalg.eigvalsh(K.smat(q, d)).min() >= -tol
        assert abs(p @ q) <= tol * (1 + np.linalg.norm(x))


def test_exp_special_cases():
    v = np.array([-1.0, 2.0, 3.0])           # in K_exp: 2 e^{-1/2} <= 3
    assert K.in_exp_cone(v)
    np.testing.assert_array_equal(K.proj_exp(v), v)
    v = np.array([1.0, 0.5, -4.0])           # -v in K_exp^*: 1*e^{0.5} <= 4e
    assert K.in_exp_dual(-v)
    np.testing.assert_array_equal(K.proj_exp(v), np.zeros(3))
    v = np.array([-2.0, -1.0, 0.7])          # x0<0, y0<0 -> (x0, 0, max(z0,0))
    np.testing.assert_array_equal(K.proj_exp(v), [-2.0, 0.0, 0.7])
    v = np.array([-2.0, -1.0, -0.7])
    np.testing.assert_array_equal(K.proj_exp(v), [-2.0, 0.0, 0.0])


def _brute_exp_distance(v):
    """Distance from v to K_exp by a dense search over the boundary rays
    {y (r, 1, e^r)}, the face {x <= 0, y = 0, z >= 0} and the apex."""
    best = np.linalg.norm(v)
    face = np.array([min(v[0], 0.0), 0.0, max(v[2], 0.0)])
    best = min(best, np.linalg.norm(v - face))
    if np.linalg.norm(v - face) <= best and K.in_exp_cone(v):
        return 0.0
    r = np.concatenate([np.linspace(-400.0, -40.0, 200001), np.linspace(-40.0, 40.0, 400001)])
    er = np.exp(r)
    dn = r * r + 1.0 + er * er
    ip = v[0] * r + v[1] + v[2] * er
    y = np.maximum(ip, 0.0) / dn
    dist2 = v @ v - y * ip
    best = min(best, math.sqrt(max(float(dist2.min()), 0.0)))
    return 0.0 if K.in_exp_cone(v) else best


def test_exp_brute_force_distance():
    for _ in range(100):
        v = RNG.standard_normal(3) * RNG.choice([0.3, 1.0, 3.0])
        p = K.proj_exp(v)
        assert K.in_exp_cone(p, 1e-12 * (1 + np.linalg.norm(v)))
        d_mine = np.linalg.norm(p - v)
        d_brute = _brute_exp_distance(v)
        # the grid distance is an upper bound on the true distance
        assert d_mine <= d_brute + 1e-9
        assert d_brute - d_mine <= 1e-6 * (1 + np.linalg.norm(v))


def test_exp_moreau():
    for _ in range(500):
        v = RNG.standard_normal(3) * RNG.choice([0.1, 1.0, 10.0])
        p = K.proj_exp(v)
        q = p - v
        nv = 1 + np.linalg.norm(v)
        assert K.in_exp_cone(p, 1e-10 * nv)
        # q's membership is ill-conditioned when q has a tiny first entry
        assert K.in_exp_dual(q, 1e-6 * nv)
        assert abs(p @ q) <= 1e-12 * nv * nv


def test_exp_dual_moreau():
    for _ in range(200):
        v = RNG.standard_normal(3)
        p = K.proj_exp_dual(v)
        q = p - v
        # membership of a point with a tiny first entry is ill-conditioned
        assert K.in_exp_dual(p, 1e-6)
        assert K.in_exp_cone(q, 1e-6)
        assert abs(p @ q) <= 1e-11 * (1 + v @ v)


def test_product_cone_dual_rules():
    cone = {"f": 2, "l": 2, "q": [3], "s": [2], "ep": 1, "ed": 1}
    m = K.cone_dim(cone)
    assert m == 2 + 2 + 3 + 3 + 3 + 3
    x = RNG.standard_normal(m)
    pk = K.proj_cone(x, cone)
    pd = K.proj_cone(x, cone, dual=True)
    np.testing.assert_array_equal(pk[:2], 0.0)         # K = {0}
    np.testing.assert_array_equal(pd[:2], x[:2])       # K^* = R
    np.testing.assert_allclose(pk[2:10], pd[2:10])     # self-dual blocks
    np.testing.assert_allclose(pk[10:13], K.proj_exp(x[10:13]))
    np.testing.assert_allclose(pd[10:13], K.proj_exp_dual(x[10:13]))
    np.testing.assert_allclose(pk[13:16], K.proj_exp_dual(x[13:16]))
    np.testing.assert_allclose(pd[13:16], K.proj_exp(x[13:16]))
    # Moreau on the product: x = Pi_K(x) - Pi_{K*}(-x)
    np.testing.assert_allclose(x, pk - K.proj_cone(-x, cone, dual=True), atol=1e-12)
