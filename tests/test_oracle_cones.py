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


# ---------------------------------------------------------------------------
# power cone and its dual (Sect. 6.1 definitions)
# ---------------------------------------------------------------------------

def test_pow_special_cases():
    a = 0.3
    v = np.array([2.0, 3.0, 1.0])            # 2^0.3 3^0.7 = 2.6 >= 1
    assert K.in_pow_cone(v, a)
    np.testing.assert_array_equal(K.proj_pow(v, a), v)
    v = np.array([-2.0, -3.0, 0.5])          # -v in the dual: (2/.3)^.3 (3/.7)^.7 >= .5
    assert K.in_pow_dual(-v, a)
    np.testing.assert_array_equal(K.proj_pow(v, a), np.zeros(3))
    v = np.array([-1.5, 2.5, 0.0])           # z0 = 0 -> (x0+, y0+, 0)
    np.testing.assert_array_equal(K.proj_pow(v, a), [0.0, 2.5, 0.0])


@pytest.mark.parametrize("a", [0.0, 1.0])
def test_pow_endpoints_reduce_to_soc_times_nonneg(a):
    # a = 1: {x >= |z|} x {y >= 0}, i.e. a second-order cone of size 2 on
    # (x, z) times the half-line on y; a = 0 swaps the roles of x and y
    for _ in range(200):
        v = RNG.standard_normal(3) * RNG.choice([0.1, 1.0, 10.0])
        p = K.proj_pow(v, a)
        if a == 1.0:
            s = K.proj_soc(np.array([v[0], v[2]]))
            ref = [s[0], max(v[1], 0.0), s[1]]
        else:
            s = K.proj_soc(np.array([v[1], v[2]]))
            ref = [max(v[0], 0.0), s[0], s[1]]
        np.testing.assert_allclose(p, ref, rtol=0, atol=1e-14 * (1 + np.linalg.norm(v)))


def test_pow_half_closed_form_point():
    # a = 1/2, v = (0, 0, 2): by symmetry x = y on the boundary x^.5 y^.5 = r,
    # so x = y = r and the nearest point minimises 2 r^2 + (2 - r)^2: r = 2/3
    p = K.proj_pow(np.array([0.0, 0.0, 2.0]), 0.5)
    np.testing.assert_allclose(p, [2 / 3, 2 / 3, 2 / 3], rtol=0, atol=1e-14)


def _brute_pow_distance(v, a):
    """Distance from v to K_pow^a by a grid search over (x, y) >= 0 (for
    fixed x, y the best z is z0 clipped to [-x^a y^(1-a), x^a y^(1-a)]),
    refined by a bounded quasi-Newton search from the best grid point."""
    from scipy.optimize import minimize

    x0, y0, z0 = v

    def d2(w):
        x, y = max(w[0], 0.0), max(w[1], 0.0)
        g = K._wpow(x, a) * K._wpow(y, 1.0 - a)
        return (x - x0) ** 2 + (y - y0) ** 2 + max(abs(z0) - g, 0.0) ** 2

    R = 2.0 * np.linalg.norm(v) + 1.0
    grid = np.linspace(0.0, R, 401)
    X, Y = np.meshgrid(grid, grid, indexing="ij")
    G = np.where(a == 0.0, 1.0, X ** a) * np.where(a == 1.0, 1.0, Y ** (1.0 - a))
    D = (X - x0) ** 2 + (Y - y0) ** 2 + np.maximum(abs(z0) - G, 0.0) ** 2
    i, j = np.unravel_index(np.argmin(D), D.shape)
    best = float(D[i, j])
    res = minimize(d2, [X[i, j], Y[i, j]], method="L-BFGS-B", bounds=[(0, None), (0, None)],
                   options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 500})
    return math.sqrt(min(best, float(res.fun)))


def test_pow_brute_force_distance():
    for _ in range(60):
        a = float(RNG.uniform(0.05, 0.95))
        v = RNG.standard_normal(3) * RNG.choice([0.3, 1.0, 3.0])
        p = K.proj_pow(v, a)
        assert K.in_pow_cone(p, a, 1e-13 * (1 + np.linalg.norm(v)))
        d_mine = np.linalg.norm(p - v)
        d_brute = _brute_pow_distance(v, a)
        # the search's distance belongs to a feasible point: an upper bound
        assert d_mine <= d_brute + 1e-9
        assert d_brute - d_mine <= 1e-6 * (1 + np.linalg.norm(v))


def test_pow_moreau():
    for _ in range(2000):
        a = float(RNG.uniform(0.0, 1.0))
        v = RNG.standard_normal(3) * RNG.choice([0.01, 1.0, 100.0])
        p = K.proj_pow(v, a)
        q = p - v
        nv = 1 + np.linalg.norm(v)
        assert K.in_pow_cone(p, a, 1e-13 * nv)
        assert K.in_pow_dual(q, a, 1e-13 * nv)
        assert abs(p @ q) <= 1e-14 * nv * nv


def test_pow_dual_moreau_and_scaling():
    # (K^a)^* = diag(a, 1-a, 1) K^a, checked on random points of K^a
    for _ in range(300):
        a = float(RNG.uniform(0.05, 0.95))
        x, y = RNG.uniform(0.0, 3.0, size=2)
        z = RNG.uniform(-1.0, 1.0) * x ** a * y ** (1 - a)
        assert K.in_pow_dual(np.array([a * x, (1 - a) * y, z]), a, 1e-14)
        v = RNG.standard_normal(3)
        p = K.proj_pow_dual(v, a)
        q = p - v
        assert K.in_pow_dual(p, a, 1e-13 * (1 + np.linalg.norm(v)))
        assert K.in_pow_cone(q, a, 1e-13 * (1 + np.linalg.norm(v)))
        assert abs(p @ q) <= 1e-13 * (1 + v @ v)


def test_product_cone_power_blocks():
    cone = {"f": 0, "l": 1, "q": [], "s": [], "ep": 0, "ed": 0, "p": [0.3, -0.6]}
    assert K.cone_dim(cone) == 7
    x = RNG.standard_normal(7)
    pk = K.proj_cone(x, cone)
    pd = K.proj_cone(x, cone, dual=True)
    np.testing.assert_allclose(pk[1:4], K.proj_pow(x[1:4], 0.3))
    np.testing.assert_allclose(pd[1:4], K.proj_pow_dual(x[1:4], 0.3))
    np.testing.assert_allclose(pk[4:7], K.proj_pow_dual(x[4:7], 0.6))
    np.testing.assert_allclose(pd[4:7], K.proj_pow(x[4:7], 0.6))
    np.testing.assert_allclose(x, pk - K.proj_cone(-x, cone, dual=True), atol=1e-12)
    assert K.in_cone(pk, cone) and K.in_cone(pd, cone, dual=True)
