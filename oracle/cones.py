"""Cone projections (oracle).  TEST INFRASTRUCTURE ONLY.

Cones follow the list of Sect. 6.1 (SCS implementation): nonnegative,
second-order, positive semidefinite, the exponential cone and its dual, and
the power cone and its dual; the zero cone carries equality rows.
Dual-cone projections use the Moreau decomposition of Sect. 3.2 (e-moreau):
x = Pi_K(x) - Pi_{K*}(-x), i.e. Pi_{K*}(v) = v + Pi_K(-v).

Vector layouts (readings where the paper is silent):

* second-order cone of size k: (t, xbar) with ||xbar||_2 <= t, bound first;
* PSD cone of side d: scaled svec of length d(d+1)/2, lower triangle in
  column-major order, off-diagonal entries multiplied by sqrt(2), so that
  <svec X, svec Y> = Tr(XY) and the cone is self-dual in R^{d(d+1)/2};
* exponential cone: triples (x, y, z) with K_exp the closure of
  {y > 0, y exp(x/y) <= z} (Sect. 6.1);
* power cone with parameter a in [0, 1]: triples (x, y, z) with
  x^a y^(1-a) >= |z|, x >= 0, y >= 0 (Sect. 6.1).  In a cone description a
  negative parameter -a denotes the dual power cone (K_pow^a)^*.
"""

from __future__ import annotations

import math

import numpy as np

SQRT2 = math.sqrt(2.0)


# ----------------------------------------------------------------------------
# nonnegative orthant and second-order cone: closed forms
# ----------------------------------------------------------------------------

def proj_nonneg(x: np.ndarray) -> np.ndarray:
    """Projection onto R_+^k: elementwise max(x, 0)."""
    return np.maximum(x, 0.0)


def proj_soc(x: np.ndarray) -> np.ndarray:
    """Projection onto {(t, xbar): ||xbar|| <= t} by the three-case closed
    form: inside -> itself; inside the polar (||xbar|| <= -t) -> 0; otherwise
    ((t + ||xbar||)/2) (1, xbar/||xbar||)."""
    x = np.asarray(x, dtype=np.float64)
    t = x[0]
    xb = x[1:]
    nrm = float(np.linalg.norm(xb))
    if nrm <= t:
        return x.copy()
    if nrm <= -t:
        return np.zeros_like(x)
    a = 0.5 * (t + nrm)
    out = np.empty_like(x)
    out[0] = a
    out[1:] = (a / nrm) * xb
    return out


# ----------------------------------------------------------------------------
# PSD cone in scaled svec
# ----------------------------------------------------------------------------

def svec_len(d: int) -> int:
    return d * (d + 1) // 2


def smat(v: np.ndarray, d: int) -> np.ndarray:
    """Scaled svec (lower triangle, column-major, off-diagonals x sqrt 2) ->
    symmetric matrix."""
    X = np.zeros((d, d))
    k = 0
    for j in range(d):
        X[j, j] = v[k]
        k += 1
        for i in range(j + 1, d):
            X[i, j] = v[k] / SQRT2
            X[j, i] = X[i, j]
            k += 1
    return X


def svec(X: np.ndarray) -> np.ndarray:
    """Symmetric matrix -> scaled svec (inverse of ``smat``)."""
    d = X.shape[0]
    out = np.empty(svec_len(d))
    k = 0
    for j in range(d):
        out[k] = X[j, j]
        k += 1
        for i in range(j + 1, d):
            out[k] = SQRT2 * X[i, j]
            k += 1
    return out


def proj_psd(v: np.ndarray, d: int) -> np.ndarray:
    """Projection onto the PSD cone of side d in scaled svec: eigendecompose
    the symmetric matrix, clamp negative eigenvalues to zero and rebuild
    (the paper does this with a LAPACK symmetric eigensolver, Sect. 6.1).
    The svec map is an isometry onto the symmetric matrices with the trace
    inner product, so the Frobenius-nearest PSD matrix is the projection."""
    X = smat(v, d)
    w, V = np.linalg.eigh(X)
    wp = np.maximum(w, 0.0)
    return svec((V * wp) @ V.T)


# ----------------------------------------------------------------------------
# exponential cone
# ----------------------------------------------------------------------------

def _safe_exp(a: float) -> float:
    return math.inf if a > 700.0 else math.exp(a)


def in_exp_cone(v, tol: float = 0.0) -> bool:
    """Membership in K_exp = cl{(x,y,z): y>0, y e^{x/y} <= z} (Sect. 6.1),
    with an absolute slack ``tol``.  The closure adds {x <= 0, y = 0, z >= 0}."""
    x, y, z = (float(t) for t in v)
    if y > 0 and y * _safe_exp(x / y) <= z + tol:
        return True
    return x <= tol and abs(y) <= tol and z >= -tol


def in_exp_dual(v, tol: float = 0.0) -> bool:
    """Membership in K_exp^* = cl{(u,v,w): u<0, -u e^{v/u} <= e w} (Sect. 6.1),
    with an absolute slack ``tol``.  The closure adds {u = 0, v >= 0, w >= 0}."""
    u, vv, w = (float(t) for t in v)
    if u < 0 and -u * _safe_exp(vv / u) <= math.e * w + tol:
        return True
    return abs(u) <= tol and vv >= -tol and w >= -tol


def _exp_stationarity(rho: float, x0: float, y0: float, z0: float) -> float:
    """Sign-preserving form of the stationarity function for the nearest
    point of the ray {y (rho, 1, e^rho): y >= 0} to v = (x0, y0, z0).

    With d(rho) = (rho, 1, e^rho) and d' = (1, 0, e^rho), maximising
    <v,d>/||d|| over rho gives <v,d'>||d||^2 - <v,d><d,d'> = 0, i.e.

      f(rho) = (x0 - rho y0) + e^{2 rho}((1 - rho) x0 - y0)
               + z0 e^{rho} (rho^2 - rho + 1) = 0.

    For rho > 0 the function is returned multiplied by e^{-2 rho} (same sign,
    no overflow)."""
    q = rho * rho - rho + 1.0
    if rho > 0:
        e1 = math.exp(-rho)
        return (x0 - rho * y0) * e1 * e1 + ((1.0 - rho) * x0 - y0) + z0 * e1 * q
    e1 = math.exp(rho)
    return (x0 - rho * y0) + e1 * e1 * ((1.0 - rho) * x0 - y0) + z0 * e1 * q


def _bisect(fun, lo: float, hi: float, flo: float) -> float:
    """Bisection on a sign-changing bracket to full double precision."""
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        fm = fun(mid)
        if fm == 0.0:
            return mid
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _exp_boundary_point(rho: float, v: np.ndarray) -> np.ndarray:
    """Nearest point to v on the ray {y (rho, 1, e^rho): y >= 0}; the ray
    direction is rescaled by e^{-rho} for rho > 0 (same ray, no overflow)."""
    if rho > 0:
        e1 = math.exp(-rho)
        d = np.array([rho * e1, e1, 1.0])
    else:
        d = np.array([rho, 1.0, math.exp(rho)])
    yy = max(float(v @ d), 0.0) / float(d @ d)
    return yy * d


def proj_exp(v: np.ndarray) -> np.ndarray:
    """Projection of v = (x0, y0, z0) onto K_exp.

    Cases (Sect. 6.1 cone definitions; the paper cites its source for the
    algorithm and gives none, so this follows the univariate formulation of
    Friberg, "Projection onto the exponential cone: a univariate root-finding
    problem", 2021, derived independently):

    1. v in K_exp -> v;
    2. -v in K_exp^* (v in the polar cone) -> 0;
    3. x0 <= 0 and y0 <= 0 -> (x0, 0, max(z0, 0));
    4. otherwise the projection is y (rho, 1, e^rho) with y > 0, where rho
       solves the stationarity equation of ``_exp_stationarity``.  Writing
       v = y d(rho) + c n(rho) with the surface normal
       n(rho) = (e^rho, (1-rho) e^rho, -1) and y, c > 0 gives the bracket
       conditions rho x0 > x0 - y0 and rho y0 < x0, which bound rho on one
       or both sides; an open side is found by doubling.
    The root is refined by bisection to full double precision, and the
    candidates are compared by distance among the feasible ones.
    """
    v = np.asarray(v, dtype=np.float64)
    x0, y0, z0 = float(v[0]), float(v[1]), float(v[2])
    if in_exp_cone(v):
        return v.copy()
    if in_exp_dual(-v):
        return np.zeros(3)
    if x0 <= 0 and y0 <= 0:
        return np.array([x0, 0.0, max(z0, 0.0)])

    fun = lambda r: _exp_stationarity(r, x0, y0, z0)  # noqa: E731
    lo = -math.inf
    hi = math.inf
    if x0 > 0:
        lo = max(lo, 1.0 - y0 / x0)
    elif x0 < 0:
        hi = min(hi, 1.0 - y0 / x0)
    if y0 > 0:
        hi = min(hi, x0 / y0)
    elif y0 < 0:
        lo = max(lo, x0 / y0)
    # close open sides by doubling away from the finite end
    if math.isinf(lo) and math.isinf(hi):
        lo, hi = -1.0, 1.0
    if math.isinf(hi):
        step = 1.0
        hi = lo + step
        while fun(hi) > 0 and step < 1e6:
            step *= 2.0
            hi = lo + step
    if math.isinf(lo):
        step = 1.0
        lo = hi - step
        while fun(lo) < 0 and step < 1e6:
            step *= 2.0
            lo = hi - step
    flo, fhi = fun(lo), fun(hi)
    # the bracket ends are candidates too: when the root sits at an end,
    # rounding in f there can hide the sign change
    cands = [np.zeros(3), np.array([min(x0, 0.0), 0.0, max(z0, 0.0)]),
             _exp_boundary_point(lo, v), _exp_boundary_point(hi, v)]
    if flo == 0.0:
        cands.append(_exp_boundary_point(lo, v))
    elif fhi == 0.0:
        cands.append(_exp_boundary_point(hi, v))
    elif (flo > 0) != (fhi > 0):
        cands.append(_exp_boundary_point(_bisect(fun, lo, hi, flo), v))
    else:
        # no sign change on the bracket: scan it for one (safety net)
        grid = np.linspace(lo, hi, 2001)
        vals = [fun(float(g)) for g in grid]
        for a, b_, fa, fb in zip(grid[:-1], grid[1:], vals[:-1], vals[1:]):
            if (fa > 0) != (fb > 0):
                cands.append(_exp_boundary_point(_bisect(fun, float(a), float(b_), fa), v))
    best = None
    bestd = math.inf
    for p in cands:
        if not in_exp_cone(p, tol=1e-12 * (1.0 + float(np.linalg.norm(p)))):
            continue
        dist = float(np.linalg.norm(p - v))
        if dist < bestd:
            best, bestd = p, dist
    return best


def proj_exp_dual(v: np.ndarray) -> np.ndarray:
    """Projection onto K_exp^* via Moreau: Pi_{K*}(v) = v + Pi_K(-v)."""
    v = np.asarray(v, dtype=np.float64)
    return v + proj_exp(-v)


# ----------------------------------------------------------------------------
# power cone
# ----------------------------------------------------------------------------

def _wpow(t: float, e: float) -> float:
    """t^e for t >= 0 with t^0 = 1 (also at t = 0 or t = inf): the factor of
    an exponent-zero coordinate drops out of the power-cone definitions."""
    if e == 0.0:
        return 1.0
    return t ** e


def in_pow_cone(v, a: float, tol: float = 0.0) -> bool:
    """Membership in K_pow^a = {(x,y,z): x^a y^(1-a) >= |z|, x >= 0, y >= 0}
    (Sect. 6.1) of v + tol (1, 1, 0): with tol > 0 a point within distance
    sqrt(2) tol of the cone passes.  (A slack on the defining inequality
    itself would be ill-conditioned: x^a has unbounded slope at x = 0.)"""
    x, y, z = (float(t) for t in v)
    x += tol
    y += tol
    if x < 0.0 or y < 0.0:
        return False
    return _wpow(x, a) * _wpow(y, 1.0 - a) >= abs(z)


def in_pow_dual(v, a: float, tol: float = 0.0) -> bool:
    """Membership in (K_pow^a)^* = {(u,v,w): (u/a)^a (v/(1-a))^(1-a) >= |w|,
    u >= 0, v >= 0} (Sect. 6.1) of v + tol (1, 1, 0), as in ``in_pow_cone``;
    a factor whose exponent is zero is 1."""
    u, vv, w = (float(t) for t in v)
    u += tol
    vv += tol
    if u < 0.0 or vv < 0.0:
        return False
    fu = 1.0 if a == 0.0 else (u / a) ** a
    fv = 1.0 if a == 1.0 else (vv / (1.0 - a)) ** (1.0 - a)
    return fu * fv >= abs(w)


def _pow_point(r: float, x0: float, y0: float, az: float, a: float):
    """The candidate (x(r), y(r)) of the power-cone projection for |z| = r.

    On the boundary x^a y^(1-a) = r the stationarity conditions of
    min |p - v|^2 with multiplier mu = |z0| - r read x^2 - x0 x - mu a r = 0
    and y^2 - y0 y - mu (1-a) r = 0; their nonnegative roots are taken.  For
    a negative x0 the root (x0 + s)/2, s = sqrt(x0^2 + 4c), is evaluated as
    2c/(s - x0), the same number without the cancellation."""
    mu = az - r

    def root(t0: float, c: float) -> float:
        s = math.sqrt(t0 * t0 + 4.0 * c)
        return 0.5 * (t0 + s) if t0 >= 0.0 else 2.0 * c / (s - t0)

    return root(x0, a * r * mu), root(y0, (1.0 - a) * r * mu)


def proj_pow(v: np.ndarray, a: float) -> np.ndarray:
    """Projection of v = (x0, y0, z0) onto K_pow^a, a in [0, 1].

    The paper defines the cone (Sect. 6.1) and gives no algorithm.  Cases:

    1. v in K -> v;
    2. -v in K^* (v in the polar cone) -> 0;
    3. z0 = 0 -> (max(x0, 0), max(y0, 0), 0);
    4. otherwise the projection lies on the boundary with z = sign(z0) r,
       0 < r < |z0|, and (x, y) = ``_pow_point(r)`` from the stationarity
       conditions of the nearest-point problem; r is the root of
       phi(r) = x(r)^a y(r)^(1-a) - r, which is positive just above 0 (else
       case 2 holds) and negative at |z0| (else case 1 holds).  The root is
       found by bisection to full double precision.
    """
    v = np.asarray(v, dtype=np.float64)
    x0, y0, z0 = float(v[0]), float(v[1]), float(v[2])
    if in_pow_cone(v, a):
        return v.copy()
    if in_pow_dual(-v, a):
        return np.zeros(3)
    if z0 == 0.0:
        return np.array([max(x0, 0.0), max(y0, 0.0), 0.0])
    az = abs(z0)

    def phi(r: float) -> float:
        x, y = _pow_point(r, x0, y0, az, a)
        return _wpow(x, a) * _wpow(y, 1.0 - a) - r

    lo, hi = 0.0, az
    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if phi(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    r = 0.5 * (lo + hi)
    x, y = _pow_point(r, x0, y0, az, a)
    return np.array([x, y, math.copysign(r, z0)])


def proj_pow_dual(v: np.ndarray, a: float) -> np.ndarray:
    """Projection onto (K_pow^a)^* via Moreau: Pi_{K*}(v) = v + Pi_K(-v)."""
    v = np.asarray(v, dtype=np.float64)
    return v + proj_pow(-v, a)


# ----------------------------------------------------------------------------
# product cones
# ----------------------------------------------------------------------------

def cone_blocks(cone):
    """Yield (kind, start, length, param) for each block of the product cone
    in row order: zero, nonneg, soc, psd, exp, dexp, pow.  ``cone`` is any
    object with attributes f, l, q, s, ep, ed and optionally p (or a dict
    with those keys).  A power block's param is its entry of p: a >= 0 for
    K_pow^a, -a < 0 for (K_pow^a)^*."""
    if isinstance(cone, dict):
        get = lambda k: cone.get(k, [] if k == "p" else 0)  # noqa: E731
    else:
        get = lambda k: getattr(cone, k, [] if k == "p" else 0)  # noqa: E731
    pos = 0
    f, l = int(get("f")), int(get("l"))
    if f:
        yield ("zero", pos, f, None)
        pos += f
    if l:
        yield ("nonneg", pos, l, None)
        pos += l
    for k in get("q"):
        yield ("soc", pos, int(k), None)
        pos += int(k)
    for d in get("s"):
        L = svec_len(int(d))
        yield ("psd", pos, L, int(d))
        pos += L
    for _ in range(int(get("ep"))):
        yield ("exp", pos, 3, None)
        pos += 3
    for _ in range(int(get("ed"))):
        yield ("dexp", pos, 3, None)
        pos += 3
    for a in get("p"):
        yield ("pow", pos, 3, float(a))
        pos += 3


def cone_dim(cone) -> int:
    return sum(L for _, _, L, _ in cone_blocks(cone))


def proj_cone(x: np.ndarray, cone, dual: bool = False) -> np.ndarray:
    """Projection onto K (``dual=False``) or K^* (``dual=True``) for the
    product cone.  Zero cone: K = {0}, K^* = R.  Nonnegative, second-order
    and PSD cones are self-dual.  Exponential and power blocks swap with
    their duals."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    for kind, a, L, d in cone_blocks(cone):
        seg = x[a:a + L]
        if kind == "zero":
            out[a:a + L] = seg if dual else 0.0
        elif kind == "nonneg":
            out[a:a + L] = proj_nonneg(seg)
        elif kind == "soc":
            out[a:a + L] = proj_soc(seg)
        elif kind == "psd":
            out[a:a + L] = proj_psd(seg, d)
        elif kind == "exp":
            out[a:a + L] = proj_exp_dual(seg) if dual else proj_exp(seg)
        elif kind == "dexp":
            out[a:a + L] = proj_exp(seg) if dual else proj_exp_dual(seg)
        elif kind == "pow":
            # a >= 0: K_pow^a; a < 0: (K_pow^|a|)^*
            primal = (d >= 0) != dual
            out[a:a + L] = proj_pow(seg, abs(d)) if primal else proj_pow_dual(seg, abs(d))
    return out


def in_cone(x: np.ndarray, cone, dual: bool = False, tol: float = 1e-9) -> bool:
    """Membership test for K or K^* with absolute slack ``tol`` (scaled by
    the block norm)."""
    for kind, a, L, d in cone_blocks(cone):
        seg = np.asarray(x[a:a + L], dtype=np.float64)
        sc = tol * (1.0 + float(np.linalg.norm(seg)))
        if kind == "zero":
            if not dual and np.any(np.abs(seg) > sc):
                return False
        elif kind == "nonneg":
            if np.any(seg < -sc):
                return False
        elif kind == "soc":
            if np.linalg.norm(seg[1:]) > seg[0] + sc:
                return False
        elif kind == "psd":
            if np.linalg.eigvalsh(smat(seg, d)).min() < -sc:
                return False
        elif kind in ("exp", "dexp"):
            primal = (kind == "exp") != dual
            ok = in_exp_cone(seg, sc) if primal else in_exp_dual(seg, sc)
            if not ok:
                return False
        elif kind == "pow":
            primal = (d >= 0) != dual
            ok = in_pow_cone(seg, abs(d), sc) if primal else in_pow_dual(seg, abs(d), sc)
            if not ok:
                return False
    return True
