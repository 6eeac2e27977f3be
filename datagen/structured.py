"""Seeded structured cone programs: the problem families of Sect. 6.2-6.5
(lasso, long-only portfolio with a factor risk model, robust PCA, and
l1-regularised logistic regression), drawn as each section's "problem
instances" paragraph describes and written in the standard form of
Sect. 2 (e-coneprob):

    minimize c^T x  subject to  A x + s = b,  s in K,

with the rows of K in the order zero, nonnegative, second-order, PSD
(scaled svec: lower triangle, column-major, off-diagonal entries times
sqrt 2), exponential.  Turning a family's model into (A, b, c, K) is
modelling, not the method: every consumer solves the same data.

Readings (the paper is silent or its text and tables disagree):

* "N(0, 0.1)" is a normal law with standard deviation 0.1.
* The tables' nonzero counts of A imply sparse data matrices with about
  10 % nonzeros (lasso's F, portfolio's F, the logistic regression's data
  points), where the text only names the entries' distribution; the
  matrices are drawn with ``density`` (default 0.1) nonzeros, uniformly
  placed, with the stated entry distribution.
* The tables' standard-form sizes come from the authors' modelling tool;
  the forms here follow the formulations printed in the text, so n, m and
  the nonzero counts differ from the tables'.
* RPCA's objective is printed as "maximize (1/2)(Tr W1 + Tr W2)"; the
  nuclear norm is the minimum of that expression over the PSD constraint,
  so the program minimises it.  The sparse part's nonzero values are
  standard normal.
* The logistic regression's objective sum log(1 + exp(y_i w^T z_i)) is
  kept as printed (the labels' sign convention does not change the
  problem's structure).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .random_cone import ConeSpec, sample_sparse_pattern


@dataclass
class Program:
    """A cone program in standard form plus what its family needs to judge
    a solution (its model data)."""

    name: str
    cone: ConeSpec
    m: int
    n: int
    indptr: np.ndarray       # (m+1,) int64
    indices: np.ndarray      # (nnz,) int32
    data: np.ndarray         # (nnz,) float64
    b: np.ndarray
    c: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])

    def csr(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.m, self.n))


class _Rows:
    """Row-by-row COO assembly."""

    def __init__(self):
        self.r, self.c, self.v = [], [], []
        self.b = []
        self.m = 0

    def add(self, cols, vals, rhs=0.0):
        cols = np.atleast_1d(np.asarray(cols, dtype=np.int64))
        vals = np.broadcast_to(np.asarray(vals, dtype=np.float64), cols.shape)
        self.r.append(np.full(cols.shape[0], self.m, dtype=np.int64))
        self.c.append(cols)
        self.v.append(np.array(vals))
        self.b.append(float(rhs))
        self.m += 1

    def add_block(self, rows, cols, vals, rhs):
        """Several rows at once: entry k of (rows, cols, vals) is in row
        self.m + rows[k]; rhs has one entry per new row."""
        rhs = np.asarray(rhs, dtype=np.float64)
        self.r.append(np.asarray(rows, dtype=np.int64) + self.m)
        self.c.append(np.asarray(cols, dtype=np.int64))
        self.v.append(np.asarray(vals, dtype=np.float64))
        self.b.extend(rhs.tolist())
        self.m += rhs.shape[0]

    def finish(self, n):
        r = np.concatenate(self.r) if self.r else np.zeros(0, np.int64)
        c = np.concatenate(self.c) if self.c else np.zeros(0, np.int64)
        v = np.concatenate(self.v) if self.v else np.zeros(0)
        order = np.lexsort((c, r))
        r, c, v = r[order], c[order], v[order]
        counts = np.bincount(r, minlength=self.m)
        indptr = np.zeros(self.m + 1, dtype=np.int64)
        np.cumsum(counts, out=indptr[1:])
        return indptr, c.astype(np.int32), v, np.array(self.b)


def _sparse(rng, rows, cols, density, std=1.0):
    """rows x cols matrix with round(density rows cols) uniformly placed
    nonzeros of law N(0, std^2), as (row, col, value) arrays."""
    nnz = int(round(density * rows * cols))
    pos = sample_sparse_pattern(rng, rows, cols, nnz)
    vals = std * rng.standard_normal(pos.shape[0])
    return pos // cols, pos % cols, vals


# ----------------------------------------------------------------------------
# lasso (Sect. 6.2)
# ----------------------------------------------------------------------------

def lasso(seed: int, p: int = 10_000, q: int = 2_000, density: float = 0.1) -> Program:
    """minimize (1/2)|F z - g|^2 + mu |z|_1 as the SOCP
        minimize (1/2) w + mu 1^T t
        s.t.  -t <= z <= t,  |(1 - w, 2(F z - g))|_2 <= 1 + w
    over x = (z, t, w).  F (q x p) has N(0, 1) entries, z_hat has p/10
    N(0, 1) nonzeros, g = F z_hat + N(0, 0.1^2) noise, mu = 0.1 |F^T g|_inf.
    Draw order: F's pattern and values, z_hat's support and values, the
    noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fr, fc, fv = _sparse(rng, q, p, density)
    k = max(1, p // 10)
    supp = np.sort(rng.choice(p, size=k, replace=False))
    zhat = np.zeros(p)
    zhat[supp] = rng.standard_normal(k)
    noise = 0.1 * rng.standard_normal(q)
    Fz = np.bincount(fr, weights=fv * zhat[fc], minlength=q)
    g = Fz + noise
    Ftg = np.bincount(fc, weights=fv * g[fr], minlength=p)
    mu = 0.1 * float(np.max(np.abs(Ftg)))
    n = 2 * p + 1
    iz, it, iw = 0, p, 2 * p
    R = _Rows()
    ar = np.arange(p)
    # t - z >= 0, t + z >= 0 (s = b - A x)
    R.add_block(np.r_[ar, ar], np.r_[iz + ar, it + ar], np.r_[np.ones(p), -np.ones(p)], np.zeros(p))
    R.add_block(np.r_[ar, ar], np.r_[iz + ar, it + ar], np.r_[-np.ones(p), -np.ones(p)], np.zeros(p))
    # second-order cone (1 + w, 1 - w, 2 (F z - g))
    R.add(iw, -1.0, 1.0)
    R.add(iw, 1.0, 1.0)
    R.add_block(fr, iz + fc, -2.0 * fv, -2.0 * g)
    indptr, indices, data, b = R.finish(n)
    c = np.zeros(n)
    c[it:it + p] = mu
    c[iw] = 0.5
    cone = ConeSpec(l=2 * p, q=[q + 2])
    return Program("lasso", cone, R.m, n, indptr, indices, data, b, c,
                   meta={"p": p, "q": q, "mu": mu, "F": (fr, fc, fv), "g": g, "zhat": zhat})


def lasso_objective(prog: Program, x: np.ndarray) -> float:
    p, q = prog.meta["p"], prog.meta["q"]
    fr, fc, fv = prog.meta["F"]
    z = x[:p]
    r = np.bincount(fr, weights=fv * z[fc], minlength=q) - prog.meta["g"]
    return 0.5 * float(r @ r) + prog.meta["mu"] * float(np.abs(z).sum())


# ----------------------------------------------------------------------------
# portfolio (Sect. 6.3)
# ----------------------------------------------------------------------------

def portfolio(seed: int, p: int = 100_000, q: int = 100, density: float = 0.1,
              gamma: float = 1.0) -> Program:
    """maximize mu^T z - gamma z^T (F F^T + D) z, 1^T z = 1, z >= 0, as
        minimize -mu^T z + gamma (t + s)
        s.t.  1^T z = 1, z >= 0, |D^{1/2} z| <= u, |F^T z| <= v,
              |(1 - t, 2u)| <= 1 + t, |(1 - s, 2v)| <= 1 + s
    over x = (z, t, s, u, v).  log(mu) ~ N(0, 1), F (p x q) with N(0, 0.1^2)
    entries, D_ii ~ U[0, 0.1].  Draw order: log(mu), F, D."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mu = np.exp(rng.standard_normal(p))
    fr, fc, fv = _sparse(rng, p, q, density, std=0.1)
    dg = rng.uniform(0.0, 0.1, size=p)
    n = p + 4
    it, is_, iu, iv = p, p + 1, p + 2, p + 3
    ar = np.arange(p)
    R = _Rows()
    R.add(ar, 1.0, 1.0)                                           # zero: 1 - 1^T z = 0
    R.add_block(ar, ar, -np.ones(p), np.zeros(p))                 # z >= 0
    R.add(iu, -1.0, 0.0)                                          # (u, D^{1/2} z)
    R.add_block(ar, ar, -np.sqrt(dg), np.zeros(p))
    R.add(iv, -1.0, 0.0)                                          # (v, F^T z)
    R.add_block(fc, fr, -fv, np.zeros(q))
    R.add(it, -1.0, 1.0)                                          # (1 + t, 1 - t, 2u)
    R.add(it, 1.0, 1.0)
    R.add(iu, -2.0, 0.0)
    R.add(is_, -1.0, 1.0)                                         # (1 + s, 1 - s, 2v)
    R.add(is_, 1.0, 1.0)
    R.add(iv, -2.0, 0.0)
    indptr, indices, data, b = R.finish(n)
    c = np.zeros(n)
    c[:p] = -mu
    c[it] = gamma
    c[is_] = gamma
    cone = ConeSpec(f=1, l=p, q=[p + 1, q + 1, 3, 3])
    return Program("portfolio", cone, R.m, n, indptr, indices, data, b, c,
                   meta={"p": p, "q": q, "gamma": gamma, "mu": mu, "F": (fr, fc, fv), "D": dg})


def portfolio_objective(prog: Program, x: np.ndarray) -> float:
    """Risk-adjusted return mu^T z - gamma z^T (F F^T + D) z (maximised)."""
    p, q = prog.meta["p"], prog.meta["q"]
    fr, fc, fv = prog.meta["F"]
    z = x[:p]
    ftz = np.bincount(fc, weights=fv * z[fr], minlength=q)
    return float(prog.meta["mu"] @ z) - prog.meta["gamma"] * (float(ftz @ ftz) + float(prog.meta["D"] @ (z * z)))


# ----------------------------------------------------------------------------
# robust PCA (Sect. 6.4)
# ----------------------------------------------------------------------------

def _svec_index(d: int, r: int, c: int) -> int:
    """Position of entry (r, c), r >= c, in the scaled svec of side d."""
    return c * d - (c * (c - 1)) // 2 + (r - c)


def rpca(seed: int, p: int = 40, rank: int = 10, frac: float = 0.1) -> Program:
    """minimize |L|_*  s.t. |S|_1 <= mu, L + S = M  (p x p), as the SDP
        minimize (1/2) Tr X,  X = [[W1, L], [L^T, W2]] PSD,
        L + S = M,  -t <= vec(S) <= t,  1^T t <= mu
    over x = (svec X, vec S, t); vec is column-major.  M = L_hat + S_hat,
    L_hat = U V^T with U, V (p x rank) standard normal, S_hat with about
    frac p^2 standard normal nonzeros, mu = |S_hat|_1.  Draw order: U, V,
    S_hat's pattern and values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = p
    U = rng.standard_normal((p, rank))
    V = rng.standard_normal((q, rank))
    Lhat = U @ V.T
    sr, sc, sv = _sparse(rng, p, q, frac)
    Shat = np.zeros((p, q))
    Shat[sr, sc] = sv
    M = Lhat + Shat
    mu = float(np.abs(Shat).sum())
    d = p + q
    nX = d * (d + 1) // 2
    pq = p * q
    iS, itt = nX, nX + pq
    n = nX + 2 * pq
    R = _Rows()
    rs2 = 1.0 / math.sqrt(2.0)
    # zero cone: L_ij + S_ij = M_ij, L_ij = svec(X)[(p + j, i)] / sqrt 2
    rows, cols, vals, rhs = [], [], [], []
    for j in range(q):
        for i in range(p):
            k = j * p + i
            rows += [k, k]
            cols += [_svec_index(d, p + j, i), iS + k]
            vals += [rs2, 1.0]
            rhs.append(M[i, j])
    R.add_block(rows, cols, vals, rhs)
    ar = np.arange(pq)
    R.add_block(np.r_[ar, ar], np.r_[iS + ar, itt + ar], np.r_[np.ones(pq), -np.ones(pq)], np.zeros(pq))
    R.add_block(np.r_[ar, ar], np.r_[iS + ar, itt + ar], np.r_[-np.ones(pq), -np.ones(pq)], np.zeros(pq))
    R.add(itt + ar, 1.0, mu)                                   # mu - 1^T t >= 0
    R.add_block(np.arange(nX), np.arange(nX), -np.ones(nX), np.zeros(nX))   # svec X in PSD
    indptr, indices, data, b = R.finish(n)
    c = np.zeros(n)
    for k in range(d):
        c[_svec_index(d, k, k)] = 0.5
    cone = ConeSpec(f=pq, l=2 * pq + 1, s=[d])
    return Program("rpca", cone, R.m, n, indptr, indices, data, b, c,
                   meta={"p": p, "q": q, "mu": mu, "M": M, "Lhat": Lhat, "Shat": Shat})


def rpca_low_rank(prog: Program, x: np.ndarray) -> np.ndarray:
    """The L block of a solution x."""
    p, q = prog.meta["p"], prog.meta["q"]
    d = p + q
    L = np.empty((p, q))
    for j in range(q):
        for i in range(p):
            L[i, j] = x[_svec_index(d, p + j, i)] / math.sqrt(2.0)
    return L


# ----------------------------------------------------------------------------
# l1-regularised logistic regression (Sect. 6.5)
# ----------------------------------------------------------------------------

def logreg(seed: int, p: int = 100, q: int = 10_000, density: float = 0.1) -> Program:
    """minimize sum_i log(1 + exp(y_i w^T z_i)) + mu |w|_1 as
        minimize 1^T t + mu 1^T s
        s.t. -s <= w <= s, u + v <= 1,
             (y_i w^T z_i - t_i, 1, u_i) in K_exp, (-t_i, 1, v_i) in K_exp
    over x = (w, s, t, u, v).  w_true has at most p/5 N(0, 1) nonzeros; the
    data points z_i (rows of Z, q x p) have N(0, 1) entries; y_i = +1 with
    probability 1/(1 + exp(-w_true^T z_i)), else -1; mu = 0.1 mu_max,
    mu_max = (1/2) |sum_i y_i z_i|_inf.  Draw order: w_true's support and
    values, Z, the label uniforms."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = max(1, p // 5)
    supp = np.sort(rng.choice(p, size=k, replace=False))
    wtrue = np.zeros(p)
    wtrue[supp] = rng.standard_normal(k)
    zr, zc, zv = _sparse(rng, q, p, density)
    lin = np.bincount(zr, weights=zv * wtrue[zc], minlength=q)
    prob = 1.0 / (1.0 + np.exp(-lin))
    y = np.where(rng.uniform(size=q) < prob, 1.0, -1.0)
    yz = np.bincount(zc, weights=zv * y[zr], minlength=p)
    mu = 0.1 * 0.5 * float(np.max(np.abs(yz)))
    iw, is_, it, iu, iv = 0, p, 2 * p, 2 * p + q, 2 * p + 2 * q
    n = 2 * p + 3 * q
    R = _Rows()
    ap, aq = np.arange(p), np.arange(q)
    R.add_block(np.r_[ap, ap], np.r_[iw + ap, is_ + ap], np.r_[np.ones(p), -np.ones(p)], np.zeros(p))
    R.add_block(np.r_[ap, ap], np.r_[iw + ap, is_ + ap], np.r_[-np.ones(p), -np.ones(p)], np.zeros(p))
    R.add_block(np.r_[aq, aq], np.r_[iu + aq, iv + aq], np.ones(2 * q), np.ones(q))   # 1 - u - v >= 0
    # exponential triples (y_i z_i^T w - t_i, 1, u_i): rows 3i, 3i+1, 3i+2
    rows = np.r_[3 * zr, 3 * aq, 3 * aq + 2]
    cols = np.r_[iw + zc, it + aq, iu + aq]
    vals = np.r_[-y[zr] * zv, np.ones(q), -np.ones(q)]
    rhs = np.zeros(3 * q)
    rhs[1::3] = 1.0
    R.add_block(rows, cols, vals, rhs)
    # (-t_i, 1, v_i)
    rows = np.r_[3 * aq, 3 * aq + 2]
    cols = np.r_[it + aq, iv + aq]
    vals = np.r_[np.ones(q), -np.ones(q)]
    R.add_block(rows, cols, vals, rhs)
    indptr, indices, data, b = R.finish(n)
    c = np.zeros(n)
    c[is_:is_ + p] = mu
    c[it:it + q] = 1.0
    cone = ConeSpec(l=2 * p + q, ep=2 * q)
    return Program("logreg", cone, R.m, n, indptr, indices, data, b, c,
                   meta={"p": p, "q": q, "mu": mu, "Z": (zr, zc, zv), "y": y, "wtrue": wtrue})


def logreg_objective(prog: Program, x: np.ndarray) -> float:
    p, q = prog.meta["p"], prog.meta["q"]
    zr, zc, zv = prog.meta["Z"]
    w = x[:p]
    a = prog.meta["y"] * np.bincount(zr, weights=zv * w[zc], minlength=q)
    return float(np.logaddexp(0.0, a).sum()) + prog.meta["mu"] * float(np.abs(w).sum())
