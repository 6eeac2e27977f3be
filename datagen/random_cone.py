"""Seeded draws for the random feasible cone programs of Sect. 6 (random cone
programs, Table 5).

The paper builds a feasible, bounded program with a known optimal value from
a random vector z, a random sparse A with standard normal entries (pattern
chosen uniformly at random) and a random x*.  This module performs exactly
those random draws and nothing else.  Every function takes an integer seed
and uses ``numpy.random.Generator(PCG64(seed))`` with a fixed draw order:

1. cone sizes,
2. z ~ N(0, 1)^m,
3. the nonzero positions of A (``round(density*m*n)`` distinct positions,
   uniform over all such sets),
4. the nonzero values of A, N(0, 1), in row-major position order,
5. x* ~ N(0, 1)^n,
6. (parametric family only) the dense matrix B.

Rows of the cone are ordered: zero cone, nonnegative, second-order, PSD
(scaled svec, lower triangle, column-major), primal exponential triples,
dual exponential triples, power-cone triples.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass
class ConeSpec:
    """Product cone K = {0}^f x R_+^l x SOC(q_1) x ... x PSD(s_1) x ... x
    K_exp^ep x (K_exp^*)^ed, in that row order.

    ``q`` holds second-order cone sizes (bound first, then the vector part).
    ``s`` holds PSD matrix sides d; each occupies d(d+1)/2 rows (scaled svec).
    ``ep``/``ed`` count primal / dual exponential-cone triples (x, y, z).
    ``p`` holds power-cone parameters, one triple (x, y, z) each, after the
    exponential triples: a in [0, 1] for the power cone with exponent a, -a
    for its dual.
    """

    f: int = 0
    l: int = 0
    q: List[int] = field(default_factory=list)
    s: List[int] = field(default_factory=list)
    ep: int = 0
    ed: int = 0
    p: List[float] = field(default_factory=list)

    @property
    def m(self) -> int:
        return (self.f + self.l + int(sum(self.q))
                + int(sum(d * (d + 1) // 2 for d in self.s))
                + 3 * (self.ep + self.ed + len(self.p)))

    def to_dict(self) -> dict:
        return {"f": self.f, "l": self.l, "q": list(map(int, self.q)),
                "s": list(map(int, self.s)), "ep": self.ep, "ed": self.ed,
                "p": list(map(float, self.p))}


@dataclass
class Draw:
    """One seeded draw: the cone, sizes, z, A in CSR form and x*."""

    cone: ConeSpec
    m: int
    n: int
    z: np.ndarray            # (m,) float64
    indptr: np.ndarray       # (m+1,) int64
    indices: np.ndarray      # (nnz,) int32, sorted within each row
    data: np.ndarray         # (nnz,) float64
    xstar: np.ndarray        # (n,) float64
    seed: int = 0

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])


def _fill_soc_sizes(rng: np.random.Generator, rows: int, lo: int, hi: int) -> List[int]:
    """Second-order cone sizes drawn uniformly from [lo, hi] in sequence until
    ``rows`` rows are used.  A draw larger than what is left is cut to the
    remainder; a remainder smaller than ``lo`` left after a draw is merged
    into the last cone (so every cone has at least ``lo`` rows unless
    ``rows < lo``)."""
    sizes: List[int] = []
    left = rows
    while left > 0:
        k = int(rng.integers(lo, hi + 1))
        k = min(k, left)
        sizes.append(k)
        left -= k
        if 0 < left < lo:
            sizes[-1] += left
            left = 0
    return sizes


def sample_sparse_pattern(rng: np.random.Generator, m: int, n: int, nnz: int) -> np.ndarray:
    """``nnz`` distinct flat positions in [0, m*n), uniform over all sets of
    that size, returned sorted (row-major order).

    Positions are drawn with replacement and de-duplicated, and the deficit is
    drawn again until exactly ``nnz`` distinct positions remain; the procedure
    is exchangeable over positions, so every ``nnz``-subset is equally likely.
    """
    total = m * n
    if nnz > total:
        raise ValueError("nnz exceeds m*n")
    if nnz == 0:
        return np.zeros(0, dtype=np.int64)
    if nnz * 4 > total:
        # dense regime: a permutation prefix is cheaper than rejection
        return np.sort(rng.permutation(total)[:nnz].astype(np.int64))
    pos = np.unique(rng.integers(0, total, size=nnz, dtype=np.int64))
    while pos.shape[0] < nnz:
        extra = rng.integers(0, total, size=nnz - pos.shape[0], dtype=np.int64)
        pos = np.unique(np.concatenate([pos, extra]))
    return pos


def _csr_from_positions(pos: np.ndarray, m: int, n: int, vals: np.ndarray):
    rows = pos // n
    cols = (pos % n).astype(np.int32)
    counts = np.bincount(rows, minlength=m)
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    return indptr, cols, vals


def draw_instance(seed: int, n: int, cone: ConeSpec, density: float) -> Draw:
    """Draw z, A and x* for a program with ``n`` variables and cone ``cone``
    (cone sizes must already be fixed; use the ``draw_*`` helpers to draw
    them from the same generator)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return _draw_rest(rng, seed, n, cone, density)


def _draw_rest(rng, seed, n, cone, density) -> Draw:
    m = cone.m
    z = rng.standard_normal(m)
    nnz = int(round(density * m * n))
    pos = sample_sparse_pattern(rng, m, n, nnz)
    vals = rng.standard_normal(pos.shape[0])
    indptr, indices, data = _csr_from_positions(pos, m, n, vals)
    xstar = rng.standard_normal(n)
    return Draw(cone=cone, m=m, n=n, z=z, indptr=indptr, indices=indices,
                data=data, xstar=xstar, seed=seed)


def draw_lp(seed: int, n: int = 100, m: int = 300, density: float = 0.1) -> Draw:
    """Random LP: nonnegative cone only (default sizes: n=100, m=300,
    density 0.1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cone = ConeSpec(l=m)
    return _draw_rest(rng, seed, n, cone, density)


def draw_socp(seed: int, n: int = 10_000, m: int = 30_000, nonneg: int = 5_000,
              soc_lo: int = 3, soc_hi: int = 50, density: float = 1e-3) -> Draw:
    """Random SOCP: ``nonneg`` nonnegative rows, then second-order cones of
    sizes uniform in [soc_lo, soc_hi] filling the remaining rows."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = _fill_soc_sizes(rng, m - nonneg, soc_lo, soc_hi)
    cone = ConeSpec(l=nonneg, q=q)
    return _draw_rest(rng, seed, n, cone, density)


def draw_mixed(seed: int, n: int = 5_000, nonneg: int = 2_000, n_soc: int = 400,
               soc_lo: int = 3, soc_hi: int = 30, n_psd: int = 60, psd_lo: int = 8,
               psd_hi: int = 40, n_exp: int = 500, n_dexp: int = 0,
               density: float = 2e-3, n_pow: int = 0) -> Draw:
    """Mixed-cone program: nonnegative rows, ``n_soc`` SOCs with sizes in
    [soc_lo, soc_hi], ``n_psd`` PSD cones with sides in [psd_lo, psd_hi]
    (scaled svec) and ``n_exp`` primal exponential triples (plus ``n_dexp``
    dual exponential triples and ``n_pow`` power-cone triples whose
    parameters are uniform in [-1, 1], a negative one meaning the dual
    cone).  With n_pow = 0 the draw is the same as before power cones
    existed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = [int(v) for v in rng.integers(soc_lo, soc_hi + 1, size=n_soc)]
    s = [int(v) for v in rng.integers(psd_lo, psd_hi + 1, size=n_psd)]
    p = [float(v) for v in rng.uniform(-1.0, 1.0, size=n_pow)] if n_pow > 0 else []
    cone = ConeSpec(l=nonneg, q=q, s=s, ep=n_exp, ed=n_dexp, p=p)
    return _draw_rest(rng, seed, n, cone, density)


def draw_batch_member(seed: int, n_lo: int = 20, n_hi: int = 400, soc_lo: int = 3,
                      soc_hi: int = 10, density: float = 0.05) -> Draw:
    """One member of the batched workload: n uniform in [n_lo, n_hi], m = 3n,
    floor(m/2) nonnegative rows and SOCs of sizes in [soc_lo, soc_hi]
    filling the rest."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rng.integers(n_lo, n_hi + 1))
    m = 3 * n
    nonneg = m // 2
    q = _fill_soc_sizes(rng, m - nonneg, soc_lo, soc_hi)
    cone = ConeSpec(l=nonneg, q=q)
    return _draw_rest(rng, seed, n, cone, density)


@dataclass
class ParametricDraw:
    """Base draw plus the dense perturbation matrix B of b(theta) = b0 + B theta."""

    base: Draw
    B: np.ndarray            # (m, p) float64
    b_std: float


def draw_parametric_family(seed: int = 5000, n: int = 2_000, m: int = 6_000,
                           nonneg: int = 1_000, soc_lo: int = 3, soc_hi: int = 50,
                           density: float = 5e-3, p: int = 64,
                           b_std: float = 0.1) -> ParametricDraw:
    """Parametric SOCP family with fixed A and c: the base draw plus a dense
    B with N(0, b_std^2) entries (``b_std`` is the standard deviation)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = _fill_soc_sizes(rng, m - nonneg, soc_lo, soc_hi)
    cone = ConeSpec(l=nonneg, q=q)
    base = _draw_rest(rng, seed, n, cone, density)
    B = b_std * rng.standard_normal((m, p))
    return ParametricDraw(base=base, B=B, b_std=b_std)


def draw_theta(seed: int, p: int = 64) -> np.ndarray:
    """theta ~ N(0, I_p) for one member of the parametric family."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(p)
