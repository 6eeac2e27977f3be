"""Random cone programs with known optimal value (oracle side).  TEST
INFRASTRUCTURE ONLY.

Sect. 6 (random cone programs): from a random z set s* = Pi_K(z) and
y* = s* - z (conic feasibility, complementarity and zero gap by the Moreau
decomposition), draw A and x*, and set b = A x* + s*, c = -A^T y*; the
optimal value is p* = c^T x*.  The random draws come from ``datagen``; the
projection here is the oracle's own.

The paper only mentions that infeasible and unbounded programs can be built
the same way (together with a certificate); ``make_infeasible`` and
``make_unbounded`` are this project's constructions by a rank-one update
(dense, so for tiny sizes only).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .cones import proj_cone


@dataclass
class Instance:
    A: sp.csr_matrix
    b: np.ndarray
    c: np.ndarray
    cone: object
    xstar: np.ndarray
    ystar: np.ndarray
    sstar: np.ndarray
    pstar: float


def from_draw(draw) -> Instance:
    A = sp.csr_matrix((draw.data, draw.indices, draw.indptr), shape=(draw.m, draw.n))
    s = proj_cone(draw.z, draw.cone, dual=False)
    y = s - draw.z
    b = A @ draw.xstar + s
    c = -(A.T @ y)
    return Instance(A=A, b=b, c=c, cone=draw.cone, xstar=draw.xstar, ystar=y,
                    sstar=s, pstar=float(c @ draw.xstar))


def make_infeasible(inst: Instance, rng: np.random.Generator):
    """Primal-infeasible variant with a known certificate y_c:
    y_c = Pi_{K*}(z') != 0, A <- A - y_c (y_c^T A)/||y_c||^2 (so A^T y_c = 0),
    b <- b - y_c (y_c^T b + 1)/||y_c||^2 (so b^T y_c = -1).  Returns
    (A, b, c, y_c)."""
    m = inst.A.shape[0]
    while True:
        yc = proj_cone(rng.standard_normal(m), inst.cone, dual=True)
        if np.linalg.norm(yc) > 1e-3:
            break
    Ad = inst.A.toarray()
    nrm2 = float(yc @ yc)
    Ad = Ad - np.outer(yc, yc @ Ad) / nrm2
    b = inst.b - yc * (float(yc @ inst.b) + 1.0) / nrm2
    return sp.csr_matrix(Ad), b, inst.c.copy(), yc


def make_unbounded(inst: Instance, rng: np.random.Generator):
    """Dual-infeasible (unbounded) variant with a known certificate x_c:
    s_c = Pi_K(z') in K, A <- A - (A x_c + s_c) x_c^T/||x_c||^2 (so
    -A x_c = s_c in K), c <- c - x_c (x_c^T c + 1)/||x_c||^2 (so
    c^T x_c = -1), and b = A x0 + s0 with s0 in K (primal stays feasible).
    Returns (A, b, c, x_c)."""
    m, n = inst.A.shape
    xc = rng.standard_normal(n)
    sc = proj_cone(rng.standard_normal(m), inst.cone, dual=False)
    Ad = inst.A.toarray()
    nrm2 = float(xc @ xc)
    Ad = Ad - np.outer(Ad @ xc + sc, xc) / nrm2
    c = inst.c - xc * (float(xc @ inst.c) + 1.0) / nrm2
    x0 = rng.standard_normal(n)
    s0 = proj_cone(rng.standard_normal(m), inst.cone, dual=False)
    b = Ad @ x0 + s0
    return sp.csr_matrix(Ad), b, c, xc
