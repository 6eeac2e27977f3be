"""Shared helpers for the GPU tests: seeded instances built by the oracle
(test infrastructure) and fed to both sides."""

import sys

import numpy as np

from datagen import draw_lp, draw_mixed, draw_socp
from oracle.instances import from_draw


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def lp_c1(seed=0):
    """Random LP: n=100, m=300, nonnegative cone, density 0.1."""
    return from_draw(draw_lp(seed))


def socp_small(seed=0, n=400, m=1200, nonneg=200, density=1e-2):
    return from_draw(draw_socp(seed, n=n, m=m, nonneg=nonneg, density=density))


def mixed_small(seed=0):
    return from_draw(draw_mixed(seed, n=150, nonneg=60, n_soc=12, soc_lo=3, soc_hi=12,
                                n_psd=5, psd_lo=2, psd_hi=9, n_exp=20, n_dexp=6,
                                density=4e-2))


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def weak_duality_bound(inst, x, y, s):
    """(objective, bound) for an approximate solution of a program with the
    planted solution (x*, y*, s*) of inst: with r_p = Ax + s - b,
    r_d = A^T y + c, s in K and y in K*, weak duality puts the mean
    objective (c^T x - b^T y)/2 within
        gap/2 + max(|r_p| |y*|, |r_d| |x*|)
    of p* = c^T x*, where gap = |c^T x + b^T y|.  The stopping criteria
    bound residuals, not the objective error, so two solutions that both
    pass them can differ in objective by up to the sum of their bounds."""
    A, b, c = inst.A, inst.b, inst.c
    pri = np.linalg.norm(A @ x + s - b)
    dua = np.linalg.norm(A.T @ y + c)
    gap = abs(c @ x + b @ y)
    obj = 0.5 * (c @ x - b @ y)
    return obj, 0.5 * gap + max(pri * np.linalg.norm(inst.ystar), dua * np.linalg.norm(inst.xstar))
