"""Subspace projection (oracle).  TEST INFRASTRUCTURE ONLY.

Sect. 4.1 (solving the linear system): solve (I+Q) u_tilde = w for the
skew-symmetric Q of the embedding (e-hsdnice).  With M = [[I, A^T], [-A, I]]
and h = (c, b), block elimination of the tau row gives

    (M + h h^T) u_xy = w_xy - w_tau h,     u_tau = w_tau + c^T u_x + b^T u_y,

and Sherman-Morrison-Woodbury with the cached g = M^{-1} h and
eta = 1 + h^T g gives u_xy = z - g (h^T z)/eta with z = M^{-1}(w_xy - w_tau h).

M^{-1}(r_x, r_y) is applied by elimination (the indirect method of Sect.
4.1):  z_x = (I + A^T A)^{-1}(r_x - A^T r_y),  z_y = r_y + A z_x.

Two modes:
* ``exact`` -- a dense Cholesky factor of I + A^T A (small n only);
* ``cg``    -- conjugate gradient on I + A^T A, warm-started from the
               previous z_x and stopped when ||(I + A^T A) z_x - rhs||_2 <= tol
               (the approximate projection of Sect. 3.3 with the residual
               test (e-approx-proj-resid); when z_y and u_tau are formed as
               above, that full residual equals the CG residual).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def cg(A: sp.csr_matrix, AT: sp.csr_matrix, rhs: np.ndarray, x0: np.ndarray,
       tol: float, max_iters: int):
    """Conjugate gradient for (I + A^T A) x = rhs from x0 (textbook CG,
    e.g. Golub & Van Loan Alg. 10.2.1).  Stops when the residual 2-norm is at
    most ``tol`` (checked before each iteration, so zero iterations are
    possible).  Returns (x, iterations, final residual norm)."""
    x = x0.copy()
    r = rhs - (x + AT @ (A @ x))
    rr = float(r @ r)
    p = r.copy()
    it = 0
    while np.sqrt(rr) > tol and it < max_iters:
        Gp = p + AT @ (A @ p)
        alpha = rr / float(p @ Gp)
        x += alpha * p
        r -= alpha * Gp
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it, float(np.sqrt(rr))


class LinSys:
    """(I+Q)^{-1} for the scaled data (A_hat, b_hat, c_hat)."""

    def __init__(self, A: sp.csr_matrix, b: np.ndarray, c: np.ndarray,
                 mode: str = "cg", cg_max_iters: int = 100,
                 g_tol_rel: float = 1e-12):
        self.A = sp.csr_matrix(A)
        self.AT = sp.csr_matrix(self.A.T)
        self.m, self.n = self.A.shape
        self.b = np.asarray(b, dtype=np.float64)
        self.c = np.asarray(c, dtype=np.float64)
        self.mode = mode
        self.cg_max_iters = cg_max_iters
        self.h = np.concatenate([self.c, self.b])
        if mode == "exact":
            G = np.eye(self.n) + (self.AT @ self.A).toarray()
            self._chol = sla.cho_factor(G, lower=True)
        elif mode != "cg":
            raise ValueError(mode)
        self.cg_iters_total = 0
        self.spmv_count = 0
        # g = M^{-1} h, computed once (Sect. 4.1, "in the first iteration")
        hn = float(np.linalg.norm(self.h))
        gx, gy, _ = self.minv(self.c, self.b, np.zeros(self.n),
                           tol=g_tol_rel * max(hn, 1.0), max_iters=10 * self.n + 100,
                           count=False)
        self.g = np.concatenate([gx, gy])
        self.eta = 1.0 + float(self.h @ self.g)

    def minv(self, rx, ry, zx0, tol, max_iters=None, count=True):
        """M^{-1}(r_x, r_y) by elimination; CG warm-started from zx0."""
        rhs = rx - self.AT @ ry
        if self.mode == "exact":
            zx = sla.cho_solve(self._chol, rhs)
            it = 0
        else:
            zx, it, _ = cg(self.A, self.AT, rhs, zx0, tol,
                           self.cg_max_iters if max_iters is None else max_iters)
        zy = ry + self.A @ zx
        if count:
            self.cg_iters_total += it
            # products with A or A^T: rhs (1), each CG iteration (2), z_y (1)
            # and the initial CG residual (2, only in cg mode)
            self.spmv_count += 2 + 2 * it + (2 if self.mode == "cg" else 0)
        return zx, zy, it

    def solve(self, w: np.ndarray, zx0: np.ndarray, tol: float):
        """u_tilde = (I+Q)^{-1} w (e-lin-sys), with M^{-1} by ``minv``.
        Returns (u_tilde, z_x, cg iterations)."""
        n, m = self.n, self.m
        wx, wy, wt = w[:n], w[n:n + m], w[n + m]
        rx = wx - wt * self.c
        ry = wy - wt * self.b
        zx, zy, it = self.minv(rx, ry, zx0, tol)
        z = np.concatenate([zx, zy])
        ut_xy = z - self.g * (float(self.h @ z) / self.eta)
        ut_tau = wt + float(self.c @ ut_xy[:n]) + float(self.b @ ut_xy[n:])
        return np.concatenate([ut_xy, [ut_tau]]), zx, it


def dense_Q(A, b, c) -> np.ndarray:
    """The skew-symmetric matrix Q of (e-hsdnice) as a dense array."""
    A = A.toarray() if sp.issparse(A) else np.asarray(A)
    m, n = A.shape
    N = n + m + 1
    Q = np.zeros((N, N))
    Q[:n, n:n + m] = A.T
    Q[:n, -1] = c
    Q[n:n + m, :n] = -A
    Q[n:n + m, -1] = b
    Q[-1, :n] = -c
    Q[-1, n:n + m] = -b
    return Q
