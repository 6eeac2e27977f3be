"""Problem-data scaling (oracle).  TEST INFRASTRUCTURE ONLY.

Sect. 5 (scaling problem data) scales the data to A_hat = D A E,
b_hat = sigma D b, c_hat = rho E c with positive diagonal D, E and positive
scalars sigma, rho, where D must be constant on every block of the cone that
is not separable elementwise (the example after the recovery formulas).  The
paper states only the goals -- columns of A and b with Euclidean norm near
one, rows of A and c with similar norms -- and no algorithm.  This module
implements the reading used throughout this project (rule R):

  D = 1, E = 1
  repeat ``passes`` times:
      r_i  = ||row_i(D A E)||_2 ;  d_i = 1/sqrt(r_i)   (1 if r_i = 0)
      on every second-order, PSD, exponential and power block, replace d_i by the
      block mean of d;  clip d_i to [lo, hi];  D <- D d
      k_j  = ||col_j(D A E)||_2 ;  e_j = 1/sqrt(k_j)   (1 if k_j = 0)
      clip e_j to [lo, hi];  E <- E e
  sigma = 1/max(||D b||_2, tiny)        (b_hat has unit norm)
  rho   = rbar / max(||E c||_2, tiny) with rbar = mean_i ||row_i(A_hat)||_2
                                      (c_hat has the mean row norm of A_hat;
                                       rbar = 1 when A has no nonzeros)

With ``enabled=False`` the scaling is the identity (D = E = 1,
sigma = rho = 1).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .cones import cone_blocks

TINY = 1e-8


@dataclass
class Scaling:
    D: np.ndarray     # (m,)
    E: np.ndarray     # (n,)
    sigma: float
    rho: float


def equilibrate(A: sp.csr_matrix, b: np.ndarray, c: np.ndarray, cone,
                passes: int = 10, lo: float = 1e-4, hi: float = 1e4,
                enabled: bool = True) -> Scaling:
    """Rule R above.  ``A`` is the original (unscaled) data."""
    m, n = A.shape
    D = np.ones(m)
    E = np.ones(n)
    if not enabled:
        return Scaling(D=D, E=E, sigma=1.0, rho=1.0)
    A = sp.csr_matrix(A)
    A2 = A.multiply(A).tocsr()          # squared entries: norms of D A E
    blocks = [(a, L) for kind, a, L, _ in cone_blocks(cone)
              if kind in ("soc", "psd", "exp", "dexp", "pow")]
    for _ in range(passes):
        # row norms of D A E: sqrt(D_i^2 sum_j A_ij^2 E_j^2)
        r = D * np.sqrt(A2 @ (E * E))
        d = np.ones(m)
        pos = r > 0
        d[pos] = 1.0 / np.sqrt(r[pos])
        for a, L in blocks:
            d[a:a + L] = d[a:a + L].mean()
        d = np.clip(d, lo, hi)
        D = D * d
        # column norms of D A E
        k = E * np.sqrt(A2.T @ (D * D))
        e = np.ones(n)
        pos = k > 0
        e[pos] = 1.0 / np.sqrt(k[pos])
        e = np.clip(e, lo, hi)
        E = E * e
    sigma = 1.0 / max(float(np.linalg.norm(D * b)), TINY)
    row_norms = D * np.sqrt(A2 @ (E * E))
    rbar = float(row_norms.mean()) if m > 0 else 1.0
    if not rbar > 0.0:
        rbar = 1.0  # A = 0: keep rho positive
    rho = rbar / max(float(np.linalg.norm(E * c)), TINY)
    return Scaling(D=D, E=E, sigma=sigma, rho=rho)


def apply(A: sp.csr_matrix, b: np.ndarray, c: np.ndarray, sc: Scaling):
    """A_hat = D A E, b_hat = sigma D b, c_hat = rho E c (Sect. 5)."""
    Ah = sp.diags(sc.D) @ sp.csr_matrix(A) @ sp.diags(sc.E)
    return sp.csr_matrix(Ah), sc.sigma * sc.D * b, sc.rho * sc.E * c
