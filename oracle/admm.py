"""ADMM on the homogeneous self-dual embedding (oracle).  TEST
INFRASTRUCTURE ONLY.

Follows the paper step by step:

* embedding and notation u = (x, y, tau), v = (r, s, kappa), cones
  C = R^n x K^* x R_+ and C^* = {0}^n x K x R_+ (Sect. 2.3, e-hsdnice);
* the iteration (e-SCS) with over-relaxation and approximate projection
  (Sect. 3.3):
      u_tilde = (I+Q)^{-1}(u + v)          (to CG tolerance zeta_k)
      u_bar   = alpha u_tilde + (1 - alpha) u
      u+      = Pi_C(u_bar - v)
      v+      = v - u_bar + u+
* the cold start u = v = (0, 0, 1) (Sect. 3.4, eliminating convergence to
  zero) and the warm start u = (x*, y*, 1), v = (0, s*, 0) (Sect. 4.2);
* termination (Sect. 3.5) in the scaled form of Sect. 5, outcome decoding
  and certificates (Sect. 2.3 cases 1-2), unscaling (Sect. 5);
* CG tolerance zeta_k = (k+1)^{-1.5} for the solve that produces
  u^{k+1} (Sect. 6.1, written there as (1/k)^{1.5} with k counted from 1);
* the reported objective is the mean of the primal and dual objectives
  (Sect. 6.1).

Readings where the paper is silent (also listed in the design notes):
the test order when several tests pass is optimality, then infeasibility,
then unboundedness; a certificate test whose normalising norm (||b|| or
||c||) is zero is disabled; the optimality test requires tau > 0; the
iterate is checked before each update, so ``iters`` is the number of
updates performed when a test first passes.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp

from . import cones as K
from .linsys import LinSys
from .scaling import Scaling, apply, equilibrate

SOLVED = 1
MAX_ITERS = 2
INFEASIBLE = 3
UNBOUNDED = 4
INDETERMINATE = 5


@dataclass
class Settings:
    eps_pri: float = 1e-4
    eps_dual: float = 1e-4
    eps_gap: float = 1e-4
    eps_unbdd: float = 1e-4
    eps_infeas: float = 1e-4
    alpha: float = 1.5
    cg_zeta_pow: float = 1.5
    cg_max_iters: int = 100
    max_iters: int = 10_000
    check_every: int = 1
    scale: bool = True
    mode: str = "cg"          # "cg" or "exact"


@dataclass
class Info:
    status: int = 0
    iters: int = 0
    res_pri: float = np.inf
    res_dual: float = np.inf
    gap: float = np.inf
    pobj: float = np.nan
    dobj: float = np.nan
    obj: float = np.nan
    tau: float = np.nan
    kappa: float = np.nan
    cg_iters: int = 0
    spmv_count: int = 0


@dataclass
class Result:
    x: np.ndarray
    y: np.ndarray
    s: np.ndarray
    info: Info
    u: np.ndarray = None
    v: np.ndarray = None
    history: list = field(default_factory=list)


class Problem:
    """Scaled problem data, the cached linear-system quantities and the
    projections onto C and C^*."""

    def __init__(self, A, b, c, cone, settings: Settings):
        self.A0 = sp.csr_matrix(A, dtype=np.float64)
        self.b0 = np.asarray(b, dtype=np.float64)
        self.c0 = np.asarray(c, dtype=np.float64)
        self.m, self.n = self.A0.shape
        if K.cone_dim(cone) != self.m:
            raise ValueError("cone dimension does not match the rows of A")
        self.cone = cone
        self.st = settings
        self.sc: Scaling = equilibrate(self.A0, self.b0, self.c0, cone,
                                       enabled=settings.scale)
        self.A, self.b, self.c = apply(self.A0, self.b0, self.c0, self.sc)
        self.AT = sp.csr_matrix(self.A.T)
        self.lin = LinSys(self.A, self.b, self.c, mode=settings.mode,
                          cg_max_iters=settings.cg_max_iters)
        self.nb = float(np.linalg.norm(self.b0))
        self.nc = float(np.linalg.norm(self.c0))

    # -- cones C and C^* (e-hsdnice) ---------------------------------------
    def proj_C(self, w: np.ndarray) -> np.ndarray:
        """Pi_C with C = R^n x K^* x R_+."""
        n, m = self.n, self.m
        out = np.empty_like(w)
        out[:n] = w[:n]
        out[n:n + m] = K.proj_cone(w[n:n + m], self.cone, dual=True)
        out[n + m] = max(w[n + m], 0.0)
        return out

    def proj_Cstar(self, w: np.ndarray) -> np.ndarray:
        """Pi_{C^*} with C^* = {0}^n x K x R_+."""
        n, m = self.n, self.m
        out = np.empty_like(w)
        out[:n] = 0.0
        out[n:n + m] = K.proj_cone(w[n:n + m], self.cone, dual=False)
        out[n + m] = max(w[n + m], 0.0)
        return out

    # -- starts -------------------------------------------------------------
    def cold_start(self):
        """u0 = v0 = (0, 0, 1) (Sect. 3.4)."""
        N = self.n + self.m + 1
        u = np.zeros(N)
        v = np.zeros(N)
        u[-1] = 1.0
        v[-1] = 1.0
        return u, v

    def warm_start(self, x, y, s):
        """u0 = (x, y, 1), v0 = (0, s, 0) in scaled variables (Sect. 4.2),
        with x_hat = sigma E^{-1} x, y_hat = rho D^{-1} y, s_hat = sigma D s
        (inverse of the recovery formulas of Sect. 5)."""
        sc = self.sc
        u = np.concatenate([sc.sigma * x / sc.E, sc.rho * y / sc.D, [1.0]])
        v = np.concatenate([np.zeros(self.n), sc.sigma * sc.D * s, [0.0]])
        return u, v

    def start_from_q(self, q):
        """u0 = Pi_C(q), v0 = Pi_{C^*}(-q): the Moreau pair of q = u - v
        (e-moreau), which is the whole ADMM state; q is in scaled variables."""
        q = np.asarray(q, dtype=np.float64)
        return self.proj_C(q), self.proj_Cstar(-q)

    # -- termination (Sect. 3.5, scaled form Sect. 5) -----------------------
    def residuals(self, u, v):
        n, m = self.n, self.m
        sc, st = self.sc, self.st
        ux, uy, tau = u[:n], u[n:n + m], u[n + m]
        vs, kappa = v[n:n + m], v[n + m]
        Aux = self.A @ ux
        ATuy = self.AT @ uy
        out = {"tau": tau, "kappa": kappa}
        if tau > 0:
            pri = np.linalg.norm((Aux + vs - self.b * tau) / sc.D) / (sc.sigma * tau)
            dua = np.linalg.norm((ATuy + self.c * tau) / sc.E) / (sc.rho * tau)
            cx = float(self.c @ ux) / (sc.rho * sc.sigma * tau)
            by = float(self.b @ uy) / (sc.rho * sc.sigma * tau)
            out.update(res_pri=pri, res_dual=dua, pobj=cx, dobj=-by,
                       gap=abs(cx + by),
                       solved=(pri <= st.eps_pri * (1 + self.nb)
                               and dua <= st.eps_dual * (1 + self.nc)
                               and abs(cx + by) <= st.eps_gap * (1 + abs(cx) + abs(by))))
        else:
            out.update(res_pri=np.inf, res_dual=np.inf, pobj=np.nan, dobj=np.nan,
                       gap=np.inf, solved=False)
        bty = float(self.b @ uy)
        cxt = float(self.c @ ux)
        out["infeasible"] = bool(self.nb > 0 and -bty > 0 and
                                 np.linalg.norm(ATuy / sc.E)
                                 <= (-bty / np.linalg.norm(self.b / sc.D)) * st.eps_infeas)
        out["unbounded"] = bool(self.nc > 0 and -cxt > 0 and
                                np.linalg.norm((Aux + vs) / sc.D)
                                <= (-cxt / np.linalg.norm(self.c / sc.E)) * st.eps_unbdd)
        out["finite"] = bool(np.all(np.isfinite(u)) and np.all(np.isfinite(v)))
        return out

    def decide(self, u, v):
        r = self.residuals(u, v)
        if not r["finite"]:
            return INDETERMINATE, r
        if r["solved"]:
            return SOLVED, r
        if r["infeasible"]:
            return INFEASIBLE, r
        if r["unbounded"]:
            return UNBOUNDED, r
        return 0, r

    # -- outputs (Sect. 2.3 outcomes, Sect. 5 recovery) ----------------------
    def outputs(self, u, v, status):
        n, m = self.n, self.m
        sc = self.sc
        ux, uy, tau = u[:n], u[n:n + m], u[n + m]
        vs = v[n:n + m]
        if status == INFEASIBLE:
            bty = float(self.b @ uy)
            y = sc.sigma * sc.D * uy / (-bty)
            return np.full(n, np.nan), y, np.full(m, np.nan)
        if status == UNBOUNDED:
            cxt = float(self.c @ ux)
            x = sc.rho * sc.E * ux / (-cxt)
            s = sc.rho * vs / sc.D / (-cxt)
            return x, np.full(m, np.nan), s
        if tau > 0:
            x = sc.E * (ux / tau) / sc.sigma
            y = sc.D * (uy / tau) / sc.rho
            s = (vs / tau) / sc.D / sc.sigma
            return x, y, s
        return np.full(n, np.nan), np.full(m, np.nan), np.full(m, np.nan)

    # -- one iteration (e-SCS with over-relaxation) -------------------------
    def step(self, u, v, zx, k):
        st = self.st
        w = u + v
        if st.mode == "exact":
            tol = 0.0
        else:
            tol = (k + 1.0) ** (-st.cg_zeta_pow)
        ut, zx, it = self.lin.solve(w, zx, tol)
        ubar = st.alpha * ut + (1.0 - st.alpha) * u
        un = self.proj_C(ubar - v)
        vn = v - ubar + un
        return un, vn, zx, it


def solve(A, b, c, cone, settings: Optional[Settings] = None, start=None,
          record: int = 0) -> Result:
    """Run the method to a termination test or ``max_iters`` updates.

    ``start`` is None (cold start), ("xys", x, y, s) (Sect. 4.2 warm start)
    or ("q", q).  ``record`` > 0 keeps (u^k, v^k) for k = 0..record."""
    st = settings or Settings()
    P = Problem(A, b, c, cone, st)
    if start is None:
        u, v = P.cold_start()
    elif start[0] == "xys":
        u, v = P.warm_start(*start[1:])
    elif start[0] == "q":
        u, v = P.start_from_q(start[1])
    else:
        raise ValueError(start)
    zx = np.zeros(P.n)
    hist = []
    status = 0
    r = None
    k = 0
    while True:
        if record and k <= record:
            hist.append((u.copy(), v.copy()))
        if k % st.check_every == 0 or k == st.max_iters:
            status, r = P.decide(u, v)
            if status:
                break
        if k == st.max_iters:
            status = MAX_ITERS if u[-1] > 0 else INDETERMINATE
            break
        u, v, zx, _ = P.step(u, v, zx, k)
        k += 1
    x, y, s = P.outputs(u, v, status)
    info = Info(status=status, iters=k, res_pri=r["res_pri"], res_dual=r["res_dual"],
                gap=r["gap"], tau=float(u[-1]), kappa=float(v[-1]),
                cg_iters=P.lin.cg_iters_total, spmv_count=P.lin.spmv_count)
    if status in (SOLVED, MAX_ITERS) and u[-1] > 0:
        info.pobj = float(P.c0 @ x)
        info.dobj = float(-P.b0 @ y)
        info.obj = 0.5 * (info.pobj + info.dobj)
    return Result(x=x, y=y, s=s, info=info, u=u, v=v, history=hist)


def iterate(P: Problem, u, v, count: int, zx=None):
    """``count`` plain updates from (u, v) with no termination tests;
    returns the list [(u^0, v^0), ..., (u^count, v^count)]."""
    zx = np.zeros(P.n) if zx is None else zx
    out = [(u.copy(), v.copy())]
    for k in range(count):
        u, v, zx, _ = P.step(u, v, zx, k)
        out.append((u.copy(), v.copy()))
    return out


def naive_admm(P: Problem, u0, v0, count: int):
    """The five-sequence ADMM (e-SCS-naive) applied to (e-consensus), with
    lambda^0 = v^0 and mu^0 = u^0, exact projections and alpha = 1.  The
    projection onto {(u, v): Q u = v} is computed from its KKT system
    (e-kkt) with a dense solve.  Used only to check that the three-step
    form (e-SCS) reproduces it (Sect. 3.2, eliminating dual variables)."""
    Q = _dense_Q_scaled(P)
    N = Q.shape[0]
    IQQ = np.eye(N) + Q.T @ Q
    u, v = u0.copy(), v0.copy()
    lam, mu = v0.copy(), u0.copy()
    out = [(u.copy(), v.copy())]
    for _ in range(count):
        a = u + lam
        bb = v + mu
        # Pi onto {(ut, vt): vt = Q ut} of (a, bb): eliminating the
        # multiplier of (e-kkt) leaves (I + Q^T Q) ut = a + Q^T bb
        ut = np.linalg.solve(IQQ, a + Q.T @ bb)
        vt = Q @ ut
        u = P.proj_C(ut - lam)
        v = P.proj_Cstar(vt - mu)
        lam = lam - ut + u
        mu = mu - vt + v
        out.append((u.copy(), v.copy()))
    return out


def _dense_Q_scaled(P: Problem) -> np.ndarray:
    from .linsys import dense_Q
    return dense_Q(P.A, P.b, P.c)
