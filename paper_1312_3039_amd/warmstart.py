"""Learned warm start for a parametric family of cone programs.

The paper's warm start (Sect. 4.2) restarts from a previous solution:
u0 = (x*, y*, 1), v0 = (0, s*, 0).  For a family with fixed A, c and cone
and b(theta) = b0 + B theta, a network predicts that starting point from
theta instead.  It outputs t = (x, w, 1) with w = y - s (n + m + 1 values);
because y and s are a complementary pair of the cone (y in K^*, s in K,
y^T s = 0), Moreau's decomposition (Sect. 3.2, e-moreau) recovers both from
w: y = Pi_{K*}(w), s = Pi_K(-w).  The start is then the paper's
(x, y, s) warm start.

Everything runs on the GPU through the library: training data are solves of
the method itself (batched, all programs sharing A), the network is trained
and evaluated by the library's own kernels, and a prediction is used only if
its residuals at the start point are below those of the cold start; the
cold start is the fallback otherwise.  For a family whose programs end in
certificates, the prediction is a scaled iterate q = u - v, and the cold
start and the predicted start race for a few updates, the winner judged by
the termination tests' own quantities.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import MLP, BatchSolver, Solver, project_cone


def _torch():
    import torch
    return torch


@dataclass
class Family:
    """b(theta) = b0 + B theta with fixed A, c, cone."""

    A: object            # scipy CSR
    b0: np.ndarray
    c: np.ndarray
    cone: dict
    B: np.ndarray        # m x p

    @property
    def m(self):
        return self.A.shape[0]

    @property
    def n(self):
        return self.A.shape[1]

    def b(self, theta: np.ndarray) -> np.ndarray:
        return self.b0 + self.B @ theta

    def bs(self, thetas: np.ndarray) -> np.ndarray:
        return self.b0[None, :] + thetas @ self.B.T


def family_from_draw(pdraw) -> Family:
    """The random feasible base program of a datagen parametric draw, built
    with the library's projection for s* = Pi_K(z)."""
    import scipy.sparse as sp
    d = pdraw.base
    A = sp.csr_matrix((d.data, d.indices, d.indptr), shape=(d.m, d.n))
    cone = d.cone.to_dict()
    s = project_cone(cone, d.z, dual=False).cpu().numpy()
    y = s - d.z
    return Family(A=A, b0=A @ d.xstar + s, c=-(A.T @ y), cone=cone, B=pdraw.B)


def solve_family(fam: Family, thetas: np.ndarray, chunk: int = 2048, with_q: bool = False,
                 **settings):
    """Solve b(theta) for every row of thetas with the batched solver
    (programs share A).  Returns dict of x (N x n), y, s (N x m), status,
    iters, and the wall time; with_q adds q (N x (n+m+1)), the scaled
    iterate u - v each program stopped at (a solution or a certificate)."""
    torch = _torch()
    N = thetas.shape[0]
    xs, ys, ss, qs, st, it = [], [], [], [], [], []
    t0 = time.perf_counter()
    for a in range(0, N, chunk):
        th = thetas[a:a + chunk]
        bs = BatchSolver.shared(fam.A, fam.bs(th), fam.c, fam.cone, **settings)
        x, y, s, infos = bs.solve()
        k = th.shape[0]
        xs.append(x.reshape(k, fam.n))
        ys.append(y.reshape(k, fam.m))
        ss.append(s.reshape(k, fam.m))
        if with_q:
            # programs of one size: program i's iterate starts at i (n + m + 1)
            u, v = bs.state()
            qs.append((u - v).reshape(k, fam.n + fam.m + 1))
        st += [i["status"] for i in infos]
        it += [i["iters"] for i in infos]
        bs.close()
        del bs
    torch.cuda.synchronize()
    out = {"x": torch.cat(xs), "y": torch.cat(ys), "s": torch.cat(ss),
           "status": np.array(st), "iters": np.array(it), "seconds": time.perf_counter() - t0}
    if with_q:
        out["q"] = torch.cat(qs)
    return out


def targets(sol) -> object:
    """t = (x, y - s, 1) per program (device, float64)."""
    torch = _torch()
    one = torch.ones((sol["x"].shape[0], 1), dtype=torch.float64, device=sol["x"].device)
    return torch.cat([sol["x"], sol["y"] - sol["s"], one], dim=1)


def _he_init(rng, ni, h, no):
    """He-normal weights and zero biases, packed as the network expects."""
    W1 = rng.standard_normal((h, ni)) * np.sqrt(2.0 / ni)
    W2 = rng.standard_normal((h, h)) * np.sqrt(2.0 / h)
    W3 = rng.standard_normal((no, h)) * np.sqrt(2.0 / h)
    return np.concatenate([W1.ravel(), np.zeros(h), W2.ravel(), np.zeros(h), W3.ravel(),
                           np.zeros(no)]).astype(np.float32)


@dataclass
class WarmStarter:
    """The network theta -> t = (x, w, 1) and its use as a start point."""

    fam: Family
    hidden: int = 512
    batch: int = 256
    seed: int = 0
    net: object = None
    mu: object = None
    sd: object = None
    losses: list = field(default_factory=list)

    def fit(self, thetas: np.ndarray, T, epochs: int = 30, lr: float = 1e-3):
        """Adam on the mean squared error of standardised targets, minibatches
        drawn without replacement each epoch."""
        torch = _torch()
        dev = T.device
        N, no = T.shape
        ni = thetas.shape[1]
        self.mu = T.mean(dim=0)
        self.sd = T.std(dim=0).clamp_min(1e-6)
        Tn = ((T - self.mu) / self.sd).to(torch.float32)
        X = torch.as_tensor(thetas, dtype=torch.float32, device=dev)
        rng = np.random.default_rng(self.seed)
        self.net = MLP(ni, self.hidden, no, self.batch, device=dev)
        self.net.set_params(_he_init(rng, ni, self.hidden, no))
        nb = N // self.batch
        for _ in range(epochs):
            perm = torch.as_tensor(rng.permutation(N), device=dev)
            tot = torch.zeros((), dtype=torch.float32, device=dev)
            for k in range(nb):
                idx = perm[k * self.batch:(k + 1) * self.batch]
                tot += self.net.train_step(X[idx], Tn[idx], lr)[0]
            self.losses.append(float(tot) / nb)
        return self.losses

    def predict(self, thetas: np.ndarray):
        """Network output mapped back to t = (x, w, 1) (device, float64)."""
        torch = _torch()
        X = torch.as_tensor(thetas, dtype=torch.float32, device=self.mu.device)
        out = []
        for a in range(0, X.shape[0], self.batch):
            out.append(self.net.forward(X[a:a + self.batch]).to(torch.float64))
        return torch.cat(out) * self.sd + self.mu

    def start_point(self, t):
        """(x, y, s) from one predicted t by the Moreau pair of w = y - s."""
        n, m = self.fam.n, self.fam.m
        w = t[n:n + m].contiguous()
        y = project_cone(self.fam.cone, w, dual=True)
        s = project_cone(self.fam.cone, -w, dual=False)
        return t[:n].contiguous(), y, s


def evaluate(fam: Family, ws: WarmStarter, thetas: np.ndarray, **settings):
    """Cold vs warm solves of b(theta) for each row of thetas on one set-up
    handle (same A, c; b replaced per program, Sect. 4.2).  The predicted
    start is used only when its primal and dual residuals (relative to
    1 + |b| and 1 + |c|) are both below the cold start's (|b| and |c| at
    x = y = s = 0); otherwise the cold start is used (fallback)."""
    torch = _torch()
    S = Solver(fam.A, fam.b(thetas[0]), fam.c, fam.cone, **settings)
    max_iters = S.settings.max_iters
    t0 = time.perf_counter()
    T = ws.predict(thetas)
    torch.cuda.synchronize()
    infer_ms = 1e3 * (time.perf_counter() - t0) / thetas.shape[0]
    nc = float(np.linalg.norm(fam.c))
    rows = []
    for k in range(thetas.shape[0]):
        b = fam.b(thetas[k])
        S.update_b(b)
        nb = float(np.linalg.norm(b))
        _, _, _, cold = S.solve()
        t1 = time.perf_counter()
        x, y, s = ws.start_point(T[k])
        S.update_settings(max_iters=0)
        S.warm_start(x, y, s)
        _, _, _, probe = S.solve()
        S.update_settings(max_iters=max_iters)
        torch.cuda.synchronize()
        prep_ms = 1e3 * (time.perf_counter() - t1)
        use_warm = (probe["res_pri"] / (1 + nb) < nb / (1 + nb)
                    and probe["res_dual"] / (1 + nc) < nc / (1 + nc))
        if use_warm:
            S.warm_start(x, y, s)
        _, _, _, warm = S.solve()
        rows.append({
            "cold_status": cold["status"], "cold_iters": cold["iters"],
            "cold_ms": cold["solve_ms"],
            "warm_status": warm["status"], "warm_iters": warm["iters"],
            "warm_ms": warm["solve_ms"] + prep_ms + infer_ms, "used_warm": bool(use_warm),
            "cold_obj": cold["obj"], "warm_obj": warm["obj"],
        })
    S.close()
    return rows


def test_score(info: dict, nb: float, nc: float, st) -> float:
    """Distance of a run's last iterate from passing a termination test
    (Sect. 3.5), as the smallest ratio of a test's quantity to its threshold
    (a value <= 1 passes): the optimality test (primal and dual residuals
    against eps (1 + |b|), eps (1 + |c|)) and the two certificate tests."""
    opt = max(info["res_pri"] / (st.eps_pri * (1.0 + nb)), info["res_dual"] / (st.eps_dual * (1.0 + nc)))
    return min(opt, info["res_infeas"] / st.eps_infeas, info["res_unbdd"] / st.eps_unbdd)


def _stopped_at_limit(info: dict, limit: int) -> bool:
    """True when a run ended only because it reached its update limit: the
    limit status is MAX_ITERS with tau > 0 and INDETERMINATE with tau = 0
    (as in the iterates of an infeasible program, whose tau goes to 0)."""
    return info["iters"] >= limit and info["status"] in (2, 5) and np.isfinite(info["tau"])


def evaluate_q(fam: Family, ws: WarmStarter, thetas: np.ndarray, probe: int = 20, **settings):
    """Cold vs warm solves of b(theta) for each row of thetas, the network
    trained on the scaled iterates q = u - v that training programs stopped
    at (for a family whose programs end in certificates).

    The warm path judges the prediction by the method's own residuals: the
    cold start and the start from the Moreau pair of the predicted q
    (hsd_start_from_q) each run ``probe`` updates, the one whose iterate is
    nearer to passing a termination test (``test_score``: the optimality
    and certificate tests of Sect. 3.5) continues from its saved state
    (hsd_get_state / hsd_set_state, so no work of the winner is repeated),
    and the other is dropped.  A probe that already stops ends the path.
    The warm path's iterations count both probes; its time is the wall time
    of the whole path including inference."""
    torch = _torch()
    S = Solver(fam.A, fam.b(thetas[0]), fam.c, fam.cone, **settings)
    st = S.settings
    max_iters = st.max_iters
    t0 = time.perf_counter()
    Q = ws.predict(thetas)
    torch.cuda.synchronize()
    infer_ms = 1e3 * (time.perf_counter() - t0) / thetas.shape[0]
    nc = float(np.linalg.norm(fam.c))
    rows = []
    for k in range(thetas.shape[0]):
        b = fam.b(thetas[k])
        nb = float(np.linalg.norm(b))
        S.update_b(b)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, _, _, cold = S.solve()
        cold_wall = 1e3 * (time.perf_counter() - t1)
        t1 = time.perf_counter()
        S.update_settings(max_iters=probe)
        _, _, _, pc = S.solve()
        used_warm = False
        spent = 0
        if not _stopped_at_limit(pc, probe):
            final = pc
        else:
            sc = S.get_state()
            S.start_from_q(Q[k].contiguous())
            _, _, _, pw = S.solve()
            if not _stopped_at_limit(pw, probe):
                final, used_warm = pw, True
            else:
                used_warm = test_score(pw, nb, nc, st) < test_score(pc, nb, nc, st)
                keep = S.get_state() if used_warm else sc
                spent = probe  # the dropped probe
                S.update_settings(max_iters=max_iters)
                S.set_state(keep)
                _, _, _, final = S.solve()
        S.update_settings(max_iters=max_iters)
        torch.cuda.synchronize()
        warm_wall = 1e3 * (time.perf_counter() - t1) + infer_ms
        rows.append({"cold_status": cold["status"], "cold_iters": cold["iters"],
                     "cold_ms": cold_wall, "warm_status": final["status"],
                     "warm_iters": final["iters"] + spent, "warm_ms": warm_wall,
                     "used_warm": bool(used_warm)})
    S.close()
    return rows
