"""CPU checks of the structured program generators (Sect. 6.2-6.5): each
standard form (A, b, c, K) encodes its model.  For a point x built by hand
from the model's variables (with every epigraph variable at its tight
value), s = b - A x lies in K and c^T x equals the model's objective
evaluated directly -- so a dropped row, a wrong sign or a misplaced block
fails.  The oracle's solve of a small instance then matches the family's
optimality conditions."""

import math

import numpy as np
import pytest

from datagen import structured as ST
from oracle import admm as AD
from oracle import cones as OC


def _s(prog, x):
    return prog.b - prog.csr() @ x


def test_lasso_form_encodes_the_model():
    prog = ST.lasso(1, p=60, q=15)
    p = prog.meta["p"]
    rng = np.random.default_rng(0)
    z = rng.standard_normal(p)
    fr, fc, fv = prog.meta["F"]
    r = np.bincount(fr, weights=fv * z[fc], minlength=prog.meta["q"]) - prog.meta["g"]
    x = np.r_[z, np.abs(z), r @ r]
    s = _s(prog, x)
    assert OC.in_cone(s, prog.cone, tol=1e-10)
    # the SOC is tight at w = |F z - g|^2
    soc = s[2 * p:]
    assert abs(soc[0] - np.linalg.norm(soc[1:])) <= 1e-9 * soc[0]
    assert abs(prog.c @ x - ST.lasso_objective(prog, x)) <= 1e-10 * (1 + abs(prog.c @ x))
    # mu = 0.1 |F^T g|_inf
    Ftg = np.bincount(fc, weights=fv * prog.meta["g"][fr], minlength=p)
    assert prog.meta["mu"] == pytest.approx(0.1 * np.abs(Ftg).max(), rel=1e-14)


def test_portfolio_form_encodes_the_model():
    prog = ST.portfolio(2, p=80, q=6)
    p, q = prog.meta["p"], prog.meta["q"]
    rng = np.random.default_rng(1)
    z = rng.uniform(size=p)
    z /= z.sum()
    fr, fc, fv = prog.meta["F"]
    u = math.sqrt(float(prog.meta["D"] @ (z * z)))
    ftz = np.bincount(fc, weights=fv * z[fr], minlength=q)
    v = float(np.linalg.norm(ftz))
    x = np.r_[z, u * u, v * v, u, v]
    s = _s(prog, x)
    assert OC.in_cone(s, prog.cone, tol=1e-10)
    assert abs(s[0]) <= 1e-14                       # budget row
    assert abs(prog.c @ x + ST.portfolio_objective(prog, x)) <= 1e-10
    # a point that breaks the budget is not in K
    assert not OC.in_cone(_s(prog, np.r_[2 * z, u * u, v * v, u, v]), prog.cone, tol=1e-10)


def test_rpca_form_encodes_the_model():
    prog = ST.rpca(3, p=7, rank=2)
    p = prog.meta["p"]
    d = 2 * p
    L, S = prog.meta["Lhat"], prog.meta["Shat"]
    Uu, sig, Vt = np.linalg.svd(L)
    X = np.block([[Uu @ np.diag(sig) @ Uu.T, L], [L.T, Vt.T @ np.diag(sig) @ Vt]])
    sv = OC.svec(X)
    x = np.r_[sv, S.ravel(order="F"), np.abs(S).ravel(order="F")]
    s = _s(prog, x)
    assert OC.in_cone(s, prog.cone, tol=1e-9)
    assert np.max(np.abs(s[:p * p])) <= 1e-12       # L + S = M
    # (1/2) Tr X = nuclear norm of L at this X
    assert abs(prog.c @ x - sig.sum()) <= 1e-10 * sig.sum()
    assert np.allclose(ST.rpca_low_rank(prog, x), L, atol=1e-12)
    assert prog.meta["mu"] == pytest.approx(np.abs(S).sum(), rel=1e-14)
    assert prog.cone.s == [d]


def test_logreg_form_encodes_the_model():
    prog = ST.logreg(4, p=8, q=50)
    p, q = prog.meta["p"], prog.meta["q"]
    rng = np.random.default_rng(2)
    w = rng.standard_normal(p)
    zr, zc, zv = prog.meta["Z"]
    a = prog.meta["y"] * np.bincount(zr, weights=zv * w[zc], minlength=q)
    t = np.logaddexp(0.0, a)
    x = np.r_[w, np.abs(w), t, np.exp(a - t), np.exp(-t)]
    s = _s(prog, x)
    assert OC.in_cone(s, prog.cone, tol=1e-9)
    assert np.max(np.abs(s[2 * p:2 * p + q])) <= 1e-12  # u + v = 1 is tight
    assert abs(prog.c @ x - ST.logreg_objective(prog, x)) <= 1e-10 * (1 + abs(prog.c @ x))


def test_oracle_lasso_meets_its_optimality_conditions():
    """Lasso optimality (subgradient): |F^T (g - F z)|_i <= mu, with equality
    and the sign of z_i on the support; checked to the eps = 1e-6 solve's
    accuracy."""
    prog = ST.lasso(5, p=60, q=15)
    st = AD.Settings(eps_pri=1e-6, eps_dual=1e-6, eps_gap=1e-6, max_iters=50_000)
    r = AD.solve(prog.csr(), prog.b, prog.c, prog.cone, st)
    assert r.info.status == 1
    p, mu = prog.meta["p"], prog.meta["mu"]
    z = r.x[:p]
    fr, fc, fv = prog.meta["F"]
    res = prog.meta["g"] - np.bincount(fr, weights=fv * z[fc], minlength=prog.meta["q"])
    grad = np.bincount(fc, weights=fv * res[fr], minlength=p)
    assert np.max(np.abs(grad)) <= mu * (1 + 1e-2)
    on = np.abs(z) > 1e-3 * np.abs(z).max()
    assert np.all(np.abs(grad[on] - mu * np.sign(z[on])) <= 1e-2 * mu)
    assert abs(r.info.obj - ST.lasso_objective(prog, r.x)) <= 1e-5 * (1 + abs(r.info.obj))
