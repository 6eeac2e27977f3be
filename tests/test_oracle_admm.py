"""Pins for the oracle's linear system, iteration, termination and
certificates (CPU only).

Each check rests on something other than the oracle itself: a dense
library solve, a property the paper proves (Sect. 3.2 elimination of the
dual variables, Sect. 3.4 invariants and nonexpansivity, Sect. 3.2
homogeneity), a known optimal value by construction (Sect. 6 random cone
programs), brute-force vertex enumeration, or a constructed certificate.
"""

import itertools
import os

import numpy as np
import pytest
import scipy.sparse as sp

from datagen import draw_lp, draw_mixed, draw_socp, sample_sparse_pattern
from oracle import admm as AD
from oracle import cones as K
from oracle.instances import from_draw, make_infeasible, make_unbounded
from oracle.linsys import LinSys, dense_Q

HERE = os.path.dirname(os.path.abspath(__file__))


def tiny_socp(seed=0, n=6, m=14):
    return from_draw(draw_socp(seed, n=n, m=m, nonneg=4, soc_lo=3, soc_hi=5, density=0.5))


def tiny_mixed(seed=0):
    return from_draw(draw_mixed(seed, n=12, nonneg=3, n_soc=2, soc_lo=3, soc_hi=4,
                                n_psd=2, psd_lo=2, psd_hi=3, n_exp=2, n_dexp=1,
                                density=0.4, n_pow=2))


# ---------------------------------------------------------------------------
# linear system (Sect. 4.1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["exact", "cg"])
def test_smw_solve_equals_dense_solve(mode):
    inst = tiny_socp(1)
    A, b, c = inst.A, inst.b, inst.c
    lin = LinSys(A, b, c, mode=mode)
    m, n = A.shape
    Q = dense_Q(A, b, c)
    rng = np.random.default_rng(0)
    for _ in range(5):
        w = rng.standard_normal(n + m + 1)
        ut, _, _ = lin.solve(w, np.zeros(n), tol=1e-14)
        ref = np.linalg.solve(np.eye(n + m + 1) + Q, w)
        np.testing.assert_allclose(ut, ref, rtol=0, atol=1e-11 * np.linalg.norm(ref))


def test_Q_skew_and_inverse_norm():
    inst = tiny_socp(2)
    Q = dense_Q(inst.A, inst.b, inst.c)
    np.testing.assert_array_equal(Q, -Q.T)
    N = Q.shape[0]
    assert np.linalg.norm(np.linalg.inv(np.eye(N) + Q), 2) <= 1.0 + 1e-12


def test_cg_residual_is_full_residual():
    """With z_y and u_tau formed exactly, ||(Q+I) u_tilde - w|| equals the
    residual of the reduced CG system (the test of e-approx-proj-resid)."""
    inst = tiny_socp(3)
    A, b, c = inst.A, inst.b, inst.c
    m, n = A.shape
    lin = LinSys(A, b, c, mode="cg")
    Q = dense_Q(A, b, c)
    rng = np.random.default_rng(1)
    w = rng.standard_normal(n + m + 1)
    # stop CG early on purpose (loose tolerance)
    ut, zx, _ = lin.solve(w, np.zeros(n), tol=1e-1)
    rx = w[:n] - w[-1] * c
    ry = w[n:n + m] - w[-1] * b
    rhs = rx - A.T @ ry
    cg_res = np.linalg.norm(rhs - (zx + A.T @ (A @ zx)))
    full = np.linalg.norm((np.eye(n + m + 1) + Q) @ ut - w)
    assert abs(cg_res - full) <= 1e-12 * (1 + full)


# ---------------------------------------------------------------------------
# the iteration (Sect. 3)
# ---------------------------------------------------------------------------

def _problem(inst, **kw):
    st = AD.Settings(**kw)
    return AD.Problem(inst.A, inst.b, inst.c, inst.cone, st)


@pytest.mark.parametrize("make", [tiny_socp, tiny_mixed])
def test_naive_admm_equals_simplified(make):
    """Sect. 3.2: with lambda^0 = v^0 and mu^0 = u^0 the five-sequence ADMM
    produces the same (u^k, v^k) as the three-step form."""
    inst = make()
    P = _problem(inst, mode="exact", alpha=1.0)
    u0, v0 = P.cold_start()
    a = AD.iterate(P, u0, v0, 15)
    bseq = AD.naive_admm(P, u0, v0, 15)
    for (ua, va), (ub, vb) in zip(a, bseq):
        scale = 1 + np.linalg.norm(ua) + np.linalg.norm(va)
        assert np.linalg.norm(ua - ub) <= 1e-10 * scale
        assert np.linalg.norm(va - vb) <= 1e-10 * scale


@pytest.mark.parametrize("make", [tiny_socp, tiny_mixed])
def test_iterate_invariants(make):
    """(e-iter-guarantees): u^k in C, v^k in C^*, (u^k)^T v^k = 0 for k >= 1;
    and v_r stays 0 (the x-block of Pi_C is the identity)."""
    inst = make()
    P = _problem(inst, mode="cg", alpha=1.5)
    u, v = P.cold_start()
    seq = AD.iterate(P, u, v, 30)
    n, m = P.n, P.m
    for u, v in seq[1:]:
        nrm = 1 + np.linalg.norm(u) + np.linalg.norm(v)
        assert K.in_cone(u[n:n + m], inst.cone, dual=True, tol=1e-9)
        assert K.in_cone(v[n:n + m], inst.cone, dual=False, tol=1e-9)
        assert u[-1] >= 0 and v[-1] >= 0
        assert abs(u @ v) <= 1e-10 * nrm * nrm
        assert np.all(v[:n] == 0.0)


def test_homogeneity():
    """Sect. 3.2: scaling (u^0, v^0) by gamma scales every iterate by gamma
    (exact projection)."""
    inst = tiny_mixed(4)
    P = _problem(inst, mode="exact")
    u, v = P.cold_start()
    a = AD.iterate(P, u, v, 10)
    b = AD.iterate(P, 3.7 * u, 3.7 * v, 10)
    for (ua, va), (ub, vb) in zip(a, b):
        np.testing.assert_allclose(ub, 3.7 * ua, rtol=1e-9, atol=1e-11)
        np.testing.assert_allclose(vb, 3.7 * va, rtol=1e-9, atol=1e-11)


def test_nonexpansive_step():
    """(e-nonexpansive) and the appendix: one iteration phi is nonexpansive."""
    inst = tiny_mixed(5)
    P = _problem(inst, mode="exact", alpha=1.0)
    N = P.n + P.m + 1
    rng = np.random.default_rng(5)
    for _ in range(30):
        q1 = rng.standard_normal(N)
        q2 = rng.standard_normal(N)
        u1, v1 = P.start_from_q(q1)
        u2, v2 = P.start_from_q(q2)
        a, b, _, _ = P.step(u1, v1, np.zeros(P.n), 0)
        c, d, _, _ = P.step(u2, v2, np.zeros(P.n), 0)
        before = np.linalg.norm(np.concatenate([u1 - u2, v1 - v2]))
        after = np.linalg.norm(np.concatenate([a - c, b - d]))
        assert after <= before * (1 + 1e-12)


# ---------------------------------------------------------------------------
# end-to-end: known optimal values, vertex enumeration, certificates
# ---------------------------------------------------------------------------

def _kkt_residuals(inst, res):
    A, b, c = inst.A, inst.b, inst.c
    pri = np.linalg.norm(A @ res.x + res.s - b)
    dua = np.linalg.norm(A.T @ res.y + c)
    gap = abs(c @ res.x + b @ res.y)
    return pri, dua, gap


@pytest.mark.parametrize("kind,seed", [("lp", 0), ("lp", 1), ("socp", 0), ("mixed", 0),
                                       ("power", 0), ("power", 1)])
def test_known_optimal_value(kind, seed):
    if kind == "lp":
        inst = from_draw(draw_lp(seed))
    elif kind == "socp":
        inst = from_draw(draw_socp(seed, n=300, m=900, nonneg=150, density=2e-2))
    elif kind == "power":
        inst = from_draw(draw_mixed(seed, n=120, nonneg=40, n_soc=8, soc_lo=3, soc_hi=8,
                                    n_psd=0, n_exp=6, n_dexp=0, n_pow=40, density=4e-2))
    else:
        inst = from_draw(draw_mixed(seed, n=200, nonneg=60, n_soc=20, soc_lo=3, soc_hi=10,
                                    n_psd=4, psd_lo=3, psd_hi=6, n_exp=15, n_dexp=5,
                                    density=3e-2))
    st = AD.Settings(eps_pri=1e-6, eps_dual=1e-6, eps_gap=1e-6, max_iters=20000)
    r = AD.solve(inst.A, inst.b, inst.c, inst.cone, st)
    assert r.info.status == AD.SOLVED
    assert abs(r.info.obj - inst.pstar) <= 1e-4 * (1 + abs(inst.pstar))
    pri, dua, gap = _kkt_residuals(inst, r)
    assert pri <= 1e-6 * (1 + np.linalg.norm(inst.b)) * 1.0001
    assert dua <= 1e-6 * (1 + np.linalg.norm(inst.c)) * 1.0001
    # conic membership of the outputs (guaranteed by the iteration)
    assert K.in_cone(r.s, inst.cone, dual=False, tol=1e-8)
    assert K.in_cone(r.y, inst.cone, dual=True, tol=1e-8)


def _vertex_enumeration_lp(A, b, c):
    """min c^T x s.t. A x <= b (s = b - A x >= 0) by trying every n-row
    subset as the active set."""
    m, n = A.shape
    best = np.inf
    for rows in itertools.combinations(range(m), n):
        As = A[list(rows)]
        if abs(np.linalg.det(As)) < 1e-10:
            continue
        x = np.linalg.solve(As, b[list(rows)])
        if np.all(A @ x <= b + 1e-9):
            best = min(best, float(c @ x))
    return best


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_tiny_lp_vertex_enumeration(seed):
    rng = np.random.default_rng(100 + seed)
    n, m = 3, 8
    A = rng.standard_normal((m, n))
    x0 = rng.standard_normal(n)
    b = A @ x0 + rng.uniform(0.1, 1.0, m)          # strictly feasible
    y0 = rng.uniform(0.1, 1.0, m)
    c = -A.T @ y0                                  # dual feasible -> bounded
    ref = _vertex_enumeration_lp(A, b, c)
    st = AD.Settings(eps_pri=1e-7, eps_dual=1e-7, eps_gap=1e-7, max_iters=100000,
                     mode="exact")
    r = AD.solve(sp.csr_matrix(A), b, c, {"f": 0, "l": m, "q": [], "s": [], "ep": 0, "ed": 0}, st)
    assert r.info.status == AD.SOLVED
    assert abs(r.info.pobj - ref) <= 1e-5 * (1 + abs(ref))


def test_infeasible_certificate():
    inst = from_draw(draw_socp(11, n=20, m=60, nonneg=20, soc_lo=3, soc_hi=6, density=0.2))
    A, b, c, yc = make_infeasible(inst, np.random.default_rng(3))
    st = AD.Settings(max_iters=20000)
    r = AD.solve(A, b, c, inst.cone, st)
    assert r.info.status == AD.INFEASIBLE
    y = r.y
    assert abs(b @ y + 1.0) <= 1e-9                     # normalised: b^T y = -1
    assert np.linalg.norm(A.T @ y) <= 1e-4 * np.linalg.norm(b) * 1.01 + 1e-12
    assert K.in_cone(y, inst.cone, dual=True, tol=1e-8)


def test_unbounded_certificate():
    inst = from_draw(draw_socp(12, n=20, m=60, nonneg=20, soc_lo=3, soc_hi=6, density=0.2))
    A, b, c, xc = make_unbounded(inst, np.random.default_rng(4))
    st = AD.Settings(max_iters=20000)
    r = AD.solve(A, b, c, inst.cone, st)
    assert r.info.status == AD.UNBOUNDED
    x, s = r.x, r.s
    assert abs(c @ x + 1.0) <= 1e-9                     # c^T x = -1
    assert np.linalg.norm(A @ x + s) <= 1e-4 * np.linalg.norm(c) * 1.01 + 1e-12
    assert K.in_cone(s, inst.cone, dual=False, tol=1e-8)


def test_warm_start_from_solution_is_fast():
    """Sect. 4.2: restarting from the previous solution terminates almost
    immediately."""
    inst = from_draw(draw_socp(5, n=200, m=600, nonneg=100, density=3e-2))
    st = AD.Settings()
    cold = AD.solve(inst.A, inst.b, inst.c, inst.cone, st)
    assert cold.info.status == AD.SOLVED
    warm = AD.solve(inst.A, inst.b, inst.c, inst.cone, st,
                    start=("xys", cold.x, cold.y, cold.s))
    assert warm.info.status == AD.SOLVED
    assert warm.info.iters <= max(5, cold.info.iters // 10)


def test_scaling_does_not_change_the_answer():
    inst = from_draw(draw_socp(6, n=150, m=450, nonneg=80, density=4e-2))
    st_on = AD.Settings(eps_pri=1e-6, eps_dual=1e-6, eps_gap=1e-6, scale=True, max_iters=50000)
    st_off = AD.Settings(eps_pri=1e-6, eps_dual=1e-6, eps_gap=1e-6, scale=False, max_iters=50000)
    a = AD.solve(inst.A, inst.b, inst.c, inst.cone, st_on)
    b = AD.solve(inst.A, inst.b, inst.c, inst.cone, st_off)
    assert a.info.status == b.info.status == AD.SOLVED
    assert abs(a.info.obj - b.info.obj) <= 1e-4 * (1 + abs(inst.pstar))


def test_scaled_criteria_match_original():
    """Sect. 5: the scaled residual formulas give the original residuals."""
    inst = from_draw(draw_socp(7, n=60, m=180, nonneg=30, density=0.1))
    P = _problem(inst)
    u, v = P.cold_start()
    seq = AD.iterate(P, u, v, 20)
    u, v = seq[-1]
    r = P.residuals(u, v)
    x, y, s = P.outputs(u, v, AD.SOLVED)
    np.testing.assert_allclose(r["res_pri"], np.linalg.norm(inst.A @ x + s - inst.b), rtol=1e-10)
    np.testing.assert_allclose(r["res_dual"], np.linalg.norm(inst.A.T @ y + inst.c), rtol=1e-10)
    np.testing.assert_allclose(r["gap"], abs(inst.c @ x + inst.b @ y), rtol=1e-9, atol=1e-12)


def test_start_from_q_roundtrip():
    """q = u - v is the whole state: u = Pi_C(q), v = Pi_{C*}(-q) recovers
    every iterate (Moreau)."""
    inst = tiny_mixed(8)
    P = _problem(inst)
    u, v = P.cold_start()
    seq = AD.iterate(P, u, v, 8)
    for u, v in seq[1:]:
        uu, vv = P.start_from_q(u - v)
        np.testing.assert_allclose(uu, u, atol=1e-12)
        np.testing.assert_allclose(vv, v, atol=1e-12)


# ---------------------------------------------------------------------------
# the paper's printed numbers and the generator
# ---------------------------------------------------------------------------

def test_table5_multiply_accounting():
    """Table t-random-socps: total multiplies = iterations x (2 avg CG + 2),
    within the rounding of the printed average CG count (one decimal)."""
    rows = []
    with open(os.path.join(HERE, "golden", "table5_random_socp.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    assert len(rows) == 3
    for row in rows:
        iters, avg_cg, mults = int(row[4]), float(row[5]), int(row[6])
        lo = iters * (2 * (avg_cg - 0.05) + 2)
        hi = iters * (2 * (avg_cg + 0.05) + 2)
        assert lo <= mults <= hi


def test_generator_pattern_and_determinism():
    a = draw_socp(3, n=500, m=1500, nonneg=300, density=1e-2)
    b = draw_socp(3, n=500, m=1500, nonneg=300, density=1e-2)
    assert a.nnz == round(1e-2 * 500 * 1500)
    np.testing.assert_array_equal(a.indices, b.indices)
    np.testing.assert_array_equal(a.data, b.data)
    pos = a.indptr
    assert pos[-1] == a.nnz
    # sorted, distinct column indices within each row
    for i in range(0, a.m, 97):
        cols = a.indices[pos[i]:pos[i + 1]]
        assert np.all(np.diff(cols) > 0)
    assert sum(a.cone.q) + a.cone.l == a.m
    assert min(a.cone.q) >= 3
    rng = np.random.Generator(np.random.PCG64(0))
    p = sample_sparse_pattern(rng, 10, 10, 100)
    np.testing.assert_array_equal(p, np.arange(100))


def test_random_program_construction():
    """Sect. 6: s* in K, y* in K*, s*^T y* = 0, and (x*, s*, y*) is optimal
    with value c^T x* = -b^T y*."""
    inst = tiny_mixed(9)
    assert K.in_cone(inst.sstar, inst.cone, dual=False, tol=1e-10)
    assert K.in_cone(inst.ystar, inst.cone, dual=True, tol=1e-10)
    assert abs(inst.sstar @ inst.ystar) <= 1e-10
    np.testing.assert_allclose(inst.A @ inst.xstar + inst.sstar, inst.b)
    assert abs(inst.pstar + inst.b @ inst.ystar) <= 1e-9 * (1 + abs(inst.pstar))


def test_objective_within_weak_duality_bound():
    """At termination the mean objective lies within
    gap/2 + max(|r_p||y*|, |r_d||x*|) of p* (weak duality with the planted
    solution); the bound is what the full-size GPU tests assert."""
    for seed in range(3):
        inst = from_draw(draw_lp(seed))
        r = AD.solve(inst.A, inst.b, inst.c, inst.cone, AD.Settings())
        assert r.info.status == AD.SOLVED
        x, y, s = r.x, r.y, r.s
        A, b, c = inst.A, inst.b, inst.c
        pri = np.linalg.norm(A @ x + s - b)
        dua = np.linalg.norm(A.T @ y + c)
        gap = abs(c @ x + b @ y)
        bound = 0.5 * gap + max(pri * np.linalg.norm(inst.ystar), dua * np.linalg.norm(inst.xstar))
        obj = 0.5 * (c @ x - b @ y)
        assert abs(obj - inst.pstar) <= bound * (1 + 1e-9)
        # the bound is informative: a planted error of twice the bound fails it
        assert not abs(obj + 2 * bound + 1e-12 - inst.pstar) <= bound


def test_matrix_without_nonzeros():
    """A = 0: the scaling keeps rho positive (rbar = 1), and the outcomes are
    the ones the problem fixes: with c = 0 every x is optimal (objective 0,
    s = b); with c != 0 the free x makes c^T x unbounded below."""
    from datagen import ConeSpec
    m, n = 40, 10
    A = sp.csr_matrix((m, n))
    b = np.abs(np.random.default_rng(2).standard_normal(m))
    r = AD.solve(A, b, np.zeros(n), ConeSpec(l=m), AD.Settings())
    assert r.info.status == AD.SOLVED and abs(r.info.obj) <= 1e-6
    assert np.linalg.norm(r.s - b) <= 1e-4 * (1 + np.linalg.norm(b))
    c = np.array([1.0, -2.0, 0.5] + [0.0] * (n - 3))
    r = AD.solve(A, np.ones(m), c, ConeSpec(l=m), AD.Settings(max_iters=5000))
    assert r.info.status == AD.UNBOUNDED
    assert abs(c @ r.x + 1.0) <= 1e-9
