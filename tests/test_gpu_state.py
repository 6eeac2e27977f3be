"""GPU tests of the solver state across calls (Sect. 4.2 repeated solves,
Sect. 3.2 homogeneity) and of the termination quantities at a fixed
iterate, through the C ABI:

* a run interrupted after k1 updates and resumed from its saved state
  (hsd_get_state / hsd_set_state with the carried products) continues bit
  for bit as the uninterrupted run, on the same handle and on a fresh one,
  in FP64 and FP32, with the default CG tolerance schedule and in
  near-exact mode; without the carried products it agrees to rounding;
* homogeneity: the iterates from (2u, 2v, 2z_x) are twice those from
  (u, v, z_x) (the embedding is a cone, Sect. 3.2);
* hsd_update_bc gives the same scaling and solve as a fresh setup;
* the residuals, gap and objectives the kernel reports at update 50 equal
  the oracle's at the same iterate (near-exact mode, 1e-9 relative); in
  FP32 mode the difference is stated.
"""

import numpy as np
import pytest

from datagen import draw_socp
from gpu_common import log, mixed_small, rel, socp_small
from oracle import admm as AD
from oracle import cones as OC
from oracle.instances import from_draw

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _hsd():
    import paper_1312_3039_amd as hsd
    return hsd


def _same(a, b):
    torch = _torch()
    return bool(torch.equal(a, b))


# eps below reach: the runs stop at the iteration limit
NEVER = dict(eps_pri=1e-14, eps_dual=1e-14, eps_gap=1e-14, eps_unbdd=1e-14, eps_infeas=1e-14)


@pytest.mark.parametrize("precision,tight,team", [(0, 0.0, 0), (0, 1e-14, 7), (1, 0.0, 0), (0, 0.0, 1)])
def test_resume_is_bit_identical(precision, tight, team):
    _torch()
    hsd = _hsd()
    inst = socp_small(4)
    K, k1 = 60, 23
    kw = dict(precision=precision, cg_tight_tol=tight, team_blocks=team, cg_max_iters=500, **NEVER)
    cone = inst.cone.to_dict()
    log(f"resume precision={precision} tight={tight} team={team}")
    full = hsd.Solver(inst.A, inst.b, inst.c, cone, max_iters=K, **kw)
    _, _, _, i_full = full.solve()
    st_full = full.get_state()
    full.close()
    assert i_full["iters"] == K and st_full["k"] == K
    part = hsd.Solver(inst.A, inst.b, inst.c, cone, max_iters=k1, **kw)
    _, _, _, i1 = part.solve()
    assert i1["status"] == 2 and i1["iters"] == k1
    st1 = part.get_state()
    assert st1["k"] == k1
    # resumed on a fresh handle
    fresh = hsd.Solver(inst.A, inst.b, inst.c, cone, max_iters=K, **kw)
    fresh.set_state(st1)
    _, _, _, i2 = fresh.solve()
    st2 = fresh.get_state()
    fresh.close()
    # resumed on the same handle
    part.update_settings(max_iters=K)
    part.set_state(st1)
    _, _, _, i3 = part.solve()
    st3 = part.get_state()
    part.close()
    for st, info in ((st2, i2), (st3, i3)):
        assert st["k"] == K and info["iters"] == K
        for key in ("u", "v", "zx", "carry"):
            assert _same(st[key], st_full[key]), key
        for key in ("res_pri", "res_dual", "gap", "pobj", "dobj", "tau", "kappa"):
            assert info[key] == i_full[key], key
    # the carried products are those of the state: A_hat z_x and A_hat u_x
    if precision == 0:
        P = AD.Problem(inst.A, inst.b, inst.c, inst.cone, AD.Settings())
        n = inst.A.shape[1]
        u = st_full["u"].cpu().numpy()
        zx = st_full["zx"].cpu().numpy()
        cr = st_full["carry"].cpu().numpy()
        m = inst.A.shape[0]
        assert rel(cr[:m], P.A @ zx) <= 1e-10
        assert rel(cr[m:], P.A @ u[:n]) <= 1e-10


def test_resume_without_carry_agrees_to_rounding():
    _torch()
    hsd = _hsd()
    inst = mixed_small(3)
    cone = inst.cone.to_dict()
    kw = dict(cg_tight_tol=1e-14, cg_max_iters=500, **NEVER)
    log("resume without the carried products")
    full = hsd.Solver(inst.A, inst.b, inst.c, cone, max_iters=50, **kw)
    full.solve()
    st_full = full.get_state(carry=False)
    full.close()
    part = hsd.Solver(inst.A, inst.b, inst.c, cone, max_iters=20, **kw)
    part.solve()
    st1 = part.get_state(carry=False)
    part.update_settings(max_iters=50)
    part.set_state(st1, carry=False)
    part.solve()
    st2 = part.get_state(carry=False)
    part.close()
    uv_full = np.concatenate([st_full["u"].cpu().numpy(), st_full["v"].cpu().numpy()])
    uv = np.concatenate([st2["u"].cpu().numpy(), st2["v"].cpu().numpy()])
    e = rel(uv, uv_full)
    log(f"  relative difference {e:.2e}")
    # Both runs are near-exact trajectories of the method; they differ only
    # in how the products of the restart point are formed (a product
    # instead of the carried recurrences), so they are held to the bar of
    # near-exact iterate parity with the oracle.
    assert e <= 1e-9


def test_homogeneity_of_the_iteration():
    """Sect. 3.2: the embedding's solution set is a cone and one update of
    the method is positively homogeneous, so from (2u, 2v) with the CG start
    2 z_x the iterates are twice those from (u, v, z_x).  Near-exact mode:
    the CG tolerance is relative, hence homogeneous too."""
    _torch()
    hsd = _hsd()
    inst = mixed_small(5)
    cone = inst.cone.to_dict()
    S = hsd.Solver(inst.A, inst.b, inst.c, cone, cg_tight_tol=1e-14, cg_max_iters=500,
                   max_iters=15, **NEVER)
    S.solve()
    st = S.get_state(carry=False)
    S.set_state(st, carry=False)
    U1, V1 = S.iterate(20)
    st2 = {k: (2.0 * v if k != "k" and v is not None else v) for k, v in st.items()}
    S.set_state(st2, carry=False)
    U2, V2 = S.iterate(20)
    S.close()
    e = rel(np.concatenate([U2.cpu().numpy(), V2.cpu().numpy()]),
            2.0 * np.concatenate([U1.cpu().numpy(), V1.cpu().numpy()]))
    log(f"homogeneity: relative difference {e:.2e}")
    assert e <= 1e-12


def test_update_bc_matches_fresh_setup():
    """Sect. 4.2 repeated solves: the same A with a new planted solution
    (new z, x*) gives new b and c; replacing both on a set-up handle gives
    the scaling and the solve of a fresh setup."""
    _torch()
    hsd = _hsd()
    inst = socp_small(6)
    A = inst.A
    m, n = A.shape
    rng = np.random.default_rng(66)
    z = rng.standard_normal(m)
    s2 = OC.proj_cone(z, inst.cone)
    y2 = s2 - z
    x2 = rng.standard_normal(n)
    b2 = A @ x2 + s2
    c2 = -(A.T @ y2)
    cone = inst.cone.to_dict()
    log("update_bc vs fresh setup")
    S = hsd.Solver(A, inst.b, inst.c, cone)
    S.solve()
    S.update_bc(b2, c2)
    _, _, _, i1 = S.solve()
    D1, E1, sig1, rho1 = S.scaling()
    S.close()
    F = hsd.Solver(A, b2, c2, cone)
    _, _, _, i2 = F.solve()
    D2, E2, sig2, rho2 = F.scaling()
    F.close()
    assert _same(D1, D2) and _same(E1, E2)
    assert sig1 == sig2 and rho1 == rho2
    assert i1["status"] == i2["status"] == 1
    assert i1["iters"] == i2["iters"]
    assert abs(i1["obj"] - i2["obj"]) <= 1e-12 * (1 + abs(i2["obj"]))
    assert abs(i1["obj"] - float(c2 @ x2)) <= 1e-3 * (1 + abs(float(c2 @ x2)))


@pytest.mark.parametrize("make", [socp_small, mixed_small])
def test_reported_tests_match_oracle_at_update_50(make):
    """The termination quantities (Sect. 3.5, scaled form of Sect. 5) that
    the kernel reports after 50 updates, in near-exact mode, against the
    oracle's at its iterate 50 (dense Cholesky projections)."""
    _torch()
    hsd = _hsd()
    inst = make(7)
    log(f"tests at update 50: {make.__name__}")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), cg_tight_tol=1e-14,
                   cg_max_iters=1000, max_iters=50, **NEVER)
    _, _, _, g = S.solve()
    S.close()
    ref = AD.solve(inst.A, inst.b, inst.c, inst.cone,
                   AD.Settings(mode="exact", max_iters=50, eps_pri=1e-14, eps_dual=1e-14,
                               eps_gap=1e-14, eps_unbdd=1e-14, eps_infeas=1e-14))
    o = ref.info
    assert g["status"] == o.status == 2 and g["iters"] == o.iters == 50
    for key, ov in (("res_pri", o.res_pri), ("res_dual", o.res_dual), ("gap", o.gap),
                    ("tau", o.tau), ("kappa", o.kappa)):
        e = abs(g[key] - ov) / max(abs(ov), 1e-300)
        log(f"  {key}: gpu {g[key]:.12e} oracle {ov:.12e} rel {e:.1e}")
        assert e <= 1e-9, key
    # objectives: the oracle reports c^T x and -b^T y of the unscaled point
    assert abs(g["pobj"] - o.pobj) <= 1e-9 * max(1.0, abs(o.pobj))
    assert abs(g["dobj"] - o.dobj) <= 1e-9 * max(1.0, abs(o.dobj))


def test_fp32_reported_tests_against_fp64_oracle():
    """FP32 mode: SpMV and CG in FP32; the residuals and the gap are still
    formed in FP64 from FP64 products (A u_x is gathered with the FP64
    values at every check).  After 50 updates with the default CG schedule
    they are compared with the FP64 oracle's at the same update: the
    difference comes from the FP32 CG solutions and is stated."""
    _torch()
    hsd = _hsd()
    inst = from_draw(draw_socp(8, n=2000, m=6000, nonneg=1000, density=2e-3))
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), precision=1, max_iters=50, **NEVER)
    _, _, _, g = S.solve()
    S.close()
    ref = AD.solve(inst.A, inst.b, inst.c, inst.cone,
                   AD.Settings(max_iters=50, eps_pri=1e-14, eps_dual=1e-14, eps_gap=1e-14,
                               eps_unbdd=1e-14, eps_infeas=1e-14))
    o = ref.info
    errs = {}
    for key, ov in (("res_pri", o.res_pri), ("res_dual", o.res_dual), ("gap", o.gap),
                    ("pobj", o.pobj), ("dobj", o.dobj)):
        errs[key] = abs(g[key] - ov) / max(abs(ov), 1e-300)
    log("  FP32 vs FP64 oracle at update 50: " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
    assert g["iters"] == 50
    for key in ("res_pri", "res_dual", "pobj", "dobj"):
        assert errs[key] <= 1e-2, key
