"""GPU parity tests: the HIP path through the C ABI against the FP64 oracle
on the same seeded inputs.

* cone projections, elementwise;
* the scaling D, E, sigma, rho;
* iterate parity: 50 updates from the cold start in near-exact projection
  mode (GPU CG to 1e-14 relative residual, oracle dense Cholesky), relative
  error of (u^k, v^k) at most 1e-9 for every k (the bound follows from the
  nonexpansivity of one iteration, appendix of the paper: per-step
  differences of ~1e-14 add up rather than grow);
* full solves at eps = 1e-4: same status, objective within 1e-4 relative
  of the oracle's and of p*.
"""

import numpy as np
import pytest

from datagen import draw_mixed
from gpu_common import log, lp_c1, mixed_small, rel, socp_small
from oracle.instances import from_draw
from oracle import admm as AD
from oracle import cones as OC

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _hsd():
    import paper_1312_3039_amd as hsd
    return hsd


MIXED_CONE = {"f": 3, "l": 40, "q": [1, 2, 3, 5, 17, 40, 64, 100], "s": [1, 2, 3, 5, 7, 16, 17, 33, 40, 64],
              "ep": 30, "ed": 11}


@pytest.mark.parametrize("dual", [False, True])
def test_project_cone_matches_oracle(dual):
    _torch()
    hsd = _hsd()
    m = OC.cone_dim(MIXED_CONE)
    rng = np.random.default_rng(7 + dual)
    for scale in [0.1, 1.0, 10.0]:
        x = rng.standard_normal(m) * scale
        log(f"project_cone dual={dual} m={m} scale={scale}")
        got = hsd.project_cone(MIXED_CONE, x, dual=dual).cpu().numpy()
        ref = OC.proj_cone(x, MIXED_CONE, dual=dual)
        for kind, a, L, d in OC.cone_blocks(MIXED_CONE):
            g, r = got[a:a + L], ref[a:a + L]
            tol = 1e-9 if kind in ("exp", "dexp") else 1e-12
            assert np.linalg.norm(g - r) <= tol * (1 + np.linalg.norm(x[a:a + L])), (kind, a, L)


def test_project_cone_rejects_bad_cone():
    _torch()
    hsd = _hsd()
    with pytest.raises(Exception):
        hsd.project_cone({"f": 0, "l": 3, "q": [], "s": [], "ep": 0, "ed": 0}, np.zeros(4))


@pytest.mark.parametrize("make", [lp_c1, socp_small, mixed_small])
def test_scaling_matches_oracle(make):
    _torch()
    hsd = _hsd()
    inst = make()
    log(f"scaling {make.__name__} m={inst.A.shape[0]} n={inst.A.shape[1]}")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict())
    D, E, sig, rho = S.scaling()
    P = AD.Problem(inst.A, inst.b, inst.c, inst.cone, AD.Settings())
    assert rel(D.cpu().numpy(), P.sc.D) <= 1e-12
    assert rel(E.cpu().numpy(), P.sc.E) <= 1e-12
    assert abs(sig - P.sc.sigma) <= 1e-12 * P.sc.sigma
    assert abs(rho - P.sc.rho) <= 1e-12 * P.sc.rho


def socp_rows_beyond_lds():
    """3,000 rows on one workgroup: the own-row stage (56 bytes per row)
    does not fit in LDS, so the fused update reads its rows from global
    memory throughout."""
    return socp_small(0, n=1000, m=3000, nonneg=1500, density=4e-3)


def mixed_psd_large():
    """Three PSD cones of sides 38, 58 and 60 (warm-started projections whose
    padded sides are not multiples of the 16 x 16 product tiles)."""
    return from_draw(draw_mixed(3, n=300, nonneg=100, n_soc=4, soc_lo=3, soc_hi=10, n_psd=3,
                                psd_lo=33, psd_hi=64, n_exp=8, density=2e-2))


@pytest.mark.parametrize("make,alpha,team", [(lp_c1, 1.5, 0), (lp_c1, 1.0, 1), (socp_small, 1.5, 0),
                                             (socp_small, 1.5, 7), (mixed_small, 1.5, 0),
                                             (mixed_psd_large, 1.5, 0),
                                             (socp_rows_beyond_lds, 1.5, 1)])
def test_iterate_parity_fp64(make, alpha, team):
    _torch()
    hsd = _hsd()
    inst = make()
    K = 50
    log(f"iterate parity {make.__name__} alpha={alpha} team={team}")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), alpha=alpha,
                   cg_tight_tol=1e-14, cg_max_iters=1000, team_blocks=team)
    U, V = S.iterate(K)
    U = U.cpu().numpy()
    V = V.cpu().numpy()
    P = AD.Problem(inst.A, inst.b, inst.c, inst.cone, AD.Settings(mode="exact", alpha=alpha))
    u, v = P.cold_start()
    seq = AD.iterate(P, u, v, K)
    worst = 0.0
    for k, (uo, vo) in enumerate(seq):
        e = rel(np.concatenate([U[k], V[k]]), np.concatenate([uo, vo]))
        worst = max(worst, e)
        assert e <= 1e-9, (k, e)
    log(f"  worst relative iterate error {worst:.3e}")


@pytest.mark.parametrize("make", [lp_c1, socp_small, mixed_small])
def test_solve_matches_oracle(make):
    _torch()
    hsd = _hsd()
    inst = make()
    log(f"solve {make.__name__}")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict())
    x, y, s, info = S.solve()
    ref = AD.solve(inst.A, inst.b, inst.c, inst.cone, AD.Settings())
    log(f"  gpu: {info['status_name']} iters={info['iters']} obj={info['obj']:.8g} "
        f"cg={info['cg_iters']} | oracle iters={ref.info.iters} obj={ref.info.obj:.8g} "
        f"p*={inst.pstar:.8g}")
    assert info["status"] == 1 and ref.info.status == 1
    assert abs(info["obj"] - ref.info.obj) <= 1e-4 * (1 + abs(ref.info.obj))
    assert abs(info["obj"] - inst.pstar) <= 1e-3 * (1 + abs(inst.pstar))
    x, y, s = (t.cpu().numpy() for t in (x, y, s))
    A, b, c = inst.A, inst.b, inst.c
    assert np.linalg.norm(A @ x + s - b) <= 1e-4 * (1 + np.linalg.norm(b)) * 1.001
    assert np.linalg.norm(A.T @ y + c) <= 1e-4 * (1 + np.linalg.norm(c)) * 1.001
    assert OC.in_cone(s, inst.cone, dual=False, tol=1e-9)
    assert OC.in_cone(y, inst.cone, dual=True, tol=1e-9)
    # iteration counts agree closely (CG stopping ties may differ)
    assert abs(info["iters"] - ref.info.iters) <= max(5, 0.2 * ref.info.iters)
    # multiply accounting of the paper's Table 5: 2 + 2 CG per iteration
    assert info["spmv_count"] == 2 * info["iters"] + 2 * info["cg_iters"]


def test_update_b_matches_fresh_setup():
    """Sect. 4.2 repeated solves: replacing b on a set-up handle gives the same
    solve as setting up from scratch with that b."""
    _torch()
    hsd = _hsd()
    inst = socp_small(3)
    rng = np.random.default_rng(9)
    # b2 = A (x* + dx) + s*: (x* + dx, s*) stays primal feasible and y* stays
    # dual optimal, so the new program is solvable (p* shifts by c^T dx)
    b2 = inst.b + inst.A @ (0.1 * rng.standard_normal(inst.A.shape[1]))
    log("update_b vs fresh setup")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict())
    S.solve()
    S.update_b(b2)
    _, _, _, i1 = S.solve()
    F = hsd.Solver(inst.A, b2, inst.c, inst.cone.to_dict())
    _, _, _, i2 = F.solve()
    assert i1["status"] == i2["status"] == 1
    assert i1["iters"] == i2["iters"]
    assert abs(i1["obj"] - i2["obj"]) <= 1e-12 * (1 + abs(i2["obj"]))


def test_solve_with_zero_iterations_reports_start_residuals():
    _torch()
    hsd = _hsd()
    inst = lp_c1(2)
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict())
    S.update_settings(max_iters=0)
    _, _, _, info = S.solve()
    assert info["iters"] == 0 and info["status"] == 2
    # at the cold start x = y = s = 0 and tau = 1: the residuals are |b| and |c|
    assert abs(info["res_pri"] - np.linalg.norm(inst.b)) <= 1e-9 * np.linalg.norm(inst.b)
    assert abs(info["res_dual"] - np.linalg.norm(inst.c)) <= 1e-9 * np.linalg.norm(inst.c)
