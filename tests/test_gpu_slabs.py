"""Column-slab sweeps (slab_cols > 0): every product with A and A^T visits
the columns in slabs and adds the per-slab row sums in LDS.  Only the
summation order inside a row changes, so the iterates must still match the
FP64 oracle to 1e-9 over 50 updates (near-exact projection mode), and full
solves must meet the same tests as without slabs.  Cases: many narrow
slabs with a ragged last slab, a single slab for A (slab wider than n)
beside two for A^T, one slab for both (streamed sweeps over the row-major
matrix, also with a team of one workgroup as in the batched kernel),
several LDS row chunks per workgroup (more than 2,048 rows per workgroup),
teams of one and several workgroups, FP32 mode."""

import numpy as np
import pytest

from datagen import draw_socp
from gpu_common import log, lp_c1, mixed_small, rel, socp_small
from oracle import admm as AD
from oracle import cones as OC
from oracle.instances import from_draw

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _iterate_parity(inst, K=50, **settings):
    import paper_1312_3039_amd as hsd
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), cg_tight_tol=1e-14,
                   cg_max_iters=1000, **settings)
    U, V = (t.cpu().numpy() for t in S.iterate(K))
    S.close()
    P = AD.Problem(inst.A, inst.b, inst.c, inst.cone, AD.Settings(mode="exact"))
    u, v = P.cold_start()
    worst = 0.0
    for k, (uo, vo) in enumerate(AD.iterate(P, u, v, K)):
        e = rel(np.concatenate([U[k], V[k]]), np.concatenate([uo, vo]))
        worst = max(worst, e)
        assert e <= 1e-9, (k, e)
    return worst


@pytest.mark.parametrize("make,slab,team", [(lp_c1, 16, 0), (lp_c1, 7, 1), (lp_c1, 200, 0),
                                            (lp_c1, 1000, 0), (socp_small, 1 << 30, 1),
                                            (socp_small, 64, 0), (socp_small, 100, 7),
                                            (mixed_small, 32, 0)])
def test_slab_iterates_match_oracle(make, slab, team):
    _torch()
    inst = make()
    log(f"slab iterate parity {make.__name__} slab_cols={slab} team={team}")
    worst = _iterate_parity(inst, slab_cols=slab, team_blocks=team)
    log(f"  worst relative iterate error {worst:.3e}")


def test_slab_row_chunks_iterates_match_oracle():
    """3,000 rows of A per workgroup: two LDS row chunks per slab sweep."""
    _torch()
    inst = from_draw(draw_socp(2, n=2000, m=6000, nonneg=1000, density=2e-3))
    log("slab iterate parity n=2000 m=6000 team=2 slab_cols=256")
    worst = _iterate_parity(inst, K=30, slab_cols=256, team_blocks=2)
    log(f"  worst relative iterate error {worst:.3e}")


@pytest.mark.parametrize("precision", [0, 1])
def test_slab_solve_matches_unslabbed(precision):
    _torch()
    import paper_1312_3039_amd as hsd
    inst = socp_small(4)
    out = []
    for slab in (-1, 50):
        S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), precision=precision,
                       slab_cols=slab)
        x, y, s, info = S.solve()
        out.append(((x.cpu().numpy(), y.cpu().numpy(), s.cpu().numpy()), info))
        S.close()
        log(f"  slab_cols={slab} precision={precision}: {info['status_name']} iters={info['iters']} "
            f"obj={info['obj']:.10g}")
    (sol, i0), (sol1, i1) = out
    assert i0["status"] == i1["status"] == 1
    assert abs(i0["iters"] - i1["iters"]) <= max(3, 0.05 * i0["iters"])
    assert abs(i0["obj"] - i1["obj"]) <= 1e-4 * (1 + abs(i0["obj"]))
    x, y, s = sol1
    assert np.linalg.norm(inst.A @ x + s - inst.b) <= 1.001e-4 * (1 + np.linalg.norm(inst.b))
    assert np.linalg.norm(inst.A.T @ y + inst.c) <= 1.001e-4 * (1 + np.linalg.norm(inst.c))
    assert OC.in_cone(s, inst.cone, dual=False, tol=1e-9)
    assert OC.in_cone(y, inst.cone, dual=True, tol=1e-9)
    assert i1["spmv_count"] == 2 * i1["iters"] + 2 * i1["cg_iters"]
