"""GPU tests of the direct subspace projection (Sect. 4.1, factorization
caching; settings linsys = 1): the setup forms G = I + A_hat^T A_hat,
factors and inverts it once, and every update applies G^{-1} exactly.
Against the oracle's exact projections (dense Cholesky of the same G):

* 50-update iterates element by element to 1e-9 (LP, SOCP, mixed cones;
  teams of 1, 7 and the automatic size);
* full solves: status, iterations (within 2) and objective (1e-4 relative,
  1e-9 in practice), KKT residuals recomputed with SciPy;
* the default SOCP (n = 10^4) at full size against the oracle's exact-mode
  solve;
* the setting is rejected in FP32 mode.
"""

import numpy as np
import pytest

from datagen import draw_socp
from gpu_common import log, lp_c1, mixed_small, socp_small
from oracle import admm as AD
from oracle.instances import from_draw

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _elementwise(U, V, seq):
    worst = 0.0
    for k, (uo, vo) in enumerate(seq):
        o = np.concatenate([uo, vo])
        g = np.concatenate([U[k], V[k]])
        scale = np.abs(o) + np.linalg.norm(o) / np.sqrt(o.size)
        e = float(np.max(np.abs(g - o) / scale))
        worst = max(worst, e)
        assert e <= 1e-9, (k, e)
    return worst


@pytest.mark.parametrize("make", [lp_c1, socp_small, mixed_small])
@pytest.mark.parametrize("team", [1, 7, 0])
def test_direct_iterates_match_exact_oracle(make, team):
    _torch()
    import paper_1312_3039_amd as hsd
    inst = make()
    K = 50
    log(f"direct iterates {make.__name__} team={team}")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), linsys=1, team_blocks=team)
    U, V = (t.cpu().numpy() for t in S.iterate(K))
    S.close()
    P = AD.Problem(inst.A, inst.b, inst.c, inst.cone, AD.Settings(mode="exact"))
    u, v = P.cold_start()
    worst = _elementwise(U, V, AD.iterate(P, u, v, K))
    log(f"  worst elementwise error {worst:.2e}")


@pytest.mark.parametrize("make", [lp_c1, socp_small, mixed_small])
def test_direct_solve_matches_exact_oracle(make):
    _torch()
    import paper_1312_3039_amd as hsd
    inst = make()
    log(f"direct solve {make.__name__}")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), linsys=1)
    x, y, s, info = S.solve()
    S.close()
    ref = AD.solve(inst.A, inst.b, inst.c, inst.cone, AD.Settings(mode="exact")).info
    d = abs(info["obj"] - ref.obj) / max(1.0, abs(ref.obj))
    log(f"  gpu {info['status_name']} iters {info['iters']} cg {info['cg_iters']} obj {info['obj']:.12g} | "
        f"oracle iters {ref.iters} obj {ref.obj:.12g} (rel diff {d:.1e})")
    assert info["status"] == ref.status == 1
    assert abs(info["iters"] - ref.iters) <= 2
    assert d <= 1e-4
    assert info["cg_iters"] == 0 and info["spmv_count"] == 2 * info["iters"]
    x, y, s = (t.cpu().numpy() for t in (x, y, s))
    A, b, c = inst.A, inst.b, inst.c
    assert np.linalg.norm(A @ x + s - b) <= 1e-4 * (1 + np.linalg.norm(b)) * 1.001
    assert np.linalg.norm(A.T @ y + c) <= 1e-4 * (1 + np.linalg.norm(c)) * 1.001


def test_direct_default_socp_full_size():
    """The default SOCP (n = 10^4, m = 3*10^4, 300k nonzeros): the GPU's
    direct solve against the oracle's solve with exact projections."""
    _torch()
    import paper_1312_3039_amd as hsd
    inst = from_draw(draw_socp(0))
    log("direct solve of the default SOCP")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), linsys=1)
    _, _, _, info = S.solve()
    S.close()
    log(f"  gpu {info['status_name']} iters {info['iters']} setup {info['setup_ms']:.1f} ms "
        f"solve {info['solve_ms']:.1f} ms; oracle exact-mode solve ...")
    ref = AD.solve(inst.A, inst.b, inst.c, inst.cone, AD.Settings(mode="exact")).info
    d = abs(info["obj"] - ref.obj) / max(1.0, abs(ref.obj))
    log(f"  oracle iters {ref.iters} obj {ref.obj:.12g}; rel diff {d:.1e}")
    assert info["status"] == ref.status == 1
    assert abs(info["iters"] - ref.iters) <= 2
    assert d <= 1e-4


def test_direct_rejects_fp32():
    _torch()
    import paper_1312_3039_amd as hsd
    from paper_1312_3039_amd import _lib
    inst = lp_c1()
    with pytest.raises(_lib.HsdError):
        hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), linsys=1, precision=1)
