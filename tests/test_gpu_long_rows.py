"""GPU tests of the long-row pass of the row-group sweeps (a row of A or of
A^T much longer than the others is taken by a whole workgroup), through the
C ABI, against the FP64 oracle:

* 50-update iterate parity (near-exact projections, element by element) on
  a random SOCP with two dense rows and two dense columns added, for teams
  of 1, 5 and the automatic size, in FP64;
* full solves of the same program in FP64 and FP32: status, iterations and
  objective against the oracle's, KKT residuals recomputed with SciPy;
* the launch reports the long-row kernels for this program and not for the
  plain one.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from datagen import draw_socp
from gpu_common import log
from oracle import admm as AD
from oracle import cones as OC
from oracle.instances import Instance

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dense_lines_program(seed=3):
    """The random SOCP recipe (Sect. 6) at n = 300, m = 900 with rows 7 and
    460 and columns 3 and 250 of A made dense (N(0,1) entries), and the
    planted solution rebuilt on that A."""
    d = draw_socp(seed, n=300, m=900, nonneg=450, soc_lo=3, soc_hi=10, density=0.02)
    A = sp.csr_matrix((d.data, d.indices, d.indptr), shape=(d.m, d.n)).tolil()
    rng = np.random.default_rng(1000 + seed)
    for r in (7, 460):
        A[r, :] = rng.standard_normal(d.n)
    for c in (3, 250):
        A[:, c] = rng.standard_normal((d.m, 1))
    A = sp.csr_matrix(A)
    A.sort_indices()
    s = OC.proj_cone(d.z, d.cone, dual=False)
    y = s - d.z
    b = A @ d.xstar + s
    c = -(A.T @ y)
    return Instance(A=A, b=b, c=c, cone=d.cone, xstar=d.xstar, ystar=y, sstar=s,
                    pstar=float(c @ d.xstar))


@pytest.mark.parametrize("team", [1, 5, 0])
def test_long_rows_iterate_parity(team):
    _torch()
    import paper_1312_3039_amd as hsd
    inst = _dense_lines_program()
    K = 50
    log(f"long rows: iterate parity team={team}")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), cg_tight_tol=1e-14,
                   cg_max_iters=1000, team_blocks=team)
    lw = S.launch()
    log(f"  launch {lw}")
    assert lw["long_rows"] == 1
    assert lw["max_row_a"] == 300 and lw["max_row_at"] == 900
    U, V = (t.cpu().numpy() for t in S.iterate(K))
    S.close()
    P = AD.Problem(inst.A, inst.b, inst.c, inst.cone, AD.Settings(mode="exact"))
    u, v = P.cold_start()
    worst = 0.0
    for k, (uo, vo) in enumerate(AD.iterate(P, u, v, K)):
        o = np.concatenate([uo, vo])
        g = np.concatenate([U[k], V[k]])
        scale = np.abs(o) + np.linalg.norm(o) / np.sqrt(o.size)
        e = float(np.max(np.abs(g - o) / scale))
        worst = max(worst, e)
        assert e <= 1e-9, (k, e)
    log(f"  worst elementwise error {worst:.2e}")


@pytest.mark.parametrize("precision", [0, 1])
def test_long_rows_solve_matches_oracle(precision):
    _torch()
    import paper_1312_3039_amd as hsd
    inst = _dense_lines_program()
    log(f"long rows: solve precision={precision}")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), precision=precision)
    x, y, s, info = S.solve()
    S.close()
    x, y, s = (t.cpu().numpy() for t in (x, y, s))
    ref = AD.solve(inst.A, inst.b, inst.c, inst.cone, AD.Settings()).info
    d = abs(info["obj"] - ref.obj) / max(1.0, abs(ref.obj))
    log(f"  gpu {info['status_name']} iters {info['iters']} obj {info['obj']:.10g} | oracle iters "
        f"{ref.iters} obj {ref.obj:.10g} (rel diff {d:.1e})")
    assert info["status"] == ref.status == 1
    assert abs(info["iters"] - ref.iters) <= 2
    assert d <= 1e-4
    A, b, c = inst.A, inst.b, inst.c
    assert np.linalg.norm(A @ x + s - b) <= 1e-4 * (1 + np.linalg.norm(b)) * 1.001
    assert np.linalg.norm(A.T @ y + c) <= 1e-4 * (1 + np.linalg.norm(c)) * 1.001


def test_plain_program_keeps_the_default_kernel():
    _torch()
    import paper_1312_3039_amd as hsd
    d = draw_socp(3, n=300, m=900, nonneg=450, soc_lo=3, soc_hi=10, density=0.02)
    from oracle.instances import from_draw
    inst = from_draw(d)
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict())
    lw = S.launch()
    S.close()
    assert lw["long_rows"] == 0
