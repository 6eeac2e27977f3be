"""GPU checks at the workloads' full sizes, where a full oracle solve would
be slow: properties that hold at any size.  The outputs' KKT residuals are
recomputed here with SciPy from A, b, c (Sect. 3.5 criteria at eps = 1e-4),
s and y are checked for cone membership, and the objective is compared with
the known optimal value p* = c^T x* of the random program (Sect. 6).

The stopping criteria bound residuals, not the objective error, so the
objective is held to the bound that weak duality gives with the planted
solution (x*, y*, s*): with r_p = Ax + s - b, r_d = A^T y + c, s in K and
y in K*,
    c^T x - p*  = s^T y* - r_p^T y*  >= -|r_p| |y*|,
    -b^T y - p* = -s*^T y - x*^T r_d <=  |r_d| |x*|,
and the two differ by the gap c^T x + b^T y, so the mean objective
(c^T x - b^T y)/2 lies within gap/2 + max(|r_p||y*|, |r_d||x*|) of p*.
FP32 mode (SpMV and CG in FP32, the rest in FP64) is compared with FP64 on
the same program: its objective difference is stated and bounded.
"""

import numpy as np
import pytest

from datagen import draw_mixed, draw_socp
from gpu_common import log
from oracle import cones as OC
from oracle.instances import from_draw

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _check_solution(inst, x, y, s, info, eps=1e-4):
    A, b, c = inst.A, inst.b, inst.c
    assert info["status"] == 1, info["status_name"]
    pri = np.linalg.norm(A @ x + s - b)
    dua = np.linalg.norm(A.T @ y + c)
    gap = abs(c @ x + b @ y)
    assert pri <= eps * (1 + np.linalg.norm(b)) * 1.001
    assert dua <= eps * (1 + np.linalg.norm(c)) * 1.001
    assert gap <= eps * (1 + abs(c @ x) + abs(b @ y)) * 1.001
    assert OC.in_cone(s, inst.cone, dual=False, tol=1e-8)
    assert OC.in_cone(y, inst.cone, dual=True, tol=1e-8)
    obj = 0.5 * (c @ x - b @ y)
    assert abs(obj - info["obj"]) <= 1e-9 * (1 + abs(obj))
    bound = 0.5 * gap + max(pri * np.linalg.norm(inst.ystar), dua * np.linalg.norm(inst.xstar))
    err = abs(obj - inst.pstar)
    log(f"  |obj - p*| = {err:.3e}, weak-duality bound {bound:.3e}, "
        f"relative {err / max(1.0, abs(inst.pstar)):.2e}")
    assert err <= bound * 1.001 + 1e-12 * (1 + abs(inst.pstar))
    return err / max(1.0, abs(inst.pstar))


@pytest.mark.parametrize("precision", [0, 1])
def test_socp_10k_full_size(precision):
    _torch()
    import paper_1312_3039_amd as hsd
    inst = from_draw(draw_socp(0))
    log(f"SOCP n=10000 m=30000 precision={precision}")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), precision=precision)
    x, y, s, info = S.solve()
    err = _check_solution(inst, *(t.cpu().numpy() for t in (x, y, s)), info)
    log(f"  iters={info['iters']} obj rel err vs p* = {err:.2e}")


def test_socp_fp32_vs_fp64():
    _torch()
    import paper_1312_3039_amd as hsd
    inst = from_draw(draw_socp(1))
    r64 = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), precision=0).solve()[3]
    r32 = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), precision=1).solve()[3]
    d = abs(r32["obj"] - r64["obj"]) / max(1.0, abs(r64["obj"]))
    log(f"FP32 vs FP64 objective: rel diff {d:.2e}; iters {r32['iters']} vs {r64['iters']}")
    assert r32["status"] == r64["status"] == 1
    assert d <= 1e-3


@pytest.mark.parametrize("precision", [1, 0])
def test_mixed_cones_full_size(precision):
    _torch()
    import paper_1312_3039_amd as hsd
    inst = from_draw(draw_mixed(0))
    m, n = inst.A.shape
    log(f"mixed cones n={n} m={m} (60 PSD, 500 exp) precision={precision}")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), precision=precision)
    x, y, s, info = S.solve()
    err = _check_solution(inst, *(t.cpu().numpy() for t in (x, y, s)), info)
    log(f"  iters={info['iters']} kernel {info['kernel_ms']:.1f} ms, obj rel err vs p* = {err:.2e}")
