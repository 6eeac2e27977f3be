"""Termination with a certificate (Sect. 2.3 outcomes, Sect. 3.5 tests in
the scaled forms of Sect. 5) on the GPU, against the FP64 oracle, on
programs with a planted certificate (rank-one updates of a random program,
oracle/instances.py):

* primal infeasible: status INFEASIBLE, y normalised to b^T y = -1, y in K*,
  |A^T y| within the tolerance the test implies;
* dual infeasible (unbounded): status UNBOUNDED, c^T x = -1, s in K,
  |A x + s| within the tolerance;
* the first 50 iterates on such a program match the oracle's to 1e-9
  (near-exact projection mode), the same bar as for feasible programs;
* the batched solver reports the same certificates per program.
"""

import numpy as np
import pytest

from datagen import draw_socp
from gpu_common import log, rel
from oracle import admm as AD
from oracle import cones as OC
from oracle.instances import from_draw, make_infeasible, make_unbounded

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _infeasible(seed=11):
    inst = from_draw(draw_socp(seed, n=20, m=60, nonneg=20, soc_lo=3, soc_hi=6, density=0.2))
    A, b, c, _ = make_infeasible(inst, np.random.default_rng(3))
    return inst.cone, A, b, c


def _unbounded(seed=12):
    inst = from_draw(draw_socp(seed, n=20, m=60, nonneg=20, soc_lo=3, soc_hi=6, density=0.2))
    A, b, c, _ = make_unbounded(inst, np.random.default_rng(4))
    return inst.cone, A, b, c


def _check_infeasible(cone, A, b, y):
    assert abs(b @ y + 1.0) <= 1e-9
    assert np.linalg.norm(A.T @ y) <= 1e-4 * np.linalg.norm(b) * 1.01 + 1e-12
    assert OC.in_cone(y, cone, dual=True, tol=1e-8)


def _check_unbounded(cone, A, c, x, s):
    assert abs(c @ x + 1.0) <= 1e-9
    assert np.linalg.norm(A @ x + s) <= 1e-4 * np.linalg.norm(c) * 1.01 + 1e-12
    assert OC.in_cone(s, cone, dual=False, tol=1e-8)


@pytest.mark.parametrize("precision", [0, 1])
def test_infeasible_certificate_matches_oracle(precision):
    _torch()
    import paper_1312_3039_amd as hsd
    cone, A, b, c = _infeasible()
    S = hsd.Solver(A, b, c, cone.to_dict(), max_iters=20000, precision=precision)
    x, y, s, info = S.solve()
    ref = AD.solve(A, b, c, cone, AD.Settings(max_iters=20000))
    log(f"infeasible precision={precision}: gpu {info['status_name']} iters={info['iters']} | "
        f"oracle status={ref.info.status} iters={ref.info.iters}")
    assert info["status"] == ref.info.status == AD.INFEASIBLE
    _check_infeasible(cone, A, b, y.cpu().numpy())
    if precision == 0:
        assert abs(info["iters"] - ref.info.iters) <= max(5, 0.2 * ref.info.iters)


@pytest.mark.parametrize("precision", [0, 1])
def test_unbounded_certificate_matches_oracle(precision):
    _torch()
    import paper_1312_3039_amd as hsd
    cone, A, b, c = _unbounded()
    S = hsd.Solver(A, b, c, cone.to_dict(), max_iters=20000, precision=precision)
    x, y, s, info = S.solve()
    ref = AD.solve(A, b, c, cone, AD.Settings(max_iters=20000))
    log(f"unbounded precision={precision}: gpu {info['status_name']} iters={info['iters']} | "
        f"oracle status={ref.info.status} iters={ref.info.iters}")
    assert info["status"] == ref.info.status == AD.UNBOUNDED
    _check_unbounded(cone, A, c, x.cpu().numpy(), s.cpu().numpy())
    if precision == 0:
        assert abs(info["iters"] - ref.info.iters) <= max(5, 0.2 * ref.info.iters)


@pytest.mark.parametrize("make", [_infeasible, _unbounded])
def test_certificate_program_iterates_match_oracle(make):
    _torch()
    import paper_1312_3039_amd as hsd
    cone, A, b, c = make()
    K = 50
    S = hsd.Solver(A, b, c, cone.to_dict(), cg_tight_tol=1e-14, cg_max_iters=1000)
    U, V = (t.cpu().numpy() for t in S.iterate(K))
    P = AD.Problem(A, b, c, cone, AD.Settings(mode="exact"))
    u, v = P.cold_start()
    worst = 0.0
    for k, (uo, vo) in enumerate(AD.iterate(P, u, v, K)):
        e = rel(np.concatenate([U[k], V[k]]), np.concatenate([uo, vo]))
        worst = max(worst, e)
        assert e <= 1e-9, (k, e)
    log(f"{make.__name__} iterate parity: worst {worst:.3e}")


def test_batch_reports_certificates():
    _torch()
    import paper_1312_3039_amd as hsd
    feas = from_draw(draw_socp(13, n=20, m=60, nonneg=20, soc_lo=3, soc_hi=6, density=0.2))
    ci, Ai, bi, c_i = _infeasible()
    cu, Au, bu, c_u = _unbounded()
    progs = [(feas.A, feas.b, feas.c, feas.cone.to_dict()), (Ai, bi, c_i, ci.to_dict()),
             (Au, bu, c_u, cu.to_dict())]
    bs = hsd.BatchSolver(progs, max_iters=20000)
    x, y, s, infos = bs.solve()
    xs, ys, ss = bs.split(x.cpu().numpy(), "x"), bs.split(y.cpu().numpy(), "y"), bs.split(s.cpu().numpy(), "y")
    log("batch statuses " + ", ".join(i["status_name"] for i in infos))
    assert [i["status"] for i in infos] == [AD.SOLVED, AD.INFEASIBLE, AD.UNBOUNDED]
    _check_infeasible(ci, Ai, bi, ys[1])
    _check_unbounded(cu, Au, c_u, xs[2], ss[2])
