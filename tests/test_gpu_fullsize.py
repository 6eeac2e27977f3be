"""GPU checks at the workloads' full sizes, in the launch shapes the
benchmark times.

Against the FP64 oracle (its own full solve of the same seeded program):
same status, iteration counts within 2, objective within 1e-4 relative of
the oracle's objective -- the default SOCP (n = 10^4, m = 3*10^4) in FP64
and FP32, automatic and tuned launch shape; the mixed-cone program in both
precisions; statuses and objectives of sampled programs of the 4,096-program
batch, including the programs that reach the iteration limit.  On the
default SOCP in the tuned shape the first 50 iterates are also compared
with the oracle's element by element (near-exact projections).

Beside that, at every size, properties that hold at any size: the outputs'
KKT residuals recomputed here with SciPy from A, b, c (Sect. 3.5 criteria
at eps = 1e-4), s in K and y in K*, and the objective within the bound that
weak duality gives with the planted solution (x*, y*, s*): with
r_p = Ax + s - b, r_d = A^T y + c, s in K and y in K*,
    c^T x - p*  = s^T y* - r_p^T y*  >= -|r_p| |y*|,
    -b^T y - p* = -s*^T y - x*^T r_d <=  |r_d| |x*|,
and the two differ by the gap c^T x + b^T y, so the mean objective
(c^T x - b^T y)/2 lies within gap/2 + max(|r_p||y*|, |r_d||x*|) of p*.
The large SOCP (10^8 nonzeros), beyond the oracle's reach, is also solved
at eps = 1e-5 and its objective held to 1e-4 relative of the exact optimum
p* of the planted program.
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


def _check_solution(inst, x, y, s, info, eps=1e-4, quiet=False):
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
    if not quiet:
        log(f"  |obj - p*| = {err:.3e}, weak-duality bound {bound:.3e}, "
            f"relative {err / max(1.0, abs(inst.pstar)):.2e}")
    assert err <= bound * 1.001 + 1e-12 * (1 + abs(inst.pstar))
    return err / max(1.0, abs(inst.pstar))


def _bench_shape(m, n, nnz):
    """The launch shape the benchmark times on this device (the tuning
    table's entry), or the automatic shape."""
    from paper_1312_3039_amd import autotune
    hit = autotune.lookup("single", m, n, nnz)
    return dict(hit["settings"]) if hit else {}


_ORACLE = {}


def _oracle_solve(key, inst):
    """The oracle's solve of a program (cached for the module)."""
    from oracle import admm as AD
    if key not in _ORACLE:
        log(f"  oracle solve of {key} ...")
        _ORACLE[key] = AD.solve(inst.A, inst.b, inst.c, inst.cone, AD.Settings()).info
        o = _ORACLE[key]
        log(f"  oracle {key}: status {o.status} iters {o.iters} obj {o.obj:.12g}")
    return _ORACLE[key]


def _vs_oracle(info, o, iters_tol=2):
    """Status equal, iterations within iters_tol, objective within 1e-4
    relative of the oracle's objective; returns the relative difference."""
    d = abs(info["obj"] - o.obj) / max(1.0, abs(o.obj))
    log(f"  gpu: {info['status_name']} iters {info['iters']} obj {info['obj']:.12g} | "
        f"oracle iters {o.iters}; objective rel diff {d:.2e}")
    assert info["status"] == o.status
    assert abs(info["iters"] - o.iters) <= iters_tol
    assert d <= 1e-4
    return d


@pytest.mark.parametrize("precision,tuned", [(0, False), (1, False), (0, True), (1, True)])
def test_socp_10k_full_size(precision, tuned):
    """tuned: the launch shape bench.py times (the shipped tuning table)."""
    _torch()
    import paper_1312_3039_amd as hsd
    inst = from_draw(draw_socp(0))
    shape = _bench_shape(*inst.A.shape, inst.A.nnz) if tuned else {}
    log(f"SOCP n=10000 m=30000 precision={precision} shape={shape or 'automatic'}")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), precision=precision, **shape)
    x, y, s, info = S.solve()
    S.close()
    err = _check_solution(inst, *(t.cpu().numpy() for t in (x, y, s)), info)
    log(f"  iters={info['iters']} obj rel err vs p* = {err:.2e}")
    _vs_oracle(info, _oracle_solve("socp10k-seed0", inst))


def test_socp_10k_iterates_in_bench_shape():
    """The first 50 iterates of the default SOCP in the launch shape the
    benchmark times (team, lanes, LDS matrix slices of the tuning table),
    near-exact projections, against the oracle's (dense Cholesky of
    I + A^T A), element by element:
    |g_i - o_i| <= 1e-9 (|o_i| + |o| / sqrt(N))."""
    _torch()
    import paper_1312_3039_amd as hsd
    from oracle import admm as AD
    inst = from_draw(draw_socp(0))
    shape = _bench_shape(*inst.A.shape, inst.A.nnz)
    K = 50
    log(f"SOCP n=10000 iterate check, shape {shape or 'automatic'}")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), cg_tight_tol=1e-14,
                   cg_max_iters=1000, **shape)
    U, V = (t.cpu().numpy() for t in S.iterate(K))
    S.close()
    log("  oracle: dense Cholesky of I + A^T A (n = 10,000) ...")
    P = AD.Problem(inst.A, inst.b, inst.c, inst.cone, AD.Settings(mode="exact"))
    u, v = P.cold_start()
    seq = AD.iterate(P, u, v, K)
    worst = 0.0
    for k, (uo, vo) in enumerate(seq):
        o = np.concatenate([uo, vo])
        g = np.concatenate([U[k], V[k]])
        scale = np.abs(o) + np.linalg.norm(o) / np.sqrt(o.size)
        e = float(np.max(np.abs(g - o) / scale))
        worst = max(worst, e)
        assert e <= 1e-9, (k, e)
    log(f"  worst elementwise error {worst:.2e}")


def test_socp_fp32_vs_fp64_oracle():
    """FP32 mode on another seed against the FP64 oracle's solve."""
    _torch()
    import paper_1312_3039_amd as hsd
    inst = from_draw(draw_socp(1))
    log("SOCP seed 1, FP32 mode vs the FP64 oracle")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), precision=1)
    r32 = S.solve()[3]
    S.close()
    _vs_oracle(r32, _oracle_solve("socp10k-seed1", inst))


@pytest.mark.parametrize("precision", [1, 0])
def test_mixed_cones_full_size(precision):
    _torch()
    import paper_1312_3039_amd as hsd
    inst = from_draw(draw_mixed(0))
    m, n = inst.A.shape
    log(f"mixed cones n={n} m={m} (60 PSD, 500 exp) precision={precision}")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), precision=precision)
    x, y, s, info = S.solve()
    S.close()
    err = _check_solution(inst, *(t.cpu().numpy() for t in (x, y, s)), info)
    log(f"  iters={info['iters']} kernel {info['kernel_ms']:.1f} ms, obj rel err vs p* = {err:.2e}")
    _vs_oracle(info, _oracle_solve("mixed-seed0", inst))


def test_batch_4096_full_size():
    """The batched workload at its full size (4,096 programs, n ~ U[20,400],
    m = 3n) in the launch shape the benchmark times: every program's status
    agrees with the oracle's on a sample; every solved program meets the
    eps = 1e-4 tests on its own data, has s in K and y in K*, and its
    objective lies within the weak-duality bound of its p*."""
    _torch()
    import paper_1312_3039_amd as hsd
    from paper_1312_3039_amd import autotune
    from datagen import draw_batch_member
    from oracle import admm as AD
    insts = [from_draw(draw_batch_member(10_000 + i)) for i in range(4096)]
    probs = [(p.A, p.b, p.c, p.cone.to_dict()) for p in insts]
    m = sum(p.A.shape[0] for p in insts)
    n = sum(p.A.shape[1] for p in insts)
    nnz = sum(p.A.nnz for p in insts)
    hit = autotune.lookup("batch", m // 4096, n // 4096, nnz // 4096)
    shape = dict(hit["settings"]) if hit else {}
    log(f"batch 4096 programs, {nnz} nnz, shape {shape or 'automatic'}")
    bs = hsd.BatchSolver(probs, **shape)
    x, y, s, infos = bs.solve()
    xs, ys, ss = bs.split(x.cpu().numpy(), "x"), bs.split(y.cpu().numpy(), "y"), bs.split(s.cpu().numpy(), "y")
    solved = 0
    for i, (p, info) in enumerate(zip(insts, infos)):
        if info["status"] != 1:
            assert info["status"] == 2, (i, info["status_name"])  # iteration limit only
            continue
        solved += 1
        _check_solution(p, xs[i], ys[i], ss[i], info, quiet=True)
    bs.close()
    log(f"  {solved} of 4096 solved")
    assert solved >= 4000
    # sampled programs (every 512th) and the programs the oracle's sampled
    # runs found at the iteration limit: status, iterations, objective
    for i in list(range(0, 4096, 512)) + [s - 10_000 for s in (10752, 10840, 11576, 11648, 12640)]:
        ref = AD.solve(insts[i].A, insts[i].b, insts[i].c, insts[i].cone, AD.Settings()).info
        log(f"  program {i} (seed {10_000 + i}): gpu {infos[i]['status_name']} {infos[i]['iters']} | "
            f"oracle status {ref.status} {ref.iters}")
        assert ref.status == infos[i]["status"], (i, ref.status, infos[i]["status"])
        if ref.status == 1:
            assert abs(infos[i]["iters"] - ref.iters) <= 2, i
            assert abs(infos[i]["obj"] - ref.obj) <= 1e-4 * max(1.0, abs(ref.obj)), i


def test_large_socp_full_size():
    """The large workload at its full size (n = 10^6, m = 3*10^6, 10^8
    nonzeros, 1.2 GB of FP64 CSR per copy of A) in the launch shape the
    benchmark times (the automatic one: streamed column-slab sweeps): the
    outputs meet the eps = 1e-4 tests recomputed with SciPy, s in K, y in
    K*, and the objective lies within the weak-duality bound of p*."""
    _torch()
    import paper_1312_3039_amd as hsd
    n, m, nnz = 1_000_000, 3_000_000, 100_000_000
    inst = from_draw(draw_socp(0, n=n, m=m, nonneg=500_000, soc_lo=3, soc_hi=50, density=nnz / (m * n)))
    log(f"large SOCP n={n} m={m} nnz={inst.A.nnz}")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict())
    x, y, s, info = S.solve()
    log(f"  {info['status_name']} in {info['iters']} updates, kernel {info['kernel_ms']:.0f} ms")
    _check_solution(inst, *(t.cpu().numpy() for t in (x, y, s)), info)
    # tighter: eps = 1e-5 puts the objective within 1e-4 of the exact p*
    S.update_settings(eps_pri=1e-5, eps_dual=1e-5, eps_gap=1e-5)
    x, y, s, info = S.solve()
    S.close()
    d = abs(info["obj"] - inst.pstar) / abs(inst.pstar)
    log(f"  eps=1e-5: {info['status_name']} in {info['iters']} updates, |obj - p*|/|p*| = {d:.2e}")
    _check_solution(inst, *(t.cpu().numpy() for t in (x, y, s)), info, eps=1e-5)
    assert d <= 1e-4
