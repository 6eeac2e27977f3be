"""GPU tests of the batched solver (one persistent, graph-captured launch
for many uneven programs) against the oracle and the single-program path."""

import numpy as np
import pytest
import scipy.sparse as sp

from datagen import draw_batch_member
from gpu_common import log, weak_duality_bound
from oracle import admm as AD
from oracle import cones as OC
from oracle.instances import from_draw

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def members(count, seed0=10_000, n_lo=20, n_hi=60):
    return [from_draw(draw_batch_member(seed0 + i, n_lo=n_lo, n_hi=n_hi)) for i in range(count)]


def problems(insts):
    return [(p.A, p.b, p.c, p.cone.to_dict()) for p in insts]


@pytest.mark.parametrize("stream", [False, True])
def test_batch_matches_oracle_and_solo(stream):
    """stream selects the block-streamed sweeps (slab_cols > 0)."""
    _torch()
    import paper_1312_3039_amd as hsd
    insts = members(24)
    log(f"batch of {len(insts)} programs, n in [20, 60], streamed sweeps {stream}")
    extra = dict(slab_cols=1 << 30) if stream else {}
    bs = hsd.BatchSolver(problems(insts), max_iters=4000, **extra)
    x, y, s, infos = bs.solve()
    xs, ys, ss = bs.split(x.cpu().numpy(), "x"), bs.split(y.cpu().numpy(), "y"), bs.split(s.cpu().numpy(), "y")
    solved = 0
    for i, (p, info) in enumerate(zip(insts, infos)):
        ref = AD.solve(p.A, p.b, p.c, p.cone, AD.Settings(max_iters=4000))
        # some members of this family need more than 4000 iterations; both
        # sides must then agree that they did
        assert info["status"] == ref.info.status, (i, info["status_name"], ref.info.status)
        if ref.info.status != 1:
            continue
        solved += 1
        # both objectives within their weak-duality bounds of p*
        obj, bound = weak_duality_bound(p, xs[i], ys[i], ss[i])
        assert abs(obj - info["obj"]) <= 1e-9 * (1 + abs(obj)), i
        assert abs(obj - p.pstar) <= bound * 1.001 + 1e-12 * (1 + abs(p.pstar)), (i, obj, p.pstar, bound)
        oobj, obound = weak_duality_bound(p, ref.x, ref.y, ref.s)
        assert abs(oobj - p.pstar) <= obound * 1.001 + 1e-12 * (1 + abs(p.pstar)), (i, oobj, obound)
        assert abs(info["iters"] - ref.info.iters) <= max(3, 0.1 * ref.info.iters), (i, info["iters"], ref.info.iters)
        assert np.linalg.norm(p.A @ xs[i] + ss[i] - p.b) <= 1e-4 * (1 + np.linalg.norm(p.b)) * 1.001
        assert np.linalg.norm(p.A.T @ ys[i] + p.c) <= 1e-4 * (1 + np.linalg.norm(p.c)) * 1.001
        assert OC.in_cone(ss[i], p.cone, dual=False, tol=1e-9)
        assert OC.in_cone(ys[i], p.cone, dual=True, tol=1e-9)
    assert solved >= 20
    # the same programs one at a time by the single-program path, both sides
    # in near-exact projection mode (CG to 1e-12 relative), where no CG
    # stopping tie can send the two trajectories apart: the same iterates up
    # to the grouping of the team reductions
    pick = [insts[0], insts[7], insts[23]]
    tight = dict(max_iters=4000, cg_tight_tol=1e-12, cg_max_iters=1000, **extra)
    _, _, _, binfo = hsd.BatchSolver(problems(pick), **tight).solve()
    for p, bi in zip(pick, binfo):
        S = hsd.Solver(p.A, p.b, p.c, p.cone.to_dict(), **tight)
        _, _, _, solo = S.solve()
        assert solo["status"] == bi["status"]
        assert abs(solo["iters"] - bi["iters"]) <= 2, (solo["iters"], bi["iters"])
        assert abs(solo["obj"] - bi["obj"]) <= 1e-6 * (1 + abs(solo["obj"])), (solo["obj"], bi["obj"])


@pytest.mark.parametrize("stream", [False, True])
def test_batch_graph_replay_is_deterministic(stream):
    torch = _torch()
    import paper_1312_3039_amd as hsd
    insts = members(40, seed0=20_000)
    log(f"batch graph replay x3 with eager work in between, streamed sweeps {stream}")
    extra = dict(slab_cols=1 << 30) if stream else {}
    bs = hsd.BatchSolver(problems(insts), **extra)
    first = bs.solve()
    for rep in range(2):
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        again = bs.solve()
        assert torch.equal(first[0], again[0]) and torch.equal(first[1], again[1])
        assert [a["iters"] for a in first[3]] == [b["iters"] for b in again[3]]
        del junk


@pytest.mark.parametrize("stream,precision", [(False, 0), (True, 0), (False, 1)])
def test_batch_vectors_in_lds_bit_identical(stream, precision):
    """The iterate vectors of each program kept in its workgroup's LDS
    (batch_vectors = 1, the default) or in global memory (0): the same
    arithmetic in the same order, so the same outputs bit for bit, on
    programs up to the batched workload's largest size (n = 400,
    m = 1,200)."""
    torch = _torch()
    import paper_1312_3039_amd as hsd
    insts = members(24, seed0=50_000, n_lo=20, n_hi=400)
    log(f"batch vectors in LDS vs global, streamed {stream}, precision {precision}")
    extra = dict(slab_cols=1 << 30) if stream else {}
    runs = []
    for bv in (1, 0):
        bs = hsd.BatchSolver(problems(insts), batch_vectors=bv, precision=precision, **extra)
        lw = bs.launch()
        log(f"  batch_vectors={bv}: launch {lw}")
        assert lw["vectors_lds"] == bv
        runs.append(bs.solve())
        bs.close()
    (x1, y1, s1, i1), (x0, y0, s0, i0) = runs

    def same(a, b):  # bit for bit, NaN outputs (certificates) in the same places
        return torch.equal(torch.isnan(a), torch.isnan(b)) and torch.equal(a.nan_to_num(0.0), b.nan_to_num(0.0))
    assert same(x1, x0) and same(y1, y0) and same(s1, s0)
    assert [a["iters"] for a in i1] == [b["iters"] for b in i0]
    assert [a["status"] for a in i1] == [b["status"] for b in i0]


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matrix_in_lds_bit_identical(precision):
    """Each program's constants (b, c, D, E, g) and then its A and A^T
    copied into its workgroup's LDS when they fit beside its vectors
    (batch_matrix = 1, the default) or read from global memory (0): the
    same arithmetic in the same order, so the same outputs bit for bit.
    Sizes from n = 20 to 400, so that some programs fit and the largest do
    not."""
    torch = _torch()
    import paper_1312_3039_amd as hsd
    insts = members(24, seed0=51_000, n_lo=20, n_hi=400)
    log(f"batch matrices in LDS vs global, precision {precision}")
    runs = []
    for bm in (1, 0):
        bs = hsd.BatchSolver(problems(insts), batch_matrix=bm, precision=precision)
        lw = bs.launch()
        log(f"  batch_matrix={bm}: launch {lw}")
        assert lw["vectors_lds"] == 1 and lw["lds_matrix"] == bm
        if bm:
            # programs whose vectors and matrix fit in the workgroup's LDS
            # (no PSD cones here, so the vectors start at offset 0)
            sv = 4 if precision else 8
            total = lw["lds_bytes"] // 8
            fit_c, fit = [], []
            for p in insts:
                m, n = p.A.shape
                vec = 2 * (n + m + 1) + m + 4 * n + 3 * m
                cst = 3 * (n + m)
                mat = (2 * p.A.nnz * sv + 4 * (2 * p.A.nnz + m + n + 2) + 7) // 8
                fit_c.append(vec + cst <= total)
                fit.append(vec + (cst if fit_c[-1] else 0) + mat <= total)
            log(f"  {sum(fit_c)} of {len(insts)} programs take their constants into LDS, {sum(fit)} their matrix")
            assert 0 < sum(fit) < len(insts) and 0 < sum(fit_c) < len(insts)
        runs.append(bs.solve())
        bs.close()
    (x1, y1, s1, i1), (x0, y0, s0, i0) = runs

    def same(a, b):
        return torch.equal(torch.isnan(a), torch.isnan(b)) and torch.equal(a.nan_to_num(0.0), b.nan_to_num(0.0))
    assert same(x1, x0) and same(y1, y0) and same(s1, s0)
    assert [a["iters"] for a in i1] == [b["iters"] for b in i0]
    assert [a["cg_iters"] for a in i1] == [b["cg_iters"] for b in i0]
    assert [a["status"] for a in i1] == [b["status"] for b in i0]


def test_batch_fp32_mode():
    _torch()
    import paper_1312_3039_amd as hsd
    insts = members(16, seed0=30_000)
    log("batch FP32 SpMV/CG mode")
    bs = hsd.BatchSolver(problems(insts), precision=1, max_iters=4000)
    _, _, _, infos = bs.solve()
    bs64 = hsd.BatchSolver(problems(insts), precision=0, max_iters=4000)
    _, _, _, infos64 = bs64.solve()
    ok = 0
    for p, info, i64 in zip(insts, infos, infos64):
        if i64["status"] != 1:
            continue
        if info["status"] == 1:
            ok += 1
            assert abs(info["obj"] - i64["obj"]) <= 1e-3 * (1 + abs(i64["obj"]))
    assert ok >= 0.8 * sum(i["status"] == 1 for i in infos64)


def test_batch_rejects_non_block_diagonal():
    _torch()
    import paper_1312_3039_amd as hsd
    insts = members(3, seed0=40_000)
    probs = problems(insts)
    # an entry of program 0 placed in program 1's columns
    A0 = insts[0].A.tolil()
    big = sp.block_diag([insts[0].A, insts[1].A, insts[2].A], format="lil")
    big[0, insts[0].A.shape[1]] = 1.0
    from paper_1312_3039_amd import _lib
    with pytest.raises(_lib.HsdError):
        bs = hsd.BatchSolver.__new__(hsd.BatchSolver)
        hsd.BatchSolver._setup_from_block(bs, big.tocsr(), probs)
    del A0


def test_batch_state_restarts_single_solver():
    """hsd_batch_get_state: the scaled iterate each program stopped at.
    Started from its q = u - v (hsd_start_from_q), a single-program handle
    of the same data (same scaling rule) reaches the same outcome within a
    few updates: a solution for a feasible program, the certificate for an
    infeasible one."""
    _torch()
    import paper_1312_3039_amd as hsd
    from datagen import draw_socp
    from oracle.instances import make_infeasible
    feas = members(1, seed0=30_000)[0]
    base = from_draw(draw_socp(11, n=20, m=60, nonneg=20, soc_lo=3, soc_hi=6, density=0.2))
    Ai, bi, ci, _ = make_infeasible(base, np.random.default_rng(3))
    progs = [(feas.A, feas.b, feas.c, feas.cone.to_dict()), (Ai, bi, ci, base.cone.to_dict())]
    bs = hsd.BatchSolver(progs, max_iters=20000)
    _, _, _, infos = bs.solve()
    u, v = bs.state()
    assert [i["status"] for i in infos] == [1, 3]
    for k, (A, b, c, cone) in enumerate(progs):
        lo = int(bs.row_off[k] + bs.col_off[k] + k)
        hi = lo + A.shape[0] + A.shape[1] + 1
        q = (u[lo:hi] - v[lo:hi]).contiguous()
        S = hsd.Solver(A, b, c, cone, max_iters=20000)
        S.start_from_q(q)
        _, _, _, info = S.solve()
        S.close()
        log(f"program {k}: batch {infos[k]['status_name']} after {infos[k]['iters']}; "
            f"restarted single solver {info['status_name']} after {info['iters']}")
        assert info["status"] == infos[k]["status"]
        assert info["iters"] <= 10
