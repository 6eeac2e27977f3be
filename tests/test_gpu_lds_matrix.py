"""The LDS-resident matrix slices (lds_matrix = 1): each workgroup copies its
rows of A and A^T into LDS once per solve and the sweeps read them there.
The arithmetic and its order are unchanged, so every output must be
bit-identical to the solve that reads the matrix from global memory with the
same launch shape; the small case is also held to the oracle's iterates."""

import numpy as np
import pytest

from datagen import draw_socp
from gpu_common import log, rel, socp_small
from oracle import admm as AD
from oracle.instances import from_draw

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_lds_matrix_iterates_match_oracle():
    _torch()
    import paper_1312_3039_amd as hsd
    inst = socp_small()
    K = 30
    log("lds_matrix=1 iterate parity socp_small team=7")
    S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), cg_tight_tol=1e-14,
                   cg_max_iters=1000, team_blocks=7, lds_matrix=1)
    U, V = (t.cpu().numpy() for t in S.iterate(K))
    P = AD.Problem(inst.A, inst.b, inst.c, inst.cone, AD.Settings(mode="exact"))
    u, v = P.cold_start()
    for k, (uo, vo) in enumerate(AD.iterate(P, u, v, K)):
        assert rel(np.concatenate([U[k], V[k]]), np.concatenate([uo, vo])) <= 1e-9, k


@pytest.mark.parametrize("precision", [0, 1])
def test_lds_matrix_full_size_bit_identical(precision):
    _torch()
    import paper_1312_3039_amd as hsd
    inst = from_draw(draw_socp(0))
    out = []
    for lm in (0, 1):
        log(f"SOCP n=10000 m=30000 team=64 precision={precision} lds_matrix={lm}")
        S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), precision=precision,
                       team_blocks=64, block_threads=512, lds_matrix=lm)
        x, y, s, info = S.solve()
        out.append(([t.cpu().numpy() for t in (x, y, s)], info))
        log(f"  iters={info['iters']} kernel {info['kernel_ms']:.2f} ms")
        S.close()
    (a, ia), (b, ib) = out
    assert ia["status"] == ib["status"] == 1
    assert ia["iters"] == ib["iters"]
    for p, q in zip(a, b):
        assert np.array_equal(p, q)
