"""Edge cases of the problem statement (Sect. 2) on the GPU, each against
the FP64 oracle on the same input: equality rows (zero cone, whose dual
cone is the whole line), empty rows and columns of A, A with no nonzeros,
b = 0 and c = 0 (the tests of Sect. 3.5 whose norm ||b|| or ||c|| is zero
are disabled), and programs of one variable and one row."""

import numpy as np
import pytest
import scipy.sparse as sp

from datagen import ConeSpec, draw_lp
from gpu_common import log
from oracle import admm as AD
from oracle import cones as OC
from oracle.instances import from_draw

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _both(A, b, c, cone, **settings):
    import paper_1312_3039_amd as hsd
    S = hsd.Solver(sp.csr_matrix(A), b, c, cone.to_dict(), **settings)
    x, y, s, info = S.solve()
    S.close()
    ref = AD.solve(sp.csr_matrix(A), b, c, cone, AD.Settings(**{k: v for k, v in settings.items()
                                                                 if k in ("max_iters",)}))
    return (x.cpu().numpy(), y.cpu().numpy(), s.cpu().numpy(), info), ref


def _check_solved(A, b, c, cone, x, y, s, info, ref):
    assert info["status"] == ref.info.status == AD.SOLVED, (info["status_name"], ref.info.status)
    assert abs(info["obj"] - ref.info.obj) <= 1e-4 * (1 + abs(ref.info.obj))
    assert np.linalg.norm(A @ x + s - b) <= 1.001e-4 * (1 + np.linalg.norm(b))
    assert np.linalg.norm(A.T @ y + c) <= 1.001e-4 * (1 + np.linalg.norm(c))
    assert OC.in_cone(s, cone, dual=False, tol=1e-9)
    assert OC.in_cone(y, cone, dual=True, tol=1e-9)


def test_equality_rows():
    """An LP whose first 20 rows are equalities (zero cone): s = 0 there."""
    _torch()
    d = draw_lp(3, n=60, m=200, density=0.1)
    cone = ConeSpec(f=20, l=180)
    d.cone = cone
    inst = from_draw(d)
    (x, y, s, info), ref = _both(inst.A, inst.b, inst.c, cone)
    log(f"equality rows: gpu {info['status_name']} iters={info['iters']} | oracle {ref.info.iters}")
    _check_solved(inst.A, inst.b, inst.c, cone, x, y, s, info, ref)
    assert np.all(s[:20] == 0.0)


def test_empty_rows_and_columns():
    """Rows and columns of A without nonzeros (a free variable that appears
    nowhere must have c_j = 0 for the program to be bounded)."""
    _torch()
    inst = from_draw(draw_lp(4, n=50, m=150, density=0.1))
    A = inst.A.tolil()
    for i in (0, 17, 149):
        A[i, :] = 0.0
    for j in (5, 49):
        A[:, j] = 0.0
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    rng = np.random.default_rng(1)
    s_star = np.maximum(rng.standard_normal(150), 0.0)
    y_star = s_star - rng.standard_normal(150) * (s_star == 0)
    y_star = np.maximum(y_star, 0.0) * (s_star == 0)
    x_star = rng.standard_normal(50)
    b = A @ x_star + s_star
    c = -(A.T @ y_star)
    assert A.getnnz(axis=1)[0] == 0 and A.getnnz(axis=0)[5] == 0
    (x, y, s, info), ref = _both(A, b, c, inst.cone)
    log(f"empty rows/cols: gpu {info['status_name']} iters={info['iters']} | oracle {ref.info.iters}")
    _check_solved(A, b, c, inst.cone, x, y, s, info, ref)


def test_no_nonzeros_with_c_zero():
    """A = 0, c = 0, b in K: every x is optimal with s = b (objective 0)."""
    _torch()
    m, n = 40, 10
    A = sp.csr_matrix((m, n))
    b = np.abs(np.random.default_rng(2).standard_normal(m))
    c = np.zeros(n)
    cone = ConeSpec(l=m)
    (x, y, s, info), ref = _both(A, b, c, cone)
    log(f"A = 0, c = 0: gpu {info['status_name']} obj={info['obj']:.3g} | oracle {ref.info.status}")
    _check_solved(A.toarray(), b, c, cone, x, y, s, info, ref)
    assert abs(info["obj"]) <= 1e-4


def test_no_nonzeros_unbounded():
    """A = 0, c != 0: c^T x is unbounded below on the free x."""
    _torch()
    m, n = 30, 4
    A = sp.csr_matrix((m, n))
    b = np.ones(m)
    c = np.array([1.0, -2.0, 0.5, 0.0])
    cone = ConeSpec(l=m)
    (x, y, s, info), ref = _both(A, b, c, cone, max_iters=5000)
    log(f"A = 0, c != 0: gpu {info['status_name']} | oracle {ref.info.status}")
    assert info["status"] == ref.info.status == AD.UNBOUNDED
    assert abs(c @ x + 1.0) <= 1e-9


def test_c_zero_feasibility_problem():
    """c = 0: any feasible point is optimal (objective 0)."""
    _torch()
    inst = from_draw(draw_lp(6, n=40, m=120, density=0.1))
    c = np.zeros(40)
    (x, y, s, info), ref = _both(inst.A, inst.b, c, inst.cone)
    log(f"c = 0: gpu {info['status_name']} iters={info['iters']} | oracle {ref.info.iters}")
    _check_solved(inst.A, inst.b, c, inst.cone, x, y, s, info, ref)


def test_b_zero_homogeneous_program():
    """b = 0: the feasible set is a cone; with c = -A^T y* for y* in K* the
    optimum is 0 at x = 0."""
    _torch()
    inst = from_draw(draw_lp(7, n=40, m=120, density=0.1))
    b = np.zeros(120)
    (x, y, s, info), ref = _both(inst.A, b, inst.c, inst.cone)
    log(f"b = 0: gpu {info['status_name']} obj={info['obj']:.3g} | oracle {ref.info.status} {ref.info.obj:.3g}")
    _check_solved(inst.A, b, inst.c, inst.cone, x, y, s, info, ref)
    assert abs(info["obj"]) <= 1e-4


def test_one_variable_one_row():
    """min x subject to x >= 1 written as -x + s = -1, s >= 0: x* = 1."""
    _torch()
    A = sp.csr_matrix(np.array([[-1.0]]))
    b = np.array([-1.0])
    c = np.array([1.0])
    cone = ConeSpec(l=1)
    (x, y, s, info), ref = _both(A, b, c, cone)
    log(f"1 x 1: gpu {info['status_name']} x={x[0]:.6f} | oracle x={ref.x[0]:.6f}")
    _check_solved(A.toarray(), b, c, cone, x, y, s, info, ref)
    assert abs(x[0] - 1.0) <= 1e-3


@pytest.mark.parametrize("case", ["nan_in_A", "inf_in_b", "nan_in_c", "row_ptr_end", "row_ptr_decreasing",
                                  "column_out_of_range", "negative_column"])
def test_setup_rejects_bad_inputs(case):
    """Set-up checks its inputs on the device before anything indexes with
    them (the structure check reads only row_ptr[0..m] and col_idx[0..nnz)):
    non-finite values give HSD_ERR_NONFINITE, a malformed CSR HSD_ERR_ARG."""
    torch = _torch()
    import paper_1312_3039_amd as hsd
    from paper_1312_3039_amd import _lib
    inst = from_draw(draw_lp(8, n=30, m=90, density=0.1))
    A = inst.A.tocsr()
    rp = torch.as_tensor(A.indptr.astype(np.int32))
    ci = torch.as_tensor(A.indices.astype(np.int32))
    va = torch.as_tensor(A.data.copy())
    b, c = inst.b.copy(), inst.c.copy()
    want = _lib.ERR_ARG
    if case == "nan_in_A":
        va[5] = float("nan")
        want = _lib.ERR_NONFINITE
    elif case == "inf_in_b":
        b[3] = np.inf
        want = _lib.ERR_NONFINITE
    elif case == "nan_in_c":
        c[0] = np.nan
        want = _lib.ERR_NONFINITE
    elif case == "row_ptr_end":
        rp[-1] = rp[-1] - 1
    elif case == "row_ptr_decreasing":
        k = 40
        rp[k] = rp[k + 1] + 1
    elif case == "column_out_of_range":
        ci[7] = 30
    elif case == "negative_column":
        ci[2] = -1
    with pytest.raises(_lib.HsdError) as e:
        hsd.Solver((rp, ci, va, A.shape), b, c, inst.cone.to_dict())
    log(f"{case}: {e.value}")
    assert e.value.code == want
