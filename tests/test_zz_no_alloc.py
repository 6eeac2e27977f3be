"""GPU test of the allocation-free projection entry point
(hsd_project_cone_noalloc) through the C ABI: its output equals that of
hsd_project_cone bit for bit, for the cone and its dual, on two calls in a
row (the second with a smaller input and fewer cones, so the shared device
scratch holds the first call's tables when the second starts); cone tables
beyond its 1 MiB scratch are rejected with an error and nothing is
written."""

from ctypes import byref, c_void_p

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

BIG = {"f": 2, "l": 30, "q": [3, 5, 17, 40, 64], "s": [2, 5, 12], "ep": 9, "ed": 4,
       "p": [0.3, -0.6, 1.0]}
SMALL = {"f": 1, "l": 4, "q": [3, 6], "s": [3], "ep": 1, "ed": 0, "p": [-0.2]}


def _run(lib, _lib, torch, cone, x, dual, noalloc):
    K, keep = _lib.make_cone(cone)
    out = torch.full_like(x, float("nan"))
    fn = lib.hsd_project_cone_noalloc if noalloc else lib.hsd_project_cone
    stream = c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = fn(byref(K), int(x.numel()), c_void_p(x.data_ptr()), c_void_p(out.data_ptr()),
            1 if dual else 0, stream)
    return rc, out


def test_noalloc_projection_matches_allocating_one():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1312_3039_amd import _lib
    from oracle import cones as OC
    lib = _lib.load()
    rng = np.random.default_rng(5)
    for dual in (False, True):
        for cone in (BIG, SMALL):  # the second call is the smaller one
            m = OC.cone_dim(cone)
            x = torch.as_tensor(rng.standard_normal(m) * 3.0, device="cuda")
            print(f"noalloc projection dual={dual} m={m}", flush=True)
            rc0, ref = _run(lib, _lib, torch, cone, x, dual, noalloc=False)
            rc1, got = _run(lib, _lib, torch, cone, x, dual, noalloc=True)
            assert rc0 == 0 and rc1 == 0, _lib.load().hsd_last_error()
            assert torch.equal(got, ref)


def test_noalloc_projection_rejects_tables_beyond_its_scratch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1312_3039_amd import _lib
    lib = _lib.load()
    nq = (1 << 20) // 8 + 1  # 8 bytes per second-order cone: one beyond 1 MiB
    cone = {"f": 0, "l": 0, "q": [1] * nq, "s": [], "ep": 0, "ed": 0}
    x = torch.ones(nq, dtype=torch.float64, device="cuda")
    print(f"noalloc projection over {nq} cones (beyond the scratch)", flush=True)
    rc, out = _run(lib, _lib, torch, cone, x, False, noalloc=True)
    assert rc == _lib.ERR_ARG
    assert "scratch" in lib.hsd_last_error().decode()
    assert bool(torch.isnan(out).all())
