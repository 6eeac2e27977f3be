"""GPU tests of the launch-shape autotuner (coordinate search over the
ABI's launch settings, median HIP-event time of capped solves, JSON cache
keyed by device and shape bucket): a forced search on a small program and
on a small batch writes its cache entry, and the shape it returns solves
the program to the same outcome as the automatic shape (the launch shape
changes only the grouping of the sums, not the method)."""

import json
import math

import pytest

from datagen import draw_batch_member
from gpu_common import log, socp_small
from oracle.instances import from_draw

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_tune_solver_search_and_cache(tmp_path):
    _torch()
    import paper_1312_3039_amd as hsd
    from paper_1312_3039_amd import autotune
    inst = socp_small(11)
    cache = str(tmp_path / "tune.json")
    log("autotune: single-program search")
    shape = autotune.tune_solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), iters=20, reps=1,
                                 path=cache, force=True)
    data = json.load(open(cache))
    (dev, entries), = data.items()
    key = autotune._bucket("single", *inst.A.shape, inst.A.nnz)
    entry = entries[key]
    log(f"  {dev} {key}: {entry}")
    assert entry["settings"] == shape and entry["trials"] >= 3
    assert math.isfinite(entry["kernel_ms"]) and entry["kernel_ms"] > 0
    # a second call is a cache hit
    assert autotune.tune_solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), path=cache) == shape
    infos = []
    for kw in ({}, shape):
        S = hsd.Solver(inst.A, inst.b, inst.c, inst.cone.to_dict(), **kw)
        infos.append(S.solve()[3])
        S.close()
    a, b = infos
    assert a["status"] == b["status"] == 1
    assert abs(a["iters"] - b["iters"]) <= 2
    assert abs(a["obj"] - b["obj"]) <= 1e-6 * (1 + abs(a["obj"]))


def test_tune_batch_search_and_cache(tmp_path):
    _torch()
    import paper_1312_3039_amd as hsd
    from paper_1312_3039_amd import autotune
    insts = [from_draw(draw_batch_member(60_000 + i, n_lo=20, n_hi=120)) for i in range(24)]
    probs = [(p.A, p.b, p.c, p.cone.to_dict()) for p in insts]
    cache = str(tmp_path / "tune.json")
    log("autotune: batched search")
    shape = autotune.tune_batch(probs, iters=50, reps=1, path=cache, force=True)
    data = json.load(open(cache))
    (dev, entries), = data.items()
    (key, entry), = entries.items()
    log(f"  {dev} {key}: {entry}")
    assert key.startswith("batch:") and entry["settings"] == shape
    bs0 = hsd.BatchSolver(probs, max_iters=4000)
    i0 = bs0.solve()[3]
    bs0.close()
    bs1 = hsd.BatchSolver(probs, max_iters=4000, **shape)
    i1 = bs1.solve()[3]
    bs1.close()
    assert [a["status"] for a in i0] == [b["status"] for b in i1]
    for a, b in zip(i0, i1):
        if a["status"] == 1:
            assert abs(a["obj"] - b["obj"]) <= 1e-3 * (1 + abs(a["obj"]))
