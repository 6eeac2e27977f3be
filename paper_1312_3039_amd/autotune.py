"""Launch-shape autotuner for the single-program and batched solvers.

The kernels take their launch shape as settings (workgroups in a team,
threads per workgroup, lanes per row of A and of A^T in the sparse
products, lanes per second-order cone).  This module times short capped
solves over a candidate grid (median of ``reps`` runs of the persistent
kernel's own HIP-event time) and caches the best shape in a JSON file keyed
by the device name and a shape bucket (powers of two of m, n and nnz per
row, and the kind of solve).  The cached shapes are plain settings, so a
tuned solve runs exactly the same kernels as an untuned one.
"""

from __future__ import annotations

import itertools
import json
import math
import os
import time

import numpy as np

from . import BatchSolver, Solver

CACHE = os.environ.get("HSD_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "hsd_autotune.json"))


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0)


def _bucket(kind: str, m: int, n: int, nnz: int) -> str:
    lg = lambda v: int(math.log2(max(1, v)))  # noqa: E731
    return f"{kind}:m{lg(m)}:n{lg(n)}:r{lg(max(1, nnz // max(1, m)))}:c{lg(max(1, nnz // max(1, n)))}"


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(kind: str, m: int, n: int, nnz: int, path: str = CACHE):
    """Cached launch shape for this device and shape bucket, or None."""
    return _load(path).get(_device_name(), {}).get(_bucket(kind, m, n, nnz))


def _pow2s(lo, hi):
    out = []
    v = 1
    while v <= hi:
        if v >= lo:
            out.append(v)
        v *= 2
    return out


def candidates_single(m, n, nnz):
    ar = nnz / max(1, m)
    ac = nnz / max(1, n)
    teams = sorted({t for t in (max(1, nnz // d) for d in (2048, 4608, 9216, 18432)) if t <= 2048})
    la = [L for L in _pow2s(1, 64) if L <= max(1, 2 * ar)]
    lt = [L for L in _pow2s(1, 64) if L <= max(1, 2 * ac)]
    return [dict(team_blocks=t, block_threads=bt, lanes_a=a, lanes_at=b)
            for t, bt, a, b in itertools.product(teams, (256, 512), la[-3:], lt[-3:])]


def candidates_batch(nnz_per_row_a, nnz_per_row_t, avg_soc):
    la = [L for L in _pow2s(1, 64) if L <= max(1, 2 * nnz_per_row_a)]
    lt = [L for L in _pow2s(1, 64) if L <= max(1, 2 * nnz_per_row_t)]
    ls = [L for L in _pow2s(1, 64) if L <= max(1, 2 * avg_soc)]
    return [dict(block_threads=bt, lanes_a=a, lanes_at=b, lanes_soc=c)
            for bt, a, b, c in itertools.product((256, 512), la[-2:], lt[-2:], ls[-2:])]


def tune_solver(A, b, c, cone, iters: int = 60, reps: int = 3, path: str = CACHE,
                force: bool = False, **settings) -> dict:
    """Best launch shape for the single-program solver on this program's
    shape bucket (cached).  Each candidate runs `iters` capped updates."""
    m, n = A.shape
    nnz = int(A.nnz)
    key = _bucket("single", m, n, nnz)
    dev = _device_name()
    data = _load(path)
    if not force and key in data.get(dev, {}):
        return data[dev][key]["settings"]
    best = None
    results = []
    for cand in candidates_single(m, n, nnz):
        try:
            S = Solver(A, b, c, cone, max_iters=iters, **settings, **cand)
        except Exception:
            continue
        ts = []
        for _ in range(reps):
            _, _, _, info = S.solve()
            ts.append(info["kernel_ms"])
        S.close()
        t = float(np.median(ts))
        results.append((t, cand))
        if best is None or t < best[0]:
            best = (t, cand)
    if best is None:
        return {}
    data.setdefault(dev, {})[key] = {"settings": best[1], "kernel_ms": best[0],
                                     "iters": iters, "candidates": len(results),
                                     "time": time.strftime("%Y-%m-%d %H:%M:%S")}
    _store(path, data)
    return best[1]


def tune_batch(problems, iters: int = 100, reps: int = 2, path: str = CACHE,
               force: bool = False, **settings) -> dict:
    """Best launch shape for the batched solver (cached by the bucket of the
    average program; pass a representative sample of the batch).  Each
    candidate solves the sample with updates capped at `iters`."""
    m = sum(p[0].shape[0] for p in problems)
    n = sum(p[0].shape[1] for p in problems)
    nnz = sum(int(p[0].nnz) for p in problems)
    B = len(problems)
    # keyed by the average program, so a representative sample tunes the batch
    key = _bucket("batch", m // B, n // B, nnz // B)
    dev = _device_name()
    data = _load(path)
    if not force and key in data.get(dev, {}):
        return data[dev][key]["settings"]
    socs = [q for p in problems for q in p[3]["q"]]
    avg_soc = float(np.mean(socs)) if socs else 1.0
    best = None
    count = 0
    for cand in candidates_batch(nnz / m, nnz / n, avg_soc):
        try:
            bs = BatchSolver(problems, max_iters=iters, **settings, **cand)
        except Exception:
            continue
        ts = []
        for _ in range(reps):
            ts.append(bs.solve()[3][0]["kernel_ms"])
        bs.close()
        count += 1
        t = float(np.median(ts))
        if best is None or t < best[0]:
            best = (t, cand)
    if best is None:
        return {}
    data.setdefault(dev, {})[key] = {"settings": best[1], "kernel_ms": best[0], "iters": iters,
                                     "candidates": count,
                                     "time": time.strftime("%Y-%m-%d %H:%M:%S")}
    _store(path, data)
    return best[1]
