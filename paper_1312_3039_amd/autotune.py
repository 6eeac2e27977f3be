"""Launch-shape autotuner for the single-program and batched solvers.

The kernels take their launch shape as settings (workgroups in a team,
threads per workgroup, lanes per row of A and of A^T in the sparse
products, lanes per second-order cone, LDS-resident matrix slices).  This
module times short capped solves (median of ``reps`` runs of the persistent
kernel's own HIP-event time) in a coordinate search that starts from the
library's automatic shape and tries, one field at a time, powers of two
around the average row lengths, and caches the best shape in a JSON file
keyed by the device (architecture and compute units) and a shape bucket
(powers of two of m, n and nnz per row, and the kind of solve).  The cached shapes are plain settings, so
a tuned solve runs exactly the same kernels as an untuned one.
"""

from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import BatchSolver, Solver

CACHE = os.environ.get("HSD_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "hsd_autotune.json"))
# Shapes measured on known devices, shipped with the package and consulted
# after the user cache (a tuning run with force=True replaces an entry in the
# user cache only).
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_shapes.json")


def _device_name() -> str:
    """Key of the device in the caches: GPU architecture and compute-unit
    count (what decides the launch shape), else the device name."""
    import torch
    props = torch.cuda.get_device_properties(0)
    arch = (getattr(props, "gcnArchName", "") or "").split(":")[0]
    if arch:
        return f"{arch}/{props.multi_processor_count}cu"
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


def _cached(path: str, dev: str, key: str):
    """The entry for (device, bucket) from the user cache, else the shipped table."""
    for src in (path, SHIPPED):
        entry = _load(src).get(dev, {}).get(key)
        if entry is not None:
            return entry
    return None


def lookup(kind: str, m: int, n: int, nnz: int, path: str = CACHE):
    """Cached launch shape for this device and shape bucket, or None."""
    return _cached(path, _device_name(), _bucket(kind, m, n, nnz))


def _pow2_around(avg: float, lo_div: float = 8.0, hi_mul: float = 2.0, cap: int = 64):
    """Powers of two from about avg/lo_div to avg*hi_mul (at least 1, at most cap)."""
    lo = max(1.0, avg / lo_div)
    hi = min(float(cap), max(1.0, avg * hi_mul))
    out, v = [], 1
    while v <= cap:
        if lo / 2 < v <= hi:
            out.append(v)
        v *= 2
    return out or [1]


def _coordinate_search(time_of, axes, start):
    """Start from `start` (0 = the library's automatic choice for a field),
    then for each axis in turn try every option with the other fields held,
    keeping any improvement.  Returns (best settings, best time, count)."""
    best = dict(start)
    t_best = time_of(best)
    count = 1
    for key, options in axes:
        for o in options:
            if o == best.get(key):
                continue
            cand = dict(best, **{key: o})
            t = time_of(cand)
            count += 1
            if t < t_best:
                best, t_best = cand, t
    return best, t_best, count


def axes_single(m, n, nnz):
    ar = nnz / max(1, m)
    ac = nnz / max(1, n)
    # teams beyond the co-resident limit fail at setup and are skipped
    teams = sorted({min(2048, max(1, nnz // d)) for d in (1152, 2304, 4608, 9216, 18432)}
                   | {t for t in (256, 512, 768, 1024) if t * 64 <= nnz})
    # lanes from 1 up: with column slabs a row has only its entries of one
    # slab per visit, far fewer than its full length
    axes = [("team_blocks", teams), ("block_threads", (256, 512)),
            ("lanes_a", _pow2_around(ar, 64.0)), ("lanes_at", _pow2_around(ac, 64.0)),
            ("lds_matrix", (1,))]
    if max(m, n) > 262144:  # column slabs are on by default: try other widths and none
        axes.insert(0, ("slab_cols", (-1, 65536, 262144)))
    return axes


def axes_batch(nnz_per_row_a, nnz_per_row_t, avg_soc):
    # slab_cols > 0 selects the block-streamed sweeps (lanes are then unused)
    # batch_vectors 0 keeps the iterate vectors in global memory (LDS is the default)
    return [("slab_cols", (1 << 30,)), ("lanes_a", _pow2_around(nnz_per_row_a)),
            ("lanes_at", _pow2_around(nnz_per_row_t)),
            ("lanes_soc", _pow2_around(avg_soc, 4.0, 2.0)), ("block_threads", (256, 512)),
            ("batch_vectors", (0,))]


def tune_solver(A, b, c, cone, iters: int = 60, reps: int = 3, path: str = CACHE,
                force: bool = False, **settings) -> dict:
    """Best launch shape for the single-program solver on this program's
    shape bucket (cached).  Each trial runs `iters` capped updates `reps`
    times; the median kernel time decides."""
    if isinstance(A, tuple):      # device CSR (row_ptr, col_idx, val, shape)
        m, n = A[3]
        nnz = int(A[1].numel())
    else:
        m, n = A.shape
        nnz = int(A.nnz)
    key = _bucket("single", m, n, nnz)
    dev = _device_name()
    if not force and (hit := _cached(path, dev, key)) is not None:
        return hit["settings"]
    data = _load(path)

    def time_of(cand):
        try:
            S = Solver(A, b, c, cone, max_iters=iters, **settings, **cand)
        except Exception:
            return math.inf
        ts = []
        for _ in range(reps):
            ts.append(S.solve()[3]["kernel_ms"])
        S.close()
        return float(np.median(ts))

    start = dict(team_blocks=0, block_threads=0, lanes_a=0, lanes_at=0, lds_matrix=0, slab_cols=0)
    best, t_best, count = _coordinate_search(time_of, axes_single(m, n, nnz), start)
    if not math.isfinite(t_best):
        return {}
    data.setdefault(dev, {})[key] = {"settings": best, "kernel_ms": t_best, "iters": iters,
                                     "trials": count, "time": time.strftime("%Y-%m-%d %H:%M:%S")}
    _store(path, data)
    return best


def tune_batch(problems, iters: int = 100, reps: int = 2, path: str = CACHE,
               force: bool = False, **settings) -> dict:
    """Best launch shape for the batched solver (cached by the bucket of the
    average program).  Pass the whole batch (or a sample several times
    larger than the number of co-resident workgroups): each trial solves it
    with updates capped at `iters`, so the time measures throughput over the
    work queue rather than the latency of the largest program."""
    m = sum(p[0].shape[0] for p in problems)
    n = sum(p[0].shape[1] for p in problems)
    nnz = sum(int(p[0].nnz) for p in problems)
    B = len(problems)
    key = _bucket("batch", m // B, n // B, nnz // B)
    dev = _device_name()
    if not force and (hit := _cached(path, dev, key)) is not None:
        return hit["settings"]
    data = _load(path)
    socs = [q for p in problems for q in p[3]["q"]]
    avg_soc = float(np.mean(socs)) if socs else 1.0

    def time_of(cand):
        try:
            bs = BatchSolver(problems, max_iters=iters, **settings, **cand)
        except Exception:
            return math.inf
        ts = [bs.solve()[3][0]["kernel_ms"] for _ in range(reps)]
        bs.close()
        return float(np.median(ts))

    start = dict(block_threads=0, lanes_a=0, lanes_at=0, lanes_soc=0, slab_cols=0, batch_vectors=1)
    best, t_best, count = _coordinate_search(time_of, axes_batch(nnz / m, nnz / n, avg_soc), start)
    if not math.isfinite(t_best):
        return {}
    data.setdefault(dev, {})[key] = {"settings": best, "kernel_ms": t_best, "iters": iters,
                                     "trials": count, "time": time.strftime("%Y-%m-%d %H:%M:%S")}
    _store(path, data)
    return best
