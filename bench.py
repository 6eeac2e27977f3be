#!/usr/bin/env python3
"""Benchmark: ADMM on the homogeneous self-dual embedding on one MI355X.

Headline workload: random feasible SOCP, n = 10,000, m = 30,000 (5,000
nonnegative rows, second-order cones of sizes uniform in [3, 50] filling the
rest), A sparse CSR at density 1e-3 (300,000 nonzeros, N(0,1)), built as in
the paper's random cone programs (s* = Pi_K(z), y* = s* - z, b = A x* + s*,
c = -A^T y*), eps = 1e-4.

One step = one complete solve of that program: setup (transpose,
equilibration, g = M^{-1} h) plus the iteration to eps = 1e-4, with A, b, c
already resident in HBM.  The reported value is whole-job ADMM iterations
per second over the timed steps; time-to-eps per solve is reported beside
it.  The FP32-SpMV/CG mode is timed on the same program.

The same JSON line carries the other workloads under "workloads" (each
with its own roofline and CPU-oracle baseline): the random LP (n = 100),
the mixed-cone program (PSD and exponential cones, FP32 and FP64), the
batch of 4,096 small SOCPs against a one-program-at-a-time loop on the same
GPU, the large SOCP (10^8 nonzeros, beyond the caches) and the learned warm
start against the cold start.  --quick leaves them out; --workload runs one
of them alone.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--quick]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

PEAK_HBM_GBS = 8000.0
WORKLOAD = {"n": 10_000, "m": 30_000, "nonneg": 5_000, "soc_lo": 3, "soc_hi": 50,
            "density": 1e-3, "seed": 0, "eps": 1e-4}
METRIC = "time-to-eps=1e-4 & ADMM iters/s; HBM GB/s vs peak; warm/batched vs plain"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# HBM traffic of one FP64 launch of the dominant kernel of a workload, from
# two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch;
# the profiles named below), each scaled by what the same counter reads for
# a plain 1 GiB device copy (FETCH_SIZE reads 512 MiB: x2.0; WRITE_SIZE reads
# 1 GiB: x1.0).  Valid only for the kernel sources they were measured on
# (hash below) and the launch shape they were measured with; otherwise the
# bench reports null.
TRAFFIC_FP64 = {"src_hash": "3c738e9e3a0b88b3",
                "shape": {"block_threads": 512, "lanes_a": 2, "lanes_at": 4, "lds_matrix": 1,
                          "slab_cols": 0, "team_blocks": 130},
                "fetch_kib": 712912.7, "write_kib": 235876.1, "fetch_scale": 2.0, "write_scale": 1.0,
                "fetch_profile": "profiles/k_solve_socp10k_fp64_traffic.md",
                "write_profile": "profiles/k_solve_socp10k_fp64_traffic.md"}
TRAFFIC_BATCH = {"src_hash": "bcc02b2b0972defd",
                 "shape": {"block_threads": 0, "lanes_a": 2, "lanes_at": 4, "lanes_soc": 0, "slab_cols": 0},
                 "fetch_kib": 180979408.1, "write_kib": 61813.7, "fetch_scale": 2.0, "write_scale": 1.0,
                 "fetch_profile": "profiles/k_batch_socp4096_fp64.md",
                 "write_profile": "profiles/k_batch_socp4096_fp64.md"}


def kernel_src_hash(kind: str = "single"):
    """Hash of the sources a kernel is built from: the single-program solve
    kernel (everything but the batched and network sources) or the batched
    kernels (everything but the single-program host file and the network)."""
    import glob
    import hashlib
    skip = {"single": ("hsd_batch.hip", "hsd_mlp.hip"), "batch": ("hsd_api.hip", "hsd_mlp.hip")}[kind]
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(HERE, "paper_1312_3039_amd", "csrc", "*"))):
        if os.path.basename(f) in skip:
            continue
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(shape, t=TRAFFIC_FP64, kind="single"):
    if kernel_src_hash(kind) != t["src_hash"] or dict(shape or {}) != t["shape"]:
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


# ---------------------------------------------------------------------------
# algorithmic bytes of the persistent solve kernel
# ---------------------------------------------------------------------------

def pair_bytes(m, n, nnz, sv):
    """One product with A and one with A^T (CSR, s_v-byte values, 4-byte
    indices): the matrix entries, the row pointers, the gathered input and
    the written output of each, every element counted once."""
    return 2 * nnz * (sv + 4) + 4 * (m + n + 2) + 2 * (m + n) * sv


def alg_bytes(m, n, nnz, sv, iters, cg_iters, checks):
    """Algorithmic bytes of one solve launch, counted per unit of work:
        per CG iteration  B_cg = (A, A^T product pair) + 9 n s_v
                                 (the fused CG vector updates);
        per ADMM update   (pair) for the right-hand side r_x - A^T r_y and
                          z_y = r_y + A z_x, plus 12 (n + m + 1) 8 bytes of
                          vector work (w, r, SMW, relaxation, projection,
                          dual update);
        per termination test  (pair) in FP64 (A u_x and A^T u_y).
    s_v = 8 in FP64, 4 in FP32 mode (tests stay FP64)."""
    pair = pair_bytes(m, n, nnz, sv)
    b_cg = pair + 9 * n * sv
    upd = pair + 12 * (n + m + 1) * 8
    return iters * upd + cg_iters * b_cg + checks * pair_bytes(m, n, nnz, 8)


def sweep_bytes(rows, cols, nnz, sv):
    """One CSR product: values and column indices once, row pointers once,
    the gathered input vector once and the output vector once."""
    return nnz * (sv + 4) + 4 * (rows + 1) + cols * sv + rows * sv


def solve_bytes(m, n, nnz, sv, iters, cg_iters, checks, fp32):
    """Algorithmic HBM bytes of one persistent solve launch: every array
    element a phase touches counted once per phase (caches ignored).

    per ADMM update   : A-phase t0 = r_y + A z0 (reads u_y, v_s, b; writes
                        z_y, t): A z0 by a product on the first update (FP32
                        mode: every 32nd), else read back from t, where the
                        update left z_y - r_y;
                        A^T-sweep (res0; reads u_x, c, z_x; writes res),
                        update (reads z, g, u, v_s; writes u, v_s, t)
    per CG iteration  : A-sweep on p formed from res and p_old (+n), writes p;
                        A^T-sweep, reads p, z_x, res, c, writes z_x, res;
                        z_y += a t over m (reads t, z_y, b, writes z_y)
    per test          : FP64 values again in FP32 mode, the gathered u_x / u_y,
                        D and E
    """
    a_rows = 3 * 8 * m + m * sv
    a_prod = sweep_bytes(m, n, nnz, sv) + a_rows
    a_carry = a_rows + 2 * m * sv
    n_prod = min(iters, 1 + (iters // 32 if fp32 else 0))
    upd = (sweep_bytes(n, m, nnz, sv) + 3 * 8 * n + 2 * n * sv
           + n * sv + m * sv + 8 * (n + m) * 3 + 8 * m * 2 + m * sv)
    cg = (sweep_bytes(m, n, nnz, sv) + n * sv + n * sv
          + sweep_bytes(n, m, nnz, sv) + 5 * n * sv + 8 * n + 3 * m * sv + 8 * m)
    chk = (2 * nnz * 8 if fp32 else 0) + 8 * n + 8 * m + 8 * m + 8 * n
    return (n_prod * a_prod + (iters - n_prod) * a_carry + iters * upd + cg_iters * cg
            + checks * chk)


# ---------------------------------------------------------------------------
# instance: seeded draw + the library's own projection for s* = Pi_K(z)
# ---------------------------------------------------------------------------

def gpu_instance(torch, hsd, draw):
    import scipy.sparse as sp
    dev = torch.device("cuda")
    A = sp.csr_matrix((draw.data, draw.indices, draw.indptr), shape=(draw.m, draw.n))
    cone = draw.cone.to_dict()
    s = hsd.project_cone(cone, draw.z, dual=False).cpu().numpy()
    y = s - draw.z
    b = A @ draw.xstar + s
    c = -(A.T @ y)
    pstar = float(c @ draw.xstar)
    Ad = (torch.as_tensor(draw.indptr.astype(np.int32), device=dev),
          torch.as_tensor(draw.indices.astype(np.int32), device=dev),
          torch.as_tensor(draw.data, device=dev), (draw.m, draw.n))
    bd = torch.as_tensor(b, device=dev)
    cd = torch.as_tensor(c, device=dev)
    return Ad, bd, cd, cone, pstar


def run_gpu(torch, hsd, Ad, bd, cd, cone, steps, warmup, **settings):
    infos = []
    for _ in range(warmup):
        S = hsd.Solver(Ad, bd, cd, cone, **settings)
        S.solve()
        S.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        S = hsd.Solver(Ad, bd, cd, cone, **settings)
        _, _, _, info = S.solve()
        S.close()
        infos.append(info)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, infos


def summarize(wall, infos, m, n, nnz, fp32, pstar):
    steps = len(infos)
    iters = sum(i["iters"] for i in infos)
    sv = 4 if fp32 else 8
    kern_ms = [i["kernel_ms"] for i in infos]
    by = [alg_bytes(m, n, nnz, sv, i["iters"], i["cg_iters"], i["iters"] + 1) for i in infos]
    by_model = [solve_bytes(m, n, nnz, sv, i["iters"], i["cg_iters"], i["iters"] + 1, fp32) for i in infos]
    achieved = [b / (k * 1e-3) / 1e9 for b, k in zip(by, kern_ms)]
    return {
        "value": iters / wall,
        "ms_per_step": 1e3 * wall / steps,
        "time_to_eps_ms": float(np.mean([i["setup_ms"] + i["solve_ms"] for i in infos])),
        "setup_ms": float(np.mean([i["setup_ms"] for i in infos])),
        "solve_ms": float(np.mean([i["solve_ms"] for i in infos])),
        "kernel_ms": float(np.mean(kern_ms)),
        "iters": int(np.mean([i["iters"] for i in infos])),
        "avg_cg": float(np.mean([i["cg_iters"] / max(1, i["iters"]) for i in infos])),
        "spmv_count": int(infos[-1]["spmv_count"]),
        "status": sorted(set(i["status_name"] for i in infos)),
        "obj": float(infos[-1]["obj"]),
        "obj_rel_err_vs_pstar": abs(infos[-1]["obj"] - pstar) / max(1.0, abs(pstar)),
        "bytes_per_launch": float(np.mean(by)),
        "achieved_gbs": float(np.mean(achieved)),
        "bytes_per_launch_touched": float(np.mean(by_model)),
        "achieved_gbs_touched": float(np.mean([b / (k * 1e-3) / 1e9 for b, k in zip(by_model, kern_ms)])),
    }


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def roofline(bound, rec, kernel, traffic=None, traffic_source=None, note=None):
    out = {"bound": bound, "achieved": rec["achieved_gbs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": rec["achieved_gbs"] / PEAK_HBM_GBS, "traffic": traffic,
           "kernel": kernel, "bytes_per_launch": rec["bytes_per_launch"],
           "kernel_ms": rec["kernel_ms"],
           "bytes_rule": "per CG iteration: A and A^T products + 9n s_v; per ADMM update: the "
                         "products for the right-hand side and z_y + 12(n+m+1)*8 vector bytes; "
                         "per test: the FP64 product pair",
           "touched_model": {"bytes_per_launch": rec["bytes_per_launch_touched"],
                             "achieved": rec["achieved_gbs_touched"]}}
    if traffic_source is not None:
        out["traffic_source"] = traffic_source
    if note:
        out["note"] = note
    return out


def oracle_solves(insts, threads):
    """Wall time and results of full oracle solves (setup + iterations) of
    the given programs with the BLAS pools limited to ``threads``."""
    from threadpoolctl import threadpool_limits
    from oracle.admm import Settings, solve
    res = []
    tot = 0.0
    for inst in insts:
        with threadpool_limits(threads):
            t0 = time.perf_counter()
            r = solve(inst.A, inst.b, inst.c, inst.cone, Settings())
            tot += time.perf_counter() - t0
        res.append(r.info)
    return tot, res


def cpu_baseline(seeds, make_inst, label):
    """The oracle (test infrastructure) on the same workload: full cold
    solves to eps = 1e-4 for the given seeds, on one thread, then with the
    BLAS pools on every usable core (SciPy's sparse products stay on one
    thread either way)."""
    insts = [make_inst(sd) for sd in seeds]
    t1, res = oracle_solves(insts, 1)
    for sd, r in zip(seeds, res):
        log(f"[cpu] {label} seed {sd}: {r.iters} iterations")
    hi = host_info()
    tN, _ = oracle_solves(insts, hi["usable_cpus"])
    it = sum(r.iters for r in res)
    return {"value": it / t1, "unit": "ADMM iters/s", "cores": 1, "kind": "oracle",
            "time_to_eps_ms": 1e3 * t1 / len(seeds),
            "sample": f"{len(seeds)} complete cold solves (setup + iterations to eps=1e-4) of the "
                      f"same workload, seeds {list(seeds)}, FP64 NumPy/SciPy oracle, 1 thread",
            "all_cores": {"value": it / tN, "cores": hi["usable_cpus"], "time_to_eps_ms": 1e3 * tN / len(seeds),
                          "note": "BLAS pools on every usable core; SciPy's CSR products run on "
                                  "one thread"},
            "host": hi,
            "oracle": [{"seed": int(sd), "status": int(r.status), "iters": int(r.iters), "obj": float(r.obj)}
                       for sd, r in zip(seeds, res)]}


LARGE = {"n": 1_000_000, "m": 3_000_000, "nonneg": 500_000, "soc_lo": 3, "soc_hi": 50,
         "nnz": 100_000_000, "seed": 0, "eps": 1e-4}


def run_large(args):  # noqa: C901
    """One large random SOCP (n = 1e6, m = 3e6, 1e8 nonzeros: 1.2 GB of FP64
    CSR per copy of A, well beyond the last-level caches), so every sweep
    streams A or A^T from HBM.  Same generator and path as the default
    workload; cold solves to eps = 1e-4, setup included."""
    import torch
    import paper_1312_3039_amd as hsd
    from datagen import draw_socp
    W = LARGE
    dens = W["nnz"] / (W["m"] * W["n"])
    t0 = time.perf_counter()
    draw = draw_socp(W["seed"], n=W["n"], m=W["m"], nonneg=W["nonneg"], soc_lo=W["soc_lo"],
                     soc_hi=W["soc_hi"], density=dens)
    log(f"[large] drew m={draw.m} n={draw.n} nnz={draw.nnz} in {time.perf_counter() - t0:.1f} s")
    Ad, bd, cd, cone, pstar = gpu_instance(torch, hsd, draw)
    eps = dict(eps_pri=W["eps"], eps_dual=W["eps"], eps_gap=W["eps"])
    shape = {}
    if args.shape is not None:
        shape = json.loads(args.shape)
    elif not args.no_tune:
        from paper_1312_3039_amd import autotune
        t0 = time.perf_counter()
        shape = autotune.tune_solver(Ad, bd, cd, cone, iters=20, reps=2, **eps)
        log(f"[large] launch shape {shape} ({time.perf_counter() - t0:.1f}s, cached per device)")
    res = {}
    for prec, name in ((0, "fp64"), (1, "fp32_spmv")):
        log(f"[large] {name}: {args.warmup} warmup + {args.steps} timed solves")
        wall, infos = run_gpu(torch, hsd, Ad, bd, cd, cone, args.steps, args.warmup,
                              precision=prec, **eps, **shape)
        res[name] = summarize(wall, infos, draw.m, draw.n, draw.nnz, prec == 1, pstar)
        log(f"[large] {name}: {res[name]['iters']} iters, {res[name]['time_to_eps_ms']:.1f} ms "
            f"to eps, {res[name]['achieved_gbs']:.0f} GB/s")
    r64 = res["fp64"]
    out = {
        "metric": METRIC, "value": r64["value"], "unit": "ADMM iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded random feasible SOCP with known optimal value)",
        "config": {"workload": "large random SOCP n=1e6 m=3e6 (5e5 nonneg + SOC sizes U[3,50]), "
                               "1e8 nnz, eps=1e-4, cold start, setup included",
                   "n": draw.n, "m": draw.m, "nnz": draw.nnz, "n_soc": len(draw.cone.q),
                   "seed": W["seed"], "global_batch": 1, "parallelism": "single GPU"},
        "time_to_eps_ms": r64["time_to_eps_ms"], "launch_shape": shape or "automatic",
        "fp64": r64, "fp32_spmv": res["fp32_spmv"],
        "roofline": roofline("hbm", r64, "k_solve<double, true, 0> (persistent cooperative solve, "
                                        "streamed column-slab sweeps)",
                             note="working set (2.4 GB of CSR per product pair) beyond the caches"),
    }
    # objective against the exact optimum of the planted program at eps = 1e-5
    S = hsd.Solver(Ad, bd, cd, cone, precision=0, eps_pri=1e-5, eps_dual=1e-5, eps_gap=1e-5, **shape)
    _, _, _, inf5 = S.solve()
    S.close()
    out["eps_1e-5"] = {"status": inf5["status_name"], "iters": inf5["iters"],
                       "time_to_eps_ms": inf5["setup_ms"] + inf5["solve_ms"],
                       "obj_rel_err_vs_pstar": abs(inf5["obj"] - pstar) / abs(pstar)}
    log(f"[large] eps=1e-5: {inf5['iters']} iters, |obj-p*|/|p*| = {out['eps_1e-5']['obj_rel_err_vs_pstar']:.2e}")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_large_baseline(draw, args.cpu_iters)
    return out


def cpu_large_baseline(draw, iters):
    """The oracle (test infrastructure) on the large program, one thread:
    set-up (scaling and g) timed once, then `iters` ADMM iterations from the
    cold start in CG mode; the rate is iterations per second of the loop."""
    from threadpoolctl import threadpool_limits
    from oracle import admm as AD
    from oracle.instances import from_draw
    inst = from_draw(draw)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        P = AD.Problem(inst.A, inst.b, inst.c, inst.cone, AD.Settings())
        t_setup = time.perf_counter() - t0
        log(f"[cpu] oracle setup {t_setup:.1f} s")
        u, v = P.cold_start()
        t0 = time.perf_counter()
        AD.iterate(P, u, v, iters)
        t_it = time.perf_counter() - t0
    log(f"[cpu] oracle {iters} iterations {t_it:.1f} s")
    return {"value": iters / t_it, "unit": "ADMM iters/s", "cores": 1, "kind": "oracle",
            "setup_s": t_setup,
            "sample": f"oracle set-up once, then {iters} ADMM iterations from the cold start "
                      "(CG mode) of the same large program, FP64 NumPy/SciPy, 1 thread",
            "host": host_info()}


# The paper's random SOCPs (Sect. 6, random cone programs; Table
# t-random-socps: small and medium columns) with this project's cone mix
# (m/6 nonnegative rows, second-order cones of sizes U[3,50]; the paper does
# not state its mix), and the paper's numbers for its indirect solver at its
# tolerance eps = 1e-3: iterations, average CG iterations, total products.
PAPER_SOCP = {"S": {"n": 10_000, "m": 30_000, "nnz": 1_000_000, "paper": (40, 4.7, 457, 0.9)},
              "M": {"n": 1_000_000, "m": 3_000_000, "nnz": 1_000_000_000, "paper": (160, 6.1, 2265, 4.3e3)}}


def run_paper(args):  # noqa: C901
    """The paper's random SOCPs S (10^6 nonzeros) and M (10^9 nonzeros, 12 GB
    of FP64 CSR per copy of A) on one GPU: cold solves at the paper's
    eps = 1e-3 and at 1e-4, set-up included, with the paper's own accounting
    (iterations, average CG iterations per iteration, total products with A
    or A^T) beside its Table's numbers, the relative objective errors the
    Table reports, and KKT residuals of the returned point recomputed on the
    host with SciPy."""
    import torch
    import paper_1312_3039_amd as hsd
    from datagen import draw_socp
    out = {"metric": METRIC, "unit": "s to eps (setup included)", "n_gpus": 1, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (the paper's random SOCP recipe, seeded)", "sizes": {}}
    for key in args.paper_sizes:
        W = PAPER_SOCP[key]
        n, m, nnz = W["n"], W["m"], W["nnz"]
        t0 = time.perf_counter()
        draw = draw_socp(0, n=n, m=m, nonneg=m // 6, soc_lo=3, soc_hi=50, density=nnz / (m * n))
        log(f"[paper {key}] drew m={m} n={n} nnz={draw.nnz} in {time.perf_counter() - t0:.1f} s")
        t0 = time.perf_counter()
        Ad, bd, cd, cone, pstar = gpu_instance(torch, hsd, draw)
        log(f"[paper {key}] data on the GPU in {time.perf_counter() - t0:.1f} s")
        rec = {"n": n, "m": m, "nnz": int(draw.nnz), "n_soc": len(draw.cone.q),
               "paper_eps_1e-3": dict(zip(("iterations", "avg_cg", "products", "seconds"), W["paper"]))}
        import scipy.sparse as sp
        A = sp.csr_matrix((draw.data, draw.indices, draw.indptr), shape=(m, n))
        b, c = bd.cpu().numpy(), cd.cpu().numpy()
        for eps in (1e-3, 1e-4):
            S = hsd.Solver(Ad, bd, cd, cone, eps_pri=eps, eps_dual=eps, eps_gap=eps)
            lw = S.launch()
            x, y, s_, info = S.solve()
            S.close()
            torch.cuda.synchronize()
            xs, ys, ss = (t.cpu().numpy() for t in (x, y, s_))
            pri = float(np.linalg.norm(A @ xs + ss - b)) / (1 + float(np.linalg.norm(b)))
            dua = float(np.linalg.norm(A.T @ ys + c)) / (1 + float(np.linalg.norm(c)))
            r = {"status": info["status_name"], "iterations": info["iters"],
                 "avg_cg": info["cg_iters"] / max(1, info["iters"]), "products": int(info["spmv_count"]),
                 "setup_s": info["setup_ms"] / 1e3, "solve_s": info["solve_ms"] / 1e3,
                 "time_to_eps_s": (info["setup_ms"] + info["solve_ms"]) / 1e3,
                 "kernel_ms": info["kernel_ms"],
                 "cx_rel_err_vs_pstar": abs(float(c @ xs) - pstar) / abs(pstar),
                 "by_rel_err_vs_pstar": abs(-float(b @ ys) - pstar) / abs(pstar),
                 "kkt_rel_primal": pri, "kkt_rel_dual": dua, "launch": lw}
            by = alg_bytes(m, n, draw.nnz, 8, info["iters"], info["cg_iters"], info["iters"] + 1)
            r["bytes_per_launch"] = by
            r["achieved_gbs"] = by / (info["kernel_ms"] * 1e-3) / 1e9
            r["frac_of_hbm_peak"] = r["achieved_gbs"] / PEAK_HBM_GBS
            log(f"[paper {key}] eps={eps:g}: {r['status']} in {r['iterations']} iterations, avg CG "
                f"{r['avg_cg']:.2f}, {r['products']} products, {r['time_to_eps_s']:.2f} s to eps "
                f"(setup {r['setup_s']:.2f} s), {r['achieved_gbs']:.0f} GB/s; |c^T x - p*|/|p*| "
                f"{r['cx_rel_err_vs_pstar']:.1e}, |b^T y + p*|/|p*| {r['by_rel_err_vs_pstar']:.1e}")
            rec[f"eps_{eps:g}"] = r
        out["sizes"][key] = rec
        del Ad, bd, cd, draw, A
        torch.cuda.empty_cache()
    last = out["sizes"][args.paper_sizes[-1]]
    out["value"] = last["eps_0.0001"]["time_to_eps_s"]
    out["config"] = {"workload": "the paper's random SOCPs (sizes " + ", ".join(args.paper_sizes) +
                                 "), eps = 1e-3 (the paper's) and 1e-4, cold start, setup included"}
    return out


BATCH = {"B": 4096, "n_lo": 20, "n_hi": 400, "soc_lo": 3, "soc_hi": 10, "density": 0.05,
         "seed0": 10_000, "eps": 1e-4}


def gpu_batch_problems(torch, hsd, draws):
    """Per-program data with the library's own projection for s* = Pi_K(z)."""
    import scipy.sparse as sp
    probs = []
    for d in draws:
        A = sp.csr_matrix((d.data, d.indices, d.indptr), shape=(d.m, d.n))
        cone = d.cone.to_dict()
        s = hsd.project_cone(cone, d.z, dual=False).cpu().numpy()
        y = s - d.z
        probs.append((A, A @ d.xstar + s, -(A.T @ y), cone))
    return probs


def run_batch(args):
    import torch
    import paper_1312_3039_amd as hsd
    from datagen import draw_batch_member
    W = BATCH
    B = args.batch_size
    t0 = time.perf_counter()
    draws = [draw_batch_member(W["seed0"] + i, n_lo=W["n_lo"], n_hi=W["n_hi"], soc_lo=W["soc_lo"],
                               soc_hi=W["soc_hi"], density=W["density"]) for i in range(B)]
    probs = gpu_batch_problems(torch, hsd, draws)
    nnz = sum(d.nnz for d in draws)
    log(f"[gpu] {B} programs generated in {time.perf_counter() - t0:.1f}s, total nnz={nnz}")
    eps = dict(eps_pri=W["eps"], eps_dual=W["eps"], eps_gap=W["eps"])
    shape = {}
    if not args.no_tune:
        from paper_1312_3039_amd import autotune
        t0 = time.perf_counter()
        shape = autotune.tune_batch(probs, **eps)
        log(f"[gpu] launch shape {shape} ({time.perf_counter() - t0:.1f}s, cached per device)")
    bs = hsd.BatchSolver(probs, **eps, **shape)
    for _ in range(args.warmup):
        bs.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for _ in range(args.steps):
        runs.append(bs.solve()[3])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    infos = runs[-1]
    solved = sum(i["status"] == 1 for i in infos)
    kern_ms = float(np.mean([r[0]["kernel_ms"] for r in runs]))
    solve_ms = float(np.mean([r[0]["solve_ms"] for r in runs]))
    by = sum(alg_bytes(d.m, d.n, d.nnz, 8, i["iters"], i["cg_iters"], i["iters"] + 1)
             for d, i in zip(draws, infos))
    achieved = by / (kern_ms * 1e-3) / 1e9
    log(f"[gpu] batch: {solved}/{B} solved, {solve_ms:.1f} ms per batch (solve kernel {kern_ms:.1f} ms)")
    # the plain method on the same GPU: one program at a time (a sample spread
    # over the sizes, extrapolated to the whole batch)
    sample = list(range(0, B, max(1, B // args.seq_sample)))[:args.seq_sample]
    seq_t = 0.0
    seq_solved = 0
    torch.cuda.synchronize()
    for i in sample:
        A, b, c, cone = probs[i]
        t1 = time.perf_counter()
        S = hsd.Solver(A, b, c, cone, **eps)
        _, _, _, inf = S.solve()
        S.close()
        torch.cuda.synchronize()
        seq_t += time.perf_counter() - t1
        seq_solved += inf["status"] == 1
    seq_rate = len(sample) / seq_t
    out = {
        "metric": METRIC,
        "value": B * args.steps / wall,
        "unit": "solves/s (eps=1e-4)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded random feasible SOCPs with known optimal values)",
        "config": {"workload": f"batched: {B} independent random SOCPs, n~U[20,400], m=3n, "
                               "floor(m/2) nonneg + SOC sizes U[3,10], density 0.05, eps=1e-4, "
                               "one persistent graph-captured launch per batch",
                   "programs": B, "total_nnz": int(nnz), "global_batch": B,
                   "parallelism": "single GPU, one workgroup per program"},
        "solved": solved,
        "launch_shape": shape,
        "batch_solve_ms": solve_ms,
        "solve_kernel_ms": kern_ms,
        "mean_iters": float(np.mean([i["iters"] for i in infos])),
        "sequential_gpu": {"solves_per_s": seq_rate, "sample": len(sample), "solved": int(seq_solved),
                           "note": "hsd.Solver (setup + solve) one program at a time, same GPU"},
        "speedup_vs_sequential": (B * args.steps / wall) / seq_rate,
        "roofline": {"bound": "latency", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": measured_traffic(shape, TRAFFIC_BATCH, "batch"),
                     "traffic_source": {"profiles": [TRAFFIC_BATCH["fetch_profile"], TRAFFIC_BATCH["write_profile"]],
                                        "kernel_src_hash": TRAFFIC_BATCH["src_hash"],
                                        "current_src_hash": kernel_src_hash("batch")},
                     "kernel": "k_batch<double, false, true> (persistent batched solve, iterate vectors in LDS)",
                     "bytes_per_launch": by, "kernel_ms": kern_ms,
                     "bytes_rule": "per program as for one program: CG iterations, updates and tests",
                     "note": "each program is a chain of dependent steps on one workgroup; the "
                             "batch's end is set by its longest programs"},
    }
    bs.close()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_batch_baseline(draws[:args.cpu_programs])
    return out


def cpu_batch_baseline(draws):
    from threadpoolctl import threadpool_limits
    from oracle.admm import Settings, solve
    from oracle.instances import from_draw
    t = 0.0
    for d in draws:
        inst = from_draw(d)
        with threadpool_limits(1):
            t0 = time.perf_counter()
            solve(inst.A, inst.b, inst.c, inst.cone, Settings())
            t += time.perf_counter() - t0
    return {"value": len(draws) / t, "unit": "solves/s (eps=1e-4)", "cores": 1, "kind": "oracle",
            "sample": f"the first {len(draws)} programs of the batch, solved one after another by the "
                      "FP64 NumPy/SciPy oracle on 1 thread", "host": host_info()}


WARM = {"seed": 5000, "n": 2000, "m": 6000, "nonneg": 1000, "soc_lo": 3, "soc_hi": 50,
        "density": 5e-3, "p": 64, "train": 20_000, "eval": 2_000, "hidden": 512}


def run_warmstart(args):
    """Parametric family: learned warm start vs cold start on one GPU."""
    import torch
    from datagen import draw_parametric_family, draw_theta
    from paper_1312_3039_amd import warmstart as Wm
    W = WARM
    out_rows = {}
    for b_std in args.b_std:
        pd = draw_parametric_family(seed=W["seed"], n=W["n"], m=W["m"], nonneg=W["nonneg"],
                                    soc_lo=W["soc_lo"], soc_hi=W["soc_hi"], density=W["density"],
                                    p=W["p"], b_std=b_std)
        fam = Wm.family_from_draw(pd)
        ntr = args.train_size
        train = np.stack([draw_theta(s, p=W["p"]) for s in range(max(ntr, args.cert_train))])
        train_all = train
        held = np.stack([draw_theta(10 ** 6 + s, p=W["p"]) for s in range(args.eval_size)])
        log(f"[warm] b_std={b_std}: generating {ntr} solves")
        # a first chunk shows whether the family is solvable at all; a mostly
        # infeasible family is reported from that chunk alone
        first = Wm.solve_family(fam, train[:2048], chunk=2048)
        if (first["status"] == 1).mean() < 0.1 or ntr <= 2048:
            sol = first
            train = train[:first["status"].shape[0]]
            ntr = train.shape[0]
        else:
            train = train[:ntr]
            rest = Wm.solve_family(fam, train[2048:], chunk=2048)
            sol = {k: (torch.cat([first[k], rest[k]]) if k in ("x", "y", "s") else
                       first[k] + rest[k] if k == "seconds" else
                       np.concatenate([first[k], rest[k]])) for k in first}
        ok = sol["status"] == 1
        rec = {"b_std": b_std, "train_solves": ntr, "train_solved": int(ok.sum()),
               "train_gen_s": sol["seconds"],
               "train_status_counts": {int(k): int(v) for k, v in zip(*np.unique(sol["status"], return_counts=True))}}
        log(f"[warm] solved {int(ok.sum())}/{ntr} in {sol['seconds']:.1f}s")
        if ok.sum() < 512:
            # A family of certificates: the network learns the scaled iterate
            # q = u - v the training programs stopped at, and the held-out
            # programs are timed to their certificates, cold vs warm.
            rec["note"] = "too few solved programs to train on (the family is mostly infeasible)"
            cert_th = train_all[:args.cert_train]
            cert = Wm.solve_family(fam, cert_th, chunk=2048, with_q=True)
            inf = cert["status"] == 3
            rec["cert_train_solves"] = int(inf.shape[0])
            rec["cert_train_infeasible"] = int(inf.sum())
            if inf.sum() >= 512:
                ws = Wm.WarmStarter(fam, hidden=W["hidden"], batch=256)
                t0 = time.perf_counter()
                losses = ws.fit(cert_th[inf], cert["q"][inf], epochs=args.epochs, lr=1e-3)
                torch.cuda.synchronize()
                rec["cert_train_s"] = time.perf_counter() - t0
                rec["cert_loss_first_last"] = [losses[0], losses[-1]]
                rows = Wm.evaluate_q(fam, ws, held[:args.cert_eval_size])
                cold_it = np.array([r["cold_iters"] for r in rows])
                warm_it = np.array([r["warm_iters"] for r in rows])
                cold_ms = np.array([r["cold_ms"] for r in rows])
                warm_ms = np.array([r["warm_ms"] for r in rows])
                rec.update({"cert_eval_programs": len(rows),
                            "cert_cold_infeasible": int(sum(r["cold_status"] == 3 for r in rows)),
                            "cert_warm_infeasible": int(sum(r["warm_status"] == 3 for r in rows)),
                            "cert_cold_mean_iters": float(cold_it.mean()),
                            "cert_warm_mean_iters": float(warm_it.mean()),
                            "cert_cold_mean_ms": float(cold_ms.mean()),
                            "cert_warm_mean_ms": float(warm_ms.mean()),
                            "cert_iters_ratio": float(warm_it.mean() / cold_it.mean()),
                            "cert_time_ratio": float(warm_ms.mean() / cold_ms.mean())})
                log(f"[warm] certificates: iterations cold {cold_it.mean():.1f} warm {warm_it.mean():.1f}; "
                    f"ms cold {cold_ms.mean():.2f} warm {warm_ms.mean():.2f}")
            out_rows[str(b_std)] = rec
            continue
        ws = Wm.WarmStarter(fam, hidden=W["hidden"], batch=256)
        t0 = time.perf_counter()
        losses = ws.fit(train[ok], Wm.targets(sol)[ok], epochs=args.epochs, lr=1e-3)
        torch.cuda.synchronize()
        rec["train_s"] = time.perf_counter() - t0
        rec["loss_first_last"] = [losses[0], losses[-1]]
        log(f"[warm] trained in {rec['train_s']:.1f}s, loss {losses[0]:.3g} -> {losses[-1]:.3g}")
        rows = Wm.evaluate(fam, ws, held)
        cold_it = np.array([r["cold_iters"] for r in rows])
        warm_it = np.array([r["warm_iters"] for r in rows])
        cold_ms = np.array([r["cold_ms"] for r in rows])
        warm_ms = np.array([r["warm_ms"] for r in rows])
        rec.update({"eval_programs": len(rows),
                    "cold_solved": int(sum(r["cold_status"] == 1 for r in rows)),
                    "warm_solved": int(sum(r["warm_status"] == 1 for r in rows)),
                    "warm_used": int(sum(r["used_warm"] for r in rows)),
                    "cold_mean_iters": float(cold_it.mean()), "warm_mean_iters": float(warm_it.mean()),
                    "cold_mean_ms": float(cold_ms.mean()), "warm_mean_ms": float(warm_ms.mean()),
                    "iters_ratio": float(warm_it.mean() / cold_it.mean()),
                    "time_ratio": float(warm_ms.mean() / cold_ms.mean())})
        log(f"[warm] iterations cold {cold_it.mean():.1f} warm {warm_it.mean():.1f}; "
            f"ms cold {cold_ms.mean():.2f} warm {warm_ms.mean():.2f}")
        out_rows[str(b_std)] = rec
    main_rec = out_rows.get(str(args.b_std[-1]), {})
    out = {"metric": METRIC, "value": main_rec.get("warm_mean_ms"), "unit": "ms to eps=1e-4 per program (warm)",
           "n_gpus": 1, "steps": 1, "warmup": 0, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64 solve, f32 network",
           "data": "synthetic parametric SOCP family",
           "config": {"workload": "learned warm start: fixed A (n=2000, m=6000, density 5e-3), "
                                  "b(theta)=b0+B theta, theta~N(0,I_64); MLP 64-512-512-8001",
                      "train": args.train_size, "eval": args.eval_size},
           "families": out_rows}
    return out


def socp_record(args):
    """The headline workload: the random SOCP n = 10^4, m = 3*10^4."""
    import torch
    import paper_1312_3039_amd as hsd
    from datagen import draw_socp

    W = WORKLOAD
    draw = draw_socp(W["seed"], n=W["n"], m=W["m"], nonneg=W["nonneg"], soc_lo=W["soc_lo"],
                     soc_hi=W["soc_hi"], density=W["density"])
    Ad, bd, cd, cone, pstar = gpu_instance(torch, hsd, draw)
    eps = dict(eps_pri=W["eps"], eps_dual=W["eps"], eps_gap=W["eps"])
    shape = {}
    untuned = None
    if args.shape is not None:
        shape = json.loads(args.shape)
        log(f"[gpu] launch shape {shape} (given)")
    elif not args.no_tune:
        import scipy.sparse as sp
        from paper_1312_3039_amd import autotune
        t0 = time.perf_counter()
        A_host = sp.csr_matrix((draw.data, draw.indices, draw.indptr), shape=(draw.m, draw.n))
        shape = autotune.tune_solver(A_host, bd, cd, cone, **eps)
        log(f"[gpu] launch shape {shape} ({time.perf_counter() - t0:.1f}s, cached per device)")
        wall_d, inf_d = run_gpu(torch, hsd, Ad, bd, cd, cone, args.steps, args.warmup, precision=0, **eps)
        untuned = summarize(wall_d, inf_d, draw.m, draw.n, draw.nnz, False, pstar)
        log(f"[gpu] FP64 automatic shape: {untuned['time_to_eps_ms']:.2f} ms to eps")
    log(f"[gpu] FP64: {args.warmup} warmup + {args.steps} timed solves, m={draw.m} n={draw.n} nnz={draw.nnz}")
    wall64, inf64 = run_gpu(torch, hsd, Ad, bd, cd, cone, args.steps, args.warmup, precision=0,
                            **eps, **shape)
    r64 = summarize(wall64, inf64, draw.m, draw.n, draw.nnz, False, pstar)
    log(f"[gpu] FP64 done: {r64['iters']} iters, {r64['time_to_eps_ms']:.2f} ms to eps")
    log(f"[gpu] FP32-SpMV/CG: {args.warmup} warmup + {args.steps} timed solves")
    wall32, inf32 = run_gpu(torch, hsd, Ad, bd, cd, cone, args.steps, args.warmup, precision=1,
                            **eps, **shape)
    r32 = summarize(wall32, inf32, draw.m, draw.n, draw.nnz, True, pstar)
    log(f"[gpu] FP32 done: {r32['iters']} iters, {r32['time_to_eps_ms']:.2f} ms to eps")
    # the direct projection (dense G^{-1} applied per update; exact
    # projections, so fewer updates than with CG's inexact ones)
    nd = max(1, min(args.steps, 5))
    log(f"[gpu] FP64 direct projection: 1 warmup + {nd} timed solves")
    # (the library's automatic team for this path: one workgroup per CU)
    walld, infd = run_gpu(torch, hsd, Ad, bd, cd, cone, nd, 1, precision=0, linsys=1, **eps,
                          **{k: v for k, v in shape.items() if k not in ("slab_cols", "team_blocks")})
    rd = summarize(walld, infd, draw.m, draw.n, draw.nnz, False, pstar)
    zb = 8.0 * draw.n * draw.n * rd["iters"]
    rd["z_bytes_per_launch"] = zb
    rd["z_gbs"] = zb / (rd["kernel_ms"] * 1e-3) / 1e9
    rd["note"] = ("Z = (I + A^T A)^{-1} formed at setup (dense Cholesky and inverse); each update "
                  "reads Z once (8 n^2 bytes); z_gbs = those bytes over the solve kernel's time")
    log(f"[gpu] direct done: {rd['iters']} iters, {rd['time_to_eps_ms']:.2f} ms to eps "
        f"(setup {rd['setup_ms']:.1f} ms), Z read at {rd['z_gbs']:.0f} GB/s")
    t = TRAFFIC_FP64
    out = {
        "metric": METRIC,
        "value": r64["value"],
        "unit": "ADMM iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded random feasible SOCP with known optimal value)",
        "config": {"workload": "random SOCP n=10000 m=30000 (5000 nonneg + SOC sizes U[3,50]), "
                               "density 1e-3 (300k nnz), eps=1e-4, cold start, setup included",
                   "n": draw.n, "m": draw.m, "nnz": draw.nnz, "n_soc": len(draw.cone.q),
                   "seed": W["seed"], "global_batch": 1, "parallelism": "single GPU"},
        "time_to_eps_ms": r64["time_to_eps_ms"],
        "launch_shape": shape or "automatic",
        "fp64": r64,
        "fp64_automatic_shape": untuned,
        "fp32_spmv": r32,
        "fp64_direct": rd,
        "roofline": roofline("latency", r64, "k_solve<double, false, 0> (persistent cooperative solve)",
                             traffic=measured_traffic(shape),
                             traffic_source={"profiles": [t["fetch_profile"], t["write_profile"]],
                                             "kernel_src_hash": t["src_hash"],
                                             "current_src_hash": kernel_src_hash("single")},
                             note="a chain of about 2.9 dependent team-barrier phases per ADMM "
                                  "iteration over a cache-resident working set (about 10 MB); the "
                                  "fraction of the HBM peak is reported for reference"),
    }
    if not args.no_cpu:
        log(f"[cpu] oracle baseline on {args.cpu_seeds} seeds")

        def make(sd):
            from oracle.instances import from_draw
            return from_draw(draw_socp(sd, n=W["n"], m=W["m"], nonneg=W["nonneg"], soc_lo=W["soc_lo"],
                                       soc_hi=W["soc_hi"], density=W["density"]))
        cb = cpu_baseline(range(args.cpu_seeds), make, "socp")
        out["cpu_baseline"] = cb
        o = cb["oracle"][0]
        for rec in (r64, r32):
            rec["obj_rel_err_vs_oracle"] = abs(rec["obj"] - o["obj"]) / max(1.0, abs(o["obj"]))
            rec["iters_vs_oracle"] = rec["iters"] - o["iters"]
    return out


def lp_record(args):
    """The random LP: n = 100, m = 300, nonnegative cone, density 0.1."""
    import torch
    import paper_1312_3039_amd as hsd
    from datagen import draw_lp
    draw = draw_lp(0)
    Ad, bd, cd, cone, pstar = gpu_instance(torch, hsd, draw)
    steps, warm = max(args.steps, 20), 3
    wall, infos = run_gpu(torch, hsd, Ad, bd, cd, cone, steps, warm)
    r = summarize(wall, infos, draw.m, draw.n, draw.nnz, False, pstar)
    log(f"[lp] {r['iters']} iters, {r['time_to_eps_ms']:.2f} ms to eps")
    out = {"workload": "random LP n=100 m=300, nonneg cone, density 0.1, eps=1e-4, setup included",
           "value": r["value"], "unit": "ADMM iters/s", "steps": steps, "fp64": r,
           "roofline": roofline("latency", r, "k_solve<double, false, 0> (persistent cooperative solve)",
                                note="80 KB working set; one workgroup's dependent chain")}
    if not args.no_cpu:
        from oracle.instances import from_draw
        cb = cpu_baseline(range(3), lambda sd: from_draw(draw_lp(sd)), "lp")
        out["cpu_baseline"] = cb
        r["obj_rel_err_vs_oracle"] = abs(r["obj"] - cb["oracle"][0]["obj"]) / max(1.0, abs(cb["oracle"][0]["obj"]))
    return out


def mixed_record(args):
    """The mixed-cone program: n = 5,000; 2,000 nonnegative rows, 400 SOCs
    in [3, 30], 60 PSD cones of side in [8, 40], 500 exponential triples,
    density 2e-3; FP32 SpMV/CG (the configuration's mode) and FP64."""
    import torch
    import paper_1312_3039_amd as hsd
    from datagen import draw_mixed
    draw = draw_mixed(0)
    Ad, bd, cd, cone, pstar = gpu_instance(torch, hsd, draw)
    steps, warm = 5, 2
    res = {}
    for prec, name in ((1, "fp32_spmv"), (0, "fp64")):
        wall, infos = run_gpu(torch, hsd, Ad, bd, cd, cone, steps, warm, precision=prec)
        res[name] = summarize(wall, infos, draw.m, draw.n, draw.nnz, prec == 1, pstar)
        log(f"[mixed] {name}: {res[name]['iters']} iters, {res[name]['time_to_eps_ms']:.2f} ms to eps")
    # projection time share: a stand-alone projection of the y-block onto K^*
    # per cone family (one grid-wide launch, 20 repetitions), times the
    # iterations, against the solve kernel's time
    share = {}
    rng = np.random.default_rng(1)
    parts = {"psd": {"f": 0, "l": 0, "q": [], "s": list(draw.cone.s), "ep": 0, "ed": 0},
             "exp": {"f": 0, "l": 0, "q": [], "s": [], "ep": draw.cone.ep, "ed": 0},
             "soc_nonneg": {"f": 0, "l": draw.cone.l, "q": list(draw.cone.q), "s": [], "ep": 0, "ed": 0}}
    from datagen import ConeSpec
    for key, sub in parts.items():
        x = torch.as_tensor(rng.standard_normal(ConeSpec(**sub).m), device="cuda")
        hsd.project_cone(sub, x, dual=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            hsd.project_cone(sub, x, dual=True)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 20
        share[key] = {"ms_per_projection": ms,
                      "share_of_fp32_kernel": ms * res["fp32_spmv"]["iters"] / res["fp32_spmv"]["kernel_ms"]}
    out = {"workload": "mixed cones n=5000: 2000 nonneg, 400 SOC U[3,30], 60 PSD sides U[8,40] "
                       "(scaled svec), 500 exp triples, density 2e-3, eps=1e-4, setup included",
           "m": draw.m, "n": draw.n, "nnz": draw.nnz,
           "value": res["fp32_spmv"]["value"], "unit": "ADMM iters/s", "steps": steps,
           "fp32_spmv": res["fp32_spmv"], "fp64": res["fp64"],
           "projection_time_share_estimate": share,
           "projection_note": "stand-alone projections start cold; inside the solve the PSD "
                              "projections start from the previous update's eigenvectors, so "
                              "a PSD share above 1 is the gain of that warm start",
           "roofline": roofline("latency", res["fp32_spmv"],
                                "k_solve<float, false, 1> (persistent cooperative solve, general kernel: warm-started PSD projections)",
                                note="cache-resident working set; PSD projections by one "
                                     "workgroup each are on the critical path")}
    if not args.no_cpu:
        from oracle.instances import from_draw
        cb = cpu_baseline(range(1), lambda sd: from_draw(draw_mixed(sd)), "mixed")
        out["cpu_baseline"] = cb
        o = cb["oracle"][0]
        for rec in res.values():
            rec["obj_rel_err_vs_oracle"] = abs(rec["obj"] - o["obj"]) / max(1.0, abs(o["obj"]))
            rec["iters_vs_oracle"] = rec["iters"] - o["iters"]
    return out


def _guarded(name, fn, args):
    """Run one extra workload; a failure is recorded instead of ending the run."""
    t0 = time.perf_counter()
    try:
        rec = fn(args)
    except Exception as e:  # noqa: BLE001 -- reported in the JSON line
        log(f"[{name}] failed: {type(e).__name__}: {e}")
        return {"error": f"{type(e).__name__}: {e}"}
    rec["bench_wall_s"] = time.perf_counter() - t0
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="the headline workload only")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--shape", default=None,
                    help="launch shape as JSON settings (skips the autotuner)")
    ap.add_argument("--cpu-seeds", type=int, default=3)
    ap.add_argument("--workload", choices=["socp", "lp", "mixed", "batch", "warmstart", "large", "paper"],
                    default="socp")
    ap.add_argument("--paper-sizes", nargs="+", default=["S", "M"], choices=["S", "M"],
                    help="paper: the random SOCP sizes to run")
    ap.add_argument("--cpu-iters", type=int, default=3, help="large: oracle iterations timed")
    ap.add_argument("--train-size", type=int, default=WARM["train"])
    ap.add_argument("--eval-size", type=int, default=WARM["eval"])
    ap.add_argument("--cert-eval-size", type=int, default=50,
                    help="held-out programs of a family that ends in certificates")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--cert-train", type=int, default=8192,
                    help="training programs of a family that ends in certificates (warm start on q)")
    ap.add_argument("--b-std", type=float, nargs="+", default=[0.1, 0.01])
    ap.add_argument("--batch-size", type=int, default=BATCH["B"])
    ap.add_argument("--seq-sample", type=int, default=64)
    ap.add_argument("--cpu-programs", type=int, default=32)
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (3 times): the "
                         "reference dispatch for scaling hardware traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(this build solves on a single MI355X)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calib:
        nb = args.copy_calib * (1 << 20)
        src = torch.empty(nb // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[calib] copied {args.copy_calib} MiB three times (reads {nb} B, writes {nb} B each)")
    single = {"lp": lp_record, "mixed": mixed_record, "batch": run_batch,
              "warmstart": run_warmstart, "large": run_large, "paper": run_paper}
    if args.workload != "socp":
        print(json.dumps(single[args.workload](args)), flush=True)
        return
    out = socp_record(args)
    if not args.quick:
        out["workloads"] = {}
        for name, fn in (("lp_n100", lp_record), ("mixed_cones", mixed_record),
                         ("batch_4096", run_batch), ("large_socp_1e8", run_large),
                         ("warmstart", run_warmstart)):
            log(f"[bench] workload {name}")
            out["workloads"][name] = _guarded(name, fn, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
