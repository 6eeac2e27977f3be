// Host-side helpers shared by the single-program and batched runtimes:
// error reporting, cone description, launch-shape helpers and the device
// exclusive scan used by the transpose.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/hsd.h"
#include "hsd_setup_kernels.h"

namespace hsd {

constexpr int MAX_TEAM = 2048;
constexpr size_t ALIGN = 256;

inline thread_local std::string g_err;

inline int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(HSD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

// ---------------------------------------------------------------------------
// host-side cone description
// ---------------------------------------------------------------------------

struct HostCone {
    int32_t f = 0, l = 0;
    std::vector<int32_t> soc_off, soc_len, psd_off, psd_dim;
    int32_t nexp = 0, exp_off = 0, nexpd = 0, expd_off = 0, max_psd = 0;
    int32_t npow = 0, pow_off = 0;
    std::vector<double> pow_a;  // power-cone parameters (sign marks the dual)
    // non-separable blocks for the scaling rule: (offset, length)
    std::vector<int32_t> blk_off, blk_len;
    int64_t m = 0;
};

inline int build_cone(const hsd_cone_t *K, HostCone &hc) {
    if (!K) return fail(HSD_ERR_ARG, "cone description is null");
    if (K->f < 0 || K->l < 0 || K->nq < 0 || K->ns < 0 || K->ep < 0 || K->ed < 0 || K->np < 0)
        return fail(HSD_ERR_CONE, "negative cone count");
    if ((K->nq > 0 && !K->q) || (K->ns > 0 && !K->s) || (K->np > 0 && !K->p))
        return fail(HSD_ERR_ARG, "cone size array is null");
    int64_t pos = 0;
    hc.f = (int32_t)K->f;
    pos += K->f;
    hc.l = (int32_t)K->l;
    pos += K->l;
    for (int i = 0; i < K->nq; ++i) {
        if (K->q[i] < 1) return fail(HSD_ERR_CONE, "second-order cone of size < 1");
        hc.soc_off.push_back((int32_t)pos);
        hc.soc_len.push_back(K->q[i]);
        hc.blk_off.push_back((int32_t)pos);
        hc.blk_len.push_back(K->q[i]);
        pos += K->q[i];
    }
    for (int i = 0; i < K->ns; ++i) {
        const int d = K->s[i];
        if (d < 1) return fail(HSD_ERR_CONE, "PSD cone of side < 1");
        if (d > 90) return fail(HSD_ERR_CONE, "PSD cone side above 90 is not supported");
        const int L = d * (d + 1) / 2;
        hc.psd_off.push_back((int32_t)pos);
        hc.psd_dim.push_back(d);
        hc.blk_off.push_back((int32_t)pos);
        hc.blk_len.push_back(L);
        hc.max_psd = std::max(hc.max_psd, d);
        pos += L;
    }
    hc.nexp = (int32_t)K->ep;
    hc.exp_off = (int32_t)pos;
    for (int64_t i = 0; i < K->ep; ++i) {
        hc.blk_off.push_back((int32_t)pos);
        hc.blk_len.push_back(3);
        pos += 3;
    }
    hc.nexpd = (int32_t)K->ed;
    hc.expd_off = (int32_t)pos;
    for (int64_t i = 0; i < K->ed; ++i) {
        hc.blk_off.push_back((int32_t)pos);
        hc.blk_len.push_back(3);
        pos += 3;
    }
    hc.npow = K->np;
    hc.pow_off = (int32_t)pos;
    for (int32_t i = 0; i < K->np; ++i) {
        const double a = K->p[i];
        if (!(a >= -1.0 && a <= 1.0)) return fail(HSD_ERR_CONE, "power-cone parameter outside [-1, 1]");
        hc.pow_a.push_back(a);
        hc.blk_off.push_back((int32_t)pos);
        hc.blk_len.push_back(3);
        pos += 3;
    }
    hc.m = pos;
    if (pos >= (int64_t)INT32_MAX) return fail(HSD_ERR_CONE, "cone dimension too large");
    return HSD_OK;
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------

inline int grid_for(int64_t work, int threads, int cap = 4096) {
    int64_t g = (work + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// Sorts the entries of every row of a CSR matrix by column (a deterministic
// order for the transpose built with atomic counters): rows of up to 256
// entries by one wavefront each, rows of up to LONG_SORT_CAP entries by one
// workgroup each (bitonic network in LDS), longer rows by one lane.  max_len
// is an upper bound on the row length.
constexpr int LONG_SORT_CAP = 8192;
inline int sort_rows(int32_t rows, const int32_t *rp, int32_t *ci, double *v, int64_t max_len,
                     hipStream_t s) {
    int32_t cap = 0;
    if (max_len > 256) {
        cap = (int32_t)std::min<int64_t>(max_len, LONG_SORT_CAP);
        int P = 512;
        while (P < cap) P <<= 1;
        const size_t lds = 12 * (size_t)P;
        if (lds > 65536)
            HIP_TRY(hipFuncSetAttribute((const void *)k_sort_rows_long,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(k_sort_rows_long, dim3(grid_for(rows, 1, 4096)), dim3(256), lds, s, rows, rp, ci, v,
                           cap);
    }
    hipLaunchKernelGGL(k_sort_rows, dim3(grid_for(rows, 4)), dim3(256), 0, s, rows, rp, ci, v, cap);
    HIP_TRY(hipGetLastError());
    return HSD_OK;
}

inline int pow2_floor(double x, int lo, int hi) {
    int p = 1;
    while (p * 2 <= x && p * 2 <= hi) p *= 2;
    return std::max(lo, std::min(hi, p));
}

inline bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// Exclusive scan of len ints from `in` to `out` (may alias); scratch from ws.
inline int scan_exclusive(const int32_t *in, int32_t *out, int64_t len, int32_t *scratch,
                          hipStream_t st) {
    const int64_t tiles = (len + 1023) / 1024;
    int32_t *sums = scratch;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(1024), 0, st, in, out, len, sums);
    HIP_TRY(hipGetLastError());
    if (tiles > 1) {
        int rc = scan_exclusive(sums, sums, tiles, scratch + tiles + 1, st);
        if (rc) return rc;
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(1024), 0, st, out, len,
                           (const int32_t *)sums);
        HIP_TRY(hipGetLastError());
    }
    return HSD_OK;
}

inline int check_settings(const hsd_settings_t *st) {
    if (!st) return fail(HSD_ERR_ARG, "settings are null");
    if (!(st->alpha > 0.0 && st->alpha < 2.0)) return fail(HSD_ERR_ARG, "alpha must lie in (0, 2)");
    if (st->cg_max_iters < 1 || st->max_iters < 0 || st->check_every < 1)
        return fail(HSD_ERR_ARG, "iteration limits must be positive");
    if (st->precision != 0 && st->precision != 1) return fail(HSD_ERR_ARG, "precision must be 0 or 1");
    if (st->team_blocks < 0 || st->team_blocks > MAX_TEAM)
        return fail(HSD_ERR_ARG, "team_blocks out of range");
    if (st->block_threads != 0 &&
        (st->block_threads < 64 || st->block_threads > 512 || st->block_threads % 64))
        return fail(HSD_ERR_ARG, "block_threads must be a multiple of 64 in [64, 512]");
    for (int L : {st->lanes_a, st->lanes_at, st->lanes_soc})
        if (L != 0 && (!is_pow2(L) || L > 64)) return fail(HSD_ERR_ARG, "lanes must be a power of two <= 64");
    if (st->lds_matrix != 0 && st->lds_matrix != 1) return fail(HSD_ERR_ARG, "lds_matrix must be 0 or 1");
    if (st->batch_vectors != 0 && st->batch_vectors != 1) return fail(HSD_ERR_ARG, "batch_vectors must be 0 or 1");
    if (st->batch_matrix != 0 && st->batch_matrix != 1) return fail(HSD_ERR_ARG, "batch_matrix must be 0 or 1");
    if (st->slab_cols < -1) return fail(HSD_ERR_ARG, "slab_cols must be -1, 0 or positive");
    if (st->linsys != 0 && st->linsys != 1) return fail(HSD_ERR_ARG, "linsys must be 0 or 1");
    if (st->linsys == 1 && st->precision != 0)
        return fail(HSD_ERR_ARG, "the direct projection (linsys 1) runs in FP64 only (precision 0)");
    if (st->linsys == 1 && st->slab_cols > 0)
        return fail(HSD_ERR_ARG, "the direct projection (linsys 1) runs with row-group sweeps (slab_cols <= 0)");
    return HSD_OK;
}

// Largest n of the direct projection (its dense factor and inverse take
// 2 * 8 * NP^2 bytes with NP = n rounded up to 64).
constexpr int32_t DIRECT_MAX_N = 32768;

// Column slabs of the sparse products (see hsd_settings_t::slab_cols):
// slab width and the slab counts of A (over its n columns) and of A^T (over
// its m columns); a count of 1 means no slabs.
constexpr int32_t SLAB_AUTO_COLS = 131072;
constexpr int32_t SLAB_CHUNK_ROWS = 1024;  // rows per chunk of a slab sweep
struct SlabPlan {
    int32_t width = SLAB_AUTO_COLS, ka = 1, kt = 1;
    bool stream = false;  // block-streamed sweeps for both products
    // A side with one slab reads the row-major matrix with its row
    // pointers as the offsets; a side with several reads a slab-major copy.
    bool on() const { return stream; }
};
inline SlabPlan slab_plan(const hsd_settings_t *st, int64_t m, int64_t n) {
    SlabPlan p;
    // the direct projection runs with row-group sweeps (its n is small)
    if (st->slab_cols < 0 || st->linsys == 1) return p;
    if (st->slab_cols > 0) {
        p.width = st->slab_cols;
        p.ka = (int32_t)((n + p.width - 1) / p.width);
        p.kt = (int32_t)((m + p.width - 1) / p.width);
        p.stream = true;
    } else {
        if (n > 2 * (int64_t)p.width) p.ka = (int32_t)((n + p.width - 1) / p.width);
        if (m > 2 * (int64_t)p.width) p.kt = (int32_t)((m + p.width - 1) / p.width);
        p.stream = p.ka > 1 || p.kt > 1;
    }
    return p;
}

}  // namespace hsd
