// Setup kernels: input validation, transpose of A on the device,
// equilibration (Sect. 5, rule in the design notes), scaled data, norms,
// row partitions and start states.  Launched once per setup; none of them
// is on the per-iteration path.
#pragma once

#include "hsd_solver.h"

namespace hsd {

// ---- generic single-workgroup reductions ---------------------------------

// Count of non-finite values in x[0..n) added to *flag.
static __global__ void k_count_nonfinite(const double *x, int64_t n, unsigned *flag) {
    unsigned c = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        c += isfinite(x[i]) ? 0u : 1u;
    c = group_sum(c, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0 && c) atomicAdd(flag, c);
}

// Counts structural errors of a CSR matrix into *flag: row pointers that
// decrease or leave [0, nnz], and column indices outside [0, n).  Run before
// any kernel indexes with them.
static __global__ void k_validate_csr(int32_t m, int32_t n, int64_t nnz, const int32_t *rp,
                               const int32_t *ci, unsigned *flag) {
    unsigned bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride) {
        const int32_t a = rp[i], b = rp[i + 1];
        if (a < 0 || b < a || (int64_t)b > nnz) ++bad;
    }
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz; k += stride) {
        const int32_t j = ci[k];
        if (j < 0 || j >= n) ++bad;
    }
    bad = group_sum(bad, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0 && bad) atomicAdd(flag, bad);
}

template <typename T>
static __global__ void k_fill(T *x, int64_t n, T val) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = val;
}

// ---- transpose: count, scan, scatter, sort ------------------------------

// Entries per column; indices outside [0, n) are skipped (the input checks
// reject them).
static __global__ void k_count_cols(const int32_t *ci, int64_t nnz, int32_t n, int32_t *cnt) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = ci[k];
        if (j >= 0 && j < n) atomicAdd(&cnt[j], 1);
    }
}

// out = max(out, max_i (rp[i+1] - rp[i])) over i in [0, rows), negative
// differences (rejected by the input checks) counted as 0.
static __global__ void k_max_diff(const int32_t *rp, int32_t rows, unsigned *out) {
    unsigned mx = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = (int64_t)rp[i + 1] - rp[i];
        if (d > (int64_t)mx) mx = (unsigned)d;
    }
    if (mx) atomicMax(out, mx);
}

// out = max(out, max_i a[i]) over i in [0, len) (nonnegative values).
static __global__ void k_max_value(const int32_t *a, int32_t len, unsigned *out) {
    unsigned mx = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        if (a[i] > 0 && (unsigned)a[i] > mx) mx = (unsigned)a[i];
    if (mx) atomicMax(out, mx);
}

// Exclusive scan of tiles of 1024 ints (one workgroup of 1024 threads per
// tile); tile totals go to sums.
static __global__ void __launch_bounds__(1024) k_scan_tiles(const int32_t *in, int32_t *out, int64_t n,
                                                     int32_t *sums) {
    __shared__ int32_t wsum[MAX_WAVES];
    const int64_t i = blockIdx.x * 1024LL + threadIdx.x;
    int32_t v = i < n ? in[i] : 0;
    // inclusive scan within the wave
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        int32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    if (wid == 0) {
        int32_t w = lane < 16 ? wsum[lane] : 0;
        for (int off = 1; off < 16; off <<= 1) {
            int32_t y = __shfl_up(w, off, 64);
            if (lane >= off) w += y;
        }
        if (lane < 16) wsum[lane] = w;
    }
    __syncthreads();
    const int32_t before = wid > 0 ? wsum[wid - 1] : 0;
    if (i < n) out[i] = before + x - v;
    if (threadIdx.x == 1023) sums[blockIdx.x] = before + x;
}

static __global__ void k_scan_add(int32_t *out, int64_t n, const int32_t *offs) {
    const int64_t i = blockIdx.x * 1024LL + threadIdx.x;
    if (i < n) out[i] += offs[blockIdx.x];
}

// Place every nonzero (i, j) of A into row j of A^T (slot order arbitrary).
static __global__ void k_scatter_t(int32_t m, const int32_t *rp, const int32_t *ci, const double *v,
                            const int32_t *rpt, int32_t *fill, int32_t *cit, double *vt) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            const int j = ci[k];
            const int pos = rpt[j] + atomicAdd(&fill[j], 1);
            cit[pos] = i;
            vt[pos] = v[k];
        }
    }
}

// Sort each row of A^T by column (= row of A) so that the transpose, and
// every sum over it, is the same on every run.  One wavefront per row: the
// keys of a row are distinct, so each element's place is the number of
// smaller keys in its row; up to 4 elements per lane are ranked in
// registers and then written.  Rows longer than 256 are sorted by one lane.
static __global__ void k_sort_rows(int32_t rows, const int32_t *rp, int32_t *ci, double *v,
                                   int32_t long_cap = 0) {
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x / 64;
    for (int r = blockIdx.x * wpb + threadIdx.x / 64; r < rows; r += gridDim.x * wpb) {
        const int b = rp[r], e = rp[r + 1], len = e - b;
        if (len > 256 && len <= long_cap) continue;  // k_sort_rows_long's rows
        if (len <= 256) {
            int key[4], rank[4];
            double val[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = b + lane + 64 * q;
                key[q] = k < e ? ci[k] : 0;
                val[q] = k < e ? v[k] : 0.0;
                rank[q] = 0;
            }
            for (int f = b; f < e; ++f) {
                const int kf = ci[f];
#pragma unroll
                for (int q = 0; q < 4; ++q) rank[q] += (kf < key[q]) ? 1 : 0;
            }
            // every lane has read its keys and counted before anyone writes
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (lane + 64 * q < len) {
                    ci[b + rank[q]] = key[q];
                    v[b + rank[q]] = val[q];
                }
            }
            continue;
        }
        if (lane != 0) continue;
        for (int k = b + 1; k < e; ++k) {
            const int key = ci[k];
            const double val = v[k];
            int q = k - 1;
            while (q >= b && ci[q] > key) {
                ci[q + 1] = ci[q];
                v[q + 1] = v[q];
                --q;
            }
            ci[q + 1] = key;
            v[q + 1] = val;
        }
    }
}

// Rows with 256 < length <= cap: one workgroup per row sorts its (column,
// value) pairs in LDS with a bitonic network over the next power of two P
// (padded with INT32_MAX keys; the columns of a row are distinct, so the
// order is unique).  Dynamic LDS: P doubles, then P ints, P >= cap.
static __global__ void __launch_bounds__(256) k_sort_rows_long(int32_t rows, const int32_t *rp, int32_t *ci,
                                                               double *v, int32_t cap) {
    extern __shared__ double sh_sort[];
    int P = 512;
    while (P < cap) P <<= 1;
    double *sv = sh_sort;
    int32_t *sk = reinterpret_cast<int32_t *>(sh_sort + P);
    for (int r = blockIdx.x; r < rows; r += gridDim.x) {
        const int b = rp[r], e = rp[r + 1], len = e - b;
        if (len <= 256 || len > cap) continue;
        int Q = 512;
        while (Q < len) Q <<= 1;
        for (int k = threadIdx.x; k < Q; k += blockDim.x) {
            sk[k] = k < len ? ci[b + k] : INT32_MAX;
            sv[k] = k < len ? v[b + k] : 0.0;
        }
        __syncthreads();
        for (int size = 2; size <= Q; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = threadIdx.x; t < Q / 2; t += blockDim.x) {
                    const int lo = 2 * t - (t & (stride - 1));
                    const int hi = lo + stride;
                    const bool up = (lo & size) == 0;
                    const int klo = sk[lo], khi = sk[hi];
                    if ((klo > khi) == up) {
                        sk[lo] = khi;
                        sk[hi] = klo;
                        const double tv = sv[lo];
                        sv[lo] = sv[hi];
                        sv[hi] = tv;
                    }
                }
                __syncthreads();
            }
        }
        for (int k = threadIdx.x; k < len; k += blockDim.x) {
            ci[b + k] = sk[k];
            v[b + k] = sv[k];
        }
        __syncthreads();
    }
}

// ---- equilibration ---------------------------------------------------------

// out_r = Drow_r * sqrt(sum_k a_rk^2 Ecol_k^2): the row norms of
// diag(Drow) A diag(Ecol) for a CSR matrix (rows of A, or rows of A^T with
// the roles of the two scalings exchanged).  One wavefront per row.
static __global__ void k_scaled_row_norms(int32_t rows, const int32_t *rp, const int32_t *ci,
                                   const double *v, const double *Drow, const double *Ecol,
                                   double *out) {
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x / 64;
    for (int r = blockIdx.x * wpb + threadIdx.x / 64; r < rows; r += gridDim.x * wpb) {
        double s = 0.0;
        for (int k = rp[r] + lane; k < rp[r + 1]; k += 64) {
            const double a = v[k] * Ecol[ci[k]];
            s += a * a;
        }
        s = group_sum(s, 64);
        if (lane == 0) out[r] = Drow[r] * sqrt(s);
    }
}

// d_r = 1/sqrt(norm_r) (1 where norm_r = 0), written over `norm`.
static __global__ void k_inv_sqrt(double *norm, int32_t rows) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
        const double x = norm[r];
        norm[r] = x > 0.0 ? 1.0 / sqrt(x) : 1.0;
    }
}

// Replace d on every non-separable block (second-order, PSD, exponential)
// by its block mean: one wavefront per block.  Blocks are listed as
// (offset, length) pairs in blk.
static __global__ void k_block_mean(double *d, int32_t nblk, const int32_t *blk_off,
                             const int32_t *blk_len) {
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x / 64;
    for (int b = blockIdx.x * wpb + threadIdx.x / 64; b < nblk; b += gridDim.x * wpb) {
        const int off = blk_off[b], len = blk_len[b];
        double s = 0.0;
        for (int e = lane; e < len; e += 64) s += d[off + e];
        s = group_sum(s, 64);
        const double mean = s / (double)len;
        for (int e = lane; e < len; e += 64) d[off + e] = mean;
    }
}

// S_r *= clip(d_r, lo, hi)
static __global__ void k_mul_clip(double *S, const double *d, int32_t rows, double lo, double hi) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
        double x = d[r];
        x = x < lo ? lo : (x > hi ? hi : x);
        S[r] *= x;
    }
}

// sigma = 1/max(|D b|, tiny); rho = mean(rownorm)/max(|E c|, tiny); also
// |b|, |c|.  Single workgroup.
static __global__ void k_sigma_rho(const double *b, const double *D, int32_t m, const double *c,
                            const double *E, int32_t n, const double *rownorm, int scale_on,
                            double *scal) {
    __shared__ double red[4 * MAX_WAVES];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // |Db|^2, |Ec|^2, sum rownorm, |b|^2 ; |c|^2 below
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double db = D[i] * b[i];
        acc[0] += db * db;
        acc[2] += rownorm[i];
        acc[3] += b[i] * b[i];
    }
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double ec = E[j] * c[j];
        acc[1] += ec * ec;
    }
    block_sum<4>(acc, red);
    double cc[1] = {0.0};
    for (int j = threadIdx.x; j < n; j += blockDim.x) cc[0] += c[j] * c[j];
    block_sum<1>(cc, red);
    if (threadIdx.x == 0) {
        const double tiny = 1e-8;
        if (scale_on) {
            scal[SC_SIGMA] = 1.0 / fmax(sqrt(acc[0]), tiny);
            // mean row norm of the scaled A; 1 when A has no nonzeros
            double rbar = m > 0 ? acc[2] / (double)m : 1.0;
            if (!(rbar > 0.0)) rbar = 1.0;
            scal[SC_RHO] = rbar / fmax(sqrt(acc[1]), tiny);
            scal[SC_RBAR] = rbar;
        } else {
            scal[SC_SIGMA] = 1.0;
            scal[SC_RHO] = 1.0;
            scal[SC_RBAR] = 1.0;
        }
        scal[SC_NORM_B] = sqrt(acc[3]);
        scal[SC_NORM_C] = sqrt(cc[0]);
    }
}

// Scaled values A_hat = D A E on a CSR array.  For the rows of A
// (TRANSPOSED = false) entry (i, j) becomes (D_i a_ij) E_j with Drow = D,
// Ecol = E; for the rows of A^T (TRANSPOSED = true, Drow = E, Ecol = D) the
// same product is formed in the same order, so both arrays hold identical
// values.  Optional FP32 copy.
template <bool TRANSPOSED>
static __global__ void k_scale_values(int32_t rows, const int32_t *rp, const int32_t *ci, double *v,
                               const double *Drow, const double *Ecol, float *v32) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
        const double dr = Drow[r];
        for (int k = rp[r]; k < rp[r + 1]; ++k) {
            const double ec = Ecol[ci[k]];
            const double x = TRANSPOSED ? (ec * v[k]) * dr : (dr * v[k]) * ec;
            v[k] = x;
            if (v32) v32[k] = (float)x;
        }
    }
}

// b_hat = sigma D b, c_hat = rho E c, and |D^{-1} b_hat|, |E^{-1} c_hat|
// (single workgroup for the norms).
static __global__ void k_scale_rhs(const double *b, const double *c, const double *D, const double *E,
                            int32_t m, int32_t n, double *bh, double *ch, double *scal) {
    __shared__ double red[2 * MAX_WAVES];
    const double sigma = scal[SC_SIGMA], rho = scal[SC_RHO];
    double acc[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double x = sigma * D[i] * b[i];
        bh[i] = x;
        const double y = x / D[i];
        acc[0] += y * y;
    }
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double x = rho * E[j] * c[j];
        ch[j] = x;
        const double y = x / E[j];
        acc[1] += y * y;
    }
    block_sum<2>(acc, red);
    if (threadIdx.x == 0) {
        scal[SC_NORM_DINV_BH] = sqrt(acc[0]);
        scal[SC_NORM_EINV_CH] = sqrt(acc[1]);
    }
}

// New right-hand side b with the same A, c and scaling: sigma, b_hat,
// |b| and |D^{-1} b_hat| (single workgroup).
static __global__ void k_update_b(const double *b, const double *D, int32_t m, int scale_on,
                                  double *bh, double *scal) {
    __shared__ double red[2 * MAX_WAVES];
    double acc[2] = {0.0, 0.0};  // |D b|^2, |b|^2
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double db = D[i] * b[i];
        acc[0] += db * db;
        acc[1] += b[i] * b[i];
    }
    block_sum<2>(acc, red);
    const double sigma = scale_on ? 1.0 / fmax(sqrt(acc[0]), 1e-8) : 1.0;
    double nrm[1] = {0.0};
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double x = sigma * D[i] * b[i];
        bh[i] = x;
        const double y = x / D[i];
        nrm[0] += y * y;
    }
    block_sum<1>(nrm, red);
    if (threadIdx.x == 0) {
        scal[SC_SIGMA] = sigma;
        scal[SC_NORM_B] = sqrt(acc[1]);
        scal[SC_NORM_DINV_BH] = sqrt(nrm[0]);
    }
}

// New cost vector c with the same A and scaling: rho = rbar / max(|E c|,
// tiny) with the mean row norm rbar of A_hat kept from setup, c_hat,
// |c| and |E^{-1} c_hat| (single workgroup).
static __global__ void k_update_c(const double *c, const double *E, int32_t n, int scale_on,
                                  double *ch, double *scal) {
    __shared__ double red[2 * MAX_WAVES];
    double acc[2] = {0.0, 0.0};  // |E c|^2, |c|^2
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double ec = E[j] * c[j];
        acc[0] += ec * ec;
        acc[1] += c[j] * c[j];
    }
    block_sum<2>(acc, red);
    const double rho = scale_on ? scal[SC_RBAR] / fmax(sqrt(acc[0]), 1e-8) : 1.0;
    double nrm[1] = {0.0};
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double x = rho * E[j] * c[j];
        ch[j] = x;
        const double y = x / E[j];
        nrm[0] += y * y;
    }
    block_sum<1>(nrm, red);
    if (threadIdx.x == 0) {
        scal[SC_RHO] = rho;
        scal[SC_NORM_C] = sqrt(acc[1]);
        scal[SC_NORM_EINV_CH] = sqrt(nrm[0]);
    }
}

// Type conversion between the FP64 state arrays of the ABI and the
// CG-precision arrays of the workspace.
template <typename To, typename From>
static __global__ void k_cast(const From *in, To *out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (To)in[i];
}

// Largest LDS footprint of one workgroup's matrix slices: values (sv bytes)
// and column indices of its rows of A and A^T plus the row pointers.
static __global__ void k_slice_bytes(const int32_t *rpA, const int32_t *rpT, const int32_t *part_a,
                                     const int32_t *part_t, int parts, int sv, unsigned *out) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < parts; r += gridDim.x * blockDim.x) {
        const int64_t na = rpA[part_a[r + 1]] - rpA[part_a[r]];
        const int64_t nt = rpT[part_t[r + 1]] - rpT[part_t[r]];
        const int64_t rows = (part_a[r + 1] - part_a[r]) + (part_t[r + 1] - part_t[r]) + 2;
        const int64_t bytes = (na + nt) * (sv + 4) + 4 * rows + 64;
        atomicMax(out, (unsigned)(bytes > 0x7fffffff ? 0x7fffffff : bytes));
    }
}

// Row-major slab boundaries: the first entry of every row in each column
// slab (slab s holds the columns [s W, (s+1) W)), off[s * rows + i] for
// s = 0..K, so off[0 * rows + i] = rp[i] and off[K * rows + i] = rp[i + 1].
// The columns of every row must be sorted.
static __global__ void k_slab_offsets(int32_t rows, const int32_t *rp, const int32_t *ci, int32_t K,
                                      int32_t W, int32_t *off) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t kb = rp[i], ke = rp[i + 1];
        int32_t sl = 0;
        off[i] = kb;
        for (int32_t e = kb; e < ke; ++e) {
            const int32_t target = ci[e] / W;
            while (sl < target) {
                ++sl;
                off[(size_t)sl * rows + i] = e;
            }
        }
        while (sl < K) {
            ++sl;
            off[(size_t)sl * rows + i] = ke;
        }
    }
}

// Entries per (slab, row) in slab-major order, cnt[s * rows + i] for s < K,
// from the row-major slab boundaries bnd of k_slab_offsets; cnt[K * rows] = 0
// so that an exclusive scan of K * rows + 1 values ends with the total.
static __global__ void k_slab_counts(int32_t rows, int32_t K, const int32_t *bnd, int32_t *cnt) {
    const int64_t total = (int64_t)K * rows;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q <= total;
         q += (int64_t)gridDim.x * blockDim.x)
        cnt[q] = q < total ? bnd[q + rows] - bnd[q] : 0;
}

// Copy every row's entries of slab s to the slab-major arrays: the entries
// of (slab s, row i) start at off[s * rows + i], so that the entries of one
// slab are contiguous, row after row.  v32 may be null (FP64 mode).
static __global__ void k_slab_scatter(int32_t rows, int32_t K, const int32_t *bnd, const int32_t *off,
                                      const int32_t *ci, const double *v, const float *v32,
                                      int32_t *ci_s, double *v_s, float *v32_s) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int32_t sl = 0; sl < K; ++sl) {
            const int32_t a = bnd[(size_t)sl * rows + i], b = bnd[(size_t)(sl + 1) * rows + i];
            int32_t d = off[(size_t)sl * rows + i];
            for (int32_t e = a; e < b; ++e, ++d) {
                ci_s[d] = ci[e];
                v_s[d] = v[e];
                if (v32) v32_s[d] = v32[e];
            }
        }
    }
}

// nnz-balanced row partition: part[r] = first row whose start is at least
// r * nnz / parts (part[0] = 0, part[parts] = rows).
// With a block table (the non-separable cones: second-order, PSD and
// exponential, in row order) a boundary that falls inside a block is moved
// to the block's first row, so that every cone lies in one part; the map is
// nondecreasing, so the parts stay ordered (some may be empty).
static __global__ void k_partition(const int32_t *rp, int32_t rows, int parts, int32_t *part,
                                   const int32_t *blk_off = nullptr, const int32_t *blk_len = nullptr,
                                   int32_t nblk = 0) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r <= parts; r += gridDim.x * blockDim.x) {
        if (r == 0) { part[0] = 0; continue; }
        if (r == parts) { part[parts] = rows; continue; }
        const int64_t nnz = rp[rows];
        const int64_t target = nnz * r / parts;
        int lo = 0, hi = rows;  // first row i with rp[i] >= target
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((int64_t)rp[mid] >= target) hi = mid; else lo = mid + 1;
        }
        if (nblk > 0) {
            int a = 0, b = nblk;  // first block starting after row lo
            while (a < b) {
                const int mid = (a + b) >> 1;
                if (blk_off[mid] <= lo) a = mid + 1; else b = mid;
            }
            if (a > 0 && lo < blk_off[a - 1] + blk_len[a - 1]) lo = blk_off[a - 1];
        }
        part[r] = lo;
    }
}

// ---- start states ----------------------------------------------------------

// u = v = 0 except u_tau = tau0, v_kappa = kappa0.
static __global__ void k_init_uv(double *u, double *v, int64_t N, double tau0, double kappa0) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        u[i] = (i == N - 1) ? tau0 : 0.0;
        v[i] = (i == N - 1) ? kappa0 : 0.0;
    }
}

// Warm start from (x, y, s) (Sect. 4.2) in scaled variables:
// u = (sigma x / E, rho y / D, 1), v = (0, sigma D s, 0).
static __global__ void k_warm_xys(const double *x, const double *y, const double *s, const double *D,
                           const double *E, const double *scal, int32_t m, int32_t n, double *u,
                           double *v) {
    const double sigma = scal[SC_SIGMA], rho = scal[SC_RHO];
    const int64_t N = (int64_t)n + m + 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < n) { u[i] = sigma * x[i] / E[i]; v[i] = 0.0; }
        else if (i < n + m) { const int64_t r = i - n; u[i] = rho * y[r] / D[r]; v[i] = sigma * D[r] * s[r]; }
        else { u[i] = 1.0; v[i] = 0.0; }
    }
}

// x-block and tau/kappa of the start from q: u_x = q_x, v_r = 0,
// u_tau = max(q_tau, 0), v_kappa = max(-q_tau, 0).
static __global__ void k_q_rest(const double *q, int32_t m, int32_t n, double *u, double *v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x) {
        if (i < n) { u[i] = q[i]; v[i] = 0.0; }
        else {
            const double qt = q[(int64_t)n + m];
            u[(int64_t)n + m] = qt > 0.0 ? qt : 0.0;
            v[(int64_t)n + m] = qt < 0.0 ? -qt : 0.0;
        }
    }
}

// out = Pi(sign * in) onto K (dual = 0) or K^*.  Grid-wide, no barrier.
static __global__ void __launch_bounds__(256) k_project(ConeDev K, int32_t m, const double *in,
                                                 double sign, double *out, int dual, int Ls) {
    extern __shared__ double lds[];
    Team tm{(int)blockIdx.x, (int)gridDim.x, nullptr};
    int64_t a0, a1;
    split_range(m, gridDim.x, blockIdx.x, a0, a1);
    project_y(K, dual != 0, tm, (int)a0, (int)a1, Ls, lds,
              [&](int i) { return sign * in[i]; },
              [&](int i, double p, double a) { out[i] = p; });
}

// ---- outputs (Sect. 2.3 outcomes, Sect. 5 recovery) ------------------------

static __global__ void k_outputs(const double *u, const double *v, const double *D, const double *E,
                          const double *scal, const double *info, int32_t m, int32_t n,
                          double *x, double *y, double *s) {
    const double sigma = scal[SC_SIGMA], rho = scal[SC_RHO];
    const int status = (int)info[INFO_STATUS];
    const double tau = u[(int64_t)n + m];
    const double bty = info[INFO_BTY], ctx = info[INFO_CTX];
    const double qnan = __builtin_nan("");
    const int64_t tot = (int64_t)n + m;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < n) {
            double xv;
            if (status == 4) xv = rho * E[i] * u[i] / (-ctx);
            else if (status == 3 || !(tau > 0.0)) xv = qnan;
            else xv = E[i] * (u[i] / tau) / sigma;
            if (x) x[i] = xv;
        } else {
            const int64_t r = i - n;
            const double uy = u[i], vs = v[i];
            double yv, sv;
            if (status == 3) { yv = sigma * D[r] * uy / (-bty); sv = qnan; }
            else if (status == 4) { yv = qnan; sv = rho * vs / D[r] / (-ctx); }
            else if (tau > 0.0) { yv = D[r] * (uy / tau) / rho; sv = (vs / tau) / D[r] / sigma; }
            else { yv = qnan; sv = qnan; }
            if (y) y[r] = yv;
            if (s) s[r] = sv;
        }
    }
}

}  // namespace hsd
