// The direct subspace projection (Sect. 4.1, direct method with
// factorization caching): the reduced system of e-linsys,
//   (I + A^T A) z_x = r_x - A^T r_y,   z_y = r_y + A z_x,
// is solved exactly with a factorization made once at setup.  Here the
// matrix G = I + A_hat^T A_hat is formed densely on the device, factored
// G = L L^T by a blocked Cholesky, and inverted (L Y = I, then L^T Z = Y),
// so that every iteration applies Z = G^{-1} as one dense product, a
// bandwidth-bound sweep over Z instead of two chains of dependent
// triangular solves.  All matrices are row-major, padded to NP = a multiple
// of TILE rows and columns with an identity block (G_pad = diag(G, I), whose
// factor and inverse are diag(L, I) and diag(G^{-1}, I)), so every tile is
// full.  Every sum is taken in a fixed order: the results are the same on
// every run.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hsd_host.h"

namespace hsd {

constexpr int DTILE = 64;   // tile side of the dense kernels
constexpr int DKC = 32;     // k-chunk of the tile product (LDS: 2 x 64 x 33 doubles)

// G = I + A_hat^T A_hat (and the identity padding): entry (j, k) is 1 on
// the diagonal plus the dot product of rows j and k of A_hat^T, whose
// column indices are sorted, by a two-pointer merge.  Block row j = blockIdx.y,
// columns k <= j by the threads; both (j, k) and (k, j) are written.
static __global__ void k_form_gram(double *W, int64_t NP, int32_t n, const int32_t *rpT,
                                   const int32_t *ciT, const double *vT) {
    const int64_t j = blockIdx.y;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k <= j; k += (int64_t)gridDim.x * blockDim.x) {
        double g = (j == k) ? 1.0 : 0.0;
        if (j < n && k < n) {
            int p = rpT[j], pe = rpT[j + 1], q = rpT[k], qe = rpT[k + 1];
            double s = 0.0;
            while (p < pe && q < qe) {
                const int a = ciT[p], b = ciT[q];
                if (a == b) {
                    s = __builtin_fma(vT[p], vT[q], s);
                    ++p;
                    ++q;
                } else if (a < b) {
                    ++p;
                } else {
                    ++q;
                }
            }
            g += s;
        }
        W[j * NP + k] = g;
        W[k * NP + j] = g;
    }
}

// Cholesky of the diagonal tile (kb, kb) in LDS by one workgroup, column by
// column with one barrier per column: every thread takes the pivot d of
// column c, the threads write column c of L (a_ic / sqrt(d), below the
// diagonal; sqrt(d) on it) straight to W, and update the trailing lower
// part by a_ij -= a_ic a_jc / d, which reads column c only.  Zeros are
// written above the diagonal.  A pivot that is not positive (G is positive
// definite, so only rounding of a badly scaled matrix can cause one) sets
// *bad and is taken as 1.
static __global__ void __launch_bounds__(256) k_potrf_tile(double *W, int64_t NP, int kb, unsigned *bad) {
    __shared__ double a[DTILE][DTILE + 1];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int ty = tid / 16, tx = tid % 16;
    const int64_t o = (int64_t)kb * DTILE;
    for (int e = tid; e < DTILE * DTILE; e += nt) a[e / DTILE][e % DTILE] = W[(o + e / DTILE) * NP + o + e % DTILE];
    __syncthreads();
    for (int c = 0; c < DTILE; ++c) {
        const double d0 = a[c][c];
        const bool ok = d0 > 0.0;
        const double d = ok ? d0 : 1.0;
        const double sd = sqrt(d), inv_d = 1.0 / d;
        if (tid == 0 && !ok) atomicAdd(bad, 1u);
        if (tid < DTILE) {
            const int i = tid;
            W[(o + i) * NP + o + c] = i > c ? a[i][c] / sd : (i == c ? sd : 0.0);
        }
        for (int i = c + 1 + ty; i < DTILE; i += 16) {
            const double f = a[i][c] * inv_d;
            for (int jj = c + 1 + tx; jj <= i; jj += 16) a[i][jj] -= f * a[jj][c];
        }
        __syncthreads();
    }
}

// The panel below the diagonal tile: every row r of the rows below solves
// x L_kk^T = a (a = its 64 entries in tile column kb), x_c = (a_c -
// sum_{p<c} x_p L_cp) / L_cc; one thread per row, L_kk in LDS (the
// division as a product with 1 / L_cc).
static __global__ void __launch_bounds__(256) k_trsm_panel(double *W, int64_t NP, int kb) {
    __shared__ double l[DTILE][DTILE + 1];
    __shared__ double rd[DTILE];  // 1 / L_cc
    const int64_t o = (int64_t)kb * DTILE;
    for (int e = threadIdx.x; e < DTILE * DTILE; e += blockDim.x) l[e / DTILE][e % DTILE] = W[(o + e / DTILE) * NP + o + e % DTILE];
    if (threadIdx.x < DTILE) rd[threadIdx.x] = 1.0 / W[(o + threadIdx.x) * NP + o + threadIdx.x];
    __syncthreads();
    const int64_t r = o + DTILE + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= NP) return;
    double x[DTILE];
    double *row = W + r * NP + o;
#pragma unroll
    for (int c = 0; c < DTILE; ++c) x[c] = row[c];
    // each sum in four interleaved partial sums (independent chains)
#pragma unroll
    for (int c = 0; c < DTILE; ++c) {
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int p = 0; p < c; ++p) s4[p & 3] = __builtin_fma(x[p], l[c][p], s4[p & 3]);
        x[c] = (x[c] - ((s4[0] + s4[1]) + (s4[2] + s4[3]))) * rd[c];
    }
#pragma unroll
    for (int c = 0; c < DTILE; ++c) row[c] = x[c];
}

// C -= op(A) op(B) on 64 x 64 output tiles with inner dimension K = kdim
// (a multiple of DKC): output tile (R, C) with R in [r0, r0 + nr), C in
// [c0, c0 + nc) (tiles with C > R skipped when lower is set).  A's 64 x K
// block for row tile R is at Abase + R * a_rstride (TA: read as its
// transpose), B's K x 64 block for column tile C at Bbase + C * b_cstride
// (TB: read as its transpose); every matrix has leading dimension NP.  256
// threads, the K dimension in chunks of DKC through LDS; each wavefront
// takes a 32 x 32 quadrant of the output as 2 x 2 tiles of 16 x 16 on the
// FP64 matrix cores (v_mfma_f64_16x16x4: lane l supplies op(A)(i0 + l % 16,
// k + l / 16) and op(B)(k + l / 16, j0 + l % 16) and accumulates
// D(i0 + l / 16 + 4 r, j0 + l % 16), r = 0..3).
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_tile_gemm(double *Cbase, const double *Abase, const double *Bbase,
                                                   int64_t NP, int64_t a_rstride, int64_t b_cstride,
                                                   int r0, int nr, int c0, int nc, int lower, int kdim) {
    __shared__ double sa[DTILE][DKC + 1];  // sa[i][p] = op(A)(i, p)
    __shared__ double sb[DTILE][DKC + 1];  // sb[j][p] = op(B)(p, j)
    const int R = r0 + blockIdx.x / nc, Cc = c0 + blockIdx.x % nc;
    if (lower && Cc > R) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;  // the wavefront's quadrant
    const int li = lane & 15, lk = lane >> 4;
    const double *A = Abase + (int64_t)R * a_rstride;
    const double *B = Bbase + (int64_t)Cc * b_cstride;
    double *C = Cbase + (int64_t)R * DTILE * NP + (int64_t)Cc * DTILE;
    typedef double f64x4 __attribute__((ext_vector_type(4)));
    f64x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    // the next chunk's entries are loaded into registers while the current
    // one is multiplied (each thread NQ entries of op(A) and of op(B))
    constexpr int NQ = DTILE * DKC / 256;
    double ra[NQ], rb[NQ];
    auto load_chunk = [&](int k0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = tid + q * 256;
            // op(A)(i, p): A[i][k0 + p], or A[k0 + p][i] when transposed
            if (TA) ra[q] = A[(int64_t)(k0 + e / DTILE) * NP + e % DTILE];
            else ra[q] = A[(int64_t)(e / DKC) * NP + k0 + e % DKC];
            // op(B)(p, j): B[k0 + p][j], or B[j][k0 + p] when transposed
            if (TB) rb[q] = B[(int64_t)(e / DKC) * NP + k0 + e % DKC];
            else rb[q] = B[(int64_t)(k0 + e / DTILE) * NP + e % DTILE];
        }
    };
    load_chunk(0);
    for (int k0 = 0; k0 < kdim; k0 += DKC) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = tid + q * 256;
            if (TA) sa[e % DTILE][e / DTILE] = ra[q];
            else sa[e / DKC][e % DKC] = ra[q];
            if (TB) sb[e / DKC][e % DKC] = rb[q];
            else sb[e % DTILE][e / DTILE] = rb[q];
        }
        __syncthreads();
        if (k0 + DKC < kdim) load_chunk(k0 + DKC);
#pragma unroll
        for (int p = 0; p < DKC; p += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = sa[wr + a * 16 + li][p + lk];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = sb[wc + b * 16 + li][p + lk];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                C[(int64_t)(wr + a * 16 + lk + 4 * r) * NP + wc + b * 16 + li] -= acc[a][b][r];
}

// Y = I on the padded matrix.
static __global__ void k_eye(double *Y, int64_t NP) {
    const int64_t tot = NP * NP;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x)
        Y[e] = (e / NP == e % NP) ? 1.0 : 0.0;
}

// Block row kb of Y (columns [0, ncol)): Y_b <- L_bb^{-1} Y_b (forward
// substitution per column, one thread per column, L_bb in LDS).
static __global__ void __launch_bounds__(256) k_trsv_rows_fwd(const double *W, double *Y, int64_t NP, int kb,
                                                              int64_t ncol) {
    __shared__ double l[DTILE][DTILE + 1];
    __shared__ double rd[DTILE];  // 1 / L_ii
    const int64_t o = (int64_t)kb * DTILE;
    for (int e = threadIdx.x; e < DTILE * DTILE; e += blockDim.x) l[e / DTILE][e % DTILE] = W[(o + e / DTILE) * NP + o + e % DTILE];
    if (threadIdx.x < DTILE) rd[threadIdx.x] = 1.0 / W[(o + threadIdx.x) * NP + o + threadIdx.x];
    __syncthreads();
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= ncol) return;
    double y[DTILE];
#pragma unroll
    for (int i = 0; i < DTILE; ++i) y[i] = Y[(o + i) * NP + j];
    // each row's sum in four interleaved partial sums (independent chains)
#pragma unroll
    for (int i = 0; i < DTILE; ++i) {
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int p = 0; p < i; ++p) s4[p & 3] = __builtin_fma(l[i][p], y[p], s4[p & 3]);
        y[i] = (y[i] - ((s4[0] + s4[1]) + (s4[2] + s4[3]))) * rd[i];
    }
#pragma unroll
    for (int i = 0; i < DTILE; ++i) Y[(o + i) * NP + j] = y[i];
}

// Block row kb of Z (all columns): Z_b <- L_bb^{-T} Z_b (back substitution
// with L_bb^T per column).
static __global__ void __launch_bounds__(256) k_trsv_rows_bwd(const double *W, double *Z, int64_t NP, int kb) {
    __shared__ double l[DTILE][DTILE + 1];
    __shared__ double rd[DTILE];  // 1 / L_ii
    const int64_t o = (int64_t)kb * DTILE;
    for (int e = threadIdx.x; e < DTILE * DTILE; e += blockDim.x) l[e / DTILE][e % DTILE] = W[(o + e / DTILE) * NP + o + e % DTILE];
    if (threadIdx.x < DTILE) rd[threadIdx.x] = 1.0 / W[(o + threadIdx.x) * NP + o + threadIdx.x];
    __syncthreads();
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= NP) return;
    double z[DTILE];
#pragma unroll
    for (int i = 0; i < DTILE; ++i) z[i] = Z[(o + i) * NP + j];
    // each row's sum in four interleaved partial sums (independent chains)
#pragma unroll
    for (int i = DTILE - 1; i >= 0; --i) {
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int p = i + 1; p < DTILE; ++p) s4[p & 3] = __builtin_fma(l[p][i], z[p], s4[p & 3]);
        z[i] = (z[i] - ((s4[0] + s4[1]) + (s4[2] + s4[3]))) * rd[i];
    }
#pragma unroll
    for (int i = 0; i < DTILE; ++i) Z[(o + i) * NP + j] = z[i];
}

// The direct projection's setup (see hsd_direct.h): W <- G = I + A^T A
// (padded to NP), W <- its Cholesky factor L (lower; tiles above the
// diagonal are not read again), Z <- G^{-1} by L Y = I then L^T Z = Y.  A
// non-positive pivot counts into *bad.
//
// All three passes work in blocks of DSUPER tiles (256 rows or columns):
// inside a block the 64-wide steps as before (a tile factored or solved,
// then the product updates that the rest of the block needs), and the
// update of everything beyond the block by one product with K = 256, so
// that the trailing matrix is read and written once per block rather than
// once per tile.
constexpr int DSUPER = 4;
inline int direct_prepare(double *W, double *Z, int64_t NP, int32_t n, const int32_t *rpT,
                          const int32_t *ciT, const double *vT, unsigned *bad, hipStream_t s) {
    const int T = (int)(NP / DTILE);
    const int64_t TS = (int64_t)DTILE * NP;  // one tile row
    hipLaunchKernelGGL(k_form_gram, dim3(grid_for(NP, 256), (unsigned)NP), dim3(256), 0, s, W, NP, n, rpT, ciT, vT);
    HIP_TRY(hipGetLastError());
    // Cholesky, right-looking by blocks of DSUPER tile columns
    for (int p0 = 0; p0 < T; p0 += DSUPER) {
        const int p1 = p0 + DSUPER < T ? p0 + DSUPER : T;
        for (int kb = p0; kb < p1; ++kb) {
            hipLaunchKernelGGL(k_potrf_tile, dim3(1), dim3(256), 0, s, W, NP, kb, bad);
            if (kb + 1 < T) {
                const int rest = T - kb - 1;
                hipLaunchKernelGGL(k_trsm_panel, dim3(grid_for((int64_t)rest * DTILE, 256, 1 << 20)), dim3(256), 0,
                                   s, W, NP, kb);
            }
            // the block's later tile columns, every row below
            if (kb + 1 < p1) {
                const int rows = T - kb - 1, cols = p1 - kb - 1;
                hipLaunchKernelGGL((k_tile_gemm<false, true>), dim3(rows * cols), dim3(256), 0, s, W,
                                   (const double *)(W + (int64_t)kb * DTILE), (const double *)(W + (int64_t)kb * DTILE),
                                   NP, TS, TS, kb + 1, rows, kb + 1, cols, 1, DTILE);
            }
            HIP_TRY(hipGetLastError());
        }
        // the trailing lower triangle beyond the block, K = the block's width
        if (p1 < T) {
            const int rest = T - p1;
            hipLaunchKernelGGL((k_tile_gemm<false, true>), dim3(rest * rest), dim3(256), 0, s, W,
                               (const double *)(W + (int64_t)p0 * DTILE), (const double *)(W + (int64_t)p0 * DTILE), NP,
                               TS, TS, p1, rest, p1, rest, 1, (p1 - p0) * DTILE);
            HIP_TRY(hipGetLastError());
        }
    }
    // L Y = I (Y lower triangular: block row b has columns [0, (b + 1) 64))
    hipLaunchKernelGGL(k_eye, dim3(grid_for(NP * NP, 256)), dim3(256), 0, s, Z, NP);
    for (int b0 = 0; b0 < T; b0 += DSUPER) {
        const int b1 = b0 + DSUPER < T ? b0 + DSUPER : T;
        for (int b = b0; b < b1; ++b) {
            const int64_t ncol = (int64_t)(b + 1) * DTILE;
            hipLaunchKernelGGL(k_trsv_rows_fwd, dim3(grid_for(ncol, 256, 1 << 20)), dim3(256), 0, s,
                               (const double *)W, Z, NP, b, ncol);
            // the block's later rows
            if (b + 1 < b1)
                hipLaunchKernelGGL((k_tile_gemm<false, false>), dim3((b1 - b - 1) * (b + 1)), dim3(256), 0, s, Z,
                                   (const double *)(W + (int64_t)b * DTILE), (const double *)(Z + (int64_t)b * TS), NP,
                                   TS, (int64_t)DTILE, b + 1, b1 - b - 1, 0, b + 1, 0, DTILE);
            HIP_TRY(hipGetLastError());
        }
        // every row below the block, K = the block's height
        if (b1 < T) {
            hipLaunchKernelGGL((k_tile_gemm<false, false>), dim3((T - b1) * b1), dim3(256), 0, s, Z,
                               (const double *)(W + (int64_t)b0 * DTILE), (const double *)(Z + (int64_t)b0 * TS), NP,
                               TS, (int64_t)DTILE, b1, T - b1, 0, b1, 0, (b1 - b0) * DTILE);
            HIP_TRY(hipGetLastError());
        }
    }
    // L^T Z = Y, from the last block up
    for (int b1 = T; b1 > 0; b1 -= DSUPER) {
        const int b0 = b1 - DSUPER > 0 ? b1 - DSUPER : 0;
        for (int b = b1 - 1; b >= b0; --b) {
            hipLaunchKernelGGL(k_trsv_rows_bwd, dim3(grid_for(NP, 256, 1 << 20)), dim3(256), 0, s, (const double *)W,
                               Z, NP, b);
            // the block's earlier rows
            if (b > b0)
                hipLaunchKernelGGL((k_tile_gemm<true, false>), dim3((b - b0) * T), dim3(256), 0, s, Z,
                                   (const double *)(W + (int64_t)b * TS), (const double *)(Z + (int64_t)b * TS), NP,
                                   (int64_t)DTILE, (int64_t)DTILE, b0, b - b0, 0, T, 0, DTILE);
            HIP_TRY(hipGetLastError());
        }
        // every row above the block, K = the block's height
        if (b0 > 0) {
            hipLaunchKernelGGL((k_tile_gemm<true, false>), dim3(b0 * T), dim3(256), 0, s, Z,
                               (const double *)(W + (int64_t)b0 * TS), (const double *)(Z + (int64_t)b0 * TS), NP,
                               (int64_t)DTILE, (int64_t)DTILE, 0, b0, 0, T, 0, (b1 - b0) * DTILE);
            HIP_TRY(hipGetLastError());
        }
    }
    return HSD_OK;
}

}  // namespace hsd
