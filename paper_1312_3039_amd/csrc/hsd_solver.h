// The per-iteration hot path as one device routine run by a "team" of
// workgroups (a cooperative grid for one large program, or one workgroup
// per program in the batched kernel):
//
//   w = u + v,  r = w_xy - w_tau h                              (Sect. 4.1)
//   z = M^{-1} r by CG on (I + A^T A) z_x = r_x - A^T r_y,
//       z_y = r_y + A z_x, warm-started from the previous z_x    (Sect. 4.1)
//   u_tilde = (z - g h^T z / eta, w_tau + h^T z / eta)           (SMW, Sect. 4.1)
//   u_bar = alpha u_tilde + (1 - alpha) u                        (Sect. 3.3)
//   u+ = Pi_C(u_bar - v),  v+ = v - u_bar + u+                   (e-SCS)
//
// with the termination tests of Sect. 3.5 (scaled forms of Sect. 5) fused
// into the first two sweeps over A and A^T of each iteration.
//
// Sweeps and barriers per ADMM iteration (CG with k_cg iterations):
//   A-sweep:   t0 = r_y + A z0  (+ A u_x for the tests)       [barrier]
//   AT-sweep:  res0 = r_x - z0 - A^T t0  (+ A^T u_y)          [barrier]
//   per CG iteration:
//     A-sweep:  t = A p with p = res + beta p_old formed on the fly,
//               |p|^2 + |t|^2 = p^T (I + A^T A) p             [barrier]
//     AT-sweep: z_x += a p, res -= a (p + A^T t), z_y += a t    [barrier]
//   update: SMW, relaxation, cone projections, dual update      [barrier]
// z_y is accumulated as t0 + sum a_k t_k, so no extra product with A is
// needed after CG: 2 + 2 k_cg products per iteration, the accounting of the
// paper's Table 5.
#pragma once

#include "hsd_device.h"

namespace hsd {

template <typename T>
__device__ __forceinline__ T tfma(T a, T b, T c);
template <>
__device__ __forceinline__ double tfma<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <>
__device__ __forceinline__ float tfma<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// CG search direction p_j = res_j + beta p_old_j (exactly res_j on the first
// CG iteration); the same expression is used by the gathering SpMV and by
// the owner that stores p, so both see identical values.
template <typename T>
__device__ __forceinline__ T cg_dir(const T *res, const T *pold, T beta, int j, bool first) {
    return first ? res[j] : tfma(beta, pold[j], res[j]);
}

// Partial dot product of one CSR row with a gathered vector for the lane
// gl of a group of L lanes: sum over k = kb+gl, kb+gl+L, ... of
// val[k] * x(ci[k]), accumulated in that order.  Four nonzeros are loaded
// per step so that their index, value and gather loads are in flight
// together (the memory latency, not bandwidth, bounds these sweeps when the
// matrix sits in cache); the summation order is the same as one at a time.
//
// With NT set the index and value loads are nontemporal: a slab sweep
// streams the matrix once, and the hint keeps it from evicting the slab of
// the gathered vector from L2.
template <bool NT, typename X>
__device__ __forceinline__ X ld(const X *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// Entries a lane gathers at once: a row's entries are visited in chunks of
// ROW_CHUNK per lane, every load of a chunk issued before the first is
// used.  Entries past the row end are neither gathered nor added, so the
// sums keep the order of a plain loop.  (Chunks of 8 wait on fewer round
// trips but cost more in registers than they save.)
constexpr int ROW_CHUNK = 4;
// A row whose group would take more than this many chunks is a long row,
// taken by the whole workgroup (see sweep).
constexpr int LONG_CHUNKS = 32;
// Entries per lane in flight in the direct projection's product with Z.
typedef double f64x2 __attribute__((ext_vector_type(2)));  // two doubles, one 16-byte access
constexpr int DIRECT_UNROLL = 8;

template <typename T, bool NT = false, typename V, typename F>
__device__ __forceinline__ T row_dot(const int32_t *__restrict__ ci, const V *__restrict__ val,
                                     int kb, int ke, int gl, int L, F x) {
    T s = T(0);
    for (int k0 = kb + gl; k0 < ke; k0 += ROW_CHUNK * L) {
        const int jf = ld<NT>(ci + k0);
        int j[ROW_CHUNK];
        T v[ROW_CHUNK];
#pragma unroll
        for (int q = 0; q < ROW_CHUNK; ++q) {
            const int k = k0 + q * L;
            const bool in = k < ke;
            j[q] = in ? ld<NT>(ci + k) : jf;
            v[q] = in ? (T)ld<NT>(val + k) : T(0);
        }
        T y[ROW_CHUNK];
#pragma unroll
        for (int q = 0; q < ROW_CHUNK; ++q) y[q] = (k0 + q * L < ke) ? x(j[q]) : T(0);
#pragma unroll
        for (int q = 0; q < ROW_CHUNK; ++q)
            if (k0 + q * L < ke) s = tfma(v[q], y[q], s);
    }
    return s;
}

// Two row products in one pass over the row: s1 with values v1 and vector
// x1 (CG precision), s2 with FP64 values v2 and vector x2 (the termination
// tests).  v1 and v2 may be the same array.  Chunks as in row_dot.
template <typename T, bool NT = false, typename F1, typename F2>
__device__ __forceinline__ void row_dot2(const int32_t *__restrict__ ci, const T *v1,
                                         const double *v2, int kb, int ke, int gl, int L,
                                         F1 x1, F2 x2, T &s1, double &s2) {
    T a = T(0);
    double b = 0.0;
    // FP64 mode: the test values are the product's own values, loaded once
    const bool same = sizeof(T) == 8 && (const void *)v1 == (const void *)v2;
    for (int k0 = kb + gl; k0 < ke; k0 += ROW_CHUNK * L) {
        const int jf = ld<NT>(ci + k0);
        int j[ROW_CHUNK];
        T va[ROW_CHUNK];
        double vb[ROW_CHUNK];
#pragma unroll
        for (int q = 0; q < ROW_CHUNK; ++q) {
            const int k = k0 + q * L;
            const bool in = k < ke;
            j[q] = in ? ld<NT>(ci + k) : jf;
            va[q] = in ? ld<NT>(v1 + k) : T(0);
            vb[q] = in ? (same ? (double)va[q] : ld<NT>(v2 + k)) : 0.0;
        }
        T y[ROW_CHUNK];
        double z[ROW_CHUNK];
#pragma unroll
        for (int q = 0; q < ROW_CHUNK; ++q) {
            const bool in = k0 + q * L < ke;
            y[q] = in ? x1(j[q]) : T(0);
            z[q] = in ? x2(j[q]) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < ROW_CHUNK; ++q) {
            if (k0 + q * L < ke) {
                a = tfma(va[q], y[q], a);
                b = __builtin_fma(vb[q], z[q], b);
            }
        }
    }
    s1 = a;
    s2 = b;
}

// One sweep over rows [r0, r1) of a CSR matrix by groups of L lanes: for
// every row i, st = sum_k v1[k] x1(ci[k]) (CG precision) and, when `two` is
// set, sc = sum_k v2[k] x2(ci[k]) (FP64); then lane 0 of the row's group
// calls epi(i, st, sc).
//
// Without SLABS: one pass per row group, row i read through rp[i - ra].
// With SLABS (K >= 1 column slabs): the matrix is stored slab-major (the
// entries of slab s, row after row, are contiguous; those of row i in slab
// s are off[s*rows + i] .. off[s*rows + i + 1]).  The rows are taken in
// chunks; for a chunk and a slab the entries form one contiguous range,
// streamed in blocks of SLAB_PER_THREAD entries per thread: every thread
// loads its entries (coalesced, all loads in flight together), gathers and
// writes the products to LDS, and after a barrier the thread owning a row
// adds the row's products of the block in entry order to the row's sum in
// LDS.  The epilogue runs once the chunk's last slab is done.  All
// workgroups walk the slabs in the same order, so the slab of the gathered
// vector they share stays in L2 while the matrix streams past.  The order of the
// additions is fixed, so results are the same on every run.
// LDS of a slab sweep: per-row sums of a chunk of rows, the chunk's slab
// offsets, and the products of one block.
template <typename T>
struct SlabLds {
    T *acc_t;        // chunk
    double *acc_d;   // chunk
    int32_t *offs;   // chunk + 1
    T *p1;           // 8 * blockDim.x
    double *p2;      // 8 * blockDim.x
    int chunk;       // rows per chunk (0 = no LDS: never launched this way)
};
constexpr int SLAB_PER_THREAD = 4;  // entries per thread and block of a slab sweep

// LDS doubles a slab sweep needs for `chunk` rows and `threads` threads.
__host__ __device__ constexpr size_t slab_lds_doubles(int chunk, int threads) {
    return 2 * (size_t)chunk + (size_t)chunk / 2 + 1 + 2 * (size_t)SLAB_PER_THREAD * threads;
}

template <typename T>
__device__ __forceinline__ SlabLds<T> slab_lds(double *base, int chunk) {
    SlabLds<T> L;
    L.chunk = chunk;
    L.acc_t = reinterpret_cast<T *>(base);
    L.acc_d = base + chunk;
    L.offs = reinterpret_cast<int32_t *>(base + 2 * chunk);
    L.p1 = reinterpret_cast<T *>(base + 2 * chunk + chunk / 2 + 1);
    L.p2 = base + 2 * chunk + chunk / 2 + 1 + SLAB_PER_THREAD * blockDim.x;
    return L;
}

//
// Long rows (row-group sweeps, long_thr > 0): a row with more than long_thr
// entries would keep its group of L lanes busy for many chunks while the
// rest of the workgroup waits (a dense row or column beside short ones, as
// in the budget row of a portfolio program).  Such a row is left out by its
// group and taken, after the other rows of the same step, by the whole
// workgroup: every thread adds a strided share of its entries, the wave sums
// are added in wave order, and thread 0 calls the epilogue.  The rows of a
// step are taken in row order, so the sums are the same on every run.
// lred: LDS scratch of 4 * MAX_WAVES doubles (free during a sweep).
template <typename T, bool SLABS, typename G1, typename G2, typename Epi>
__device__ __forceinline__ void sweep(int r0, int r1, int L, bool two, const int32_t *rp, int ra,
                                      int K, const int32_t *off, int rows, const SlabLds<T> &sl,
                                      const int32_t *ci, const T *v1, const double *v2, G1 x1,
                                      G2 x2, Epi epi, int long_thr = 0, double *lred = nullptr) {
    const int ng = blockDim.x / L, gid = threadIdx.x / L, gl = threadIdx.x % L;
    if constexpr (!SLABS) {
        for (int base = r0; base < r1; base += ng) {
            const int i = base + gid;
            const bool act = i < r1;
            T st = T(0);
            double sc = 0.0;
            bool lng = false;
            int kb = 0, ke = 0;
            if (act) {
                kb = rp[i - ra];
                ke = rp[i - ra + 1];
                lng = long_thr > 0 && ke - kb > long_thr;
                if (!lng) {
                    if (two) row_dot2<T>(ci, v1, v2, kb, ke, gl, L, x1, x2, st, sc);
                    else st = row_dot<T>(ci, v1, kb, ke, gl, L, x1);
                }
            }
            st = group_sum(st, L);
            if (two) sc = group_sum(sc, L);
            if (act && gl == 0 && !lng) epi(i, st, sc);
            if (long_thr > 0) {
                // the long rows of this step: one mask word per wave, in a
                // buffer that alternates from step to step (a thread may
                // write the next step's word while another still reads
                // these; the barrier of that step keeps it two steps away)
                const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
                const int nw = blockDim.x / WAVE;
                unsigned long long *msk = reinterpret_cast<unsigned long long *>(lred + 2 * MAX_WAVES) +
                                          (((base - r0) / ng) & 1) * MAX_WAVES;
                const unsigned long long bm = __ballot(act && gl == 0 && lng);
                if (lane == 0) msk[wid] = bm;
                __syncthreads();
                for (int w = 0; w < nw; ++w) {
                    unsigned long long mw = msk[w];
                    while (mw) {
                        const int b = __builtin_ctzll(mw);
                        mw &= mw - 1;
                        const int r = base + (w * WAVE + b) / L;
                        const int rb = rp[r - ra], re = rp[r - ra + 1];
                        T a = T(0);
                        double d = 0.0;
                        if (two) row_dot2<T>(ci, v1, v2, rb, re, threadIdx.x, blockDim.x, x1, x2, a, d);
                        else a = row_dot<T>(ci, v1, rb, re, threadIdx.x, blockDim.x, x1);
                        a = group_sum(a, WAVE);
                        if (two) d = group_sum(d, WAVE);
                        if (lane == 0) { lred[wid] = (double)a; lred[MAX_WAVES + wid] = d; }
                        __syncthreads();
                        if (threadIdx.x == 0) {
                            T ta = T(0);
                            double td = 0.0;
                            for (int q = 0; q < nw; ++q) { ta += (T)lred[q]; td += lred[MAX_WAVES + q]; }
                            epi(r, ta, two ? td : 0.0);
                        }
                        __syncthreads();
                    }
                }
            }
        }
        return;
    }
    const int nt = blockDim.x, tid = threadIdx.x;
    const int chunk = sl.chunk;
    if (chunk <= 0) return;  // no LDS for the slab sweep: never launched this way
    for (int c0 = r0; c0 < r1; c0 += chunk) {
        const int nr = (c0 + chunk < r1 ? c0 + chunk : r1) - c0;
        for (int r = tid; r < nr; r += nt) {
            sl.acc_t[r] = T(0);
            sl.acc_d[r] = 0.0;
        }
        for (int s = 0; s < K; ++s) {
            const int32_t *o = off + (size_t)s * rows + c0;
            __syncthreads();  // the previous slab's offsets and products are no longer read
            for (int r = tid; r <= nr; r += nt) sl.offs[r] = o[r];
            __syncthreads();
            const int E0 = sl.offs[0], E1 = sl.offs[nr];
            for (int eb = E0; eb < E1; eb += SLAB_PER_THREAD * nt) {
                // stage 1: the block's products, the loads of all its entries issued together
                int jj[SLAB_PER_THREAD];
                T aa[SLAB_PER_THREAD];
                double bb[SLAB_PER_THREAD];
#pragma unroll
                for (int q = 0; q < SLAB_PER_THREAD; ++q) {
                    const int e = eb + tid + q * nt;
                    jj[q] = 0;
                    aa[q] = T(0);
                    bb[q] = 0.0;
                    if (e < E1) {
                        jj[q] = ld<true>(ci + e);
                        aa[q] = (T)ld<true>(v1 + e);
                        if (two) bb[q] = ld<true>(v2 + e);
                    }
                }
#pragma unroll
                for (int q = 0; q < SLAB_PER_THREAD; ++q) {
                    const int e = eb + tid + q * nt;
                    if (e < E1) {
                        sl.p1[tid + q * nt] = aa[q] * x1(jj[q]);
                        if (two) sl.p2[tid + q * nt] = bb[q] * x2(jj[q]);
                    }
                }
                __syncthreads();
                // stage 2: every row adds its entries of the block in order
                const int ee = eb + SLAB_PER_THREAD * nt < E1 ? eb + SLAB_PER_THREAD * nt : E1;
                for (int r = tid; r < nr; r += nt) {
                    const int lo = sl.offs[r] > eb ? sl.offs[r] : eb;
                    const int hi = sl.offs[r + 1] < ee ? sl.offs[r + 1] : ee;
                    if (lo < hi) {
                        T a = sl.acc_t[r];
                        for (int e = lo; e < hi; ++e) a += sl.p1[e - eb];
                        sl.acc_t[r] = a;
                        if (two) {
                            double b = sl.acc_d[r];
                            for (int e = lo; e < hi; ++e) b += sl.p2[e - eb];
                            sl.acc_d[r] = b;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int r = tid; r < nr; r += nt) epi(c0 + r, sl.acc_t[r], two ? sl.acc_d[r] : 0.0);
    }
}

// End of a phase: workgroup sums of ND double and NT CG-precision values,
// written as partials, then the team barrier.  The team totals are formed
// by phase_collect after this barrier or a later one (the partial slot is
// not written again before that).  With a team of one workgroup the sums
// are formed in every thread and are already the totals; otherwise only
// thread 0 forms them (wave sums through LDS, added in wave order), and the
// values in vd and vt are left as they were.  Returns false if the team
// aborted.
template <int ND, int NT, typename T>
__device__ __forceinline__ bool phase_put(const Team &tm, double *part, int slot,
                                          double *vd, T *vt, double *red_d, T *red_t) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int nw = blockDim.x / WAVE;
    if (tm.size == 1) {
        // the workgroup sums of all ND + NT values behind one barrier (each
        // summed over the waves in wave order, as block_sum does); the
        // barrier after them is the team's.  The T partials sit after the
        // ND double ones, so red_t may be red_d.
        static_assert(ND + NT <= 8, "phase_put: at most 8 values");
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            const double w = group_sum(vd[k], WAVE);
            if (lane == 0) red_d[k * MAX_WAVES + wid] = w;
        }
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            const T w = group_sum(vt[k], WAVE);
            if (lane == 0) red_t[(ND + k) * MAX_WAVES + wid] = w;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            double a = 0.0;
            for (int w = 0; w < nw; ++w) a += red_d[k * MAX_WAVES + w];
            vd[k] = uniform(a);
        }
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            T a = T(0);
            for (int w = 0; w < nw; ++w) a += red_t[(ND + k) * MAX_WAVES + w];
            vt[k] = uniform(a);
        }
        __syncthreads();
        return true;
    }
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        const double w = group_sum(vd[k], WAVE);
        if (lane == 0) red_d[k * MAX_WAVES + wid] = w;
    }
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const T w = group_sum(vt[k], WAVE);
        if (lane == 0) red_t[k * MAX_WAVES + wid] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *dst = part + ((size_t)slot * tm.size + tm.rank) * PART_STRIDE;
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            double a = 0.0;
            for (int w = 0; w < nw; ++w) a += red_d[k * MAX_WAVES + w];
            dst[k] = a;
        }
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            T a = T(0);
            for (int w = 0; w < nw; ++w) a += red_t[k * MAX_WAVES + w];
            dst[ND + k] = (double)a;
        }
    }
    // team_sync starts with a workgroup barrier: red_d and red_t are free
    // again once every workgroup has passed it
    return team_sync(tm);
}

// Team totals of one phase (slot: ND doubles, NT CG-precision values) and,
// if NE > 0, of an earlier phase (slot_e: NE doubles).  The first wavefront
// loads the partials of both slots in one pass (lane l adds workgroups l,
// l + 64, ... in order), adds across its lanes in a fixed butterfly order
// and hands the totals to the workgroup through LDS: every workgroup forms
// bit-identical totals.  The FP64 totals are summed in FP64, the
// CG-precision totals in T.
struct NoSide {
    __device__ void operator()() const {}
};

// side() runs once in every thread, in the threads past the first wavefront
// while that wavefront waits on the partials; what it writes to LDS is
// visible to the workgroup when phase_collect returns.
template <int ND, int NT, int NE = 0, typename T, typename Side = NoSide>
__device__ __forceinline__ void phase_collect(const Team &tm, const double *part, int slot,
                                              double *vd, T *vt, double *red_d, T *red_t,
                                              int slot_e = 0, double *ve = nullptr,
                                              Side side = Side()) {
    if (tm.size == 1 || blockDim.x <= WAVE) {
        side();
        __syncthreads();
        if (tm.size == 1) return;
    } else if (threadIdx.x >= WAVE) {
        side();
    }
    constexpr int NV = ND + NT + NE;
    static_assert(NV <= 16, "phase_collect: at most 16 totals");
    // written by the first wavefront, read by all threads after the
    // workgroup barrier below; the next write is behind at least one more
    // workgroup barrier (every phase_put has one)
    __shared__ double s_tot[16];
    if (threadIdx.x < WAVE) {
        // FP64 totals in FP64; the NT CG-precision totals (the CG inner
        // products) are added in T, so that in FP32 mode they are FP32 sums
        // of FP32 partials throughout
        double a[NV];
        T at[NT > 0 ? NT : 1];
#pragma unroll
        for (int k = 0; k < NV; ++k) a[k] = 0.0;
#pragma unroll
        for (int k = 0; k < NT; ++k) at[k] = T(0);
        for (int r = threadIdx.x; r < tm.size; r += WAVE) {
            const double *src = part + ((size_t)slot * tm.size + r) * PART_STRIDE;
#pragma unroll
            for (int k = 0; k < ND; ++k) a[k] += src[k];
#pragma unroll
            for (int k = 0; k < NT; ++k) at[k] += (T)src[ND + k];
            if constexpr (NE > 0) {
                const double *se = part + ((size_t)slot_e * tm.size + r) * PART_STRIDE;
#pragma unroll
                for (int k = 0; k < NE; ++k) a[ND + NT + k] += se[k];
            }
        }
#pragma unroll
        for (int k = 0; k < NT; ++k) a[ND + k] = (double)group_sum(at[k], WAVE);
#pragma unroll
        for (int k = 0; k < ND; ++k) a[k] = group_sum(a[k], WAVE);
#pragma unroll
        for (int k = ND + NT; k < NV; ++k) a[k] = group_sum(a[k], WAVE);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < NV; ++k) s_tot[k] = a[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ND; ++k) vd[k] = s_tot[k];
#pragma unroll
    for (int k = 0; k < NT; ++k) vt[k] = (T)s_tot[ND + k];
#pragma unroll
    for (int k = 0; k < NE; ++k) ve[k] = s_tot[ND + NT + k];
}

// phase_put followed by phase_collect of the same slot.
template <int ND, int NT, typename T>
__device__ __forceinline__ bool phase_end(const Team &tm, double *part, int slot,
                                          double *vd, T *vt, double *red_d, T *red_t) {
    if (!phase_put<ND, NT>(tm, part, slot, vd, vt, red_d, red_t)) return false;
    phase_collect<ND, NT>(tm, part, slot, vd, vt, red_d, red_t);
    return true;
}

// Projection of the y-block onto K (dual = false) or K^* (dual = true).
// fin(i) returns argument row i; fout(i, p, a) stores result p of row i
// with argument a.  Rows [a0, a1) of the zero/nonnegative part are handled
// by this workgroup; second-order cones go to groups of Ls lanes across the
// team, PSD cones to whole workgroups, exponential triples to threads.
template <typename Fin, typename Fout>
__device__ void project_y(const ConeDev &K, bool dual, const Team &tm, int a0, int a1, int Ls,
                          double *lds_psd, Fin fin, Fout fout) {
    const int tid = threadIdx.x, nt = blockDim.x;
    // zero cone and nonnegative orthant: elementwise, this workgroup's rows
    {
        const int fl = K.f + K.l;
        const int lo = a0, hi = a1 < fl ? a1 : fl;
        for (int i = lo + tid; i < hi; i += nt) {
            const double a = fin(i);
            double p;
            if (i < K.f) p = dual ? a : 0.0;
            else p = a > 0.0 ? a : 0.0;
            fout(i, p, a);
        }
    }
    // second-order cones: (t, xbar), closed form
    if (K.nsoc > 0) {
        const int gpb = nt / Ls;
        const int G = gpb * tm.size;
        const int g = tm.rank * gpb + tid / Ls;
        const int gl = tid % Ls;
        for (int c0 = 0; c0 < K.nsoc; c0 += G) {
            const int cidx = c0 + g;
            const bool act = cidx < K.nsoc;
            int off = 0, len = 0;
            if (act) { off = K.soc_off[cidx]; len = K.soc_len[cidx]; }
            double ss = 0.0;
            for (int e = 1 + gl; e < len; e += Ls) {
                const double a = fin(off + e);
                ss += a * a;
            }
            ss = group_sum(ss, Ls);
            if (act) {
                const double t = fin(off);
                const double nrm = sqrt(ss);
                if (nrm <= t) {
                    for (int e = gl; e < len; e += Ls) { const double a = fin(off + e); fout(off + e, a, a); }
                } else if (nrm <= -t) {
                    for (int e = gl; e < len; e += Ls) { const double a = fin(off + e); fout(off + e, 0.0, a); }
                } else {
                    const double h = 0.5 * (t + nrm);
                    const double f = h / nrm;
                    for (int e = gl; e < len; e += Ls) {
                        const double a = fin(off + e);
                        fout(off + e, e == 0 ? h : f * a, a);
                    }
                }
            }
        }
    }
    // PSD cones: one workgroup each (self-dual)
    for (int cidx = tm.rank; cidx < K.npsd; cidx += tm.size) {
        const int off = K.psd_off[cidx];
        const int d = K.psd_dim[cidx];
        proj_psd_block(d, lds_psd,
                       [&](int e) { return fin(off + e); },
                       [&](int e, double p, double a) { fout(off + e, p, a); });
    }
    // exponential triples: one thread each; K^* of a primal exponential
    // block is K_exp^*, of a dual exponential block K_exp
    {
        const int gt = tm.rank * nt + tid;
        const int GT = tm.size * nt;
        const int tot = K.nexp + K.nexpd;
        for (int e = gt; e < tot; e += GT) {
            const bool primal_block = e < K.nexp;
            const int off = primal_block ? K.exp_off + 3 * e : K.expd_off + 3 * (e - K.nexp);
            const double a0v = fin(off), a1v = fin(off + 1), a2v = fin(off + 2);
            double x = a0v, y = a1v, z = a2v;
            const bool use_dual_proj = (primal_block == dual);
            if (use_dual_proj) proj_exp_dual_dev(x, y, z);
            else proj_exp_dev(x, y, z);
            fout(off, x, a0v);
            fout(off + 1, y, a1v);
            fout(off + 2, z, a2v);
        }
    }
    // power-cone triples: one thread each; parameter a >= 0 marks K_pow^a,
    // -a a dual block (K_pow^a)^*, whose own dual is K_pow^a again
    {
        const int gt = tm.rank * nt + tid;
        const int GT = tm.size * nt;
        for (int e = gt; e < K.npow; e += GT) {
            const int off = K.pow_off + 3 * e;
            const double pa = K.pow_a[e];
            const double a0v = fin(off), a1v = fin(off + 1), a2v = fin(off + 2);
            double x = a0v, y = a1v, z = a2v;
            const bool primal_block = !(pa < 0.0);
            if (primal_block == dual) proj_pow_dual_dev(x, y, z, fabs(pa));
            else proj_pow_dev(x, y, z, fabs(pa));
            fout(off, x, a0v);
            fout(off + 1, y, a1v);
            fout(off + 2, z, a2v);
        }
    }
}

// u_x of an update (Sect. 3.3 relaxation of the SMW solution z_x - g_x s):
// alpha (z_x - g_x s) + (1 - alpha) u_x, with explicit fused operations so
// that every site that forms it rounds the same way.
__device__ __forceinline__ double relaxed_ux(double zj, double gj, double uj, double sfac, double alpha) {
    return __builtin_fma(alpha, __builtin_fma(-gj, sfac, zj), (1.0 - alpha) * uj);
}

// First index k in [0, len) with a[k] >= x (len if none).
__device__ __forceinline__ int lower_bound_i32(const int32_t *a, int len, int x) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// The cones of the y-block that lie in rows [a0, a1): the part boundaries
// of the rows of A never split a cone, so every cone belongs to exactly one
// workgroup of the team.
struct OwnCones {
    int soc0, soc1, psd0, psd1, exp0, exp1, expd0, expd1, pow0, pow1;
};

__device__ __forceinline__ int triple_index(int row, int off, int count) {
    // first triple of a block of `count` triples at `off` starting at or after `row`
    const int t = row <= off ? 0 : (row - off + 2) / 3;
    return t < count ? t : count;
}

__device__ __forceinline__ OwnCones own_cones(const ConeDev &K, int a0, int a1) {
    OwnCones c;
    c.soc0 = lower_bound_i32(K.soc_off, K.nsoc, a0);
    c.soc1 = lower_bound_i32(K.soc_off, K.nsoc, a1);
    c.psd0 = lower_bound_i32(K.psd_off, K.npsd, a0);
    c.psd1 = lower_bound_i32(K.psd_off, K.npsd, a1);
    c.exp0 = triple_index(a0, K.exp_off, K.nexp);
    c.exp1 = triple_index(a1, K.exp_off, K.nexp);
    c.expd0 = triple_index(a0, K.expd_off, K.nexpd);
    c.expd1 = triple_index(a1, K.expd_off, K.nexpd);
    c.pow0 = triple_index(a0, K.pow_off, K.npow);
    c.pow1 = triple_index(a1, K.pow_off, K.npow);
    return c;
}

// Projection of rows [a0, a1) of the y-block onto K^*, by this workgroup
// alone (its own cones, see OwnCones); the same formulas as project_y.
template <bool WARM = false, typename Fin, typename Fout>
__device__ void project_y_own(const ConeDev &K, const OwnCones &oc, int a0, int a1, int Ls,
                              double *lds_psd, Fin fin, Fout fout, double *psd_v = nullptr,
                              const int64_t *psd_voff = nullptr, bool psd_warm = false) {
    const int tid = threadIdx.x, nt = blockDim.x;
    {
        const int fl = K.f + K.l;
        const int hi = a1 < fl ? a1 : fl;
        for (int i = a0 + tid; i < hi; i += nt) {
            const double a = fin(i);
            const double p = i < K.f ? a : (a > 0.0 ? a : 0.0);
            fout(i, p, a);
        }
    }
    if (oc.soc1 > oc.soc0) {
        const int gpb = nt / Ls, g = tid / Ls, gl = tid % Ls;
        for (int c0 = oc.soc0; c0 < oc.soc1; c0 += gpb) {
            const int cidx = c0 + g;
            const bool act = cidx < oc.soc1;
            int off = 0, len = 0;
            if (act) { off = K.soc_off[cidx]; len = K.soc_len[cidx]; }
            double ss = 0.0;
            for (int e = 1 + gl; e < len; e += Ls) {
                const double a = fin(off + e);
                ss += a * a;
            }
            ss = group_sum(ss, Ls);
            if (act) {
                const double t = fin(off);
                const double nrm = sqrt(ss);
                if (nrm <= t) {
                    for (int e = gl; e < len; e += Ls) { const double a = fin(off + e); fout(off + e, a, a); }
                } else if (nrm <= -t) {
                    for (int e = gl; e < len; e += Ls) { const double a = fin(off + e); fout(off + e, 0.0, a); }
                } else {
                    const double h = 0.5 * (t + nrm);
                    const double f = h / nrm;
                    for (int e = gl; e < len; e += Ls) {
                        const double a = fin(off + e);
                        fout(off + e, e == 0 ? h : f * a, a);
                    }
                }
            }
        }
    }
    for (int cidx = oc.psd0; cidx < oc.psd1; ++cidx) {
        const int off = K.psd_off[cidx];
        const int d = K.psd_dim[cidx];
        proj_psd_block<WARM>(d, lds_psd, [&](int e) { return fin(off + e); },
                             [&](int e, double p, double a) { fout(off + e, p, a); },
                             (WARM && psd_v != nullptr) ? psd_v + psd_voff[cidx] : nullptr, psd_warm);
    }
    // the dual cone of a primal exponential block is K_exp^*, of a dual block K_exp
    for (int e = oc.exp0 + tid; e < oc.exp1; e += nt) {
        const int off = K.exp_off + 3 * e;
        const double a0v = fin(off), a1v = fin(off + 1), a2v = fin(off + 2);
        double x = a0v, y = a1v, z = a2v;
        proj_exp_dual_dev(x, y, z);
        fout(off, x, a0v);
        fout(off + 1, y, a1v);
        fout(off + 2, z, a2v);
    }
    for (int e = oc.expd0 + tid; e < oc.expd1; e += nt) {
        const int off = K.expd_off + 3 * e;
        const double a0v = fin(off), a1v = fin(off + 1), a2v = fin(off + 2);
        double x = a0v, y = a1v, z = a2v;
        proj_exp_dev(x, y, z);
        fout(off, x, a0v);
        fout(off + 1, y, a1v);
        fout(off + 2, z, a2v);
    }
    // the dual cone of a power block K_pow^a is (K_pow^a)^*, of a dual block K_pow^a
    for (int e = oc.pow0 + tid; e < oc.pow1; e += nt) {
        const int off = K.pow_off + 3 * e;
        const double pa = K.pow_a[e];
        const double a0v = fin(off), a1v = fin(off + 1), a2v = fin(off + 2);
        double x = a0v, y = a1v, z = a2v;
        if (pa < 0.0) proj_pow_dev(x, y, z, -pa);
        else proj_pow_dual_dev(x, y, z, pa);
        fout(off, x, a0v);
        fout(off + 1, y, a1v);
        fout(off + 2, z, a2v);
    }
}

// Arrays of the own-row stage (FUSE kernels, rows of the workgroup's slice
// of A, ROW_STAGE x row_cap doubles of dynamic LDS), kept for the whole
// launch: the projection's argument, b, D, A u_x, A z0 of the next CG
// start, u_y, v_s, z_y and g_y.
using lds_f64 = __attribute__((address_space(3))) double;  // a double in LDS
constexpr int ROW_STAGE = 9;
enum RowStage { RS_ARG = 0, RS_B, RS_D, RS_AUX, RS_AZ, RS_UY, RS_VS, RS_ZY, RS_G };
// Arrays of the own-column stage (FUSE kernels, the workgroup's columns,
// COL_STAGE x col_cap doubles), kept for the whole launch: u_x, v_x, c, E,
// z_x and g_x.
constexpr int COL_STAGE = 6;
enum ColStage { CS_UX = 0, CS_V, CS_C, CS_E, CS_ZX, CS_G };

// Doubles of dynamic LDS that the iterate's vectors of a program take when
// they live in LDS (VLDS): u, v (n + m + 1 each), A u_x (m), then z_x, res,
// p0, p1 (n each) and z_y, t, A z_x (m each), each array in a double slot
// whatever T is.
__host__ __device__ constexpr int64_t vec_lds_doubles(int64_t n, int64_t m) {
    return 2 * (n + m + 1) + m + 4 * n + 3 * m;
}

// LDS doubles of a program's constants as run_solver copies them (lds_cst:
// b and D over m, c and E over n, g over n + m).
__host__ __device__ constexpr int64_t cst_lds_doubles(int64_t n, int64_t m) { return 3 * (n + m); }

// LDS doubles of a whole program's A and A^T as run_solver copies them
// (lds_mat: values in T, column indices, row pointers of both).
template <typename T>
__host__ __device__ constexpr int64_t mat_lds_doubles(int64_t n, int64_t m, int64_t nnz) {
    return (2 * nnz * (int64_t)sizeof(T) + 4 * (2 * nnz + m + n + 2) + 7) / 8;
}

// The method on one program.  Runs MODE_SOLVE, MODE_G or MODE_ITERATE.
// LONGR: the general instantiation, for matrices with long rows of A or
// A^T (taken by whole workgroups, see sweep) and cones with warm-started
// PSD projections (P.psd_v, see proj_psd_block); the default one keeps
// neither path.
// VLDS (a team of one workgroup): the iterate's vectors live in LDS at
// lds_vec (layout of vec_lds_doubles) instead of the program's global
// arrays, so every gather of a sweep and every update reads LDS; the caller
// fills them before and copies what it needs out after.
// DIRECT: the subspace projection applies P.Z = (I + A^T A)^{-1} (the
// direct method) instead of running CG; a separate instantiation.
template <typename T, bool SLABS = false, bool FUSE = false, bool PAIRS = false, bool LONGR = false,
          bool VLDS = false, bool DIRECT = false>
__device__ __forceinline__ void run_solver(const Prob<T> &P, const Settings &S, const Team &tm,
                           double *part, double *red_d, T *red_t, double *lds_psd,
                           double *lds_mat = nullptr, double *lds_vec = nullptr,
                           double *lds_cst = nullptr) {
    const int n = P.n, m = P.m;
    // the iterate's vectors (see VLDS)
    const int64_t NV = (int64_t)n + m + 1;
    double *const Pu = VLDS ? lds_vec : P.u;
    double *const Pv = VLDS ? lds_vec + NV : P.v;
    double *const Paux = VLDS ? lds_vec + 2 * NV : P.aux;
    T *const Pzx = VLDS ? reinterpret_cast<T *>(lds_vec + 2 * NV + m) : P.zx;
    T *const Pres = VLDS ? reinterpret_cast<T *>(lds_vec + 2 * NV + m + n) : P.res;
    T *const Pp0 = VLDS ? reinterpret_cast<T *>(lds_vec + 2 * NV + m + 2 * n) : P.p0;
    T *const Pp1 = VLDS ? reinterpret_cast<T *>(lds_vec + 2 * NV + m + 3 * n) : P.p1;
    T *const Pzy = VLDS ? reinterpret_cast<T *>(lds_vec + 2 * NV + m + 4 * n) : P.zy;
    T *const Pt = VLDS ? reinterpret_cast<T *>(lds_vec + 2 * NV + 2 * m + 4 * n) : P.t;
    T *const Pazc = VLDS ? reinterpret_cast<T *>(lds_vec + 2 * NV + 3 * m + 4 * n) : P.azc;
    const int tid = threadIdx.x, nt = blockDim.x;
    const bool is_g = S.mode == MODE_G;
    // The program's constants b, c, D, E and g: from global memory or,
    // given lds_cst (cst_lds_doubles(n, m)), copied there once per solve
    // (g only outside MODE_G, which writes it).
    const double *Pb = P.b, *Pc = P.c, *PD = P.D, *PE = P.E, *Pg = P.g;
    if (lds_cst != nullptr) {
        double *cb = lds_cst, *cD = cb + m, *cc = cD + m, *cE = cc + n, *cg = cE + n;
        for (int i = tid; i < m; i += nt) { cb[i] = P.b[i]; cD[i] = P.D[i]; }
        for (int j = tid; j < n; j += nt) { cc[j] = P.c[j]; cE[j] = P.E[j]; }
        if (!is_g)
            for (int e = tid; e < n + m; e += nt) cg[e] = P.g[e];
        __syncthreads();
        Pb = cb;
        PD = cD;
        Pc = cc;
        PE = cE;
        if (!is_g) Pg = cg;
    }
    const int a0 = P.part_a[tm.rank], a1 = P.part_a[tm.rank + 1];
    const int t0 = P.part_t[tm.rank], t1 = P.part_t[tm.rank + 1];
    const int LA = S.lanes_a, LT = S.lanes_t;
    // t_i and the gathered copy of u_y: in the gather pairs (PAIRS) or in
    // their own arrays.  Gather pairs halve the requests of the A^T test
    // sweep, which pays where the gathers are latency-bound; where they
    // stream through L2 (slab sweeps) separate arrays keep more values per
    // line.
    auto t_get = [&](int i) -> T { if constexpr (PAIRS) return P.tu[i].a; else return Pt[i]; };
    auto t_set = [&](int i, T x) { if constexpr (PAIRS) P.tu[i].a = x; else Pt[i] = x; };
    auto uy_get = [&](int i) -> double { if constexpr (PAIRS) return P.tu[i].b; else return Pu[n + i]; };
    // This workgroup's rows of A and A^T: from global memory, or copied once
    // into LDS (values, column indices, row pointers rebased to the slice)
    // when lds_mat is given.  Row i is read through rpa[i - ra] and
    // rpa[i - ra + 1], with ra = a0 for the slice and 0 otherwise.  The
    // offset is applied to the index, never to the pointer: an LDS pointer
    // moved below the start of the LDS window wraps in 32 bits, and once
    // widened to a generic address the later add carries out of the LDS
    // aperture.  In FP32 mode the tests' FP64 values stay in global memory,
    // offset to the same local positions.
    const int32_t *rpa = P.A.rp, *cia = P.A.ci, *rpt = P.AT.rp, *cit = P.AT.ci;
    int ra = 0, rt = 0;
    const T *va = P.Ac.v, *vt = P.ATc.v;
    const double *va64 = P.A.v, *vt64 = P.AT.v;
    if (lds_mat != nullptr) {
        const int ka0 = P.A.rp[a0], ka1 = P.A.rp[a1];
        const int kt0 = P.AT.rp[t0], kt1 = P.AT.rp[t1];
        const int na = ka1 - ka0, nt_ = kt1 - kt0;
        T *lva = reinterpret_cast<T *>(lds_mat);
        T *lvt = lva + na;
        int32_t *lca = reinterpret_cast<int32_t *>(lvt + nt_);
        int32_t *lct = lca + na;
        int32_t *lra = lct + nt_;
        int32_t *lrt = lra + (a1 - a0 + 1);
        for (int k = tid; k < na; k += nt) { lva[k] = P.Ac.v[ka0 + k]; lca[k] = P.A.ci[ka0 + k]; }
        for (int k = tid; k < nt_; k += nt) { lvt[k] = P.ATc.v[kt0 + k]; lct[k] = P.AT.ci[kt0 + k]; }
        for (int r = tid; r <= a1 - a0; r += nt) lra[r] = P.A.rp[a0 + r] - ka0;
        for (int r = tid; r <= t1 - t0; r += nt) lrt[r] = P.AT.rp[t0 + r] - kt0;
        __syncthreads();
        rpa = lra;
        ra = a0;
        rpt = lrt;
        rt = t0;
        cia = lca;
        cit = lct;
        va = lva;
        vt = lvt;
        if constexpr (sizeof(T) == 8) {
            va64 = reinterpret_cast<const double *>(lva);
            vt64 = reinterpret_cast<const double *>(lvt);
        } else {
            va64 = P.A.v + ka0;
            vt64 = P.AT.v + kt0;
        }
    }
    // Long rows of this workgroup's slices of A and A^T (row-group sweeps):
    // a row is long when its group of L lanes would take more than
    // LONG_CHUNKS chunks for it.  Found once per launch; a workgroup without
    // any keeps the plain row-group sweeps.
    auto long_threshold = [&](const int32_t *rp, int ra_, int r0, int r1, int L) -> int {
        if (SLABS || !LONGR || L >= nt) return 0;
        const int thr = LONG_CHUNKS * ROW_CHUNK * L;
        bool f = false;
        for (int i = r0 + tid; i < r1; i += nt) f |= (rp[i - ra_ + 1] - rp[i - ra_]) > thr;
        return block_any(f, reinterpret_cast<unsigned long long *>(red_d)) ? thr : 0;
    };
    const int long_a = LONGR ? long_threshold(rpa, ra, a0, a1, LA) : 0;
    const int long_t = LONGR ? long_threshold(rpt, rt, t0, t1, LT) : 0;
    // LDS of the slab sweeps (unused without slabs)
    const SlabLds<T> sll = slab_lds<T>(lds_psd + (S.slab_lds > 0 ? S.slab_lds : 0), SLABS ? S.slab_rows : 0);
    const double sigma = uniform(P.scal[SC_SIGMA]), rho = uniform(P.scal[SC_RHO]);
    const double eta = is_g ? 1.0 : uniform(P.scal[SC_ETA]);
    const double nb = uniform(P.scal[SC_NORM_B]), nc = uniform(P.scal[SC_NORM_C]);
    const double ndb = uniform(P.scal[SC_NORM_DINV_BH]), nec = uniform(P.scal[SC_NORM_EINV_CH]);
    const double alpha = S.alpha;
    double tau = uniform(Pu[n + m]);
    double kappa = uniform(Pv[n + m]);
    long long cg_total = 0, spmv = 0;
    int k = 0;
    int status = 0;
    bool ok = true;
    const double qnan = __builtin_nan("");
    double r_pri = HUGE_VAL, r_dual = HUGE_VAL, r_gap = HUGE_VAL, pobj = qnan, dobj = qnan;
    double r_inf = HUGE_VAL, r_unb = HUGE_VAL;  // certificate test ratios (pass at <= eps)
    double last_bty = 0.0, last_ctx = 0.0;
    T *pold = Pp0, *pnew = Pp1;

    // The update of an iteration (SMW, relaxation, projection, dual
    // update) needs no barrier of its own (FUSE): its y-block part runs at
    // the start of the next A-sweep phase on the workgroup's own rows and
    // cones, its x-block part in the next A^T-sweep phase on the workgroup's
    // own columns.  In between, nothing reads another workgroup's u_x: the
    // A-sweep's test takes A u_x from the row-wise product carried by the
    // y-block part (Paux).
    //
    // FUSE is set for the cooperative kernel with row-group sweeps, whose
    // phases are short enough for a team barrier to matter.  The slab
    // kernel's phases last about a millisecond, and the batched kernel's
    // barrier is a workgroup barrier: there the update is applied at the end
    // of the iteration, followed by a team barrier.
    const OwnCones own = own_cones(P.cone, a0, a1);
    // The own-row and own-column stages: the workgroup's rows and columns
    // of every vector the fused updates, the A-phase and the A^T-sweep's
    // epilogue read, filled once per launch and kept current wherever the
    // launch writes those vectors, so that none of them waits on global
    // memory after a team barrier.  The global arrays are still written for
    // the other workgroups, the product sweeps, the state and the outputs.
    // (has_rs / has_cs say whether the stages exist; rs and cs are LDS
    // pointers, so that every stage access is an LDS access; a generic
    // pointer that may point into LDS, used in vector code, trips the
    // gfx950 instruction selector)
    const bool has_rs = FUSE && S.row_cap > 0, has_cs = FUSE && S.col_cap > 0;
    lds_f64 *const rs = (lds_f64 *)(lds_psd + (has_rs ? S.row_lds : 0));
    const int rcap = S.row_cap;
    auto RS = [&](int a, int i) -> lds_f64 & { return rs[a * rcap + (i - a0)]; };
    lds_f64 *const cs = (lds_f64 *)(lds_psd + (has_cs ? S.col_lds : 0));
    const int ccap = S.col_cap;
    auto CS = [&](int a, int j) -> lds_f64 & { return cs[a * ccap + (j - t0)]; };
    if (has_rs) {
        for (int i = a0 + tid; i < a1; i += nt) {
            RS(RS_B, i) = Pb[i];
            RS(RS_D, i) = PD[i];
            RS(RS_G, i) = Pg[n + i];
            RS(RS_UY, i) = Pu[n + i];
            RS(RS_VS, i) = Pv[n + i];
            RS(RS_AUX, i) = Paux[i];
            RS(RS_AZ, i) = (double)Pazc[i];
            RS(RS_ZY, i) = (double)Pzy[i];
        }
    }
    if (has_cs) {
        for (int j = t0 + tid; j < t1; j += nt) {
            CS(CS_UX, j) = Pu[j];
            CS(CS_V, j) = Pv[j];
            CS(CS_C, j) = Pc[j];
            CS(CS_E, j) = PE[j];
            CS(CS_ZX, j) = (double)Pzx[j];
            CS(CS_G, j) = Pg[j];
        }
    }
    if (has_rs || has_cs) __syncthreads();
    const bool record = S.mode == MODE_ITERATE && P.hist_u != nullptr;
    // With both stages, FP64 and no recording, the global copies of the
    // vectors no other workgroup reads during the launch (u, v, z_y, A u_x,
    // A z0 of the own rows; u_x, z_x of the own columns) are written once,
    // from the stages, when the launch ends.
    const bool defer = has_rs && has_cs && sizeof(T) == 8 && !record;
    // PSD projections start from the previous update's eigenvectors once
    // this launch has made one (P.psd_v; see proj_psd_block)
    bool psd_warm = false;
    bool pending = false;  // an update whose writes are still to be made
    double sfac = 0.0;     // h^T z / eta of the pending update
    double wt_upd = 0.0;   // tau + kappa of the iterate the pending update starts from
    // y-block part of the pending update: own rows and cones, tau and kappa
    auto apply_y = [&]() {
        const double *gy = Pg + n;
        double *uy = Pu + n;
        double *vs = Pv + n;
        const T *zy = Pzy;
        if (has_rs) {
            // the same arithmetic as below, on the stage
            for (int i = a0 + tid; i < a1; i += nt) {
                const double uo = RS(RS_UY, i), vo = RS(RS_VS, i), bi = RS(RS_B, i);
                const double zi = RS(RS_ZY, i), gi = RS(RS_G, i);
                const double ao = RS(RS_AUX, i);
                const double ry = (uo + vo) - wt_upd * bi;
                const double azx = zi - ry;
                const double agx = gi - bi;
                const double an = alpha * (azx - sfac * agx) + (1.0 - alpha) * ao;
                if (!defer) Paux[i] = an;
                const T az = T(azx);
                if (!defer) Pazc[i] = az;
                const double ut = zi - gi * sfac;
                const double ub = alpha * ut + (1.0 - alpha) * uo;
                RS(RS_ARG, i) = ub - vo;
                RS(RS_AUX, i) = an;
                RS(RS_AZ, i) = (double)az;
            }
            __syncthreads();
            auto fin = [&](int i) -> double { return RS(RS_ARG, i); };
            auto fout = [&](int i, double pv, double a) {
                if (!defer) uy[i] = pv;
                if (!defer) vs[i] = pv - a;
                if constexpr (PAIRS) P.tu[i].b = pv;
                RS(RS_UY, i) = pv;
                RS(RS_VS, i) = pv - a;
            };
            project_y_own<LONGR>(P.cone, own, a0, a1, S.lanes_soc, lds_psd, fin, fout, P.psd_v, P.psd_voff,
                                 psd_warm);
            psd_warm = true;
            if (tm.rank == 0 && tid == 0) { Pu[n + m] = tau; Pv[n + m] = kappa; }
            return;
        }
        // A u_x of the new iterate by linearity: u_x+ = alpha (z_x - g_x s)
        // + (1 - alpha) u_x with A z_x = z_y - r_y (CG accumulates z_y =
        // r_y + A z_x) and A g_x = g_y - b (the g pass has r_y = b); r_y of
        // the update from the old u_y, v_s.  |1 - alpha| < 1, so rounding
        // does not grow from one update to the next.
        // A z_x itself is kept in azc: z_x is the next CG's start point z0,
        // so the next A-sweep can take A z0 from there instead of a product.
        for (int i = a0 + tid; i < a1; i += nt) {
            const double ry = (uy[i] + vs[i]) - wt_upd * Pb[i];
            const double azx = (double)zy[i] - ry;
            const double agx = gy[i] - Pb[i];
            Paux[i] = alpha * (azx - sfac * agx) + (1.0 - alpha) * Paux[i];
            Pazc[i] = T(azx);
        }
        __syncthreads();  // the projection below overwrites u_y and v_s
        auto fin = [&](int i) -> double {
            const double ut = (double)zy[i] - gy[i] * sfac;
            const double ub = alpha * ut + (1.0 - alpha) * uy[i];
            return ub - vs[i];
        };
        auto fout = [&](int i, double pv, double a) {
            uy[i] = pv;
            vs[i] = pv - a;
            if constexpr (PAIRS) P.tu[i].b = pv;
        };
        project_y_own<LONGR>(P.cone, own, a0, a1, S.lanes_soc, lds_psd, fin, fout, P.psd_v, P.psd_voff,
                             psd_warm);
        psd_warm = true;
        if (tm.rank == 0 && tid == 0) { Pu[n + m] = tau; Pv[n + m] = kappa; }
    };
    // x-block part of the pending update: own columns (v_x stays 0)
    auto apply_x = [&]() {
        if (has_cs) {
            for (int j = t0 + tid; j < t1; j += nt) {
                const double ux = relaxed_ux(CS(CS_ZX, j), CS(CS_G, j), CS(CS_UX, j), sfac, alpha);
                if (!defer) Pu[j] = ux;
                CS(CS_UX, j) = ux;
            }
            return;
        }
        for (int j = t0 + tid; j < t1; j += nt) Pu[j] = relaxed_ux((double)Pzx[j], Pg[j], Pu[j], sfac, alpha);
    };
    // u_x of the current iterate as the A-sweep's test gather sees it.  With
    // FUSE the x-block part of the pending update is applied only after the
    // A-phase, so there u_x is formed here from the same values by the same
    // expression as apply_x will store.
    auto ux_now = [&](int j) -> double {
        if (FUSE && pending) return relaxed_ux((double)Pzx[j], Pg[j], Pu[j], sfac, alpha);
        return Pu[j];
    };
    // the gather pairs of the start point (own rows and columns), visible to
    // the team before the first sweep
    if constexpr (PAIRS) {
        for (int i = a0 + tid; i < a1; i += nt) P.tu[i].b = Pu[n + i];
        if (!team_sync(tm)) ok = false;
    }
    while (ok) {
        // the own-row stage holds this update's rows (FUSE: the update is
        // applied just below)
        const bool pending_rows = FUSE && pending;
        if (FUSE && pending) {
            apply_y();
            __syncthreads();  // own rows of u_y and v_s are read below by other threads
        }
        if (record && k <= S.record) {
            const size_t N = (size_t)n + m + 1;
            double *hu = P.hist_u + (size_t)k * N;
            double *hv = P.hist_v + (size_t)k * N;
            for (int i = a0 + tid; i < a1; i += nt) { hu[n + i] = Pu[n + i]; hv[n + i] = Pv[n + i]; }
            if (tm.rank == 0 && tid == 0) { hu[n + m] = tau; hv[n + m] = kappa; }
        }
        // kk: the iteration number (k0 > 0 for a resumed state)
        const int kk = S.k0 + k;
        const bool check = (S.mode == MODE_SOLVE) &&
                           ((kk % S.check_every) == 0 || kk >= S.max_iters);
        const double wt = tau + kappa;
        // the products of the start point: carried from a saved state, or
        // made on the first update of the launch
        const bool first_products = k == 0 && !S.carried;
        // the test product A u_x: gathered on the first update of a launch
        // (also without tests, so that the carried value of a saved state
        // is valid), carried row by row (Paux) after that.  In FP32 mode
        // the carried value would rest on the FP32 products of CG, so every
        // check gathers it with the FP64 values and the tests stay FP64
        // tests.
        const bool gather_ax = (first_products && !is_g) || (check && sizeof(T) == 4);


        // ---------------- A-sweep: t0 = r_y + A z0, tests: A u_x ----------------
        double accA[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // |r_y|^2, pri^2, unb^2, b^T u_y, b^T z_y
        T noT[1] = {T(0)};
        auto epi_a = [&](int i, T st, double sg) {
            const double uy = Pu[n + i], vs = Pv[n + i], bi = Pb[i];
            const double ry = (uy + vs) - wt * bi;
            const T tv = T(ry) + st;
            Pzy[i] = tv;
            t_set(i, tv);
            accA[0] += ry * ry;
            accA[4] += bi * (double)tv;
            if (has_rs) RS(RS_ZY, i) = (double)tv;
            if (gather_ax) {
                Paux[i] = sg;
                if (has_rs) RS(RS_AUX, i) = sg;
            }
            if (check) {
                const double sc = gather_ax ? sg : Paux[i];
                const double Di = PD[i];
                const double pr = (sc + vs - bi * tau) / Di;
                const double un = (sc + vs) / Di;
                accA[1] += pr * pr;
                accA[2] += un * un;
                accA[3] += bi * uy;
            }
        };
        // A z0 by a product on the first update of a launch; after that
        // from the previous CG (kept in azc by the update: z_y - r_y), in
        // FP32 mode recomputed every 32 updates, since that recurrence,
        // unlike the one for A u_x, does not damp rounding.  A sweep made
        // for the FP64 gather of A u_x computes it too.
        const bool product_a = first_products || gather_ax || (sizeof(T) == 4 && (kk & 31) == 0);
        if (product_a) {
            sweep<T, SLABS>(a0, a1, LA, gather_ax, rpa, ra, P.slabs_a, P.off_a, m, sll,
                            cia, va, va64, [&](int j) { return Pzx[j]; }, ux_now, epi_a, long_a, red_d);
        } else if (has_rs && pending_rows) {
            // epi_a on the own-row stage (no check gathers after the first update)
            for (int i = a0 + tid; i < a1; i += nt) {
                const double uy = RS(RS_UY, i), vs = RS(RS_VS, i), bi = RS(RS_B, i);
                const double ry = (uy + vs) - wt * bi;
                const T tv = T(ry) + T(RS(RS_AZ, i));
                if (!defer) Pzy[i] = tv;
                RS(RS_ZY, i) = (double)tv;
                t_set(i, tv);
                accA[0] += ry * ry;
                accA[4] += bi * (double)tv;
                if (check) {
                    const double sc = RS(RS_AUX, i);
                    const double Di = RS(RS_D, i);
                    const double pr = (sc + vs - bi * tau) / Di;
                    const double un = (sc + vs) / Di;
                    accA[1] += pr * pr;
                    accA[2] += un * un;
                    accA[3] += bi * uy;
                }
            }
        } else {
            for (int i = a0 + tid; i < a1; i += nt) epi_a(i, Pazc[i], 0.0);
        }
        // The totals of accA are first needed after the next phase.  The
        // slot alternates between iterations: a workgroup may write the next
        // iteration's partials before another has read these.
        const int slot_a = (k & 1) ? SLOT_A2 : SLOT_A;
        if (!phase_put<5, 0>(tm, part, slot_a, accA, noT, red_d, red_t)) { ok = false; break; }

        // the pending x-block update on the own columns
        const bool colst = has_cs;
        if (FUSE && pending) {
            apply_x();
            pending = false;
            __syncthreads();  // read below by the threads that finish the columns
        }
        if (record && k <= S.record) {
            const size_t N = (size_t)n + m + 1;
            double *hu = P.hist_u + (size_t)k * N;
            double *hv = P.hist_v + (size_t)k * N;
            for (int j = t0 + tid; j < t1; j += nt) { hu[j] = Pu[j]; hv[j] = Pv[j]; }
        }

        // ---------------- AT-sweep: res0 = r_x - z0 - A^T t0, tests: A^T u_y ----------------
        double accB[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // |r_x|^2, dual^2, inf^2, c^T u_x, c^T z_x
        T accBt[1] = {T(0)};                         // |res|^2
        sweep<T, SLABS>(t0, t1, LT, check, rpt, rt, P.slabs_t, P.off_t, n, sll,
                 cit, vt, vt64, t_get, uy_get,
                 [&](int j, T st, double sc) {
                     const double ux = colst ? CS(CS_UX, j) : Pu[j];
                     const double cj = colst ? CS(CS_C, j) : Pc[j];
                     const double vj = colst ? CS(CS_V, j) : Pv[j];
                     const double rx = (ux + vj) - wt * cj;
                     const T zxj = colst ? T(CS(CS_ZX, j)) : Pzx[j];
                     const T r = (T(rx) - zxj) - st;
                     Pres[j] = r;
                     accBt[0] = tfma(r, r, accBt[0]);
                     accB[0] += rx * rx;
                     accB[4] += cj * (double)zxj;
                     if (check) {
                         const double Ej = colst ? CS(CS_E, j) : PE[j];
                         const double dr = (sc + cj * tau) / Ej;
                         const double fi = sc / Ej;
                         accB[1] += dr * dr;
                         accB[2] += fi * fi;
                         accB[3] += cj * ux;
                     }
                 }, long_t, red_d);
        if (!phase_put<5, 1>(tm, part, SLOT_B, accB, accBt, red_d, red_t)) { ok = false; break; }
        // the CG tolerance of this update, (k + 1)^-zeta, computed while
        // the first wavefront gathers the partials
        __shared__ double s_tolk;
        phase_collect<5, 1, 5>(tm, part, SLOT_B, accB, accBt, red_d, red_t, slot_a, accA, [&]() {
            if (threadIdx.x == blockDim.x - 1) s_tolk = pow((double)kk + 1.0, -S.zeta_pow);
        });
        const double tolk = s_tolk;

        T rho_cg = accBt[0];
        double hz = accA[4] + accB[4];
        const double rnorm = sqrt(accA[0] + accB[0]);

        if (check) {
            const bool finite = isfinite(accA[1] + accA[2] + accA[3] + accB[1] + accB[2] + accB[3]) &&
                                isfinite((double)rho_cg) && isfinite(tau) && isfinite(kappa) &&
                                isfinite(rnorm);
            const double bty = accA[3], ctx = accB[3];
            last_bty = bty;
            last_ctx = ctx;
            bool solved = false;
            if (tau > 0.0) {
                r_pri = sqrt(accA[1]) / (sigma * tau);
                r_dual = sqrt(accB[1]) / (rho * tau);
                const double cx = ctx / (rho * sigma * tau);
                const double by = bty / (rho * sigma * tau);
                r_gap = fabs(cx + by);
                pobj = cx;
                dobj = -by;
                solved = r_pri <= S.eps_pri * (1.0 + nb) && r_dual <= S.eps_dual * (1.0 + nc) &&
                         r_gap <= S.eps_gap * (1.0 + fabs(cx) + fabs(by));
            } else {
                r_pri = HUGE_VAL; r_dual = HUGE_VAL; r_gap = HUGE_VAL;
                pobj = qnan; dobj = qnan;
            }
            const bool infeas = nb > 0.0 && -bty > 0.0 && sqrt(accB[2]) <= (-bty / ndb) * S.eps_infeas;
            const bool unbdd = nc > 0.0 && -ctx > 0.0 && sqrt(accA[2]) <= (-ctx / nec) * S.eps_unbdd;
            r_inf = (nb > 0.0 && -bty > 0.0) ? sqrt(accB[2]) * ndb / -bty : HUGE_VAL;
            r_unb = (nc > 0.0 && -ctx > 0.0) ? sqrt(accA[2]) * nec / -ctx : HUGE_VAL;
            if (!finite) status = 5;
            else if (solved) status = 1;
            else if (infeas) status = 3;
            else if (unbdd) status = 4;
            if (status) break;
            if (kk >= S.max_iters) { status = tau > 0.0 ? 2 : 5; break; }
        }
        if (!is_g && kk >= S.max_iters) { status = 2; break; }

        // ---------------- CG on (I + A^T A) z_x = r_x - A^T r_y ----------------
        double tol;
        if (is_g) {
            // g = M^{-1} h to a tight relative tolerance, once (Sect. 4.1);
            // r = h here, so rnorm = |h|
            tol = S.tight_tol * fmax(rnorm, 1.0);
        } else if (S.tight_tol > 0.0) {
            tol = S.tight_tol * rnorm;
        } else {
            tol = tolk;
            if (sizeof(T) == 4) tol = fmax(tol, S.fp32_floor * rnorm);
        }
        int it = 0;
        T beta = T(0);
        if constexpr (DIRECT) {
            // Direct projection (Sect. 4.1, cached factorization): with
            // res0 = rhs - (I + A^T A) z0 from the A^T-sweep, the exact
            // solution is z_x = z0 + p with p = Z res0 (Z = (I + A^T A)^{-1},
            // formed at setup), and z_y = t0 + A p.  Phase 1: p on the own
            // columns, one wavefront per row of Z, lanes striding over its
            // entries, summed in a fixed order.
            {
                // lane l of a wavefront takes the entry pairs (2l, 2l + 1),
                // (2l + 128, 2l + 129), ... of the row (16-byte loads; the
                // rows are padded to an even length with zeros beyond n)
                // into DIRECT_UNROLL accumulators (their loads in flight
                // together), added in order, then across the lanes
                constexpr int U = DIRECT_UNROLL;
                const int lane = tid & (WAVE - 1), wid = tid / WAVE, nw = nt / WAVE;
                for (int j = t0 + wid; j < t1; j += nw) {
                    const f64x2 *zr = reinterpret_cast<const f64x2 *>(P.Z + (int64_t)j * P.ldz);
                    double acc[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) acc[u] = 0.0;
                    for (int q0 = lane; 2 * q0 < n; q0 += U * WAVE) {
                        f64x2 zv[U];
                        double r0[U], r1[U];
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const int q = 2 * (q0 + u * WAVE);
                            zv[u] = q < n ? __builtin_nontemporal_load(zr + q0 + u * WAVE) : f64x2{0.0, 0.0};
                            r0[u] = q < n ? (double)Pres[q] : 0.0;
                            r1[u] = q + 1 < n ? (double)Pres[q + 1] : 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            acc[u] = __builtin_fma(zv[u].y, r1[u], __builtin_fma(zv[u].x, r0[u], acc[u]));
                    }
                    double a = acc[0];
#pragma unroll
                    for (int u = 1; u < U; ++u) a += acc[u];
                    a = group_sum(a, WAVE);
                    if (lane == 0) pnew[j] = T(a);
                }
            }
            if (!team_sync(tm)) { ok = false; break; }
            // Phase 2: t = A p on the own rows, z_y = t0 + t; z_x += p on
            // the own columns; c^T z_x and b^T z_y for h^T z
            double accQ[2] = {0.0, 0.0};
            T noT[1] = {T(0)};
            sweep<T, SLABS>(a0, a1, LA, false, rpa, ra, P.slabs_a, P.off_a, m, sll,
                     cia, va, va64, [&](int j) { return pnew[j]; }, [&](int) { return 0.0; },
                     [&](int i, T st, double) {
                         const T z = (has_rs ? T(RS(RS_ZY, i)) : Pzy[i]) + st;
                         if (!defer) Pzy[i] = z;
                         if (has_rs) RS(RS_ZY, i) = (double)z;
                         accQ[1] += Pb[i] * (double)z;
                     }, long_a, red_d);
            for (int j = t0 + tid; j < t1; j += nt) {
                const T z = (has_cs ? T(CS(CS_ZX, j)) : Pzx[j]) + pnew[j];
                if (!defer) Pzx[j] = z;
                if (has_cs) CS(CS_ZX, j) = (double)z;
                accQ[0] += Pc[j] * (double)z;
            }
            if (!phase_end<2, 0>(tm, part, SLOT_P2, accQ, noT, red_d, red_t)) { ok = false; break; }
            hz = accQ[0] + accQ[1];
            rho_cg = T(0);  // no CG iterations follow
        }
        while (!DIRECT && sqrt((double)rho_cg) > tol && it < S.cg_max) {
            const bool first = (it == 0);
            // A-sweep: t = A p
            T accP[2] = {T(0), T(0)};  // |t|^2, |p|^2
            double noD[1] = {0.0};
            sweep<T, SLABS>(a0, a1, LA, false, rpa, ra, P.slabs_a, P.off_a, m, sll,
                     cia, va, va64, [&](int j) { return cg_dir(Pres, pold, beta, j, first); },
                     [&](int) { return 0.0; },
                     [&](int i, T st, double) {
                         t_set(i, st);
                         accP[0] = tfma(st, st, accP[0]);
                     }, long_a, red_d);
            for (int j = t0 + tid; j < t1; j += nt) {
                const T pj = cg_dir(Pres, pold, beta, j, first);
                pnew[j] = pj;
                accP[1] = tfma(pj, pj, accP[1]);
            }
            if (!phase_end<0, 2>(tm, part, SLOT_P1, noD, accP, red_d, red_t)) { ok = false; break; }
            const T a_cg = rho_cg / (accP[0] + accP[1]);
            // A^T-sweep: z_x += a p, res -= a (p + A^T t); z_y += a t
            double accQ[2] = {0.0, 0.0};  // c^T z_x, b^T z_y
            T accQt[1] = {T(0)};          // |res|^2
            sweep<T, SLABS>(t0, t1, LT, false, rpt, rt, P.slabs_t, P.off_t, n, sll,
                     cit, vt, vt64, t_get, [&](int) { return 0.0; },
                     [&](int j, T st, double) {
                         const T pj = pnew[j];
                         const T z = tfma(a_cg, pj, has_cs ? T(CS(CS_ZX, j)) : Pzx[j]);
                         if (!defer) Pzx[j] = z;
                         if (has_cs) CS(CS_ZX, j) = (double)z;
                         const T r = Pres[j] - a_cg * (pj + st);
                         Pres[j] = r;
                         accQt[0] = tfma(r, r, accQt[0]);
                         accQ[0] += Pc[j] * (double)z;
                     }, long_t, red_d);
            for (int i = a0 + tid; i < a1; i += nt) {
                const T z = tfma(a_cg, t_get(i), has_rs ? T(RS(RS_ZY, i)) : Pzy[i]);
                if (!defer) Pzy[i] = z;
                if (has_rs) RS(RS_ZY, i) = (double)z;
                accQ[1] += Pb[i] * (double)z;
            }
            if (!phase_end<2, 1>(tm, part, SLOT_P2, accQ, accQt, red_d, red_t)) { ok = false; break; }
            const T rho_new = accQt[0];
            beta = rho_new / rho_cg;
            rho_cg = rho_new;
            hz = accQ[0] + accQ[1];
            T *sw = pold; pold = pnew; pnew = sw;
            ++it;
        }
        if (!ok) break;
        cg_total += it;
        spmv += 2 + 2 * it;

        if (is_g) {
            for (int j = t0 + tid; j < t1; j += nt) P.g[j] = (double)Pzx[j];
            for (int i = a0 + tid; i < a1; i += nt) P.g[n + i] = (double)Pzy[i];
            if (tm.rank == 0 && tid == 0) P.scal[SC_ETA] = 1.0 + hz;
            status = 1;
            break;
        }

        // ---------------- SMW, relaxation, projection, dual update ----------------
        // the scalars now; the vector writes at the start of the next phases
        sfac = hz / eta;
        wt_upd = wt;
        const double ut_tau = wt + sfac;
        const double ub_tau = alpha * ut_tau + (1.0 - alpha) * tau;
        const double tau_new = fmax(ub_tau - kappa, 0.0);
        const double kappa_new = (kappa - ub_tau) + tau_new;
        tau = tau_new;
        kappa = kappa_new;
        pending = true;
        if constexpr (!FUSE) {
            apply_y();
            apply_x();
            pending = false;
            if (!team_sync(tm)) { ok = false; break; }
        }
        ++k;
    }

    if (defer) {
        for (int i = a0 + tid; i < a1; i += nt) {
            Pu[n + i] = RS(RS_UY, i);
            Pv[n + i] = RS(RS_VS, i);
            Paux[i] = RS(RS_AUX, i);
            Pazc[i] = T(RS(RS_AZ, i));
            Pzy[i] = T(RS(RS_ZY, i));
        }
        for (int j = t0 + tid; j < t1; j += nt) {
            Pu[j] = CS(CS_UX, j);
            Pzx[j] = T(CS(CS_ZX, j));
        }
    }
    if (tm.rank == 0 && tid == 0) {
        double *inf = P.info;
        inf[INFO_ABORT] = ok ? 0.0 : 1.0;
        inf[INFO_STATUS] = ok ? (double)status : 5.0;
        inf[INFO_ITERS] = (double)(S.k0 + k);
        inf[INFO_RES_PRI] = r_pri;
        inf[INFO_RES_DUAL] = r_dual;
        inf[INFO_GAP] = r_gap;
        inf[INFO_POBJ] = pobj;
        inf[INFO_DOBJ] = dobj;
        inf[INFO_TAU] = tau;
        inf[INFO_KAPPA] = kappa;
        inf[INFO_CG_ITERS] = (double)cg_total;
        inf[INFO_SPMV] = (double)spmv;
        inf[INFO_BTY] = last_bty;
        inf[INFO_CTX] = last_ctx;
        inf[INFO_RES_INF] = r_inf;
        inf[INFO_RES_UNB] = r_unb;
    }
}

}  // namespace hsd
