// Batched solves: many independent cone programs in one persistent launch.
//
// One workgroup solves one program at a time, taking programs from a device
// queue over the programs sorted largest first: the preparation takes them
// in that order, the solve from both ends alternately (see k_batch).
// Everything a solve needs after the one-off
// structural setup runs inside the launch: the equilibration of that
// program (Sect. 5), g = M^{-1} h (Sect. 4.1), the iteration with its
// termination tests (Sect. 3) and the outputs.  The launch (and the reset of
// the queue before it) is captured once into a hipGraph and replayed by
// every hsd_batch_solve.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "hsd_host.h"
#include "hsd_solver.h"

namespace hsd {

// Per-program description (offsets into the block-diagonal arrays and the
// concatenated cone tables).
struct InstDesc {
    int32_t r0, c0, m, n;      // first row / column in the block-diagonal matrix
    int32_t u0;                // first entry of this program's u and v (r0 + c0 + index)
    int32_t soc0, nsoc, psd0, npsd, blk0, nblk;
    int32_t f, l, nexp, exp_off, nexpd, expd_off;
    int32_t npow, pow_off, pow0;
};

struct BatchArgs {
    int32_t B;
    const InstDesc *desc;
    const int32_t *order;     // programs, largest first (the queue order of the preparation)
    int32_t *queue;           // next queue position
    const int32_t *parts;     // per program {0, m, 0, n}
    const int32_t *rpA, *ciA, *rpT, *ciT;
    const double *vA0, *vT0;  // original values
    double *vA, *vT;          // scaled values
    float *vA32, *vT32;       // FP32 copies (FP32 mode) or null
    const double *b0, *c0;    // original right-hand sides
    double *bh, *ch, *D, *E, *dtmp, *g, *u, *v;
    double *zx, *zy, *res, *p0, *p1, *t;   // sized for doubles
    double *tu;                       // gather pairs (16 bytes per entry)
    double *aux;                      // A u_x per row
    double *azc;                      // A z_x of the last CG per row (sized for doubles)
    double *scal, *info;      // SC_COUNT / INFO_COUNT per program
    const int32_t *soc_off, *soc_len, *psd_off, *psd_dim, *blk_off, *blk_len;
    const double *pow_a;      // power-cone parameters of every program, concatenated
    double *x_out, *y_out, *s_out;
    int32_t scale;
    const void *probs_g;      // Prob<double>[B] for the g pass
    const void *probs_t;      // Prob<T>[B] for the solve
};

// Per-program descriptors are built on the host and read from device memory.
// The kernels refer to a program's descriptor in place (a reference into
// this read-only array) instead of copying it: a copy of its ~50 pointers
// would be held in registers for the whole solve, while fields read in place
// are loaded where they are used.

template <typename T>
__host__ __device__ Prob<T> inst_prob(const BatchArgs &BA, const InstDesc &d, int i) {
    Prob<T> P{};
    P.m = d.m;
    P.n = d.n;
    P.A = {BA.rpA + d.r0, BA.ciA, BA.vA};
    P.AT = {BA.rpT + d.c0, BA.ciT, BA.vT};
    if constexpr (sizeof(T) == 4) {
        P.Ac = {P.A.rp, P.A.ci, BA.vA32};
        P.ATc = {P.AT.rp, P.AT.ci, BA.vT32};
    } else {
        P.Ac = P.A;
        P.ATc = P.AT;
    }
    ConeDev &K = P.cone;
    K.f = d.f;
    K.l = d.l;
    K.nsoc = d.nsoc;
    K.soc_off = BA.soc_off + d.soc0;
    K.soc_len = BA.soc_len + d.soc0;
    K.npsd = d.npsd;
    K.psd_off = BA.psd_off + d.psd0;
    K.psd_dim = BA.psd_dim + d.psd0;
    K.nexp = d.nexp;
    K.exp_off = d.exp_off;
    K.nexpd = d.nexpd;
    K.expd_off = d.expd_off;
    K.npow = d.npow;
    K.pow_off = d.pow_off;
    K.pow_a = BA.pow_a + d.pow0;
    P.b = BA.bh + d.r0;
    P.c = BA.ch + d.c0;
    P.D = BA.D + d.r0;
    P.E = BA.E + d.c0;
    P.g = BA.g + d.r0 + d.c0;
    P.u = BA.u + d.u0;
    P.v = BA.v + d.u0;
    P.zx = reinterpret_cast<T *>(BA.zx) + d.c0;
    P.res = reinterpret_cast<T *>(BA.res) + d.c0;
    P.p0 = reinterpret_cast<T *>(BA.p0) + d.c0;
    P.p1 = reinterpret_cast<T *>(BA.p1) + d.c0;
    P.zy = reinterpret_cast<T *>(BA.zy) + d.r0;
    P.t = reinterpret_cast<T *>(BA.t) + d.r0;
    P.tu = reinterpret_cast<Pair<T> *>(BA.tu) + d.r0;
    P.aux = BA.aux + d.r0;
    P.azc = reinterpret_cast<T *>(BA.azc) + d.r0;
    P.scal = BA.scal + (size_t)SC_COUNT * i;
    P.info = BA.info + (size_t)INFO_COUNT * i;
    // streamed sweeps (one slab): the row pointers are the offsets
    P.slabs_a = 1;
    P.slabs_t = 1;
    P.off_a = P.A.rp;
    P.off_t = P.AT.rp;
    P.hist_u = nullptr;
    P.hist_v = nullptr;
    P.part_a = BA.parts + 4 * i;
    P.part_t = BA.parts + 4 * i + 2;
    return P;
}

// Equilibration of one program by one workgroup: the same rule as the
// single-program setup (ten passes of row then column normalisation by
// 1/sqrt of the scaled norms, block means on non-separable cones, factors
// clipped to [1e-4, 1e4], sigma = 1/|D b|, rho = mean row norm / |E c|),
// then the scaled values, b_hat, c_hat and the norms the tests use.
__device__ void scale_program(const BatchArgs &BA, const InstDesc &d, int i, double *red) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int m = d.m, n = d.n;
    const int32_t *rpA = BA.rpA + d.r0, *rpT = BA.rpT + d.c0;
    double *D = BA.D + d.r0, *E = BA.E + d.c0, *dt = BA.dtmp + d.r0;
    for (int r = tid; r < m; r += nt) D[r] = 1.0;
    for (int j = tid; j < n; j += nt) E[j] = 1.0;
    __syncthreads();
    if (BA.scale) {
        for (int pass = 0; pass < 10; ++pass) {
            for (int r = tid; r < m; r += nt) {
                double sacc = 0.0;
                for (int k = rpA[r]; k < rpA[r + 1]; ++k) {
                    const double a = BA.vA0[k] * E[BA.ciA[k]];
                    sacc += a * a;
                }
                const double nr = D[r] * sqrt(sacc);
                dt[r] = nr > 0.0 ? 1.0 / sqrt(nr) : 1.0;
            }
            __syncthreads();
            for (int bidx = tid; bidx < d.nblk; bidx += nt) {
                const int off = BA.blk_off[d.blk0 + bidx], len = BA.blk_len[d.blk0 + bidx];
                double sacc = 0.0;
                for (int e = 0; e < len; ++e) sacc += dt[off + e];
                const double mean = sacc / (double)len;
                for (int e = 0; e < len; ++e) dt[off + e] = mean;
            }
            __syncthreads();
            for (int r = tid; r < m; r += nt) D[r] *= fmin(fmax(dt[r], 1e-4), 1e4);
            __syncthreads();
            for (int j = tid; j < n; j += nt) {
                double sacc = 0.0;
                for (int k = rpT[j]; k < rpT[j + 1]; ++k) {
                    const double a = BA.vT0[k] * D[BA.ciT[k]];
                    sacc += a * a;
                }
                const double nc = E[j] * sqrt(sacc);
                const double e = nc > 0.0 ? 1.0 / sqrt(nc) : 1.0;
                E[j] *= fmin(fmax(e, 1e-4), 1e4);
            }
            __syncthreads();
        }
    }
    const double *b0 = BA.b0 + d.r0, *c0 = BA.c0 + d.c0;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // |Db|^2, |Ec|^2, sum row norms, |b|^2, |c|^2
    for (int r = tid; r < m; r += nt) {
        double sacc = 0.0;
        for (int k = rpA[r]; k < rpA[r + 1]; ++k) {
            const double a = BA.vA0[k] * E[BA.ciA[k]];
            sacc += a * a;
        }
        acc[2] += D[r] * sqrt(sacc);
        const double db = D[r] * b0[r];
        acc[0] += db * db;
        acc[3] += b0[r] * b0[r];
    }
    for (int j = tid; j < n; j += nt) {
        const double ec = E[j] * c0[j];
        acc[1] += ec * ec;
        acc[4] += c0[j] * c0[j];
    }
    block_sum<5>(acc, red);
    double *sc = BA.scal + (size_t)SC_COUNT * i;
    const double sigma = BA.scale ? 1.0 / fmax(sqrt(acc[0]), 1e-8) : 1.0;
    double rbar = m > 0 ? acc[2] / (double)m : 1.0;  // mean row norm; 1 when A has no nonzeros
    if (!(rbar > 0.0)) rbar = 1.0;
    const double rho = BA.scale ? rbar / fmax(sqrt(acc[1]), 1e-8) : 1.0;
    // scaled values (same product order for A and A^T) and right-hand sides
    for (int r = tid; r < m; r += nt) {
        const double dr = D[r];
        for (int k = rpA[r]; k < rpA[r + 1]; ++k) {
            const double x = (dr * BA.vA0[k]) * E[BA.ciA[k]];
            BA.vA[k] = x;
            if (BA.vA32) BA.vA32[k] = (float)x;
        }
    }
    for (int j = tid; j < n; j += nt) {
        const double ej = E[j];
        for (int k = rpT[j]; k < rpT[j + 1]; ++k) {
            const double x = (D[BA.ciT[k]] * BA.vT0[k]) * ej;
            BA.vT[k] = x;
            if (BA.vT32) BA.vT32[k] = (float)x;
        }
    }
    double nrm[2] = {0.0, 0.0};
    double *bh = BA.bh + d.r0, *ch = BA.ch + d.c0;
    for (int r = tid; r < m; r += nt) {
        const double x = sigma * D[r] * b0[r];
        bh[r] = x;
        const double y = x / D[r];
        nrm[0] += y * y;
    }
    for (int j = tid; j < n; j += nt) {
        const double x = rho * E[j] * c0[j];
        ch[j] = x;
        const double y = x / E[j];
        nrm[1] += y * y;
    }
    block_sum<2>(nrm, red);
    if (tid == 0) {
        sc[SC_SIGMA] = sigma;
        sc[SC_RHO] = rho;
        sc[SC_NORM_B] = sqrt(acc[3]);
        sc[SC_NORM_C] = sqrt(acc[4]);
        sc[SC_NORM_DINV_BH] = sqrt(nrm[0]);
        sc[SC_NORM_EINV_CH] = sqrt(nrm[1]);
    }
    __syncthreads();
}

template <typename T>
__device__ void init_state(const Prob<T> &P, double tau0, double kappa0) {
    const int N = P.n + P.m + 1;
    for (int e = threadIdx.x; e < N; e += blockDim.x) {
        P.u[e] = (e == N - 1) ? tau0 : 0.0;
        P.v[e] = (e == N - 1) ? kappa0 : 0.0;
    }
    for (int j = threadIdx.x; j < P.n; j += blockDim.x) P.zx[j] = T(0);
    __syncthreads();
}

__device__ void outputs_program(const BatchArgs &BA, const InstDesc &d, int i) {
    const double *sc = BA.scal + (size_t)SC_COUNT * i;
    const double *inf = BA.info + (size_t)INFO_COUNT * i;
    const double sigma = sc[SC_SIGMA], rho = sc[SC_RHO];
    const int status = (int)inf[INFO_STATUS];
    const double *u = BA.u + d.u0, *v = BA.v + d.u0;
    const double *D = BA.D + d.r0, *E = BA.E + d.c0;
    const int n = d.n, m = d.m;
    const double tau = u[n + m];
    const double bty = inf[INFO_BTY], ctx = inf[INFO_CTX];
    const double qnan = __builtin_nan("");
    for (int e = threadIdx.x; e < n + m; e += blockDim.x) {
        if (e < n) {
            double xv;
            if (status == 4) xv = rho * E[e] * u[e] / (-ctx);
            else if (status == 3 || !(tau > 0.0)) xv = qnan;
            else xv = E[e] * (u[e] / tau) / sigma;
            if (BA.x_out) BA.x_out[d.c0 + e] = xv;
        } else {
            const int r = e - n;
            const double uy = u[e], vs = v[e];
            double yv, sv;
            if (status == 3) { yv = sigma * D[r] * uy / (-bty); sv = qnan; }
            else if (status == 4) { yv = qnan; sv = rho * vs / D[r] / (-ctx); }
            else if (tau > 0.0) { yv = D[r] * (uy / tau) / rho; sv = (vs / tau) / D[r] / sigma; }
            else { yv = qnan; sv = qnan; }
            if (BA.y_out) BA.y_out[d.r0 + r] = yv;
            if (BA.s_out) BA.s_out[d.r0 + r] = sv;
        }
    }
}

// The batched launch is two persistent kernels, each a loop in which every
// workgroup takes the next program from its queue or exits when the queue is
// empty: first the preparation of each program (equilibration and
// g = M^{-1} h in FP64), then its solve.  (One kernel holding both makes the
// register allocator spill heavily.)
// STREAM selects the block-streamed sweeps (one slab per product).
//
// VLDS: every program's iterate vectors live in the workgroup's LDS during
// its solve (see run_solver), at S.vec_lds doubles into the dynamic LDS; set
// up when the largest program's vectors fit.  A program is then a chain of
// LDS accesses and streamed matrix loads instead of dependent global round
// trips.  The start is written into LDS; after the solve u and v (the
// outputs and the state) and z_x go back to the program's global arrays.
// With S.lds_total > 0, the LDS left after a program's vectors takes its
// constants (b, c, D, E, g) when they fit, and after them its A and A^T
// when those fit too (both copied by run_solver): the small programs,
// whose updates are otherwise chains of global round trips on a few
// hundred nonzeros.
template <typename T>
struct BatchLds {
    double *cst = nullptr, *mat = nullptr;
};
template <typename T>
__device__ BatchLds<T> batch_lds(const Prob<T> &P, const Settings &S, double *vec) {
    BatchLds<T> r;
    if (vec == nullptr || S.lds_total <= 0) return r;
    double *next = vec + vec_lds_doubles(P.n, P.m);
    int64_t end = S.vec_lds + vec_lds_doubles(P.n, P.m);
    if (end + cst_lds_doubles(P.n, P.m) <= S.lds_total) {
        r.cst = next;
        next += cst_lds_doubles(P.n, P.m);
        end += cst_lds_doubles(P.n, P.m);
    }
    const int64_t nnz = (int64_t)uniform((unsigned)(P.A.rp[P.m] - P.A.rp[0]));
    if (end + mat_lds_doubles<T>(P.n, P.m, nnz) <= S.lds_total) r.mat = next;
    return r;
}
template <typename T>
__device__ void init_state_lds(double *vec, int n, int m, double tau0, double kappa0) {
    const int N = n + m + 1;
    for (int e = threadIdx.x; e < N; e += blockDim.x) {
        vec[e] = (e == N - 1) ? tau0 : 0.0;
        vec[N + e] = (e == N - 1) ? kappa0 : 0.0;
    }
    T *zx = reinterpret_cast<T *>(vec + 2 * (int64_t)N + m);
    for (int j = threadIdx.x; j < n; j += blockDim.x) zx[j] = T(0);
    __syncthreads();
}

template <bool STREAM, bool VLDS>
__global__ void __launch_bounds__(512) k_batch_prep(BatchArgs BA, Settings S) {
    extern __shared__ double lds_psd[];
    __shared__ double red_d[8 * MAX_WAVES];
    __shared__ int s_q;
    const Team tm{0, 1, nullptr};
    double *vec = VLDS ? lds_psd + S.vec_lds : nullptr;
    for (;;) {
        if (threadIdx.x == 0) s_q = atomicAdd(BA.queue, 1);
        __syncthreads();
        const int q = (int)uniform((unsigned)s_q);  // the same for the whole workgroup
        __syncthreads();
        if (q >= BA.B) break;
        const int i = (int)uniform((unsigned)BA.order[q]);
        const InstDesc d = BA.desc[i];
        scale_program(BA, d, i, red_d);
        const Prob<double> &Pg = static_cast<const Prob<double> *>(BA.probs_g)[i];
        if constexpr (VLDS) init_state_lds<double>(vec, d.n, d.m, -1.0, 0.0);
        else init_state(Pg, -1.0, 0.0);
        Settings Sg = S;
        Sg.mode = MODE_G;
        Sg.tight_tol = 1e-12;  // relative to max(|h|, 1)
        Sg.cg_max = 10 * d.n + 100;
        Sg.max_iters = 1;
        Sg.check_every = 1 << 30;
        // g and eta go to global memory directly
        const BatchLds<double> xl = batch_lds(Pg, Sg, vec);
        run_solver<double, STREAM, false, false, false, VLDS>(Pg, Sg, tm, nullptr, red_d, red_d, lds_psd,
                                                              xl.mat, vec, xl.cst);
        __syncthreads();
    }
}

template <typename T, bool STREAM, bool VLDS>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_batch(BatchArgs BA, Settings S) {
    extern __shared__ double lds_psd[];
    __shared__ double red_d[8 * MAX_WAVES];
    __shared__ T red_t[8 * MAX_WAVES];
    __shared__ int s_q;
    const Team tm{0, 1, nullptr};
    double *vec = VLDS ? lds_psd + S.vec_lds : nullptr;
    for (;;) {
        if (threadIdx.x == 0) s_q = atomicAdd(BA.queue + 1, 1);
        __syncthreads();
        const int q = (int)uniform((unsigned)s_q);  // the same for the whole workgroup
        __syncthreads();
        if (q >= BA.B) break;
        // queue positions alternate between the largest and the smallest
        // programs left: the iterations a program needs vary far more than
        // its size (from tens to the iteration limit, small programs
        // included), so a small program that runs to the limit, started
        // last in size order, would finish long after the rest
        const int qq = (q & 1) ? BA.B - 1 - (q >> 1) : (q >> 1);
        const int i = (int)uniform((unsigned)BA.order[qq]);
        const Prob<T> &P = static_cast<const Prob<T> *>(BA.probs_t)[i];
        if constexpr (VLDS) init_state_lds<T>(vec, P.n, P.m, 1.0, 1.0);
        else init_state(P, 1.0, 1.0);
        const BatchLds<T> xl = batch_lds(P, S, vec);
        run_solver<T, STREAM, false, false, false, VLDS>(P, S, tm, nullptr, red_d, red_t, lds_psd, xl.mat,
                                                         vec, xl.cst);
        __syncthreads();
        if constexpr (VLDS) {
            const int n = P.n, N = P.n + P.m + 1;
            for (int e = threadIdx.x; e < N; e += blockDim.x) {
                P.u[e] = vec[e];
                P.v[e] = vec[N + e];
            }
            const T *zx = reinterpret_cast<const T *>(vec + 2 * (int64_t)N + P.m);
            for (int j = threadIdx.x; j < n; j += blockDim.x) P.zx[j] = zx[j];
            __syncthreads();
        }
    }
}

// Every nonzero of program i must lie in its own column range.
__global__ void k_validate_blockdiag(const InstDesc *desc, int32_t B, const int32_t *rp,
                                     const int32_t *ci, unsigned *flag) {
    for (int i = blockIdx.x; i < B; i += gridDim.x) {
        const InstDesc d = desc[i];
        unsigned bad = 0;
        for (int64_t k = rp[d.r0] + threadIdx.x; k < rp[d.r0 + d.m]; k += blockDim.x) {
            const int j = ci[k];
            if (j < d.c0 || j >= d.c0 + d.n) ++bad;
        }
        bad = group_sum(bad, WAVE);
        if ((threadIdx.x & (WAVE - 1)) == 0 && bad) atomicAdd(flag, bad);
    }
}

// Column indices of A and row indices of A^T made local to each program.
__global__ void k_localize(const InstDesc *desc, int32_t B, const int32_t *rpA, int32_t *ciA,
                           const int32_t *rpT, int32_t *ciT) {
    for (int i = blockIdx.x; i < B; i += gridDim.x) {
        const InstDesc d = desc[i];
        for (int64_t k = rpA[d.r0] + threadIdx.x; k < rpA[d.r0 + d.m]; k += blockDim.x) ciA[k] -= d.c0;
        for (int64_t k = rpT[d.c0] + threadIdx.x; k < rpT[d.c0 + d.n]; k += blockDim.x) ciT[k] -= d.r0;
    }
}

struct BatchLayout {
    size_t total = 0;
    size_t rpA, ciA, vA0, vA, vA32, rpT, ciT, vT0, vT, vT32;
    size_t b0, c0, bh, ch, D, E, dtmp, g, u, v, zx, res, p0, p1, zy, t, tu, aux, azc;
    size_t scal, info, desc, order, parts, queue, flag, cnt, scan;
    size_t soc_off, soc_len, psd_off, psd_dim, blk_off, blk_len, pow_a, probs_g, probs_t;
    size_t take(size_t bytes) {
        size_t off = total;
        total += (bytes + ALIGN - 1) / ALIGN * ALIGN;
        return off;
    }
};

struct BatchHost {
    std::vector<InstDesc> desc;
    std::vector<int32_t> order, parts, soc_off, soc_len, psd_off, psd_dim, blk_off, blk_len;
    std::vector<double> pow_a;
    int64_t M = 0, N = 0;
    int max_psd = 0;
    double avg_soc = 0.0;
};

static int build_batch(int32_t B, const hsd_csr_t *A, const int64_t *row_off, const int64_t *col_off,
                       const hsd_cone_t *cones, BatchHost &bh) {
    if (B < 1 || !A || !row_off || !col_off || !cones) return fail(HSD_ERR_ARG, "bad batch arguments");
    if (row_off[0] != 0 || col_off[0] != 0) return fail(HSD_ERR_ARG, "offsets must start at 0");
    if (row_off[B] != A->m || col_off[B] != A->n) return fail(HSD_ERR_ARG, "offsets must end at m and n");
    bh.desc.resize(B);
    bh.parts.resize(4 * (size_t)B);
    int64_t nsoc_tot = 0;
    std::vector<int64_t> work(B);
    for (int i = 0; i < B; ++i) {
        const int64_t mi = row_off[i + 1] - row_off[i], ni = col_off[i + 1] - col_off[i];
        if (mi < 1 || ni < 1) return fail(HSD_ERR_ARG, "every program needs m >= 1 and n >= 1");
        HostCone hc;
        int rc = build_cone(&cones[i], hc);
        if (rc) return rc;
        if (hc.m != mi) return fail(HSD_ERR_CONE, "cone dimension of program " + std::to_string(i) + " does not match its rows");
        InstDesc d{};
        d.r0 = (int32_t)row_off[i];
        d.c0 = (int32_t)col_off[i];
        d.m = (int32_t)mi;
        d.n = (int32_t)ni;
        d.u0 = (int32_t)(row_off[i] + col_off[i] + i);
        d.soc0 = (int32_t)bh.soc_off.size();
        d.nsoc = (int32_t)hc.soc_off.size();
        d.psd0 = (int32_t)bh.psd_off.size();
        d.npsd = (int32_t)hc.psd_off.size();
        d.blk0 = (int32_t)bh.blk_off.size();
        d.nblk = (int32_t)hc.blk_off.size();
        d.f = hc.f;
        d.l = hc.l;
        d.nexp = hc.nexp;
        d.exp_off = hc.exp_off;
        d.nexpd = hc.nexpd;
        d.expd_off = hc.expd_off;
        d.npow = hc.npow;
        d.pow_off = hc.pow_off;
        d.pow0 = (int32_t)bh.pow_a.size();
        bh.pow_a.insert(bh.pow_a.end(), hc.pow_a.begin(), hc.pow_a.end());
        bh.soc_off.insert(bh.soc_off.end(), hc.soc_off.begin(), hc.soc_off.end());
        bh.soc_len.insert(bh.soc_len.end(), hc.soc_len.begin(), hc.soc_len.end());
        bh.psd_off.insert(bh.psd_off.end(), hc.psd_off.begin(), hc.psd_off.end());
        bh.psd_dim.insert(bh.psd_dim.end(), hc.psd_dim.begin(), hc.psd_dim.end());
        bh.blk_off.insert(bh.blk_off.end(), hc.blk_off.begin(), hc.blk_off.end());
        bh.blk_len.insert(bh.blk_len.end(), hc.blk_len.begin(), hc.blk_len.end());
        for (int q : hc.soc_len) bh.avg_soc += q;
        nsoc_tot += hc.soc_len.size();
        bh.max_psd = std::max(bh.max_psd, hc.max_psd);
        bh.desc[i] = d;
        bh.parts[4 * i + 0] = 0;
        bh.parts[4 * i + 1] = d.m;
        bh.parts[4 * i + 2] = 0;
        bh.parts[4 * i + 3] = d.n;
        work[i] = mi * ni;
    }
    if (nsoc_tot) bh.avg_soc /= (double)nsoc_tot;
    bh.order.resize(B);
    std::iota(bh.order.begin(), bh.order.end(), 0);
    std::stable_sort(bh.order.begin(), bh.order.end(), [&](int a, int b) { return work[a] > work[b]; });
    bh.M = A->m;
    bh.N = A->n;
    return HSD_OK;
}

static BatchLayout batch_layout(const BatchHost &bh, int32_t B, int64_t nnz, int precision) {
    BatchLayout L;
    const int64_t M = bh.M, N = bh.N;
    L.rpA = L.take(4 * (M + 1));
    L.ciA = L.take(4 * nnz);
    L.vA0 = L.take(8 * nnz);
    L.vA = L.take(8 * nnz);
    L.vA32 = L.take(precision ? 4 * nnz : 0);
    L.rpT = L.take(4 * (N + 1));
    L.ciT = L.take(4 * nnz);
    L.vT0 = L.take(8 * nnz);
    L.vT = L.take(8 * nnz);
    L.vT32 = L.take(precision ? 4 * nnz : 0);
    L.b0 = L.take(8 * M);
    L.c0 = L.take(8 * N);
    L.bh = L.take(8 * M);
    L.ch = L.take(8 * N);
    L.D = L.take(8 * M);
    L.E = L.take(8 * N);
    L.dtmp = L.take(8 * M);
    L.g = L.take(8 * (M + N));
    L.u = L.take(8 * (M + N + B));
    L.v = L.take(8 * (M + N + B));
    L.zx = L.take(8 * N);
    L.res = L.take(8 * N);
    L.p0 = L.take(8 * N);
    L.p1 = L.take(8 * N);
    L.zy = L.take(8 * M);
    L.t = L.take(8 * M);
    L.tu = L.take(16 * M);
    L.aux = L.take(8 * M);
    L.azc = L.take(8 * M);
    L.scal = L.take(8 * (size_t)SC_COUNT * B);
    L.info = L.take(8 * (size_t)INFO_COUNT * B);
    L.desc = L.take(sizeof(InstDesc) * (size_t)B);
    L.order = L.take(4 * (size_t)B);
    L.parts = L.take(16 * (size_t)B);
    L.queue = L.take(64);
    L.flag = L.take(64);
    L.cnt = L.take(4 * (N + 1));
    size_t scan_ints = 0;
    for (int64_t len = N + 1; len > 1; len = (len + 1023) / 1024) scan_ints += (len + 1023) / 1024 + 1;
    L.scan = L.take(4 * (scan_ints + 16));
    L.soc_off = L.take(4 * bh.soc_off.size());
    L.soc_len = L.take(4 * bh.soc_len.size());
    L.psd_off = L.take(4 * bh.psd_off.size());
    L.psd_dim = L.take(4 * bh.psd_dim.size());
    L.blk_off = L.take(4 * bh.blk_off.size());
    L.blk_len = L.take(4 * bh.blk_len.size());
    L.pow_a = L.take(8 * bh.pow_a.size());
    L.probs_g = L.take(sizeof(Prob<double>) * (size_t)B);
    L.probs_t = L.take(sizeof(Prob<double>) * (size_t)B);
    return L;
}

}  // namespace hsd

using namespace hsd;

struct hsd_batch {
    int32_t B = 0;
    int64_t nnz = 0;
    int64_t state_len = 0;          // entries of u (and v): M + N + B
    hsd_settings_t st{};
    BatchHost bh;
    BatchLayout L;
    char *ws = nullptr;
    hipStream_t stream = nullptr;   // caller's stream
    hipStream_t cap = nullptr;      // private stream used for graph capture
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    BatchArgs args{};
    Settings S{};
    int grid = 1, grid_prep = 1, threads = 256;
    bool streamed = false;          // block-streamed sweeps
    bool vlds = false;              // iterate vectors in LDS (see k_batch)
    size_t lds = 0;
    double setup_ms = 0.0;
    double *out_x = nullptr, *out_y = nullptr, *out_s = nullptr;
    template <typename X>
    X *ptr(size_t off) const { return reinterpret_cast<X *>(ws + off); }
    ~hsd_batch() {
        for (int k = 0; k < 2; ++k) {
            if (exec[k]) (void)hipGraphExecDestroy(exec[k]);
            if (graph[k]) (void)hipGraphDestroy(graph[k]);
        }
        if (cap) (void)hipStreamDestroy(cap);
    }
};

extern "C" int hsd_batch_workspace_bytes(int32_t B, const hsd_csr_t *A, const int64_t *row_off,
                                         const int64_t *col_off, const hsd_cone_t *cones,
                                         const hsd_settings_t *st, size_t *bytes) {
    if (!bytes) return fail(HSD_ERR_ARG, "null argument");
    int rc = check_settings(st);
    if (rc) return rc;
    if (!A || A->m < 1 || A->n < 1 || A->nnz < 0 || A->nnz >= (int64_t)INT32_MAX)
        return fail(HSD_ERR_ARG, "bad matrix dimensions");
    BatchHost bh;
    rc = build_batch(B, A, row_off, col_off, cones, bh);
    if (rc) return rc;
    *bytes = batch_layout(bh, B, A->nnz, st->precision).total;
    return HSD_OK;
}

// The preparation and solve kernels of one variant.
using BatchKernel = void (*)(BatchArgs, Settings);
static BatchKernel batch_prep_fn(bool streamed, bool vlds) {
    if (streamed) return vlds ? k_batch_prep<true, true> : k_batch_prep<true, false>;
    return vlds ? k_batch_prep<false, true> : k_batch_prep<false, false>;
}
template <typename T>
static BatchKernel batch_fn(bool streamed, bool vlds) {
    if (streamed) return vlds ? k_batch<T, true, true> : k_batch<T, true, false>;
    return vlds ? k_batch<T, false, true> : k_batch<T, false, false>;
}

// Two graphs: the queue reset and the preparation kernel, then the solve
// kernel (kept apart so that the solve kernel can be timed on its own).
template <typename T>
static int capture_batch(hsd_batch *bt) {
    hipStream_t c = bt->cap;
    for (int part = 0; part < 2; ++part) {
        HIP_TRY(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal));
        if (part == 0) {
            hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(64), 0, c, bt->args.queue, (int64_t)2, 0);
            hipLaunchKernelGGL(batch_prep_fn(bt->streamed, bt->vlds), dim3(bt->grid_prep), dim3(bt->threads),
                               bt->lds, c, bt->args, bt->S);
        } else {
            hipLaunchKernelGGL(batch_fn<T>(bt->streamed, bt->vlds), dim3(bt->grid), dim3(bt->threads), bt->lds,
                               c, bt->args, bt->S);
        }
        hipError_t le = hipGetLastError();
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(c, &g);
        if (le != hipSuccess) return fail(HSD_ERR_HIP, std::string("batch launch capture: ") + hipGetErrorString(le));
        if (ee != hipSuccess) return fail(HSD_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
        bt->graph[part] = g;
        HIP_TRY(hipGraphInstantiate(&bt->exec[part], g, nullptr, nullptr, 0));
    }
    return HSD_OK;
}

extern "C" int hsd_batch_setup(int32_t B, const hsd_csr_t *A, const int64_t *row_off,
                               const int64_t *col_off, const double *b, const double *c,
                               const hsd_cone_t *cones, const hsd_settings_t *st, void *ws,
                               size_t ws_bytes, void *stream, hsd_batch_t **out) {
    if (!A || !b || !c || !ws || !out) return fail(HSD_ERR_ARG, "null argument");
    if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val))) return fail(HSD_ERR_ARG, "null matrix array");
    if (((uintptr_t)ws) % ALIGN) return fail(HSD_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    size_t need = 0;
    int rc = hsd_batch_workspace_bytes(B, A, row_off, col_off, cones, st, &need);
    if (rc) return rc;
    if (ws_bytes < need) return fail(HSD_ERR_WORKSPACE, "workspace too small");
    hsd_batch *bt = new hsd_batch();
    auto cleanup = [&](int code) { delete bt; return code; };
    bt->B = B;
    bt->nnz = A->nnz;
    bt->st = *st;
    build_batch(B, A, row_off, col_off, cones, bt->bh);
    bt->L = batch_layout(bt->bh, B, A->nnz, st->precision);
    bt->ws = (char *)ws;
    bt->stream = (hipStream_t)stream;
    hipStream_t s = bt->stream;
    const BatchLayout &L = bt->L;
    const int64_t M = bt->bh.M, N = bt->bh.N, nnz = A->nnz;
    bt->state_len = M + N + B;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return cleanup(fail(HSD_ERR_HIP, "hipEventCreate failed"));
    (void)hipEventRecord(e0, s);
    auto run = [&]() -> int {
        auto up = [&](size_t off, const void *src, size_t bytes) -> int {
            if (bytes) HIP_TRY(hipMemcpyAsync(bt->ws + off, src, bytes, hipMemcpyHostToDevice, s));
            return HSD_OK;
        };
        const BatchHost &H = bt->bh;
        int r;
        if ((r = up(L.desc, H.desc.data(), sizeof(InstDesc) * H.desc.size())) ||
            (r = up(L.order, H.order.data(), 4 * H.order.size())) ||
            (r = up(L.parts, H.parts.data(), 4 * H.parts.size())) ||
            (r = up(L.soc_off, H.soc_off.data(), 4 * H.soc_off.size())) ||
            (r = up(L.soc_len, H.soc_len.data(), 4 * H.soc_len.size())) ||
            (r = up(L.psd_off, H.psd_off.data(), 4 * H.psd_off.size())) ||
            (r = up(L.psd_dim, H.psd_dim.data(), 4 * H.psd_dim.size())) ||
            (r = up(L.blk_off, H.blk_off.data(), 4 * H.blk_off.size())) ||
            (r = up(L.blk_len, H.blk_len.data(), 4 * H.blk_len.size())) ||
            (r = up(L.pow_a, H.pow_a.data(), 8 * H.pow_a.size())))
            return r;
        HIP_TRY(hipMemcpyAsync(bt->ptr<int32_t>(L.rpA), A->row_ptr, 4 * (size_t)(M + 1), hipMemcpyDeviceToDevice, s));
        if (nnz > 0) {
            HIP_TRY(hipMemcpyAsync(bt->ptr<int32_t>(L.ciA), A->col_idx, 4 * (size_t)nnz, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(bt->ptr<double>(L.vA0), A->val, 8 * (size_t)nnz, hipMemcpyDeviceToDevice, s));
        }
        HIP_TRY(hipMemcpyAsync(bt->ptr<double>(L.b0), b, 8 * (size_t)M, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(bt->ptr<double>(L.c0), c, 8 * (size_t)N, hipMemcpyDeviceToDevice, s));
        // inputs: finite values, a valid CSR, and a block-diagonal pattern
        unsigned *flag = bt->ptr<unsigned>(L.flag);
        unsigned hflag = 0;
        hipLaunchKernelGGL(k_fill<unsigned>, dim3(1), dim3(64), 0, s, flag, (int64_t)4, 0u);
        hipLaunchKernelGGL(k_count_nonfinite, dim3(grid_for(nnz, 1024, 256)), dim3(1024), 0, s, (const double *)bt->ptr<double>(L.vA0), nnz, flag);
        hipLaunchKernelGGL(k_count_nonfinite, dim3(grid_for(M, 1024, 256)), dim3(1024), 0, s, (const double *)bt->ptr<double>(L.b0), M, flag);
        hipLaunchKernelGGL(k_count_nonfinite, dim3(grid_for(N, 1024, 256)), dim3(1024), 0, s, (const double *)bt->ptr<double>(L.c0), N, flag);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hflag) return fail(HSD_ERR_NONFINITE, "A, b or c holds a NaN or Inf");
        int32_t first = -1, last = -1;
        HIP_TRY(hipMemcpy(&first, A->row_ptr, 4, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(&last, A->row_ptr + M, 4, hipMemcpyDeviceToHost));
        if (first != 0 || last != nnz) return fail(HSD_ERR_ARG, "row_ptr must start at 0 and end at nnz");
        hipLaunchKernelGGL(k_fill<unsigned>, dim3(1), dim3(64), 0, s, flag, (int64_t)4, 0u);
        hipLaunchKernelGGL(k_validate_csr, dim3(grid_for(std::max<int64_t>(M, nnz), 256, 1024)), dim3(256), 0, s,
                           (int32_t)M, (int32_t)N, nnz, (const int32_t *)bt->ptr<int32_t>(L.rpA),
                           (const int32_t *)bt->ptr<int32_t>(L.ciA), flag);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hflag) return fail(HSD_ERR_ARG, "row_ptr is not monotone or a column index is outside [0, n)");
        hipLaunchKernelGGL(k_validate_blockdiag, dim3(std::min(B, 4096)), dim3(256), 0, s,
                           (const InstDesc *)bt->ptr<InstDesc>(L.desc), B,
                           (const int32_t *)bt->ptr<int32_t>(L.rpA), (const int32_t *)bt->ptr<int32_t>(L.ciA), flag);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hflag) return fail(HSD_ERR_ARG, "A is not block diagonal with the given row and column offsets");
        // transpose of the whole block-diagonal matrix
        int32_t *cnt = bt->ptr<int32_t>(L.cnt);
        int32_t *rpT = bt->ptr<int32_t>(L.rpT);
        hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(N + 1, 256)), dim3(256), 0, s, cnt, N + 1, 0);
        if (nnz > 0)
            hipLaunchKernelGGL(k_count_cols, dim3(grid_for(nnz, 256)), dim3(256), 0, s,
                               (const int32_t *)bt->ptr<int32_t>(L.ciA), nnz, (int32_t)N, cnt);
        HIP_TRY(hipGetLastError());
        if ((r = scan_exclusive(cnt, rpT, N + 1, bt->ptr<int32_t>(L.scan), s))) return r;
        hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(N + 1, 256)), dim3(256), 0, s, cnt, N + 1, 0);
        hipLaunchKernelGGL(k_scatter_t, dim3(grid_for(M, 256)), dim3(256), 0, s, (int32_t)M,
                           (const int32_t *)bt->ptr<int32_t>(L.rpA), (const int32_t *)bt->ptr<int32_t>(L.ciA),
                           (const double *)bt->ptr<double>(L.vA0), (const int32_t *)rpT, cnt,
                           bt->ptr<int32_t>(L.ciT), bt->ptr<double>(L.vT0));
        // a column of program i has at most m_i entries
        int64_t max_col = 0;
        for (const InstDesc &d : bt->bh.desc) max_col = std::max<int64_t>(max_col, d.m);
        if ((r = sort_rows((int32_t)N, (const int32_t *)rpT, bt->ptr<int32_t>(L.ciT), bt->ptr<double>(L.vT0),
                           max_col, s)))
            return r;
        hipLaunchKernelGGL(k_localize, dim3(std::min(B, 4096)), dim3(256), 0, s,
                           (const InstDesc *)bt->ptr<InstDesc>(L.desc), B, (const int32_t *)bt->ptr<int32_t>(L.rpA),
                           bt->ptr<int32_t>(L.ciA), (const int32_t *)rpT, bt->ptr<int32_t>(L.ciT));
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(s));

        // kernel arguments and launch shape
        BatchArgs &BA = bt->args;
        BA.B = B;
        BA.desc = bt->ptr<InstDesc>(L.desc);
        BA.order = bt->ptr<int32_t>(L.order);
        BA.queue = bt->ptr<int32_t>(L.queue);
        BA.parts = bt->ptr<int32_t>(L.parts);
        BA.rpA = bt->ptr<int32_t>(L.rpA);
        BA.ciA = bt->ptr<int32_t>(L.ciA);
        BA.rpT = bt->ptr<int32_t>(L.rpT);
        BA.ciT = bt->ptr<int32_t>(L.ciT);
        BA.vA0 = bt->ptr<double>(L.vA0);
        BA.vT0 = bt->ptr<double>(L.vT0);
        BA.vA = bt->ptr<double>(L.vA);
        BA.vT = bt->ptr<double>(L.vT);
        BA.vA32 = st->precision ? bt->ptr<float>(L.vA32) : nullptr;
        BA.vT32 = st->precision ? bt->ptr<float>(L.vT32) : nullptr;
        BA.b0 = bt->ptr<double>(L.b0);
        BA.c0 = bt->ptr<double>(L.c0);
        BA.bh = bt->ptr<double>(L.bh);
        BA.ch = bt->ptr<double>(L.ch);
        BA.D = bt->ptr<double>(L.D);
        BA.E = bt->ptr<double>(L.E);
        BA.dtmp = bt->ptr<double>(L.dtmp);
        BA.g = bt->ptr<double>(L.g);
        BA.u = bt->ptr<double>(L.u);
        BA.v = bt->ptr<double>(L.v);
        BA.zx = bt->ptr<double>(L.zx);
        BA.res = bt->ptr<double>(L.res);
        BA.p0 = bt->ptr<double>(L.p0);
        BA.p1 = bt->ptr<double>(L.p1);
        BA.zy = bt->ptr<double>(L.zy);
        BA.t = bt->ptr<double>(L.t);
        BA.tu = bt->ptr<double>(L.tu);
        BA.aux = bt->ptr<double>(L.aux);
        BA.azc = bt->ptr<double>(L.azc);
        BA.scal = bt->ptr<double>(L.scal);
        BA.info = bt->ptr<double>(L.info);
        BA.soc_off = bt->ptr<int32_t>(L.soc_off);
        BA.soc_len = bt->ptr<int32_t>(L.soc_len);
        BA.psd_off = bt->ptr<int32_t>(L.psd_off);
        BA.psd_dim = bt->ptr<int32_t>(L.psd_dim);
        BA.blk_off = bt->ptr<int32_t>(L.blk_off);
        BA.blk_len = bt->ptr<int32_t>(L.blk_len);
        BA.pow_a = bt->ptr<double>(L.pow_a);
        BA.scale = st->scale;
        // outputs are written into a fixed region and copied out per solve
        BA.x_out = nullptr;
        BA.y_out = nullptr;
        BA.s_out = nullptr;
        Settings &S = bt->S;
        S.vec_lds = -1;
        S.lds_total = 0;
        S.eps_pri = st->eps_pri;
        S.eps_dual = st->eps_dual;
        S.eps_gap = st->eps_gap;
        S.eps_unbdd = st->eps_unbdd;
        S.eps_infeas = st->eps_infeas;
        S.alpha = st->alpha;
        S.zeta_pow = st->cg_zeta_pow;
        S.tight_tol = st->cg_tight_tol;
        S.fp32_floor = 10.0 * 5.9604644775390625e-08;
        S.cg_max = st->cg_max_iters;
        S.max_iters = st->max_iters;
        S.check_every = st->check_every;
        S.mode = MODE_SOLVE;
        S.record = 0;
        const double avg_a = nnz / (double)std::max<int64_t>(1, M);
        const double avg_t = nnz / (double)std::max<int64_t>(1, N);
        S.lanes_a = st->lanes_a ? st->lanes_a : pow2_floor(avg_a / 4.0, 1, 64);
        S.lanes_t = st->lanes_at ? st->lanes_at : pow2_floor(avg_t / 4.0, 1, 64);
        S.lanes_soc = st->lanes_soc ? st->lanes_soc : pow2_floor(std::max(1.0, bt->bh.avg_soc), 1, 64);
        // per-program descriptors, built here and read as constants by the kernel
        {
            std::vector<Prob<double>> pg(B);
            for (int i = 0; i < B; ++i) pg[i] = inst_prob<double>(BA, bt->bh.desc[i], i);
            if ((r = up(L.probs_g, pg.data(), sizeof(Prob<double>) * B))) return r;
            if (st->precision) {
                static_assert(sizeof(Prob<float>) == sizeof(Prob<double>), "descriptor layout");
                std::vector<Prob<float>> pt(B);
                for (int i = 0; i < B; ++i) pt[i] = inst_prob<float>(BA, bt->bh.desc[i], i);
                if ((r = up(L.probs_t, pt.data(), sizeof(Prob<float>) * B))) return r;
            } else {
                if ((r = up(L.probs_t, pg.data(), sizeof(Prob<double>) * B))) return r;
            }
            HIP_TRY(hipStreamSynchronize(s));
            BA.probs_g = bt->ws + L.probs_g;
            BA.probs_t = bt->ws + L.probs_t;
        }
        bt->threads = st->block_threads ? st->block_threads : 256;
        bt->lds = bt->bh.max_psd > 0 ? 8 * (size_t)psd_lds_doubles(bt->bh.max_psd) : 0;
        // streamed sweeps: their LDS after the PSD scratch
        bt->streamed = st->slab_cols > 0;
        if (bt->streamed) {
            const size_t psd = (bt->lds + 15) / 16 * 16;
            S.slab_rows = SLAB_CHUNK_ROWS;
            S.slab_lds = (int)(psd / 8);
            bt->lds = psd + 8 * slab_lds_doubles(S.slab_rows, bt->threads);
        }
        // iterate vectors in LDS when the largest program's fit beside the
        // other dynamic LDS (the kernels' static LDS and a margin stay free)
        int dv = 0, maxsh = 0;
        HIP_TRY(hipGetDevice(&dv));
        HIP_TRY(hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dv));
        {
            int64_t vmax = 0;
            for (const InstDesc &d : bt->bh.desc) vmax = std::max(vmax, vec_lds_doubles(d.n, d.m));
            const size_t base = (bt->lds + 15) / 16 * 16;
            const size_t with_vec = base + 8 * (size_t)vmax;
            bt->vlds = st->batch_vectors != 0 && with_vec + 4096 <= (size_t)maxsh;
            if (bt->vlds) {
                S.vec_lds = (int)(base / 8);
                bt->lds = with_vec;
                // the LDS beside the largest program's vectors holds the
                // constants and matrices of the programs they fit
                // (row-group sweeps)
                if (st->batch_matrix != 0 && !bt->streamed) S.lds_total = (int)(bt->lds / 8);
            }
        }
        const void *kb = st->precision ? (const void *)batch_fn<float>(bt->streamed, bt->vlds)
                                       : (const void *)batch_fn<double>(bt->streamed, bt->vlds);
        const void *kp = (const void *)batch_prep_fn(bt->streamed, bt->vlds);
        if (bt->lds > 65536) {
            if (bt->lds + 4096 > (size_t)maxsh) return fail(HSD_ERR_ARG, "batched solve needs more LDS than the device allows");
            HIP_TRY(hipFuncSetAttribute(kb, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bt->lds));
            HIP_TRY(hipFuncSetAttribute(kp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bt->lds));
        }
        int bpc = 0, dev = 0, cus = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, kb, bt->threads, bt->lds));
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        bt->grid = std::max(1, std::min(B, std::max(1, bpc) * cus));
        int bpcp = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpcp, kp, bt->threads, bt->lds));
        bt->grid_prep = std::max(1, std::min(B, std::max(1, bpcp) * cus));
        if (st->team_blocks > 0) bt->grid = std::min(B, st->team_blocks);
        HIP_TRY(hipStreamCreateWithFlags(&bt->cap, hipStreamNonBlocking));
        return st->precision ? capture_batch<float>(bt) : capture_batch<double>(bt);
    };
    rc = run();
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return cleanup(rc);
    bt->setup_ms = ms;
    *out = bt;
    return HSD_OK;
}

// Copies the per-program outputs (computed inside the launch into the
// u/v-based outputs) to the caller's arrays.
__global__ void k_batch_outputs(BatchArgs BA, double *x, double *y, double *s) {
    BatchArgs A2 = BA;
    A2.x_out = x;
    A2.y_out = y;
    A2.s_out = s;
    for (int i = blockIdx.x; i < BA.B; i += gridDim.x) {
        const InstDesc d = BA.desc[i];
        outputs_program(A2, d, i);
    }
}

extern "C" int hsd_batch_solve(hsd_batch_t *bt, double *x, double *y, double *s, hsd_info_t *infos) {
    if (!bt || !bt->exec[0] || !bt->exec[1]) return fail(HSD_ERR_STATE, "batch handle is not set up");
    if (!infos) return fail(HSD_ERR_ARG, "infos is null");
    hipStream_t st = bt->stream;
    hipEvent_t ev[4];
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) return fail(HSD_ERR_HIP, "hipEventCreate failed");
    (void)hipEventRecord(ev[0], st);
    hipError_t ge = hipGraphLaunch(bt->exec[0], st);
    (void)hipEventRecord(ev[1], st);
    if (ge == hipSuccess) ge = hipGraphLaunch(bt->exec[1], st);
    (void)hipEventRecord(ev[2], st);
    if (ge != hipSuccess) return fail(HSD_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(ge));
    hipLaunchKernelGGL(k_batch_outputs, dim3(std::min(bt->B, 4096)), dim3(256), 0, st, bt->args, x, y, s);
    HIP_TRY(hipGetLastError());
    (void)hipEventRecord(ev[3], st);
    std::vector<double> h((size_t)INFO_COUNT * bt->B);
    HIP_TRY(hipMemcpyAsync(h.data(), bt->args.info, 8 * h.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    float kms = 0.f, tms = 0.f;
    (void)hipEventElapsedTime(&kms, ev[1], ev[2]);
    (void)hipEventElapsedTime(&tms, ev[0], ev[3]);
    for (auto &e : ev) (void)hipEventDestroy(e);
    for (int i = 0; i < bt->B; ++i) {
        const double *hi = h.data() + (size_t)INFO_COUNT * i;
        hsd_info_t &f = infos[i];
        std::memset(&f, 0, sizeof(f));
        f.status = (int)hi[INFO_STATUS];
        f.iters = (int)hi[INFO_ITERS];
        f.res_pri = hi[INFO_RES_PRI];
        f.res_dual = hi[INFO_RES_DUAL];
        f.gap = hi[INFO_GAP];
        f.pobj = hi[INFO_POBJ];
        f.dobj = hi[INFO_DOBJ];
        f.obj = 0.5 * (hi[INFO_POBJ] + hi[INFO_DOBJ]);
        f.tau = hi[INFO_TAU];
        f.kappa = hi[INFO_KAPPA];
        f.cg_iters = (int64_t)hi[INFO_CG_ITERS];
        f.spmv_count = (int64_t)hi[INFO_SPMV];
        f.setup_ms = bt->setup_ms;
        f.solve_ms = tms;
        f.kernel_ms = kms;
        f.res_infeas = hi[INFO_RES_INF];
        f.res_unbdd = hi[INFO_RES_UNB];
    }
    return HSD_OK;
}

extern "C" int hsd_batch_get_state(hsd_batch_t *bt, double *u, double *v) {
    if (!bt || !bt->exec[0] || !bt->exec[1]) return fail(HSD_ERR_STATE, "batch handle is not set up");
    if (!u || !v) return fail(HSD_ERR_ARG, "null argument");
    const size_t bytes = 8 * (size_t)bt->state_len;
    HIP_TRY(hipMemcpyAsync(u, bt->args.u, bytes, hipMemcpyDeviceToDevice, bt->stream));
    HIP_TRY(hipMemcpyAsync(v, bt->args.v, bytes, hipMemcpyDeviceToDevice, bt->stream));
    HIP_TRY(hipStreamSynchronize(bt->stream));
    return HSD_OK;
}

extern "C" int hsd_batch_get_launch(hsd_batch_t *bt, hsd_launch_t *out) {
    if (!bt || !out) return fail(HSD_ERR_ARG, "null argument");
    hsd_launch_t o{};
    o.team_blocks = bt->grid;
    o.block_threads = bt->threads;
    o.lanes_a = bt->S.lanes_a;
    o.lanes_at = bt->S.lanes_t;
    o.lanes_soc = bt->S.lanes_soc;
    o.slabs_a = 1;
    o.slabs_at = 1;
    o.lds_bytes = (int64_t)bt->lds;
    o.vectors_lds = bt->vlds ? 1 : 0;
    o.lds_matrix = bt->S.lds_total > 0 ? 1 : 0;
    *out = o;
    return HSD_OK;
}

extern "C" void hsd_batch_finish(hsd_batch_t *bt) { delete bt; }
