// C ABI of the solver (include/hsd.h): host runtime around the kernels.
// Validation, workspace layout, setup pipeline, the cooperative persistent
// solve launch, outputs and error reporting.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hsd_direct.h"
#include "hsd_host.h"
#include "hsd_solver.h"

namespace hsd {

// ---------------------------------------------------------------------------
// the solver kernel (one team = the whole grid)
// ---------------------------------------------------------------------------

// Partition weight of a PSD cone of side d, in nonzeros per unit of side
// (see the row partition in hsd_setup).
constexpr int64_t PSD_COST_PER_SIDE = 500;

// SLABS selects the column-slab sweeps (large programs); it is a separate
// instantiation so that the register allocation of the default kernel is
// not shaped by the slab path.
//
// Register budget: the slab kernel runs teams of several 256-thread
// workgroups per CU (3 waves per SIMD); the row-group kernel runs one
// 512-thread workgroup per CU, so it may use the register file of 2 waves
// per SIMD and keeps its working set out of scratch.
//
// LONGR (row-group sweeps only) adds the whole-workgroup pass for long rows;
// it is instantiated apart for the same reason.
// VAR: 0 = the plain row-group (or slab) kernel, 1 = with the long-row pass,
// 2 = the direct projection (with the long-row pass), each its own
// instantiation.
template <typename T, bool SLABS, int VAR>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(SLABS ? 3 : 2, 8))) k_solve(Prob<T> P, Settings S, double *part, unsigned *bar) {
    extern __shared__ double lds_psd[];
    __shared__ double red_d[8 * MAX_WAVES];
    __shared__ T red_t[8 * MAX_WAVES];
    Team tm{(int)blockIdx.x, (int)gridDim.x, bar};
    if (!team_init(tm)) {
        if (tm.rank == 0 && threadIdx.x == 0) { P.info[INFO_ABORT] = 1.0; P.info[INFO_STATUS] = 5.0; }
        return;
    }
    // fused updates and gather pairs for the row-group sweeps (see run_solver)
    run_solver<T, SLABS, !SLABS, !SLABS, (VAR >= 1), false, (VAR == 2)>(
        P, S, tm, part, red_d, red_t, lds_psd, S.mat_lds >= 0 ? lds_psd + S.mat_lds : nullptr);
}

// The same routine in MODE_G at setup (g = M^{-1} h), under its own name so
// that profiles separate it from the solve launches.
template <bool SLABS, int VAR>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_setup_g(Prob<double> P, Settings S, double *part, unsigned *bar) {
    extern __shared__ double lds_psd[];
    __shared__ double red_d[8 * MAX_WAVES];
    __shared__ double red_t[8 * MAX_WAVES];
    Team tm{(int)blockIdx.x, (int)gridDim.x, bar};
    if (!team_init(tm)) {
        if (tm.rank == 0 && threadIdx.x == 0) { P.info[INFO_ABORT] = 1.0; P.info[INFO_STATUS] = 5.0; }
        return;
    }
    run_solver<double, SLABS, false, false, (VAR >= 1), false, (VAR == 2)>(
        P, S, tm, part, red_d, red_t, lds_psd, S.mat_lds >= 0 ? lds_psd + S.mat_lds : nullptr);
}

// The solve and g-pass kernels of one variant: slab sweeps, or row-group
// sweeps with or without the long-row pass, or the direct projection (FP64,
// row-group sweeps).
template <typename T>
static const void *solve_fn(bool slabs, bool longr = false, bool direct = false) {
    if (slabs) return (const void *)k_solve<T, true, 0>;
    if constexpr (sizeof(T) == 8) {
        if (direct) return (const void *)k_solve<T, false, 2>;
    }
    return longr ? (const void *)k_solve<T, false, 1> : (const void *)k_solve<T, false, 0>;
}
static const void *setup_g_fn(bool slabs, bool longr = false, bool direct = false) {
    if (slabs) return (const void *)k_setup_g<true, 0>;
    if (direct) return (const void *)k_setup_g<false, 2>;
    return longr ? (const void *)k_setup_g<false, 1> : (const void *)k_setup_g<false, 0>;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------

struct Layout {
    size_t total = 0;
    size_t rpA, ciA, vA, vA32, rpT, ciT, vT, vT32;
    size_t bh, ch, D, E, dtmp, g, u, v;
    size_t zx, zy, res, p0, p1, t, tu, aux, azc;
    size_t part, bar, scal, info, flag;
    size_t soc_off, soc_len, psd_off, psd_dim, blk_off, blk_len, pow_a;
    size_t part_a, part_t, cnt, scan;
    size_t off_a, off_t;  // column-slab offsets (empty without slabs)
    size_t bnd;           // row-major slab boundaries (setup scratch)
    size_t ciA_s, vA_s, vA32_s, ciT_s, vT_s, vT32_s;  // slab-major matrix copies
    size_t dW, dZ;        // direct projection: Cholesky factor, then G^{-1} (NP x NP)
    size_t psdv, psdvoff; // PSD eigenvectors of the last projection per cone, their offsets
    int64_t np = 0;       // their padded side
    size_t take(size_t bytes) {
        size_t off = total;
        total += (bytes + ALIGN - 1) / ALIGN * ALIGN;
        return off;
    }
};

static Layout make_layout(int64_t m, int64_t n, int64_t nnz, const HostCone &hc, int precision,
                          const SlabPlan &sp, bool direct) {
    Layout L;
    L.np = direct ? (n + DTILE - 1) / DTILE * DTILE : 0;
    L.dW = L.take(8 * (size_t)L.np * (size_t)L.np);
    L.dZ = L.take(8 * (size_t)L.np * (size_t)L.np);
    // warm-started PSD projections (cones up to PSD_WARM_MAX)
    size_t pv = 0;
    if (hc.max_psd > 0 && hc.max_psd <= PSD_WARM_MAX)
        for (int d : hc.psd_dim) pv += (size_t)(d + (d & 1)) * (d + (d & 1));
    L.psdv = L.take(8 * pv);
    L.psdvoff = L.take(pv > 0 ? 8 * hc.psd_dim.size() : 0);
    // CG vectors hold floats in the FP32 mode, but g = M^{-1} h is computed
    // in FP64 through the same buffers at setup: size them for doubles.
    (void)precision;
    const size_t vs = sizeof(double);
    const int64_t N = n + m + 1;
    L.rpA = L.take(4 * (m + 1));
    L.ciA = L.take(4 * nnz);
    L.vA = L.take(8 * nnz);
    L.vA32 = L.take(precision ? 4 * nnz : 0);
    L.rpT = L.take(4 * (n + 1));
    L.ciT = L.take(4 * nnz);
    L.vT = L.take(8 * nnz);
    L.vT32 = L.take(precision ? 4 * nnz : 0);
    L.bh = L.take(8 * m);
    L.ch = L.take(8 * n);
    L.D = L.take(8 * m);
    L.E = L.take(8 * n);
    L.dtmp = L.take(8 * std::max(m, n));
    L.g = L.take(8 * (n + m));
    L.u = L.take(8 * N);
    L.v = L.take(8 * N);
    L.zx = L.take(vs * n);
    L.res = L.take(vs * n);
    L.p0 = L.take(vs * n);
    L.p1 = L.take(vs * n);
    L.zy = L.take(vs * m);
    L.t = L.take(vs * m);
    L.tu = L.take(16 * m);
    L.aux = L.take(8 * m);
    L.azc = L.take(vs * m);
    L.part = L.take(8 * (size_t)NSLOTS * MAX_TEAM * PART_STRIDE);
    L.bar = L.take(4 * BAR_WORDS);
    L.scal = L.take(8 * SC_COUNT);
    L.info = L.take(8 * INFO_COUNT);
    L.flag = L.take(64);
    L.soc_off = L.take(4 * hc.soc_off.size());
    L.soc_len = L.take(4 * hc.soc_len.size());
    L.psd_off = L.take(4 * hc.psd_off.size());
    L.psd_dim = L.take(4 * hc.psd_dim.size());
    L.blk_off = L.take(4 * hc.blk_off.size());
    L.blk_len = L.take(4 * hc.blk_len.size());
    L.pow_a = L.take(8 * hc.pow_a.size());
    L.part_a = L.take(4 * (MAX_TEAM + 1));
    L.part_t = L.take(4 * (MAX_TEAM + 1));
    L.cnt = L.take(4 * (n + 1));
    // scan scratch: tile sums at every level of the longest scan
    int64_t scan_len = n + 1;
    if (sp.ka > 1) scan_len = std::max(scan_len, (int64_t)sp.ka * m + 1);
    if (sp.kt > 1) scan_len = std::max(scan_len, (int64_t)sp.kt * n + 1);
    size_t scan_ints = 0;
    for (int64_t len = scan_len; len > 1; len = (len + 1023) / 1024) scan_ints += (len + 1023) / 1024 + 1;
    L.scan = L.take(4 * (scan_ints + 16));
    // slab-major copies only for a side with several slabs
    const bool sa = sp.ka > 1, st_ = sp.kt > 1;
    L.off_a = L.take(sa ? 4 * ((size_t)sp.ka * m + 1) : 0);
    L.off_t = L.take(st_ ? 4 * ((size_t)sp.kt * n + 1) : 0);
    L.bnd = L.take(4 * std::max(sa ? (size_t)(sp.ka + 1) * m : 0, st_ ? (size_t)(sp.kt + 1) * n : 0));
    L.ciA_s = L.take(sa ? 4 * nnz : 0);
    L.vA_s = L.take(sa ? 8 * nnz : 0);
    L.vA32_s = L.take(sa && precision ? 4 * nnz : 0);
    L.ciT_s = L.take(st_ ? 4 * nnz : 0);
    L.vT_s = L.take(st_ ? 8 * nnz : 0);
    L.vT32_s = L.take(st_ && precision ? 4 * nnz : 0);
    return L;
}

}  // namespace hsd

using namespace hsd;

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------

struct hsd_work {
    int32_t m = 0, n = 0;
    int64_t nnz = 0;
    hsd_settings_t st{};
    HostCone hc;
    Layout L;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    int team = 1, threads = 256, lanes_a = 8, lanes_t = 8, lanes_soc = 8;
    size_t lds_bytes = 0;       // dynamic LDS of the g pass (PSD scratch)
    size_t lds_solve = 0;       // dynamic LDS of the solve kernel (PSD scratch + matrix slices)
    int max_row_a = 0, max_row_t = 0;  // longest row of A and of A^T (entries)
    bool longr = false;         // the kernels with the long-row pass (see sweep)
    bool psd_warm = false;      // PSD projections warm-started from the last eigenvectors
    std::vector<int64_t> psd_voff;  // their offsets (host copy)
    int mat_lds = -1;           // offset of the matrix slices in doubles, -1 = not cached
    bool g_mat = false;         // the g pass reads the matrix slices too (FP64 slices)
    SlabPlan sp;                // column slabs of the sparse products
    int slab_lds = 0;           // offset of the slab row accumulators in doubles
    int slab_rows = 0;          // rows per slab chunk
    int row_lds = 0;            // offset of the own-row stage in doubles
    int row_cap = 0;            // rows per array of the own-row stage, 0 = none
    int col_lds = 0;            // offset of the own-column stage in doubles
    int col_cap = 0;            // columns per array of the own-column stage, 0 = none
    bool start_set = false;     // u, v hold a start for the next run
    bool zx_set = false;        // z_x holds the CG start of a restored state
    int32_t k0 = 0;             // iteration number of a restored state
    bool carried = false;       // the carried products of a restored state are in place
    bool has_state = false;     // u, v, z_x hold the state where the last run stopped
    int32_t k_last = 0;         // its iteration number
    bool ready = false;
    double setup_ms = 0.0;
    hipEvent_t kev0 = nullptr, kev1 = nullptr;  // around the persistent launch
    template <typename X>
    X *ptr(size_t off) const { return reinterpret_cast<X *>(ws + off); }
};

extern "C" const char *hsd_version(void) { return "hsd-gfx950 0.1"; }

extern "C" const char *hsd_last_error(void) { return g_err.c_str(); }

extern "C" void hsd_default_settings(hsd_settings_t *st) {
    if (!st) return;
    std::memset(st, 0, sizeof(*st));
    st->eps_pri = st->eps_dual = st->eps_gap = st->eps_unbdd = st->eps_infeas = 1e-4;
    st->alpha = 1.5;
    st->cg_zeta_pow = 1.5;
    st->cg_tight_tol = 0.0;
    st->cg_max_iters = 100;
    st->max_iters = 10000;
    st->check_every = 1;
    st->scale = 1;
    st->precision = 0;
    st->batch_vectors = 1;
    st->batch_matrix = 1;
}

extern "C" int hsd_workspace_bytes(const hsd_csr_t *A, const hsd_cone_t *K,
                                   const hsd_settings_t *st, size_t *bytes) {
    if (!A || !bytes) return fail(HSD_ERR_ARG, "null argument");
    int rc = check_settings(st);
    if (rc) return rc;
    if (A->m < 1 || A->n < 1 || A->nnz < 0) return fail(HSD_ERR_ARG, "bad matrix dimensions");
    if (A->nnz >= (int64_t)INT32_MAX) return fail(HSD_ERR_ARG, "nnz must be below 2^31");
    HostCone hc;
    rc = build_cone(K, hc);
    if (rc) return rc;
    if (hc.m != A->m) return fail(HSD_ERR_CONE, "cone dimension does not equal the rows of A");
    if (st->linsys == 1 && A->n > DIRECT_MAX_N)
        return fail(HSD_ERR_ARG, "the direct projection takes n <= " + std::to_string(DIRECT_MAX_N));
    *bytes = make_layout(A->m, A->n, A->nnz, hc, st->precision, slab_plan(st, A->m, A->n), st->linsys == 1).total;
    return HSD_OK;
}

template <typename T>
static Prob<T> make_prob(const hsd_work *w, double *hist_u, double *hist_v) {
    Prob<T> P{};
    const Layout &L = w->L;
    P.m = w->m;
    P.n = w->n;
    P.nnz = w->nnz;
    // a side with several column slabs reads its slab-major copy
    const bool sa = w->sp.ka > 1, sb = w->sp.kt > 1;
    P.A = {w->ptr<int32_t>(L.rpA), w->ptr<int32_t>(sa ? L.ciA_s : L.ciA), w->ptr<double>(sa ? L.vA_s : L.vA)};
    P.AT = {w->ptr<int32_t>(L.rpT), w->ptr<int32_t>(sb ? L.ciT_s : L.ciT), w->ptr<double>(sb ? L.vT_s : L.vT)};
    if constexpr (sizeof(T) == 4) {
        P.Ac = {P.A.rp, P.A.ci, w->ptr<float>(sa ? L.vA32_s : L.vA32)};
        P.ATc = {P.AT.rp, P.AT.ci, w->ptr<float>(sb ? L.vT32_s : L.vT32)};
    } else {
        P.Ac = P.A;
        P.ATc = P.AT;
    }
    ConeDev &K = P.cone;
    K.f = w->hc.f;
    K.l = w->hc.l;
    K.nsoc = (int32_t)w->hc.soc_off.size();
    K.soc_off = w->ptr<int32_t>(L.soc_off);
    K.soc_len = w->ptr<int32_t>(L.soc_len);
    K.npsd = (int32_t)w->hc.psd_off.size();
    K.psd_off = w->ptr<int32_t>(L.psd_off);
    K.psd_dim = w->ptr<int32_t>(L.psd_dim);
    K.nexp = w->hc.nexp;
    K.exp_off = w->hc.exp_off;
    K.nexpd = w->hc.nexpd;
    K.expd_off = w->hc.expd_off;
    K.npow = w->hc.npow;
    K.pow_off = w->hc.pow_off;
    K.pow_a = w->ptr<double>(L.pow_a);
    K.max_psd_dim = w->hc.max_psd;
    P.b = w->ptr<double>(L.bh);
    P.c = w->ptr<double>(L.ch);
    P.D = w->ptr<double>(L.D);
    P.E = w->ptr<double>(L.E);
    P.g = w->ptr<double>(L.g);
    P.u = w->ptr<double>(L.u);
    P.v = w->ptr<double>(L.v);
    P.zx = w->ptr<T>(L.zx);
    P.zy = w->ptr<T>(L.zy);
    P.res = w->ptr<T>(L.res);
    P.p0 = w->ptr<T>(L.p0);
    P.p1 = w->ptr<T>(L.p1);
    P.t = w->ptr<T>(L.t);
    P.tu = w->ptr<Pair<T>>(L.tu);
    P.aux = w->ptr<double>(L.aux);
    P.azc = w->ptr<T>(L.azc);
    P.scal = w->ptr<double>(L.scal);
    P.info = w->ptr<double>(L.info);
    P.hist_u = hist_u;
    P.hist_v = hist_v;
    P.part_a = w->ptr<int32_t>(L.part_a);
    P.part_t = w->ptr<int32_t>(L.part_t);
    P.slabs_a = w->sp.ka;
    P.slabs_t = w->sp.kt;
    // streamed sweeps: slab-major offsets, or the row pointers for one slab
    P.off_a = !w->sp.on() ? nullptr : sa ? w->ptr<int32_t>(L.off_a) : P.A.rp;
    P.off_t = !w->sp.on() ? nullptr : sb ? w->ptr<int32_t>(L.off_t) : P.AT.rp;
    P.Z = L.np > 0 ? w->ptr<double>(L.dZ) : nullptr;
    P.ldz = L.np;
    P.psd_v = w->psd_warm ? w->ptr<double>(L.psdv) : nullptr;
    P.psd_voff = w->psd_warm ? w->ptr<int64_t>(L.psdvoff) : nullptr;
    return P;
}

static Settings make_settings(const hsd_work *w, int mode, int max_iters, int record) {
    const hsd_settings_t &s = w->st;
    Settings S{};
    S.vec_lds = -1;
    S.eps_pri = s.eps_pri;
    S.eps_dual = s.eps_dual;
    S.eps_gap = s.eps_gap;
    S.eps_unbdd = s.eps_unbdd;
    S.eps_infeas = s.eps_infeas;
    S.alpha = s.alpha;
    S.zeta_pow = s.cg_zeta_pow;
    S.tight_tol = s.cg_tight_tol;
    S.fp32_floor = 10.0 * 5.9604644775390625e-08;  // 10 * 2^-24
    S.cg_max = s.cg_max_iters;
    S.max_iters = max_iters;
    S.check_every = s.check_every;
    S.mode = mode;
    S.record = record;
    S.k0 = (mode == MODE_G) ? 0 : w->k0;
    S.carried = (mode != MODE_G && w->carried) ? 1 : 0;
    S.lanes_a = w->lanes_a;
    S.lanes_t = w->lanes_t;
    S.lanes_soc = w->lanes_soc;
    // the g pass is FP64 in every mode: it reads the LDS matrix slices only
    // when they hold FP64 values
    S.mat_lds = (mode == MODE_G && !w->g_mat) ? -1 : w->mat_lds;
    S.slab_lds = w->slab_lds;
    S.slab_rows = w->slab_rows;
    S.row_lds = w->row_lds;
    S.row_cap = (mode == MODE_G) ? 0 : w->row_cap;
    S.col_lds = w->col_lds;
    S.col_cap = (mode == MODE_G) ? 0 : w->col_cap;
    return S;
}

// One cooperative launch of the persistent kernel.
template <typename T>
static int launch_solve(hsd_work *w, const Settings &S, double *hist_u, double *hist_v,
                        bool setup_g = false) {
    Prob<T> P = make_prob<T>(w, hist_u, hist_v);
    double *part = w->ptr<double>(w->L.part);
    unsigned *bar = w->ptr<unsigned>(w->L.bar);
    hipLaunchKernelGGL(k_fill<unsigned>, dim3(1), dim3(256), 0, w->stream, bar, (int64_t)BAR_WORDS, 0u);
    HIP_TRY(hipGetLastError());
    void *args[] = {(void *)&P, (void *)&S, (void *)&part, (void *)&bar};
    const bool slabs = w->sp.on();
    const void *fn = setup_g ? setup_g_fn(slabs, w->longr, w->L.np > 0) : solve_fn<T>(slabs, w->longr, w->L.np > 0);
    if (w->kev0 && !setup_g) HIP_TRY(hipEventRecord(w->kev0, w->stream));
    // the g pass takes the solve kernel's LDS when it reads the matrix slices
    const size_t lds = (setup_g && S.mat_lds < 0) ? w->lds_bytes : w->lds_solve;
    HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(w->team), dim3(w->threads), args, (unsigned)lds, w->stream));
    if (w->kev1 && !setup_g) HIP_TRY(hipEventRecord(w->kev1, w->stream));
    return HSD_OK;
}

static int run_mode(hsd_work *w, int mode, int max_iters, int record, double *hu, double *hv) {
    Settings S = make_settings(w, mode, max_iters, record);
    if (mode == MODE_G) {
        S.tight_tol = 1e-12;  // relative to max(|h|, 1)
        S.cg_max = 10 * w->n + 100;
        S.max_iters = 1;
        S.check_every = 1 << 30;
        // g is computed in FP64 in every precision mode
        return launch_solve<double>(w, S, nullptr, nullptr, true);
    }
    return w->st.precision ? launch_solve<float>(w, S, hu, hv) : launch_solve<double>(w, S, hu, hv);
}

static int read_info(hsd_work *w, double *h) {
    HIP_TRY(hipMemcpyAsync(h, w->ptr<double>(w->L.info), 8 * INFO_COUNT, hipMemcpyDeviceToHost,
                           w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    if (h[INFO_ABORT] != 0.0)
        return fail(HSD_ERR_ABORTED, "a device-side bounded wait expired; the solve was abandoned");
    return HSD_OK;
}

// Dynamic LDS above 64 KB must be allowed per kernel before launch (and
// before occupancy queries); the kernels' static LDS and a margin stay free.
static int allow_lds(size_t bytes) {
    if (bytes <= 65536) return HSD_OK;
    int dev = 0, maxsh = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (bytes + 4096 > (size_t)maxsh)
        return fail(HSD_ERR_ARG, "the solve needs " + std::to_string(bytes) +
                                     " bytes of LDS per workgroup, more than the device allows");
    for (bool sl : {false, true}) {
        for (bool lr : {false, true}) {
            for (bool dr : {false, true}) {
                HIP_TRY(hipFuncSetAttribute(solve_fn<double>(sl, lr, dr), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
                HIP_TRY(hipFuncSetAttribute(solve_fn<float>(sl, lr, dr), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
                HIP_TRY(hipFuncSetAttribute(setup_g_fn(sl, lr, dr), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
            }
        }
    }
    return HSD_OK;
}

static int occupancy(const void *kern, int threads, size_t lds, int *blocks_per_cu) {
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kern, threads, lds));
    return HSD_OK;
}

extern "C" int hsd_setup(const hsd_csr_t *A, const double *b, const double *c,
                         const hsd_cone_t *K, const hsd_settings_t *st, void *ws,
                         size_t ws_bytes, void *stream, hsd_work_t **out) {
    if (!A || !b || !c || !out || !ws) return fail(HSD_ERR_ARG, "null argument");
    if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)))
        return fail(HSD_ERR_ARG, "null matrix array");
    if (((uintptr_t)ws) % ALIGN) return fail(HSD_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    size_t need = 0;
    int rc = hsd_workspace_bytes(A, K, st, &need);
    if (rc) return rc;
    if (ws_bytes < need) return fail(HSD_ERR_WORKSPACE, "workspace too small");
    hsd_work *w = new hsd_work();
    w->m = A->m;
    w->n = A->n;
    w->nnz = A->nnz;
    w->st = *st;
    build_cone(K, w->hc);
    w->sp = slab_plan(st, A->m, A->n);
    w->L = make_layout(w->m, w->n, w->nnz, w->hc, st->precision, w->sp, st->linsys == 1);
    w->ws = (char *)ws;
    w->stream = (hipStream_t)stream;
    hipStream_t s = w->stream;
    const Layout &L = w->L;
    const int m = w->m, n = w->n;
    const int64_t nnz = w->nnz;
    auto cleanup = [&](int code) { delete w; return code; };

    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return cleanup(fail(HSD_ERR_HIP, "hipEventCreate failed"));
    hipEventRecord(e0, s);
    auto run = [&]() -> int {
        // cone tables
        auto up = [&](size_t off, const std::vector<int32_t> &v) -> int {
            if (!v.empty())
                HIP_TRY(hipMemcpyAsync(w->ptr<int32_t>(off), v.data(), 4 * v.size(),
                                       hipMemcpyHostToDevice, s));
            return HSD_OK;
        };
        int r;
        if ((r = up(L.soc_off, w->hc.soc_off)) || (r = up(L.soc_len, w->hc.soc_len)) ||
            (r = up(L.psd_off, w->hc.psd_off)) || (r = up(L.psd_dim, w->hc.psd_dim)) ||
            (r = up(L.blk_off, w->hc.blk_off)) || (r = up(L.blk_len, w->hc.blk_len)))
            return r;
        if (!w->hc.pow_a.empty())
            HIP_TRY(hipMemcpyAsync(w->ptr<double>(L.pow_a), w->hc.pow_a.data(), 8 * w->hc.pow_a.size(),
                                   hipMemcpyHostToDevice, s));
        // copy A
        HIP_TRY(hipMemcpyAsync(w->ptr<int32_t>(L.rpA), A->row_ptr, 4 * (size_t)(m + 1),
                               hipMemcpyDeviceToDevice, s));
        if (nnz > 0) {
            HIP_TRY(hipMemcpyAsync(w->ptr<int32_t>(L.ciA), A->col_idx, 4 * (size_t)nnz,
                                   hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(w->ptr<double>(L.vA), A->val, 8 * (size_t)nnz,
                                   hipMemcpyDeviceToDevice, s));
        }
        // Input checks, read back together: flag[0] counts non-finite
        // entries of A, b, c; flag[1] structural errors of the CSR (row
        // pointers that decrease or leave [0, nnz], column indices outside
        // [0, n)); flag[2], flag[3] are row_ptr[0] and row_ptr[m].  The
        // structure kernel only reads rp[0..m] and ci[0..nnz), so it is safe
        // on any values; nothing indexes with them before these checks.
        unsigned *flag = w->ptr<unsigned>(L.flag);
        hipLaunchKernelGGL(k_fill<unsigned>, dim3(1), dim3(64), 0, s, flag, (int64_t)6, 0u);
        hipLaunchKernelGGL(k_count_nonfinite, dim3(grid_for(nnz, 1024, 256)), dim3(1024), 0, s, (const double *)w->ptr<double>(L.vA), nnz, flag);
        hipLaunchKernelGGL(k_count_nonfinite, dim3(grid_for(m, 1024, 256)), dim3(1024), 0, s, b, (int64_t)m, flag);
        hipLaunchKernelGGL(k_count_nonfinite, dim3(grid_for(n, 1024, 256)), dim3(1024), 0, s, c, (int64_t)n, flag);
        hipLaunchKernelGGL(k_validate_csr, dim3(grid_for(std::max<int64_t>(m, nnz), 256, 1024)), dim3(256), 0, s,
                           m, n, nnz, (const int32_t *)w->ptr<int32_t>(L.rpA),
                           (const int32_t *)w->ptr<int32_t>(L.ciA), flag + 1);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(flag + 2, w->ptr<int32_t>(L.rpA), 4, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(flag + 3, w->ptr<int32_t>(L.rpA) + m, 4, hipMemcpyDeviceToDevice, s));
        // the entries per column of A (the transpose's row lengths; column
        // indices outside [0, n) are skipped here and rejected below) and
        // the longest row of A and of A^T: flag[4], flag[5]
        int32_t *cnt = w->ptr<int32_t>(L.cnt);
        int32_t *rpT = w->ptr<int32_t>(L.rpT);
        hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n + 1, 256)), dim3(256), 0, s, cnt, (int64_t)n + 1, 0);
        if (nnz > 0)
            hipLaunchKernelGGL(k_count_cols, dim3(grid_for(nnz, 256)), dim3(256), 0, s,
                               (const int32_t *)w->ptr<int32_t>(L.ciA), nnz, n, cnt);
        hipLaunchKernelGGL(k_max_diff, dim3(grid_for(m, 256, 1024)), dim3(256), 0, s,
                           (const int32_t *)w->ptr<int32_t>(L.rpA), m, flag + 4);
        hipLaunchKernelGGL(k_max_value, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s,
                           (const int32_t *)cnt, n, flag + 5);
        HIP_TRY(hipGetLastError());
        unsigned hflag[6] = {0, 0, 0, 0, 0, 0};
        HIP_TRY(hipMemcpyAsync(hflag, flag, 24, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hflag[0]) return fail(HSD_ERR_NONFINITE, "A, b or c holds a NaN or Inf");
        if ((int32_t)hflag[2] != 0 || (int64_t)(int32_t)hflag[3] != nnz)
            return fail(HSD_ERR_ARG, "row_ptr must start at 0 and end at nnz");
        if (hflag[1]) return fail(HSD_ERR_ARG, "row_ptr is not monotone or a column index is outside [0, n)");
        w->max_row_a = (int)hflag[4];
        w->max_row_t = (int)hflag[5];

        // transpose of A (cnt holds the entries per column)
        if ((r = scan_exclusive(cnt, rpT, (int64_t)n + 1, w->ptr<int32_t>(L.scan), s))) return r;
        hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n + 1, 256)), dim3(256), 0, s, cnt, (int64_t)n + 1, 0);
        hipLaunchKernelGGL(k_scatter_t, dim3(grid_for(m, 256)), dim3(256), 0, s, m,
                           (const int32_t *)w->ptr<int32_t>(L.rpA), (const int32_t *)w->ptr<int32_t>(L.ciA),
                           (const double *)w->ptr<double>(L.vA), (const int32_t *)rpT, cnt,
                           w->ptr<int32_t>(L.ciT), w->ptr<double>(L.vT));
        if ((r = sort_rows(n, (const int32_t *)rpT, w->ptr<int32_t>(L.ciT), w->ptr<double>(L.vT), w->max_row_t, s)))
            return r;

        // column slabs: rows of A sorted by column (the slab-major copies
        // are made after the scaling below)
        const SlabPlan &sp = w->sp;
        if (sp.ka > 1 && (r = sort_rows(m, (const int32_t *)w->ptr<int32_t>(L.rpA), w->ptr<int32_t>(L.ciA),
                                        w->ptr<double>(L.vA), w->max_row_a, s)))
            return r;

        // equilibration (Sect. 5): D, E, sigma, rho
        double *D = w->ptr<double>(L.D), *E = w->ptr<double>(L.E), *dt = w->ptr<double>(L.dtmp);
        hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(m, 256)), dim3(256), 0, s, D, (int64_t)m, 1.0);
        hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, E, (int64_t)n, 1.0);
        const int nblk = (int)w->hc.blk_off.size();
        if (st->scale) {
            for (int pass = 0; pass < 10; ++pass) {
                hipLaunchKernelGGL(k_scaled_row_norms, dim3(grid_for(m, 4)), dim3(256), 0, s, m,
                                   (const int32_t *)w->ptr<int32_t>(L.rpA), (const int32_t *)w->ptr<int32_t>(L.ciA),
                                   (const double *)w->ptr<double>(L.vA), (const double *)D, (const double *)E, dt);
                hipLaunchKernelGGL(k_inv_sqrt, dim3(grid_for(m, 256)), dim3(256), 0, s, dt, m);
                if (nblk > 0)
                    hipLaunchKernelGGL(k_block_mean, dim3(grid_for(nblk, 4)), dim3(256), 0, s, dt, nblk,
                                       (const int32_t *)w->ptr<int32_t>(L.blk_off),
                                       (const int32_t *)w->ptr<int32_t>(L.blk_len));
                hipLaunchKernelGGL(k_mul_clip, dim3(grid_for(m, 256)), dim3(256), 0, s, D, (const double *)dt, m, 1e-4, 1e4);
                hipLaunchKernelGGL(k_scaled_row_norms, dim3(grid_for(n, 4)), dim3(256), 0, s, n,
                                   (const int32_t *)rpT, (const int32_t *)w->ptr<int32_t>(L.ciT),
                                   (const double *)w->ptr<double>(L.vT), (const double *)E, (const double *)D, dt);
                hipLaunchKernelGGL(k_inv_sqrt, dim3(grid_for(n, 256)), dim3(256), 0, s, dt, n);
                hipLaunchKernelGGL(k_mul_clip, dim3(grid_for(n, 256)), dim3(256), 0, s, E, (const double *)dt, n, 1e-4, 1e4);
            }
        }
        // row norms of the final D A E for rho
        hipLaunchKernelGGL(k_scaled_row_norms, dim3(grid_for(m, 4)), dim3(256), 0, s, m,
                           (const int32_t *)w->ptr<int32_t>(L.rpA), (const int32_t *)w->ptr<int32_t>(L.ciA),
                           (const double *)w->ptr<double>(L.vA), (const double *)D, (const double *)E, dt);
        double *scal = w->ptr<double>(L.scal);
        hipLaunchKernelGGL(k_sigma_rho, dim3(1), dim3(1024), 0, s, b, (const double *)D, m, c,
                           (const double *)E, n, (const double *)dt, st->scale, scal);
        hipLaunchKernelGGL(k_scale_values<false>, dim3(grid_for(m, 256)), dim3(256), 0, s, m,
                           (const int32_t *)w->ptr<int32_t>(L.rpA), (const int32_t *)w->ptr<int32_t>(L.ciA),
                           w->ptr<double>(L.vA), (const double *)D, (const double *)E,
                           st->precision ? w->ptr<float>(L.vA32) : (float *)nullptr);
        hipLaunchKernelGGL(k_scale_values<true>, dim3(grid_for(n, 256)), dim3(256), 0, s, n,
                           (const int32_t *)rpT, (const int32_t *)w->ptr<int32_t>(L.ciT),
                           w->ptr<double>(L.vT), (const double *)E, (const double *)D,
                           st->precision ? w->ptr<float>(L.vT32) : (float *)nullptr);
        hipLaunchKernelGGL(k_scale_rhs, dim3(1), dim3(1024), 0, s, b, c, (const double *)D,
                           (const double *)E, m, n, w->ptr<double>(L.bh), w->ptr<double>(L.ch), scal);
        HIP_TRY(hipGetLastError());

        // slab-major copies of the scaled A and A^T: row-major slab
        // boundaries, entries per (slab, row), their exclusive scan (the
        // slab-major offsets), then the scatter
        if (sp.on()) {
            struct Side { int32_t rows, K; size_t rp, ci, v, v32, off, ci_s, v_s, v32_s; };
            const Side sides[2] = {{m, sp.ka, L.rpA, L.ciA, L.vA, L.vA32, L.off_a, L.ciA_s, L.vA_s, L.vA32_s},
                                   {n, sp.kt, L.rpT, L.ciT, L.vT, L.vT32, L.off_t, L.ciT_s, L.vT_s, L.vT32_s}};
            int32_t *bnd = w->ptr<int32_t>(L.bnd);
            for (const Side &sd : sides) {
                if (sd.K <= 1) continue;  // one slab: the row-major matrix as it is
                int32_t *off = w->ptr<int32_t>(sd.off);
                const int64_t cnt_len = (int64_t)sd.K * sd.rows + 1;
                hipLaunchKernelGGL(k_slab_offsets, dim3(grid_for(sd.rows, 256)), dim3(256), 0, s, sd.rows,
                                   (const int32_t *)w->ptr<int32_t>(sd.rp), (const int32_t *)w->ptr<int32_t>(sd.ci),
                                   sd.K, sp.width, bnd);
                hipLaunchKernelGGL(k_slab_counts, dim3(grid_for(cnt_len, 256)), dim3(256), 0, s, sd.rows, sd.K,
                                   (const int32_t *)bnd, off);
                HIP_TRY(hipGetLastError());
                if ((r = scan_exclusive(off, off, cnt_len, w->ptr<int32_t>(L.scan), s))) return r;
                hipLaunchKernelGGL(k_slab_scatter, dim3(grid_for(sd.rows, 256)), dim3(256), 0, s, sd.rows, sd.K,
                                   (const int32_t *)bnd, (const int32_t *)off,
                                   (const int32_t *)w->ptr<int32_t>(sd.ci), (const double *)w->ptr<double>(sd.v),
                                   st->precision ? (const float *)w->ptr<float>(sd.v32) : (const float *)nullptr,
                                   w->ptr<int32_t>(sd.ci_s), w->ptr<double>(sd.v_s),
                                   st->precision ? w->ptr<float>(sd.v32_s) : (float *)nullptr);
                HIP_TRY(hipGetLastError());
            }
        }

        // launch shape
        // defaults from a sweep on the 10k x 30k random SOCP (300k nonzeros):
        // 512 threads, about 4 nonzeros per lane, ~4.7k nonzeros per workgroup
        // slab sweeps: 256 threads, so that three workgroups share a CU (LDS
        // of the slab blocks and 168 VGPRs); otherwise 512
        w->threads = st->block_threads ? st->block_threads : (sp.on() ? 256 : 512);
        const double avg_a = nnz / (double)std::max(1, m);
        const double avg_t = nnz / (double)std::max(1, n);
        // with column slabs a row is visited once per slab: size the lanes
        // by the entries a row has in one slab
        const double per_a = sp.on() ? avg_a / sp.ka : avg_a;
        const double per_t = sp.on() ? avg_t / sp.kt : avg_t;
        w->lanes_a = st->lanes_a ? st->lanes_a : pow2_floor(per_a / 4.0, 1, 64);
        w->lanes_t = st->lanes_at ? st->lanes_at : pow2_floor(per_t / 4.0, 1, 64);
        double avg_soc = 0.0;
        for (int q : w->hc.soc_len) avg_soc += q;
        if (!w->hc.soc_len.empty()) avg_soc /= w->hc.soc_len.size();
        w->lanes_soc = st->lanes_soc ? st->lanes_soc : pow2_floor(std::max(1.0, avg_soc), 1, 64);
        w->psd_warm = w->hc.max_psd > 0 && w->hc.max_psd <= PSD_WARM_MAX && !sp.on();
        w->lds_bytes = w->hc.max_psd > 0 ? 8 * (size_t)psd_lds_doubles(w->hc.max_psd, w->psd_warm) : 0;
        if (w->psd_warm) {
            // (host copy kept in the handle: the copy is asynchronous)
            std::vector<int64_t> &voff = w->psd_voff;
            voff.assign(w->hc.psd_dim.size(), 0);
            int64_t acc = 0;
            for (size_t i = 0; i < voff.size(); ++i) {
                const int d = w->hc.psd_dim[i], dp = d + (d & 1);
                voff[i] = acc;
                acc += (int64_t)dp * dp;
            }
            HIP_TRY(hipMemcpyAsync(w->ptr<int64_t>(L.psdvoff), voff.data(), 8 * voff.size(), hipMemcpyHostToDevice, s));
        }
        // slab sweeps keep per-row partial sums of a chunk of rows in LDS
        // (one CG-precision and one FP64 slot per row) after the PSD scratch
        const bool slabs = sp.on();
        w->slab_lds = 0;
        w->slab_rows = 0;
        if (slabs) {
            const size_t psd = (w->lds_bytes + 15) / 16 * 16;
            w->slab_rows = SLAB_CHUNK_ROWS;
            w->slab_lds = (int)(psd / 8);
            w->lds_bytes = psd + 8 * slab_lds_doubles(w->slab_rows, w->threads);
        }
        if ((r = allow_lds(w->lds_bytes))) return r;
        int bpc64 = 0, bpc32 = 0, dev = 0, cus = 0;
        // long rows or warm-started PSD projections: the general kernels
        w->longr = !slabs && (w->max_row_a > LONG_CHUNKS * ROW_CHUNK * w->lanes_a ||
                              w->max_row_t > LONG_CHUNKS * ROW_CHUNK * w->lanes_t || w->psd_warm);
        const bool direct = L.np > 0;
        if ((r = occupancy(solve_fn<double>(slabs, w->longr, direct), w->threads, w->lds_bytes, &bpc64))) return r;
        if ((r = occupancy(solve_fn<float>(slabs, w->longr, direct), w->threads, w->lds_bytes, &bpc32))) return r;
        int bpcg = 0;
        if ((r = occupancy(setup_g_fn(slabs, w->longr, direct), w->threads, w->lds_bytes, &bpcg))) return r;
        bpc64 = std::min(bpc64, bpcg);
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const int cap = std::min(MAX_TEAM, std::max(1, std::min(bpc64, bpc32) * cus));
        int team = st->team_blocks;
        // automatic: about 4,608 nonzeros per workgroup; with the direct
        // projection one workgroup per CU, since the dense product with
        // G^{-1} wants every CU's loads in flight
        if (team == 0)
            team = direct ? std::min(cap, cus)
                          : (int)std::min<int64_t>(cap, std::max<int64_t>(1, nnz / 4608));
        if (team > cap) return fail(HSD_ERR_ARG, "team_blocks exceeds the co-resident limit " + std::to_string(cap));
        w->team = team;
        // rows of A: cone-aligned, so that each workgroup projects its own
        // cones, and balanced by nonzeros plus, for a PSD cone of side d,
        // PSD_COST_PER_SIDE * d more (its projection, one workgroup's
        // Jacobi rounds, outlasts the products of thousands of nonzeros),
        // so that large PSD cones go to different workgroups
        const int32_t *row_cost = w->ptr<int32_t>(L.rpA);
        if (!w->hc.psd_dim.empty() && !slabs) {
            std::vector<int32_t> rph((size_t)m + 1), cst((size_t)m + 1);
            HIP_TRY(hipMemcpyAsync(rph.data(), w->ptr<int32_t>(L.rpA), 4 * ((size_t)m + 1), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            int64_t extra = 0;
            size_t q = 0;
            bool fits = true;
            for (int64_t i = 0; i <= m && fits; ++i) {
                while (q < w->hc.psd_off.size() && w->hc.psd_off[q] < i) extra += PSD_COST_PER_SIDE * w->hc.psd_dim[q++];
                const int64_t c = rph[i] + extra;
                fits = c <= (int64_t)INT32_MAX;
                cst[i] = (int32_t)c;
            }
            if (fits) {
                // the scaling's scratch is free again at this point
                HIP_TRY(hipMemcpyAsync(w->ptr<double>(L.dtmp), cst.data(), 4 * ((size_t)m + 1), hipMemcpyHostToDevice, s));
                HIP_TRY(hipStreamSynchronize(s));  // cst is freed at the end of this block
                row_cost = reinterpret_cast<const int32_t *>(w->ptr<double>(L.dtmp));
            }
        }
        hipLaunchKernelGGL(k_partition, dim3(grid_for(team + 1, 256)), dim3(256), 0, s, row_cost, m, team,
                           w->ptr<int32_t>(L.part_a), (const int32_t *)w->ptr<int32_t>(L.blk_off),
                           (const int32_t *)w->ptr<int32_t>(L.blk_len), (int32_t)w->hc.blk_off.size());
        hipLaunchKernelGGL(k_partition, dim3(grid_for(team + 1, 256)), dim3(256), 0, s,
                           (const int32_t *)rpT, n, team, w->ptr<int32_t>(L.part_t));
        HIP_TRY(hipGetLastError());

        // The own-row and own-column stages of the solve kernel (row-group
        // sweeps): ROW_STAGE doubles per row and COL_STAGE per column of the
        // widest workgroup, after the PSD scratch, each when it fits beside
        // the kernel's static LDS.
        w->lds_solve = w->lds_bytes;
        w->mat_lds = -1;
        w->g_mat = false;
        w->row_lds = w->row_cap = 0;
        w->col_lds = w->col_cap = 0;
        size_t lds_base = (w->lds_bytes + 15) / 16 * 16;
        // the largest LDS matrix slice, read back with the partitions
        const bool want_slices = st->lds_matrix == 1 && !slabs;
        unsigned slice = 0;
        if (want_slices) {
            hipLaunchKernelGGL(k_fill<unsigned>, dim3(1), dim3(64), 0, s, flag, (int64_t)4, 0u);
            hipLaunchKernelGGL(k_slice_bytes, dim3(grid_for(team, 256)), dim3(256), 0, s,
                               (const int32_t *)w->ptr<int32_t>(L.rpA), (const int32_t *)rpT,
                               (const int32_t *)w->ptr<int32_t>(L.part_a), (const int32_t *)w->ptr<int32_t>(L.part_t),
                               team, st->precision ? 4 : 8, flag);
            HIP_TRY(hipGetLastError());
        }
        if (!slabs) {
            std::vector<int32_t> pa((size_t)team + 1), pt((size_t)team + 1);
            HIP_TRY(hipMemcpyAsync(pa.data(), w->ptr<int32_t>(L.part_a), 4 * ((size_t)team + 1),
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(pt.data(), w->ptr<int32_t>(L.part_t), 4 * ((size_t)team + 1),
                                   hipMemcpyDeviceToHost, s));
            if (want_slices) HIP_TRY(hipMemcpyAsync(&slice, flag, 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            int rows = 0, cols = 0;
            for (int q = 0; q < team; ++q) {
                rows = std::max(rows, pa[q + 1] - pa[q]);
                cols = std::max(cols, pt[q + 1] - pt[q]);
            }
            int maxsh = 0;
            HIP_TRY(hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
            const void *fn = st->precision ? solve_fn<float>(false, w->longr, direct) : solve_fn<double>(false, w->longr, direct);
            // true when `total` bytes of dynamic LDS keep the team co-resident
            auto fits = [&](size_t total, bool &ok) -> int {
                ok = false;
                if (total + 4096 > (size_t)maxsh) return HSD_OK;
                HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)total));
                int bpc = 0;
                if (int e = occupancy(fn, w->threads, total, &bpc)) return e;
                ok = bpc >= 1 && team <= bpc * cus;
                return HSD_OK;
            };
            bool ok = false;
            const size_t rstage = ((size_t)ROW_STAGE * 8 * rows + 15) / 16 * 16;
            if (rows > 0) {
                if ((r = fits(lds_base + rstage, ok))) return r;
                if (ok) {
                    w->row_lds = (int)(lds_base / 8);
                    w->row_cap = rows;
                    lds_base += rstage;
                }
            }
            const size_t cstage = ((size_t)COL_STAGE * 8 * cols + 15) / 16 * 16;
            if (cols > 0) {
                if ((r = fits(lds_base + cstage, ok))) return r;
                if (ok) {
                    w->col_lds = (int)(lds_base / 8);
                    w->col_cap = cols;
                    lds_base += cstage;
                }
            }
            w->lds_solve = lds_base;
            // leave the attribute at what the launch uses
            if ((r = fits(lds_base, ok))) return r;
        }
        // LDS-resident matrix slices for the solve kernel when they fit
        if (want_slices) {
            int maxsh = 0;
            HIP_TRY(hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
            const size_t psd = lds_base;
            const size_t total = psd + ((size_t)slice + 15) / 16 * 16;
            // static LDS of the kernel (reductions) and a margin stay free
            if (total + 4096 <= (size_t)maxsh) {
                const void *fn = st->precision ? solve_fn<float>(false, w->longr, direct) : solve_fn<double>(false, w->longr, direct);
                HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)total));
                int bpc = 0;
                if ((r = occupancy(fn, w->threads, total, &bpc))) return r;
                if (bpc >= 1 && team <= bpc * cus) {
                    w->lds_solve = total;
                    w->mat_lds = (int)(psd / 8);
                    // the FP64 g pass reads the same slices when its team
                    // stays co-resident with this much LDS
                    if (!st->precision) {
                        const void *gfn = setup_g_fn(false, w->longr, direct);
                        HIP_TRY(hipFuncSetAttribute(gfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)total));
                        int gbpc = 0;
                        if ((r = occupancy(gfn, w->threads, total, &gbpc))) return r;
                        w->g_mat = gbpc >= 1 && team <= gbpc * cus;
                    }
                }
            }
        }

        // direct projection: G = I + A_hat^T A_hat, its Cholesky factor and
        // its inverse, once (factorization caching)
        if (L.np > 0) {
            unsigned *flag = w->ptr<unsigned>(L.flag);
            hipLaunchKernelGGL(k_fill<unsigned>, dim3(1), dim3(64), 0, s, flag, (int64_t)1, 0u);
            if ((r = direct_prepare(w->ptr<double>(L.dW), w->ptr<double>(L.dZ), L.np, n, (const int32_t *)rpT,
                                    (const int32_t *)w->ptr<int32_t>(L.ciT), (const double *)w->ptr<double>(L.vT),
                                    flag, s)))
                return r;
            unsigned hbad = 0;
            HIP_TRY(hipMemcpyAsync(&hbad, flag, 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (hbad) return fail(HSD_ERR_NONFINITE, "the Cholesky factorization of I + A^T A met a non-positive pivot");
        }

        // g = M^{-1} h (Sect. 4.1): the solver in MODE_G with u = v = 0,
        // u_tau = -1 (so r = h) and z_x = 0; g and eta stay in FP64
        const int64_t N = (int64_t)n + m + 1;
        hipLaunchKernelGGL(k_init_uv, dim3(grid_for(N, 256)), dim3(256), 0, s, w->ptr<double>(L.u),
                           w->ptr<double>(L.v), N, -1.0, 0.0);
        hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, w->ptr<double>(L.zx), (int64_t)n, 0.0);
        HIP_TRY(hipGetLastError());
        if ((r = run_mode(w, MODE_G, 1, 0, nullptr, nullptr))) return r;
        double hinfo[INFO_COUNT];
        if ((r = read_info(w, hinfo))) return r;
        return HSD_OK;
    };
    rc = run();
    hipEventRecord(e1, s);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return cleanup(rc);
    if (hipEventCreate(&w->kev0) != hipSuccess || hipEventCreate(&w->kev1) != hipSuccess)
        return cleanup(fail(HSD_ERR_HIP, "hipEventCreate failed"));
    w->setup_ms = ms;
    w->ready = true;
    *out = w;
    return HSD_OK;
}

static int prepare_start(hsd_work *w) {
    hipStream_t s = w->stream;
    const Layout &L = w->L;
    const int64_t N = (int64_t)w->n + w->m + 1;
    if (!w->start_set) {
        hipLaunchKernelGGL(k_init_uv, dim3(grid_for(N, 256)), dim3(256), 0, s, w->ptr<double>(L.u),
                           w->ptr<double>(L.v), N, 1.0, 1.0);
        w->zx_set = false;
        w->k0 = 0;
        w->carried = false;
    }
    if (!w->zx_set) {
        if (w->st.precision)
            hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(w->n, 256)), dim3(256), 0, s, w->ptr<float>(L.zx), (int64_t)w->n, 0.f);
        else
            hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(w->n, 256)), dim3(256), 0, s, w->ptr<double>(L.zx), (int64_t)w->n, 0.0);
    }
    HIP_TRY(hipGetLastError());
    return HSD_OK;
}

// After a run: the next run starts cold unless a start is set in between.
static void clear_start(hsd_work *w) {
    w->start_set = false;
    w->zx_set = false;
    w->k0 = 0;
    w->carried = false;
}

extern "C" int hsd_solve(hsd_work_t *w, double *x, double *y, double *s, hsd_info_t *info) {
    if (!w || !w->ready) return fail(HSD_ERR_STATE, "handle is not set up");
    if (!info) return fail(HSD_ERR_ARG, "info is null");
    hipStream_t st = w->stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(HSD_ERR_HIP, "hipEventCreate failed");
    hipEventRecord(e0, st);
    int rc = prepare_start(w);
    if (!rc) rc = run_mode(w, MODE_SOLVE, w->st.max_iters, 0, nullptr, nullptr);
    clear_start(w);
    if (!rc) {
        const Layout &L = w->L;
        hipLaunchKernelGGL(k_outputs, dim3(grid_for((int64_t)w->n + w->m, 256)), dim3(256), 0, st,
                           (const double *)w->ptr<double>(L.u), (const double *)w->ptr<double>(L.v),
                           (const double *)w->ptr<double>(L.D), (const double *)w->ptr<double>(L.E),
                           (const double *)w->ptr<double>(L.scal), (const double *)w->ptr<double>(L.info),
                           w->m, w->n, x, y, s);
        if (hipGetLastError() != hipSuccess) rc = fail(HSD_ERR_HIP, "output kernel launch failed");
    }
    hipEventRecord(e1, st);
    double h[INFO_COUNT];
    if (!rc) rc = read_info(w, h);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    w->has_state = true;
    w->k_last = (int32_t)h[INFO_ITERS];
    std::memset(info, 0, sizeof(*info));
    info->status = (int)h[INFO_STATUS];
    info->iters = (int)h[INFO_ITERS];
    info->res_pri = h[INFO_RES_PRI];
    info->res_dual = h[INFO_RES_DUAL];
    info->gap = h[INFO_GAP];
    info->pobj = h[INFO_POBJ];
    info->dobj = h[INFO_DOBJ];
    info->obj = 0.5 * (h[INFO_POBJ] + h[INFO_DOBJ]);
    info->tau = h[INFO_TAU];
    info->kappa = h[INFO_KAPPA];
    info->cg_iters = (int64_t)h[INFO_CG_ITERS];
    info->spmv_count = (int64_t)h[INFO_SPMV];
    info->setup_ms = w->setup_ms;
    info->solve_ms = ms;
    info->res_infeas = h[INFO_RES_INF];
    info->res_unbdd = h[INFO_RES_UNB];
    float kms = 0.f;
    if (hipEventElapsedTime(&kms, w->kev0, w->kev1) == hipSuccess) info->kernel_ms = kms;
    return HSD_OK;
}

extern "C" int hsd_warm_start(hsd_work_t *w, const double *x, const double *y, const double *s) {
    if (!w || !w->ready) return fail(HSD_ERR_STATE, "handle is not set up");
    if (!x || !y || !s) return fail(HSD_ERR_ARG, "null argument");
    const Layout &L = w->L;
    const int64_t N = (int64_t)w->n + w->m + 1;
    hipLaunchKernelGGL(k_warm_xys, dim3(grid_for(N, 256)), dim3(256), 0, w->stream, x, y, s,
                       (const double *)w->ptr<double>(L.D), (const double *)w->ptr<double>(L.E),
                       (const double *)w->ptr<double>(L.scal), w->m, w->n, w->ptr<double>(L.u),
                       w->ptr<double>(L.v));
    HIP_TRY(hipGetLastError());
    clear_start(w);
    w->start_set = true;
    return HSD_OK;
}

static ConeDev cone_dev(const hsd_work *w) {
    ConeDev K = make_prob<double>(w, nullptr, nullptr).cone;
    return K;
}

extern "C" int hsd_start_from_q(hsd_work_t *w, const double *q) {
    if (!w || !w->ready) return fail(HSD_ERR_STATE, "handle is not set up");
    if (!q) return fail(HSD_ERR_ARG, "null argument");
    const Layout &L = w->L;
    const int n = w->n, m = w->m;
    ConeDev K = cone_dev(w);
    const int blocks = std::max(1, std::min(1024, (m + 255) / 256));
    const int Ls = w->lanes_soc;
    double *u = w->ptr<double>(L.u), *v = w->ptr<double>(L.v);
    // u_y = Pi_{K*}(q_y), v_s = Pi_K(-q_y)
    hipLaunchKernelGGL(k_project, dim3(blocks), dim3(256), w->lds_bytes, w->stream, K, m, q + n, 1.0,
                       u + n, 1, Ls);
    hipLaunchKernelGGL(k_project, dim3(blocks), dim3(256), w->lds_bytes, w->stream, K, m, q + n, -1.0,
                       v + n, 0, Ls);
    hipLaunchKernelGGL(k_q_rest, dim3(grid_for(n + 1, 256)), dim3(256), 0, w->stream, q, m, n, u, v);
    HIP_TRY(hipGetLastError());
    clear_start(w);
    w->start_set = true;
    return HSD_OK;
}

extern "C" int hsd_iterate(hsd_work_t *w, int32_t count, double *u_hist, double *v_hist) {
    if (!w || !w->ready) return fail(HSD_ERR_STATE, "handle is not set up");
    if (count < 0 || !u_hist || !v_hist) return fail(HSD_ERR_ARG, "bad argument");
    int rc = prepare_start(w);
    if (rc) return rc;
    // count updates from the start point (a restored state included)
    rc = run_mode(w, MODE_ITERATE, w->k0 + count, count, u_hist, v_hist);
    clear_start(w);
    if (rc) return rc;
    double h[INFO_COUNT];
    rc = read_info(w, h);
    if (rc) return rc;
    w->has_state = true;
    w->k_last = (int32_t)h[INFO_ITERS];
    return HSD_OK;
}

extern "C" int hsd_get_scaling(hsd_work_t *w, double *D, double *E, double *sigma, double *rho) {
    if (!w || !w->ready) return fail(HSD_ERR_STATE, "handle is not set up");
    const Layout &L = w->L;
    if (D) HIP_TRY(hipMemcpyAsync(D, w->ptr<double>(L.D), 8 * (size_t)w->m, hipMemcpyDeviceToDevice, w->stream));
    if (E) HIP_TRY(hipMemcpyAsync(E, w->ptr<double>(L.E), 8 * (size_t)w->n, hipMemcpyDeviceToDevice, w->stream));
    double sc[SC_COUNT];
    HIP_TRY(hipMemcpyAsync(sc, w->ptr<double>(L.scal), 8 * SC_COUNT, hipMemcpyDeviceToHost, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    if (sigma) *sigma = sc[SC_SIGMA];
    if (rho) *rho = sc[SC_RHO];
    return HSD_OK;
}

static int compute_g(hsd_work *w) {
    const Layout &L = w->L;
    w->has_state = false;  // the g pass runs through u, v and z_x
    const int64_t N = (int64_t)w->n + w->m + 1;
    hipLaunchKernelGGL(k_init_uv, dim3(grid_for(N, 256)), dim3(256), 0, w->stream, w->ptr<double>(L.u),
                       w->ptr<double>(L.v), N, -1.0, 0.0);
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(w->n, 256)), dim3(256), 0, w->stream,
                       w->ptr<double>(L.zx), (int64_t)w->n, 0.0);
    HIP_TRY(hipGetLastError());
    int r = run_mode(w, MODE_G, 1, 0, nullptr, nullptr);
    if (r) return r;
    double h[INFO_COUNT];
    return read_info(w, h);
}

extern "C" int hsd_update_b(hsd_work_t *w, const double *b) {
    if (!w || !w->ready) return fail(HSD_ERR_STATE, "handle is not set up");
    if (!b) return fail(HSD_ERR_ARG, "b is null");
    const Layout &L = w->L;
    unsigned *flag = w->ptr<unsigned>(L.flag);
    unsigned hflag = 0;
    hipLaunchKernelGGL(k_fill<unsigned>, dim3(1), dim3(64), 0, w->stream, flag, (int64_t)4, 0u);
    hipLaunchKernelGGL(k_count_nonfinite, dim3(grid_for(w->m, 1024, 256)), dim3(1024), 0, w->stream, b,
                       (int64_t)w->m, flag);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    if (hflag) return fail(HSD_ERR_NONFINITE, "b holds a NaN or Inf");
    hipLaunchKernelGGL(k_update_b, dim3(1), dim3(1024), 0, w->stream, b, (const double *)w->ptr<double>(L.D),
                       w->m, w->st.scale, w->ptr<double>(L.bh), w->ptr<double>(L.scal));
    HIP_TRY(hipGetLastError());
    clear_start(w);
    return compute_g(w);
}

extern "C" int hsd_update_bc(hsd_work_t *w, const double *b, const double *c) {
    if (!w || !w->ready) return fail(HSD_ERR_STATE, "handle is not set up");
    if (!b || !c) return fail(HSD_ERR_ARG, "b or c is null");
    const Layout &L = w->L;
    unsigned *flag = w->ptr<unsigned>(L.flag);
    unsigned hflag = 0;
    hipLaunchKernelGGL(k_fill<unsigned>, dim3(1), dim3(64), 0, w->stream, flag, (int64_t)4, 0u);
    hipLaunchKernelGGL(k_count_nonfinite, dim3(grid_for(w->m, 1024, 256)), dim3(1024), 0, w->stream, b,
                       (int64_t)w->m, flag);
    hipLaunchKernelGGL(k_count_nonfinite, dim3(grid_for(w->n, 1024, 256)), dim3(1024), 0, w->stream, c,
                       (int64_t)w->n, flag);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    if (hflag) return fail(HSD_ERR_NONFINITE, "b or c holds a NaN or Inf");
    hipLaunchKernelGGL(k_update_b, dim3(1), dim3(1024), 0, w->stream, b, (const double *)w->ptr<double>(L.D),
                       w->m, w->st.scale, w->ptr<double>(L.bh), w->ptr<double>(L.scal));
    hipLaunchKernelGGL(k_update_c, dim3(1), dim3(1024), 0, w->stream, c, (const double *)w->ptr<double>(L.E),
                       w->n, w->st.scale, w->ptr<double>(L.ch), w->ptr<double>(L.scal));
    HIP_TRY(hipGetLastError());
    clear_start(w);
    return compute_g(w);
}

extern "C" int hsd_get_state(hsd_work_t *w, double *u, double *v, double *zx, double *carry,
                             int32_t *k) {
    if (!w || !w->ready) return fail(HSD_ERR_STATE, "handle is not set up");
    if (!w->has_state) return fail(HSD_ERR_STATE, "no hsd_solve or hsd_iterate has run on this handle");
    const Layout &L = w->L;
    hipStream_t s = w->stream;
    const int64_t N = (int64_t)w->n + w->m + 1;
    const int m = w->m, n = w->n;
    if (u) HIP_TRY(hipMemcpyAsync(u, w->ptr<double>(L.u), 8 * (size_t)N, hipMemcpyDeviceToDevice, s));
    if (v) HIP_TRY(hipMemcpyAsync(v, w->ptr<double>(L.v), 8 * (size_t)N, hipMemcpyDeviceToDevice, s));
    if (w->st.precision) {
        if (zx) hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(n, 256)), dim3(256), 0, s,
                                   (const float *)w->ptr<float>(L.zx), zx, (int64_t)n);
        if (carry) hipLaunchKernelGGL((k_cast<double, float>), dim3(grid_for(m, 256)), dim3(256), 0, s,
                                      (const float *)w->ptr<float>(L.azc), carry, (int64_t)m);
    } else {
        if (zx) HIP_TRY(hipMemcpyAsync(zx, w->ptr<double>(L.zx), 8 * (size_t)n, hipMemcpyDeviceToDevice, s));
        if (carry) HIP_TRY(hipMemcpyAsync(carry, w->ptr<double>(L.azc), 8 * (size_t)m, hipMemcpyDeviceToDevice, s));
    }
    HIP_TRY(hipGetLastError());
    if (carry) HIP_TRY(hipMemcpyAsync(carry + m, w->ptr<double>(L.aux), 8 * (size_t)m, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (k) *k = w->k_last;
    return HSD_OK;
}

extern "C" int hsd_set_state(hsd_work_t *w, const double *u, const double *v, const double *zx,
                             const double *carry, int32_t k) {
    if (!w || !w->ready) return fail(HSD_ERR_STATE, "handle is not set up");
    if (!u || !v || !zx) return fail(HSD_ERR_ARG, "u, v and z_x are required");
    if (k < 0) return fail(HSD_ERR_ARG, "the iteration number must be nonnegative");
    const Layout &L = w->L;
    hipStream_t s = w->stream;
    const int64_t N = (int64_t)w->n + w->m + 1;
    const int m = w->m, n = w->n;
    HIP_TRY(hipMemcpyAsync(w->ptr<double>(L.u), u, 8 * (size_t)N, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(w->ptr<double>(L.v), v, 8 * (size_t)N, hipMemcpyDeviceToDevice, s));
    if (w->st.precision) {
        hipLaunchKernelGGL((k_cast<float, double>), dim3(grid_for(n, 256)), dim3(256), 0, s, zx,
                           w->ptr<float>(L.zx), (int64_t)n);
        if (carry) hipLaunchKernelGGL((k_cast<float, double>), dim3(grid_for(m, 256)), dim3(256), 0, s, carry,
                                      w->ptr<float>(L.azc), (int64_t)m);
    } else {
        HIP_TRY(hipMemcpyAsync(w->ptr<double>(L.zx), zx, 8 * (size_t)n, hipMemcpyDeviceToDevice, s));
        if (carry) HIP_TRY(hipMemcpyAsync(w->ptr<double>(L.azc), carry, 8 * (size_t)m, hipMemcpyDeviceToDevice, s));
    }
    HIP_TRY(hipGetLastError());
    if (carry) HIP_TRY(hipMemcpyAsync(w->ptr<double>(L.aux), carry + m, 8 * (size_t)m, hipMemcpyDeviceToDevice, s));
    clear_start(w);
    w->start_set = true;
    w->zx_set = true;
    w->k0 = k;
    w->carried = carry != nullptr;
    return HSD_OK;
}

extern "C" int hsd_update_settings(hsd_work_t *w, const hsd_settings_t *st) {
    if (!w || !w->ready) return fail(HSD_ERR_STATE, "handle is not set up");
    int rc = check_settings(st);
    if (rc) return rc;
    const hsd_settings_t &o = w->st;
    if (st->scale != o.scale || st->precision != o.precision || st->team_blocks != o.team_blocks ||
        st->block_threads != o.block_threads || st->lanes_a != o.lanes_a ||
        st->lanes_at != o.lanes_at || st->lanes_soc != o.lanes_soc || st->lds_matrix != o.lds_matrix ||
        st->slab_cols != o.slab_cols)
        return fail(HSD_ERR_ARG, "scale, precision and launch-shape settings are fixed at setup");
    w->st = *st;
    return HSD_OK;
}

extern "C" int hsd_get_launch(hsd_work_t *w, hsd_launch_t *out) {
    if (!w || !out) return fail(HSD_ERR_ARG, "null argument");
    if (!w->ready) return fail(HSD_ERR_STATE, "handle is not set up");
    hsd_launch_t o{};
    o.team_blocks = w->team;
    o.block_threads = w->threads;
    o.lanes_a = w->lanes_a;
    o.lanes_at = w->lanes_t;
    o.lanes_soc = w->lanes_soc;
    o.slabs_a = w->sp.on() ? w->sp.ka : 1;
    o.slabs_at = w->sp.on() ? w->sp.kt : 1;
    o.lds_matrix = w->mat_lds >= 0 ? 1 : 0;
    o.row_stage = w->row_cap > 0 ? 1 : 0;
    o.col_stage = w->col_cap > 0 ? 1 : 0;
    o.long_rows = w->longr ? 1 : 0;
    o.max_row_a = w->max_row_a;
    o.max_row_at = w->max_row_t;
    o.lds_bytes = (int64_t)w->lds_solve;
    *out = o;
    return HSD_OK;
}

extern "C" void hsd_finish(hsd_work_t *w) {
    if (!w) return;
    if (w->kev0) (void)hipEventDestroy(w->kev0);
    if (w->kev1) (void)hipEventDestroy(w->kev1);
    delete w;
}

// The projection's cone tables in one device block: int32 SOC offsets and
// lengths and PSD offsets and sides, then (8-byte aligned) the power-cone
// parameters.
static size_t cone_table_bytes(const HostCone &hc) {
    const size_t ints = 2 * hc.soc_off.size() + 2 * hc.psd_off.size();
    return (4 * ints + 7) / 8 * 8 + 8 * hc.pow_a.size();
}

static std::vector<unsigned char> cone_table_host(const HostCone &hc) {
    std::vector<unsigned char> buf(cone_table_bytes(hc), 0);
    size_t o = 0;
    for (const std::vector<int32_t> *v : {&hc.soc_off, &hc.soc_len, &hc.psd_off, &hc.psd_dim}) {
        if (!v->empty()) std::memcpy(buf.data() + o, v->data(), 4 * v->size());
        o += 4 * v->size();
    }
    o = (o + 7) / 8 * 8;
    if (!hc.pow_a.empty()) std::memcpy(buf.data() + o, hc.pow_a.data(), 8 * hc.pow_a.size());
    return buf;
}

static ConeDev cone_from_table(const HostCone &hc, unsigned char *tab) {
    const size_t nq = hc.soc_off.size(), ns = hc.psd_off.size();
    const int32_t *ti = reinterpret_cast<const int32_t *>(tab);
    ConeDev Kd{};
    Kd.f = hc.f;
    Kd.l = hc.l;
    Kd.nsoc = (int32_t)nq;
    Kd.soc_off = ti;
    Kd.soc_len = ti + nq;
    Kd.npsd = (int32_t)ns;
    Kd.psd_off = ti + 2 * nq;
    Kd.psd_dim = ti + 2 * nq + ns;
    Kd.nexp = hc.nexp;
    Kd.exp_off = hc.exp_off;
    Kd.nexpd = hc.nexpd;
    Kd.expd_off = hc.expd_off;
    Kd.npow = hc.npow;
    Kd.pow_off = hc.pow_off;
    Kd.pow_a = reinterpret_cast<const double *>(tab + (4 * (2 * nq + 2 * ns) + 7) / 8 * 8);
    Kd.max_psd_dim = hc.max_psd;
    return Kd;
}

// Launch of the projection kernel over a cone whose tables are at tab.
static int launch_project(const HostCone &hc, unsigned char *tab, int32_t m, const double *in,
                          double *out, int32_t dual, hipStream_t s) {
    const ConeDev Kd = cone_from_table(hc, tab);
    double avg = 0.0;
    for (int q : hc.soc_len) avg += q;
    if (!hc.soc_len.empty()) avg /= (double)hc.soc_len.size();
    const int Ls = pow2_floor(std::max(1.0, avg), 1, 64);
    const size_t lds = hc.max_psd > 0 ? 8 * (size_t)psd_lds_doubles(hc.max_psd) : 0;
    const int blocks = std::max(1, std::min(1024, (m + 255) / 256));
    hipLaunchKernelGGL(k_project, dim3(blocks), dim3(256), lds, s, Kd, m, in, 1.0, out, dual, Ls);
    HIP_TRY(hipGetLastError());
    return HSD_OK;
}

// The allocation-free projection keeps the cone tables in this file-scope
// device array, one copy per GPU, held until the process ends.  In host
// code its name is only a stand-in for the symbol: its device address on
// each GPU comes from hipGetSymbolAddress, taken once per device on the
// first call there (with that device current) and kept in scratch_dev.
constexpr size_t NOALLOC_TABLE_BYTES = (size_t)1 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[NOALLOC_TABLE_BYTES];
static unsigned char *scratch_dev[NOALLOC_MAX_DEVICES];
static std::mutex scratch_mu;

static int scratch_ptr(unsigned char **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(HSD_ERR_ARG, "device ordinal beyond the allocation-free projection's table");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_dev[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(HSD_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        scratch_dev[dev] = static_cast<unsigned char *>(p);
    }
    *out = scratch_dev[dev];
    return HSD_OK;
}

extern "C" int hsd_project_cone_noalloc(const hsd_cone_t *K, int32_t m, const double *in,
                                        double *out, int32_t dual, void *stream) {
    if (!in || !out) return fail(HSD_ERR_ARG, "null argument");
    HostCone hc;
    int rc = build_cone(K, hc);
    if (rc) return rc;
    if (hc.m != m) return fail(HSD_ERR_CONE, "cone dimension does not equal m");
    if (m == 0) return HSD_OK;
    const std::vector<unsigned char> host = cone_table_host(hc);
    if (host.size() > NOALLOC_TABLE_BYTES)
        return fail(HSD_ERR_ARG, "the cone tables need " + std::to_string(host.size()) +
                                     " bytes, more than the " + std::to_string(NOALLOC_TABLE_BYTES) +
                                     "-byte scratch of the allocation-free projection");
    unsigned char *tab = nullptr;
    if ((rc = scratch_ptr(&tab))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (!host.empty())
        HIP_TRY(hipMemcpyAsync(tab, host.data(), host.size(), hipMemcpyHostToDevice, s));
    rc = launch_project(hc, tab, m, in, out, dual, s);
    if (rc) return rc;
    // return after the projection, as hsd_project_cone does: the host copy
    // of the tables is released on return
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(HSD_ERR_HIP, std::string("projection: ") + hipGetErrorString(e));
    return HSD_OK;
}

extern "C" int hsd_project_cone(const hsd_cone_t *K, int32_t m, const double *in, double *out,
                                int32_t dual, void *stream) {
    if (!in || !out) return fail(HSD_ERR_ARG, "null argument");
    HostCone hc;
    int rc = build_cone(K, hc);
    if (rc) return rc;
    if (hc.m != m) return fail(HSD_ERR_CONE, "cone dimension does not equal m");
    if (m == 0) return HSD_OK;
    hipStream_t s = (hipStream_t)stream;
    const std::vector<unsigned char> host = cone_table_host(hc);
    unsigned char *tab = nullptr;
    if (!host.empty()) HIP_TRY(hipMalloc(&tab, host.size()));
    if (!host.empty()) {
        hipError_t e = hipMemcpyAsync(tab, host.data(), host.size(), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            (void)hipFree(tab);
            return fail(HSD_ERR_HIP, std::string("cone table copy: ") + hipGetErrorString(e));
        }
    }
    rc = launch_project(hc, tab, m, in, out, dual, s);
    hipError_t e2 = hipStreamSynchronize(s);
    if (tab) (void)hipFree(tab);
    if (rc) return rc;
    if (e2 != hipSuccess) return fail(HSD_ERR_HIP, std::string("projection: ") + hipGetErrorString(e2));
    return HSD_OK;
}
