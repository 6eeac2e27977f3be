// Internal layout shared by the host runtime and the kernels.  Not part of
// the public ABI (see include/hsd.h).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace hsd {

// Partial sums: each workgroup writes PART_STRIDE doubles per phase slot.
constexpr int PART_STRIDE = 8;
// SLOT_A alternates with SLOT_A2 from one iteration to the next: its totals
// are read one barrier later than written.
constexpr int SLOT_A = 0, SLOT_B = 1, SLOT_P1 = 2, SLOT_P2 = 3, SLOT_A2 = 4, NSLOTS = 5;

// Kernel modes.
constexpr int MODE_SOLVE = 0;    // iterate with termination tests
constexpr int MODE_G = 1;        // compute g = M^{-1} h (u = 0, v = 0, u_tau = -1)
constexpr int MODE_ITERATE = 2;  // fixed number of updates, no tests, record iterates

// Layout of the device info area (doubles).
enum InfoSlot {
    INFO_STATUS = 0, INFO_ITERS, INFO_RES_PRI, INFO_RES_DUAL, INFO_GAP, INFO_POBJ,
    INFO_DOBJ, INFO_TAU, INFO_KAPPA, INFO_CG_ITERS, INFO_SPMV, INFO_ETA, INFO_ABORT,
    INFO_BTY, INFO_CTX, INFO_RES_INF, INFO_RES_UNB,
    INFO_COUNT = 18
};

// Device scalars computed at setup.
enum ScalarSlot {
    SC_SIGMA = 0, SC_RHO, SC_ETA, SC_NORM_B, SC_NORM_C, SC_NORM_DINV_BH, SC_NORM_EINV_CH,
    SC_RBAR,  // mean row norm of A_hat (the numerator of rho)
    SC_COUNT = 8
};

// Cone description on the device.  Row offsets are relative to the first
// row of the y-block (0..m-1).
struct ConeDev {
    int32_t f, l;                 // zero rows [0,f), nonnegative rows [f, f+l)
    int32_t nsoc;
    const int32_t *soc_off;       // nsoc
    const int32_t *soc_len;       // nsoc
    int32_t npsd;
    const int32_t *psd_off;       // npsd
    const int32_t *psd_dim;       // npsd
    int32_t nexp, exp_off;        // primal exponential triples
    int32_t nexpd, expd_off;      // dual exponential triples
    int32_t npow, pow_off;        // power-cone triples
    const double *pow_a;          // npow parameters: a >= 0 for K_pow^a, -a for (K_pow^a)^*
    int32_t max_psd_dim;
};

template <typename T>
struct CsrDev {
    const int32_t *rp;            // rows + 1
    const int32_t *ci;            // nnz
    const T *v;                   // nnz
};

// Everything one solve needs (one program).  T is the precision of the
// SpMV/CG part (double, or float in the mixed mode).
template <typename T>
struct alignas(16) Pair {
    T a;       // CG precision
    double b;  // FP64
};

template <typename T>
struct Prob {
    int32_t m, n;
    int64_t nnz;
    CsrDev<double> A, AT;         // FP64 values (always present)
    CsrDev<T> Ac, ATc;            // values used by CG (same arrays when T = double)
    ConeDev cone;
    const double *b, *c;          // scaled data (b_hat, c_hat)
    const double *D, *E;          // scaling
    double *g;                    // n + m (written in MODE_G)
    double *u, *v;                // n + m + 1
    T *zx, *zy, *res, *p0, *p1, *t;
    // gather pairs (kernels that use them): t_i and u_y,i, which the A^T test
    // sweep gathers at the same index, side by side so that one 16-byte load
    // serves both (m entries; t then lives only here)
    Pair<T> *tu;
    // A u_x of the current iterate, row by row (m entries), carried from one
    // update to the next by the owners of the rows (the A test sweep's
    // product without a gather)
    double *aux;
    // A z_x of the last CG solution, row by row (m entries): the next CG
    // starts from that z_x, so its first product is carried from here
    T *azc;
    double *scal;                 // ScalarSlot
    double *info;                 // InfoSlot
    double *hist_u, *hist_v;      // (record + 1) x (n + m + 1), or null
    // workgroup row partitions (team_size + 1 entries each), nnz-balanced
    const int32_t *part_a;        // rows of A
    const int32_t *part_t;        // rows of A^T (= the n-slice owned by each workgroup)
    // column slabs: the products with A visit the columns in slabs_a slabs
    // and A (A.ci, A.v, Ac.v) is then stored slab-major: the entries of row i
    // in slab s are off_a[s * m + i] .. off_a[s * m + i + 1] (slabs_a * m + 1
    // offsets).  Likewise for A^T with off_t.
    int32_t slabs_a, slabs_t;     // 0 or 1 = no slabs
    const int32_t *off_a, *off_t;
    // direct projection: Z = (I + A_hat^T A_hat)^{-1}, dense row-major with
    // leading dimension ldz (null: the indirect projection by CG)
    const double *Z;
    int64_t ldz;
    // eigenvectors of each PSD cone's last projection (warm starts of the
    // Jacobi sweeps), at psd_voff[cone]; null: every projection starts cold
    double *psd_v;
    const int64_t *psd_voff;
};

struct Settings {
    double eps_pri, eps_dual, eps_gap, eps_unbdd, eps_infeas;
    double alpha, zeta_pow, tight_tol, fp32_floor;
    int32_t cg_max, max_iters, check_every, mode, record;
    int32_t k0;        // iteration number of the start point (a resumed state); 0 otherwise
    int32_t carried;   // 1: aux and azc hold the products of the start point (no
                       // product or gather on the first update)
    int32_t lanes_a, lanes_t, lanes_soc;
    int32_t mat_lds;   // offset (doubles) of the LDS matrix slices in dynamic LDS, -1 = off
    int32_t slab_lds;  // offset (doubles) of the slab row accumulators in dynamic LDS
    int32_t slab_rows; // rows per chunk of a slab sweep (accumulator capacity)
    int32_t row_lds;   // offset (doubles) of the own-row stage in dynamic LDS
    int32_t row_cap;   // rows per array of the own-row stage, 0 = no stage
    int32_t col_lds;   // offset (doubles) of the own-column stage in dynamic LDS
    int32_t col_cap;   // columns per array of the own-column stage, 0 = no stage
    int32_t vec_lds;   // offset (doubles) of the iterate vectors in dynamic LDS
                       // (batched kernels with the vectors in LDS), -1 = off
    int32_t lds_total; // batched kernels: dynamic LDS per workgroup (doubles); a
                       // program whose matrix fits after its vectors takes it
                       // into LDS (0 = never)
};

}  // namespace hsd
