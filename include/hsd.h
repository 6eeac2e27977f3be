/*
 * hsd.h -- C ABI of the MI355X (gfx950) solver for cone programs by ADMM on
 * the homogeneous self-dual embedding (O'Donoghue, Chu, Parikh, Boyd,
 * "Conic Optimization via Operator Splitting and Homogeneous Self-Dual
 * Embedding").
 *
 * Problem (paper Sect. 2, e-coneprob):
 *     minimize c^T x  s.t.  A x + s = b,  s in K
 *     maximize -b^T y s.t. -A^T y + r = c, r = 0, y in K^*
 * with A (m x n, sparse), b (m), c (n) and K a product of the zero cone,
 * the nonnegative orthant, second-order cones, PSD cones (scaled svec),
 * primal / dual exponential cones and primal / dual power cones (Sect. 6.1
 * cone list).
 *
 * Conventions for every entry point:
 *  - Every pointer documented as "device" must point to memory allocated on
 *    the current HIP device (hipMalloc or a torch CUDA tensor); "host" means
 *    ordinary host memory.  The library never frees caller memory.
 *  - The library performs no device allocation after setup: the caller
 *    supplies the workspace (size from the *_workspace_bytes call).  Host
 *    metadata owned by a handle is freed by the matching *_finish call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    All work is enqueued on it; calls that return results on the host
 *    synchronise it.
 *  - Return value: 0 (HSD_OK) on success, a negative HSD_ERR_* code
 *    otherwise; hsd_last_error() returns a message for the calling thread.
 *    Solver outcomes are reported in hsd_info_t.status, not as errors.
 *  - Index arrays are int32; nnz must be below 2^31.
 */
#ifndef HSD_H
#define HSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define HSD_OK              0
#define HSD_ERR_ARG        -1  /* null pointer, negative size, bad setting   */
#define HSD_ERR_CONE       -2  /* cone sizes do not add up to m, or a bad size */
#define HSD_ERR_NONFINITE  -3  /* NaN or Inf in A, b or c                     */
#define HSD_ERR_WORKSPACE  -4  /* workspace too small or misaligned          */
#define HSD_ERR_HIP        -5  /* a HIP runtime call failed                  */
#define HSD_ERR_STATE      -6  /* handle not set up / used out of order      */
#define HSD_ERR_ABORTED    -7  /* a device-side bounded wait expired         */

/* ---- solver outcomes (paper Sect. 2.3 cases, Sect. 3.5 tests) ---------- */
#define HSD_SOLVED          1  /* x, y, s approximately optimal              */
#define HSD_MAX_ITERS       2  /* iteration limit; last iterate returned     */
#define HSD_INFEASIBLE      3  /* y is a certificate: A^T y ~ 0, y in K^*, b^T y = -1 */
#define HSD_UNBOUNDED       4  /* x, s certificate: A x + s ~ 0, s in K, c^T x = -1  */
#define HSD_INDETERMINATE   5  /* non-finite iterate, or limit with tau = 0  */

/* Product cone K = {0}^f x R_+^l x SOC(q_0) x ... x PSD(s_0) x ... x
 * K_exp^ep x (K_exp^*)^ed x POW(p_0) x ..., rows in exactly that order
 * (Sect. 6.1 cone list).  SOC rows are (t, xbar) with ||xbar|| <= t.  A PSD
 * cone of side d (1..90) uses d(d+1)/2 rows: the lower triangle of the
 * symmetric matrix in column-major order with off-diagonal entries
 * multiplied by sqrt(2).  Exponential rows are triples (x, y, z) in
 * cl{y > 0, y exp(x/y) <= z}.  Each power-cone entry p_i is one triple:
 * p_i = a in [0, 1] for K_pow^a = {(x, y, z): x^a y^(1-a) >= |z|, x, y >= 0},
 * p_i = -a in [-1, 0) for its dual {(u, v, w): (u/a)^a (v/(1-a))^(1-a) >= |w|,
 * u, v >= 0} (a factor with exponent 0 is 1).  q, s and p are host arrays. */
typedef struct {
    int64_t f;
    int64_t l;
    const int32_t *q;
    int32_t nq;
    const int32_t *s;
    int32_t ns;
    int64_t ep;
    int64_t ed;
    const double *p;
    int32_t np;
} hsd_cone_t;

/* Sparse A in CSR form (row pointers m+1, column indices and values nnz),
 * all device pointers.  Columns need not be sorted within a row. */
typedef struct {
    int32_t m;
    int32_t n;
    int64_t nnz;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
} hsd_csr_t;

/* Settings.  hsd_default_settings fills the defaults listed here. */
typedef struct {
    double eps_pri, eps_dual, eps_gap, eps_unbdd, eps_infeas; /* 1e-4 (Sect. 3.5) */
    double alpha;          /* over-relaxation in (0, 2), default 1.5 (Sect. 3.3)   */
    double cg_zeta_pow;    /* CG tolerance (k+1)^-pow, default 1.5 (Sect. 6.1)     */
    double cg_tight_tol;   /* > 0: CG runs to ||res|| <= cg_tight_tol * ||rhs||
                              every iteration (near-exact projection); default 0 */
    int32_t cg_max_iters;  /* per subspace projection, default 100                */
    int32_t max_iters;     /* ADMM updates, default 10000                         */
    int32_t check_every;   /* termination test cadence, default 1                 */
    int32_t scale;         /* 1 = equilibrate the data (Sect. 5), default 1       */
    int32_t precision;     /* 0 = FP64 everywhere; 1 = FP32 SpMV and CG (matrix
                              values, CG vectors and CG inner products) with FP64
                              tau/kappa, projections, residuals and tests        */
    int32_t team_blocks;   /* workgroups cooperating on one solve; 0 = automatic  */
    int32_t block_threads; /* threads per workgroup (64..512, multiple of 64);
                              0 = automatic (256)                                */
    int32_t lanes_a;       /* lanes per row of A in SpMV (1,2,..,64); 0 = auto    */
    int32_t lanes_at;      /* lanes per row of A^T in SpMV; 0 = auto              */
    int32_t lanes_soc;     /* lanes per second-order cone; 0 = auto               */
    int32_t lds_matrix;    /* 1 = each workgroup copies its rows of A and A^T
                              into LDS once per solve when they fit (else
                              global memory); 0 = always read the matrix from
                              global memory (default); other values: error.
                              Ignored when column slabs are in use.           */
    int32_t slab_cols;     /* block-streamed sweeps with column slabs: each sweep
                              streams the nonzeros in coalesced blocks and
                              visits the columns of A (of A^T) in slabs of this
                              many columns, so that the slab of the gathered
                              vector stays in L2 while the matrix streams (one
                              slab when the width covers all columns).
                              0 = automatic (131072 columns, streamed sweeps
                              when n or m exceeds 262144); -1 = row-group
                              sweeps; > 0 = streamed sweeps with this width.
                              With several slabs for A the rows of the
                              workspace copy of A are sorted by column (a
                              different summation order).  Batched solves:
                              > 0 selects streamed sweeps (one slab).        */
    int32_t batch_vectors; /* batched solves: 1 = each program's iterate
                              vectors (u, v, the CG vectors, z_y, t) live in
                              its workgroup's LDS during its solve when the
                              largest program's fit (default); 0 = global
                              memory.  Ignored by single-program solves.     */
    int32_t linsys;        /* subspace projection (Sect. 4.1): 0 = indirect,
                              CG on I + A^T A (default); 1 = direct: setup
                              forms G = I + A_hat^T A_hat densely, factors it
                              (Cholesky) and inverts it once (factorization
                              caching), and every iteration applies G^{-1}
                              exactly.  Needs precision 0 and n <= 32768
                              (2 * 8 * ceil(n/64)^2 * 64^2 bytes of
                              workspace); single-program solves only.  The
                              automatic team (team_blocks 0) is then one
                              workgroup per CU.                            */
    int32_t batch_matrix;  /* batched solves with the vectors in LDS: 1 = a
                              program's constants (b, c, D, E, g) and then
                              its A and A^T (values, indices, row pointers)
                              are copied into its workgroup's LDS for its
                              solve when they fit in the LDS left beside its
                              vectors (default); 0 = read from global
                              memory.  The arithmetic is the same either
                              way.  Ignored by single-program solves.      */
} hsd_settings_t;

/* Results.  Residuals are those of the original (unscaled) problem
 * (Sect. 3.5 and the scaled forms of Sect. 5); obj is the mean of the
 * primal and dual objectives (Sect. 6.1).  spmv_count counts products with
 * A or A^T of the subspace projections as the paper's Table 5 does: 2 per
 * ADMM iteration plus 2 per CG iteration.  The product A z0 that starts each
 * CG counts even when it is carried from the previous CG instead of being
 * recomputed; products made by termination tests are not counted. */
typedef struct {
    int32_t status;
    int32_t iters;
    double res_pri, res_dual, gap;
    double pobj, dobj, obj;
    double tau, kappa;
    int64_t cg_iters;
    int64_t spmv_count;
    double setup_ms;   /* hsd_setup wall time on the stream (HIP events)      */
    double solve_ms;   /* hsd_solve: start kernels, persistent kernel, outputs */
    double kernel_ms;  /* the persistent solve kernel alone (HIP events)      */
    /* The certificate tests of Sect. 3.5 at the last check, as ratios that
     * pass at <= eps: res_infeas = |E^-1 A_hat^T u_y| |D^-1 b_hat| /
     * (-b_hat^T u_y), res_unbdd = |D^-1 (A_hat u_x + v_s)| |E^-1 c_hat| /
     * (-c_hat^T u_x); +Inf where the denominator is not positive. */
    double res_infeas, res_unbdd;
} hsd_info_t;

typedef struct hsd_work hsd_work_t;
typedef struct hsd_batch hsd_batch_t;

/* Library version string (static storage). */
const char *hsd_version(void);

/* Message describing the last error on the calling thread (static storage,
 * valid until the next call on this thread). */
const char *hsd_last_error(void);

/* Fill *st with the defaults documented in hsd_settings_t. */
void hsd_default_settings(hsd_settings_t *st);

/* Bytes of device workspace that hsd_setup needs for this problem and these
 * settings.  A, K, st: host structs (A's pointers are not read).  Errors:
 * HSD_ERR_ARG, HSD_ERR_CONE. */
int hsd_workspace_bytes(const hsd_csr_t *A, const hsd_cone_t *K,
                        const hsd_settings_t *st, size_t *bytes);

/* Set up a solve: validate the cone (Sect. 2, e-coneprob), copy A, b, c into
 * the workspace, build the transpose of A on the device, equilibrate
 * (Sect. 5), and compute the cached g = M^{-1} h and eta = 1 + h^T g
 * (Sect. 4.1).  A (device arrays), b (device, m), c (device, n); ws is a
 * device buffer of ws_bytes (256-byte aligned) owned by the caller and kept
 * alive until hsd_finish.  The inputs are not modified.  *out receives a
 * handle.  Errors: HSD_ERR_ARG, HSD_ERR_CONE, HSD_ERR_NONFINITE,
 * HSD_ERR_WORKSPACE, HSD_ERR_HIP. */
int hsd_setup(const hsd_csr_t *A, const double *b, const double *c,
              const hsd_cone_t *K, const hsd_settings_t *st,
              void *ws, size_t ws_bytes, void *stream, hsd_work_t **out);

/* Run the method (Sect. 3, e-SCS with over-relaxation and approximate
 * projection) from the current start until a termination test passes
 * (Sect. 3.5) or max_iters updates.  x (device, n), y (device, m),
 * s (device, m) receive the solution, or a normalised certificate
 * (Sect. 2.3): HSD_INFEASIBLE fills y (x and s are NaN), HSD_UNBOUNDED fills
 * x and s (y is NaN).  info (host) receives the results; the stream is
 * synchronised.  The next call starts from the cold start again unless a
 * start was set in between.  Errors: HSD_ERR_STATE, HSD_ERR_HIP,
 * HSD_ERR_ABORTED. */
int hsd_solve(hsd_work_t *w, double *x, double *y, double *s, hsd_info_t *info);

/* Warm start for the next hsd_solve from a previous solution (Sect. 4.2):
 * u0 = (x, y, 1), v0 = (0, s, 0) in scaled variables.  x (device, n),
 * y (device, m), s (device, m), unscaled.  Errors: HSD_ERR_ARG, HSD_ERR_STATE. */
int hsd_warm_start(hsd_work_t *w, const double *x, const double *y, const double *s);

/* Start the next hsd_solve from q = u - v (device, n+m+1, scaled variables):
 * u0 = Pi_C(q), v0 = Pi_{C^*}(-q) (the Moreau pair of q, Sect. 3.2).
 * Errors: HSD_ERR_ARG, HSD_ERR_STATE. */
int hsd_start_from_q(hsd_work_t *w, const double *q);

/* Repeated solves with the same A and c (Sect. 4.2): replace b (device, m)
 * and recompute what depends on it (sigma, b_hat, the norms used by the
 * tests, g = M^{-1} h and eta); the transpose, D, E, rho, A_hat and c_hat
 * are kept.  The next solve starts cold unless a start is set afterwards.
 * Errors: HSD_ERR_STATE, HSD_ERR_ARG, HSD_ERR_NONFINITE, HSD_ERR_HIP. */
int hsd_update_b(hsd_work_t *w, const double *b);

/* Repeated solves with the same A (Sect. 4.2): replace b (device, m) and
 * c (device, n) and recompute what depends on them: sigma and rho (Sect. 5,
 * rho from the mean row norm of A_hat kept from setup), b_hat, c_hat, the
 * norms used by the tests, g = M^{-1} h and eta.  The transpose, D, E and
 * A_hat are kept, so the result equals a fresh setup on (A, b, c).  The
 * next solve starts cold unless a start is set afterwards.  Errors:
 * HSD_ERR_STATE, HSD_ERR_ARG, HSD_ERR_NONFINITE, HSD_ERR_HIP. */
int hsd_update_bc(hsd_work_t *w, const double *b, const double *c);

/* The state where the last hsd_solve or hsd_iterate stopped, in scaled
 * variables (Sect. 5): u and v (device, n+m+1 each: the x, y and tau / the
 * r = 0, s and kappa blocks of Sect. 3), the CG start point z_x of the next
 * subspace projection (device, n: the last CG solution, which warm-starts
 * the next CG, Sect. 4.1), and the iteration number k (host).  By the
 * homogeneity of the embedding (Sect. 3.2) any positive multiple of (u, v)
 * is an equally valid start.  carry (device, 2m, may be NULL) receives the
 * two row products the kernel carries from one update to the next instead
 * of recomputing them: A_hat z_x (first m) and A_hat u_x (last m).  In FP32
 * mode z_x and A_hat z_x are the FP32 values, widened.  Synchronises the
 * stream.  Errors: HSD_ERR_STATE (no run since setup, hsd_update_b or
 * hsd_update_bc), HSD_ERR_HIP. */
int hsd_get_state(hsd_work_t *w, double *u, double *v, double *zx, double *carry, int32_t *k);

/* Start the next hsd_solve or hsd_iterate from a state as returned by
 * hsd_get_state (possibly from another handle set up on the same data and
 * settings): u, v (device, n+m+1), z_x (device, n) and the iteration number
 * k >= 0, which continues the CG tolerance schedule (k+1)^-pow, the
 * termination-test cadence and the iteration limit (max_iters counts from
 * 0, so the run makes max_iters - k more updates; hsd_iterate makes `count`
 * more).  With carry (device, 2m, may be NULL) the first update takes its
 * two carried products from there, and a run resumed on the same launch
 * shape continues bit for bit as the uninterrupted run would; without it
 * they are recomputed, which agrees to rounding.  The arrays are copied
 * before the call returns (stream order).  Errors: HSD_ERR_STATE,
 * HSD_ERR_ARG. */
int hsd_set_state(hsd_work_t *w, const double *u, const double *v, const double *zx,
                  const double *carry, int32_t k);

/* Change the iteration settings of a set-up handle (tolerances, alpha, CG
 * tolerance and limits, max_iters, check_every); scale, precision and the
 * launch-shape fields must equal their setup values.  Errors: HSD_ERR_STATE,
 * HSD_ERR_ARG. */
int hsd_update_settings(hsd_work_t *w, const hsd_settings_t *st);

/* Run exactly `count` updates from the current start (cold unless set) with
 * no termination tests, and copy (u^k, v^k), k = 0..count, into u_hist and
 * v_hist (device, (count+1) x (n+m+1) each, row k = iterate k, scaled
 * variables).  Used to compare iterates with a reference.  Errors:
 * HSD_ERR_ARG, HSD_ERR_STATE, HSD_ERR_HIP, HSD_ERR_ABORTED. */
int hsd_iterate(hsd_work_t *w, int32_t count, double *u_hist, double *v_hist);

/* Scaling computed at setup: D (device, m), E (device, n) and host scalars
 * sigma, rho (Sect. 5).  Any output pointer may be NULL. */
int hsd_get_scaling(hsd_work_t *w, double *D, double *E, double *sigma, double *rho);

/* The launch shape a set-up handle uses (automatic or from the settings),
 * for inspection: team size, threads, lanes, the column slabs of each side
 * (1 = none), whether the matrix slices and the own-row / own-column stages
 * sit in LDS, and whether the general kernels are used: those with the
 * whole-workgroup pass for long rows (a row of A or A^T longer than 128
 * entries per lane of its row group: a dense row or column beside short
 * ones, the imbalance the paper notes for its multi-threaded products,
 * Sect. 6.3 and 6.5) and with PSD projections warm-started from the
 * previous update's eigenvectors (PSD cones of side up to 64).
 * Errors: HSD_ERR_ARG (null), HSD_ERR_STATE. */
typedef struct {
    int32_t team_blocks, block_threads, lanes_a, lanes_at, lanes_soc;
    int32_t slabs_a, slabs_at;      /* column slabs per sweep of A, of A^T   */
    int32_t lds_matrix;             /* 1: matrix slices in LDS (batched: the
                                       programs whose matrices fit beside
                                       their vectors read them from LDS)     */
    int32_t row_stage, col_stage;   /* 1: own-row / own-column stage in LDS   */
    int32_t long_rows;              /* 1: general (long-row, warm-PSD) kernels*/
    int32_t max_row_a, max_row_at;  /* longest row of A and of A^T (entries)  */
    int64_t lds_bytes;              /* dynamic LDS per workgroup of the solve */
    int32_t vectors_lds;            /* batched: 1 = iterate vectors in LDS    */
} hsd_launch_t;
int hsd_get_launch(hsd_work_t *w, hsd_launch_t *out);

/* Release the handle's host metadata (the workspace stays the caller's). */
void hsd_finish(hsd_work_t *w);

/* Projection of in (device, m) onto K (dual = 0) or K^* (dual = 1), written
 * to out (device, m; may equal in).  Zero cone: K = {0}, K^* = R; the
 * exponential cone and its dual swap.  Uses the solver's own projection
 * kernels (Sect. 6.1 cones; Moreau, Sect. 3.2, for the duals).  Allocates a
 * small device table for the cone description and frees it before
 * returning.  Errors: HSD_ERR_ARG, HSD_ERR_CONE, HSD_ERR_HIP. */
int hsd_project_cone(const hsd_cone_t *K, int32_t m, const double *in, double *out,
                     int32_t dual, void *stream);

/* hsd_project_cone for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and the same results, bit for bit, with the
 * cone tables staged in a 1 MiB device array of the library (one per GPU,
 * held until the process ends) instead of a fresh allocation.  The caller
 * still passes in and out (device, m doubles).  Every call on a GPU shares
 * that GPU's array: calls that overlap on one GPU (different host threads
 * or streams) race; calls on one stream are ordered.  Returns once the
 * projection has finished.  Errors: HSD_ERR_ARG (null pointer, or cone
 * tables beyond 1 MiB: 8 bytes per second-order cone, per PSD cone and per
 * power-cone triple), HSD_ERR_CONE, HSD_ERR_HIP. */
int hsd_project_cone_noalloc(const hsd_cone_t *K, int32_t m, const double *in, double *out,
                             int32_t dual, void *stream);

/* ---- batched solves ----------------------------------------------------
 * B independent programs solved in one persistent launch, one workgroup per
 * program at a time (programs taken largest first from a device queue).
 * The programs are given as one block-diagonal CSR matrix: program i owns
 * rows row_off[i]..row_off[i+1]-1 and columns col_off[i]..col_off[i+1]-1
 * (host arrays of B+1 entries); b and c are the concatenated right-hand
 * sides (device).  cones is a host array of B cone descriptions.  Settings
 * are shared; team_blocks, if positive, caps the number of workgroups of
 * the launch (each still solves one program at a time).  Outputs of
 * hsd_batch_solve are concatenated the same way; infos is a host array of
 * B.  Each hsd_batch_solve replays two captured graphs: the per-program
 * preparation (equilibration, g = M^{-1} h), then the solve kernel; in
 * every info, solve_ms covers both plus the outputs and kernel_ms the solve
 * kernel alone.  Errors: as hsd_setup / hsd_solve, plus HSD_ERR_ARG when A
 * is not block diagonal with the given offsets.
 */
int hsd_batch_workspace_bytes(int32_t B, const hsd_csr_t *A, const int64_t *row_off,
                              const int64_t *col_off, const hsd_cone_t *cones,
                              const hsd_settings_t *st, size_t *bytes);
int hsd_batch_setup(int32_t B, const hsd_csr_t *A, const int64_t *row_off,
                    const int64_t *col_off, const double *b, const double *c,
                    const hsd_cone_t *cones, const hsd_settings_t *st,
                    void *ws, size_t ws_bytes, void *stream, hsd_batch_t **out);
int hsd_batch_solve(hsd_batch_t *bt, double *x, double *y, double *s, hsd_info_t *infos);
/* The iterates (u, v) the last hsd_batch_solve ended on, in each program's
 * scaled variables (Sect. 5): program i's u_x, u_y, u_tau occupy entries
 * row_off[i] + col_off[i] + i onwards (n_i + m_i + 1 of them), likewise v.
 * u and v are caller-owned device arrays of row_off[B] + col_off[B] + B
 * doubles.  With q = u - v of a program, hsd_start_from_q on a single-program
 * handle of the same data starts from where that program stopped (a
 * solution or a certificate).  Synchronises the batch's stream.  Errors:
 * HSD_ERR_STATE, HSD_ERR_ARG, HSD_ERR_HIP. */
int hsd_batch_get_state(hsd_batch_t *bt, double *u, double *v);

/* The launch shape of a batched handle (hsd_launch_t; team_blocks is the
 * number of workgroups of the persistent launch, each solving one program
 * at a time; vectors_lds tells whether the iterate vectors live in LDS).
 * Errors: HSD_ERR_ARG (null). */
int hsd_batch_get_launch(hsd_batch_t *bt, hsd_launch_t *out);
void hsd_batch_finish(hsd_batch_t *bt);

/* ---- warm-start network ------------------------------------------------
 * A two-hidden-layer MLP n_in -> h -> h -> n_out with ReLU, FP32, trained
 * with mean-squared error and Adam; it maps a parametric program's
 * parameters to a starting point of the method (a learned variant of the
 * warm start of Sect. 4.2).  Parameters are packed as W1 (h x n_in), b1 (h),
 * W2 (h x h), b2 (h), W3 (n_out x h), b3 (n_out), row-major, each layer
 * y = x W^T + b.  x, t and y are device arrays of batch x n_in / n_out
 * floats, row-major.  The caller owns the workspace (256-byte aligned); the
 * handle owns only host metadata. */
typedef struct hsd_mlp hsd_mlp_t;

/* Workspace bytes for a network of these sizes and batches up to
 * max_batch.  Errors: HSD_ERR_ARG. */
int hsd_mlp_workspace_bytes(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch,
                            size_t *bytes);
/* Create a network in ws (Adam moments zeroed; parameters undefined until
 * hsd_mlp_set_params).  Errors: HSD_ERR_ARG, HSD_ERR_WORKSPACE, HSD_ERR_HIP. */
int hsd_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch, void *ws,
                   size_t ws_bytes, void *stream, hsd_mlp_t **out);
/* Number of packed parameters (-1 for a null handle). */
int64_t hsd_mlp_param_count(const hsd_mlp_t *net);
/* Copy packed parameters in (device; resets Adam) or out (device). */
int hsd_mlp_set_params(hsd_mlp_t *net, const float *params);
int hsd_mlp_get_params(hsd_mlp_t *net, float *params);
/* y = net(x) for 1 <= batch <= max_batch.  Errors: HSD_ERR_ARG, HSD_ERR_HIP. */
int hsd_mlp_forward(hsd_mlp_t *net, int32_t batch, const float *x, float *y);
/* Gradient of L = mean over batch x n_out of (net(x) - t)^2 with respect
 * to the packed parameters, into grads (device, param_count floats, may be
 * NULL); L into *loss (device float, may be NULL). */
int hsd_mlp_gradients(hsd_mlp_t *net, int32_t batch, const float *x, const float *t,
                      float *grads, float *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on L;
 * the loss before the step goes to *loss (device float, may be NULL). */
int hsd_mlp_train_step(hsd_mlp_t *net, int32_t batch, const float *x, const float *t, float lr,
                       float *loss);
void hsd_mlp_destroy(hsd_mlp_t *net);

#ifdef __cplusplus
}
#endif

#endif /* HSD_H */
