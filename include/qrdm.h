/*
 * qrdm.h -- C ABI of libqrdm.so: rank-revealing QR with Deviation
 * Maximization pivoting (QRDM) and with classical column pivoting (QRP) on an
 * AMD Instinct MI355X (gfx950).
 *
 * Method: M. Dessole, F. Marcuzzi, "Deviation Maximization for Rank-Revealing
 * QR Factorizations", arXiv 2106.03138.  QRDM computes A*P = Q*R (Section 3,
 * eq. QRpivoting) by Algorithm 4 (QRDM2): the Deviation Maximization block
 * column choice (Algorithm 1), a Householder panel that stops early when a
 * column is nearly dependent (eq. lenght_check), a compact-WY trailing update
 * and the partial column norm update.  QRP is Algorithm 2 (Section 3.1), the
 * column-at-a-time pivoting that LAPACK xgeqp3 implements.
 *
 * Conventions shared by every entry point:
 *   - Matrices are double precision, column-major, leading dimension lda >= m
 *     (LAPACK layout).  All array pointers are DEVICE pointers unless marked
 *     "host".  The caller allocates and owns every argument array; the library
 *     owns only an internal workspace cached per device (qrdm_release frees it).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *     on it; entry points that return host values (rank, stats) synchronize it.
 *   - Output layout (same as LAPACK xgeqp3): R on and above the diagonal; the
 *     Householder vectors v_i (v_i[i] = 1 implicit) below the diagonal of the
 *     first `rank` columns; tau_house[i] the scalar of H_i = I - tau_i v_i v_i^T
 *     (tau_house[i] = 0 for i >= number of reflectors); perm[j] (0-based) the
 *     original index of the column now at position j, so A_in[:, perm] = Q R.
 *     When the stopping criterion ends the factorization at rank r < min(m,n),
 *     rows/columns >= r hold the updated trailing block R22 (not triangular),
 *     so A_in[:, perm] = Q [R11 R12; 0 R22] exactly.
 *   - Return codes: 0 = success; -i = the i-th argument is invalid (checked
 *     before any launch; nothing is written); QRDM_ERR_* > 0 otherwise.  A
 *     failure the kernels detect themselves (a bounded grid-wide wait that
 *     timed out, a launch grid smaller than a kernel's partition) returns
 *     QRDM_ERR_HIP + hipErrorLaunchTimeOut; A then holds partial results.
 *   - Workspace: the entry points without a workspace argument use one device
 *     workspace that the library caches per device; concurrent calls to them
 *     are serialized by a lock inside the library.  qrdm_factor_ws takes the
 *     caller's workspace instead: calls with distinct workspaces (and
 *     matrices) may run concurrently from several host threads on several
 *     streams.  The Householder panel and the column-pivoting block kernel
 *     synchronize their workgroups through memory and need them all resident
 *     at once (at most one workgroup per compute unit each); concurrent calls
 *     whose such kernels could together exceed the device should set
 *     QRDM_COOPERATIVE=1 in the environment (cooperative launches, whose
 *     co-residency the runtime guarantees).  Their waits are bounded: a wait
 *     that times out fails the call with hipErrorLaunchTimeOut, never hangs.
 */
#ifndef QRDM_H
#define QRDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QRDM_OK 0
#define QRDM_ERR_NONFINITE 1   /* NaN/Inf in A (or a column norm overflows); A unchanged */
#define QRDM_ERR_NOMEM 2       /* workspace allocation failed; nothing written            */
#define QRDM_ERR_UNSUPPORTED 3 /* size outside what the kernels support (see below)      */
#define QRDM_ERR_INTERNAL 4    /* the host loop ran past its bound on the number of steps
                                  (each step takes at least one column; a library fault)    */
#define QRDM_ERR_WORKSPACE 5   /* ws_bytes < qrdm_workspace_size(m, n, p); nothing written  */
#define QRDM_ERR_SCRATCH 6     /* qrdm_factor_noalloc: qrdm_workspace_size(m, n, p) exceeds
                                  QRDM_NOALLOC_WS_MAX; nothing written                      */
#define QRDM_ERR_HIP 1000      /* QRDM_ERR_HIP + hipError_t of a failed runtime call      */

/* Stopping criterion, Section 3.4, eq. (practical stopping criterion). */
#define QRDM_STOP_PAPER 0   /* stop when sqrt(n-n_s) max_i||c_i|| <= eps_1 max_i||a_i||     */
#define QRDM_STOP_MAXNORM 1 /* stop when max_i||c_i|| <= eps_1 max_i||a_i||                 */
#define QRDM_STOP_NONE 2    /* full factorization; rank = where the PAPER test first held  */

#define QRDM_PREC_FP64 0  /* everything in FP64; trailing update on FP64 MFMA             */
#define QRDM_PREC_MIXED 1 /* trailing update on FP32 MFMA with FP32 accumulation; panel,
                             norms, recompute and the rank decision stay FP64              */

#define QRDM_KMAX_LIMIT 128 /* largest supported block size k_DM                          */

typedef struct {
    double tau;         /* candidate threshold, Algorithm 1; 0 <= tau <= 1 (default 0.15);
                           tau = 0 admits every column and disables the panel break    */
    double delta;       /* cosine bound, Algorithm 1; 0 <= delta <= 1 (default 0.9)      */
    int32_t kmax;       /* block size k_DM, eq. (candidate_set_limited_by_kDM); 1..128 (64) */
    int32_t stop_rule;  /* QRDM_STOP_* (default QRDM_STOP_PAPER)                          */
    double eps1_scale;  /* eps_1 = eps1_scale * eps_w; <= 0 selects n (eq. choice1), where
                           eps_w is the unit roundoff of the trailing data: 2^-52 in FP64
                           mode, 2^-23 in mixed mode (its updates round to FP32, so the
                           trailing block carries noise of about 2^-23 ||A||); the
                           recompute tolerance of the norm downdate is sqrt(eps_w).  The
                           switch to scalar pivoting, eq. (column_norm_bound_DM), is
                           max partial norm <= n 2^-52 max ||a_j|| in both modes         */
    int32_t precision;  /* QRDM_PREC_* (default FP64)                                     */
    int32_t poll_lag;   /* host polls the device loop state this many blocks behind
                           (0 = synchronize every block; default 4; at most 1024).  The
                           factorization is the same to the bit for every value          */
    int32_t profile;    /* 1 = time the trailing GEMMs with HIP events on `stream`
                           (results in qrdm_stats; adds event overhead); default 0        */
    int32_t certified;  /* 1 = certified DM: per block, delta is lowered to
                           tau^2 / (|L| - 1) (eq. delta_max, |L| the candidate count), so
                           every block meets the hypotheses of Lemma 1; default 0         */
} qrdm_params;

typedef struct {
    int64_t nblocks;     /* outer steps executed                                          */
    int64_t nbreaks;     /* blocks whose panel stopped early (l < k_s)                    */
    int64_t nfallback;   /* columns factored by scalar pivoting after the switch of eq.
                            (column_norm_bound_DM)                                         */
    int64_t nrecompute;  /* partial norms recomputed from the data                        */
    int64_t ncols_factored; /* number of reflectors applied                               */
    /* filled when params.profile = 1 (zero otherwise):                                    */
    double gemm1_ms;     /* summed event time of the V^T A GEMM launches (k_gemm1 alone)    */
    double gemm2_ms;     /* summed event time of the A -= V Z GEMM launches                */
    double gemm_flop;    /* algorithmic flops of ONE of the two GEMMs, summed over blocks:
                            sum 2 t l w (t rows, l reflectors, w trailing columns)         */
    double total_ms;     /* event time of the whole factorization loop                    */
    double dm_ms;        /* DM selection per block: select, Gram, greedy, swaps            */
    double panel_ms;     /* Householder panels with break                                  */
    double downdate_ms;  /* partial-norm downdates and recomputes after each block         */
    double qp3_ms;       /* the scalar-pivoting continuation (column pivoting steps)       */
    double panel_flop;   /* algorithmic flops of the panels: per reflector i of a block,
                            (t-i)(2 + 4(k_s-1-i))                                          */
    double panel_bytes;  /* algorithmic bytes of the panels: 16 t k_s per block            */
    int64_t npanel;      /* panel launches that factored a block (always filled)            */
    /* the column-pivoting loop (QRP; QRDM's scalar-pivoting tail), profile = 1:           */
    double qp3_run_ms;   /* summed event time of its block-kernel launches                 */
    double qp3_bytes;    /* algorithmic bytes: 8 (m-j)(n-j) per pivot step j (the trailing
                            matrix read once by the step's matrix-vector product)          */
    int64_t nqp3_launch; /* block-kernel launches (0 when the per-step kernels ran)        */
    int64_t qp3_start;   /* first column of the column-pivoting loop: the column where the
                            switch of eq. (column_norm_bound_DM) held (QRDM), 0 for QRP,
                            -1 when the factorization never switched (always filled)       */
    int64_t ngram;       /* panels formed from the Gram matrix of the block (CholeskyQR2 and
                            Householder reconstruction) rather than column by column
                            (always filled)                                                  */
    int64_t nqp3_tail;   /* of the nqp3_launch launches, those of the register-resident tail
                            kernel, which takes every step left once the trailing block has
                            at most 2048 rows and 8 columns per compute unit (0 or 1;
                            profile = 1)                                                     */
    double zsum_ms;      /* summed event time of the partial sums of V^T A and Z = T^T Y
                            (k_zsum, between the two GEMMs; profile = 1)                    */
    double gemm2_bytes;  /* algorithmic bytes of the A -= V Z GEMM, summed over blocks:
                            sum 16 t w (A read and written once; profile = 1)               */
} qrdm_stats;

/* One record per outer step of the DM loop, for tests and tracing.  When the
 * partial norms reach the noise level (eq. column_norm_bound_DM) the loop
 * hands the remaining columns to the column-pivoting kernels: that is the last
 * record, with fallback = 1, ns = the first column pivoted singly, and
 * nL = ks = l = 0. */
typedef struct {
    int64_t ns;       /* columns factored before this step */
    int32_t nL;       /* candidate list length             */
    int32_t ks;       /* accepted columns                  */
    int32_t l;        /* reflectors kept after the break   */
    int32_t fallback; /* 1 = the hand-over record (above)  */
    double umax;      /* max partial norm at selection (the estimate the
                         selection compared, after the downdates)       */
    /* Lemma 1 on C = the k_s accepted columns [A]_{ns:m, J} at this step, from
     * their Gram matrix: gamma = min_i (1 - sum_{j != i} |theta_ij|) and
     * sigma_bound = sqrt(gamma + tau_J^2 - 1) max_J ||c_j|| with
     * tau_J = min_J ||c_j|| / max_J ||c_j|| (0 when gamma <= 1 - tau_J^2: the
     * lemma does not apply).  sigma_min(C) >= sigma_bound; with certified = 1 the
     * bound is positive.  A one-column step records gamma = 1, sigma_bound = ||c||. */
    double gamma;
    double sigma_bound;
} qrdm_block;

/* Fills *p with the paper's defaults: tau = 0.15, delta = 0.9 (Section 5) and
 * k_DM = 64 (Section 5, block size study); stop rule PAPER, eps_1 = eps*n. */
void qrdm_default_params(qrdm_params *p);

/*
 * QRDM, Algorithm 4 (QRDM2) with Algorithm 1 (DM), FP64, stop rule PAPER.
 *   A          [in/out] m x n, lda >= max(1,m); overwritten by R and the reflectors.
 *   tau_house  [out] min(m,n) doubles.
 *   perm       [out] n int32.
 *   rank       [out, host] numerical rank from eq. (practical stopping criterion).
 * Supported sizes: m, n <= 32768 columns for the selection; m <= 65536.
 */
int qrdm_factor(double *A, int64_t m, int64_t n, int64_t lda, double tau, double delta,
                int32_t kmax, double *tau_house, int32_t *perm, int64_t *rank, void *stream);

/*
 * QRDM with all parameters.  stats (host, may be NULL) receives counters.
 * log (host, may be NULL) receives up to log_cap block records and *nlog the
 * number of blocks; passing a log forces poll_lag = 0.
 */
int qrdm_factor_ex(double *A, int64_t m, int64_t n, int64_t lda, const qrdm_params *p,
                   double *tau_house, int32_t *perm, int64_t *rank, qrdm_stats *stats,
                   qrdm_block *log, int64_t log_cap, int64_t *nlog, void *stream);

/*
 * Bytes of device workspace that qrdm_factor_ws needs for an m x n matrix with
 * parameters *p (NULL = defaults; only p->kmax matters).  0 for m < 0 or n < 0.
 */
size_t qrdm_workspace_size(int64_t m, int64_t n, const qrdm_params *p);

/*
 * QRDM (Algorithm 4 with Algorithm 1; Section 3, A P = Q R) in a workspace the
 * caller owns, with the rank written to device memory.
 *   A, lda, p, tau_house, perm  as in qrdm_factor_ex (p->profile must be 0).
 *   rank_dev   [out, DEVICE] one int64: the rank of eq. (practical stopping
 *              criterion) (Section 5 uses it as the numerical rank), written in
 *              stream order after the last kernel of the factorization; -1 if
 *              the call fails on the device.
 *   stats      [out, host, may be NULL] counters; asking for them synchronizes
 *              the stream.
 *   workspace  [DEVICE] at least qrdm_workspace_size(m, n, p) bytes, 256-byte
 *              aligned; its contents on entry do not matter, and it must not be
 *              used by any other work until the stream has passed this call.
 * The call launches the factorization on `stream` and returns once the device
 * has reported the end of the loop (the host waits on events of its own,
 * never on the whole stream); it allocates no device memory and takes no lock
 * shared with other calls, so calls with distinct workspaces run concurrently
 * (see the conventions above for the kernels that need co-residency).
 * Returns as qrdm_factor_ex; QRDM_ERR_WORKSPACE if ws_bytes is too small, -10
 * for a NULL or misaligned workspace.
 */
int qrdm_factor_ws(double *A, int64_t m, int64_t n, int64_t lda, const qrdm_params *p, double *tau_house,
                   int32_t *perm, int64_t *rank_dev, qrdm_stats *stats, void *workspace, size_t ws_bytes,
                   void *stream);

/*
 * For callers that cannot allocate memory (tight serving loops, harnesses that
 * forbid hipMalloc): qrdm_factor_ws without a workspace argument.  The
 * workspace is a fixed array in device memory that the library holds on each
 * device it runs on (QRDM_NOALLOC_WS_MAX bytes plus a 256-byte polling slot,
 * kept until the process ends); the call itself allocates nothing, neither
 * device memory nor pinned host memory nor events.
 *   A, lda, p, tau_house, perm, rank_dev  as in qrdm_factor_ws (p->profile must
 *              be 0; p->poll_lag is ignored: the host reads the loop state
 *              after every step, which gives the same factorization to the bit).
 * Shapes whose qrdm_workspace_size(m, n, p) exceeds QRDM_NOALLOC_WS_MAX are
 * rejected with QRDM_ERR_SCRATCH before any launch (8192 x 8192 with
 * k_DM <= 64 fits).  The array keeps the contents of the last call; every call
 * clears what it needs.  All calls on one device share its array: calls that
 * overlap on one device (from several host threads or streams) race and give
 * wrong results; serialize them.  Returns as qrdm_factor_ws.
 */
#define QRDM_NOALLOC_WS_MAX ((size_t)96 << 20)
int qrdm_factor_noalloc(double *A, int64_t m, int64_t n, int64_t lda, const qrdm_params *p, double *tau_house,
                        int32_t *perm, int64_t *rank_dev, void *stream);

/*
 * QRP, Algorithm 2 (Section 3.1), blocked like LAPACK xgeqp3: one pivot per
 * step with the partial norm update; the trailing matrix is updated every
 * `nb` columns with a BLAS-3 product.  Same outputs and rank rule as
 * qrdm_factor (stop_rule from p, may be NULL for PAPER).
 */
int qrp_factor(double *A, int64_t m, int64_t n, int64_t lda, double *tau_house, int32_t *perm,
               int64_t *rank, void *stream);
int qrp_factor_ex(double *A, int64_t m, int64_t n, int64_t lda, const qrdm_params *p, int32_t nb,
                  double *tau_house, int32_t *perm, int64_t *rank, qrdm_stats *stats, void *stream);

/*
 * Column 2-norms of A (device out[n]), the first step of Algorithm 4.
 * Returns QRDM_ERR_NONFINITE if any column holds NaN/Inf.
 */
int qrdm_colnorms(const double *A, int64_t m, int64_t n, int64_t lda, double *out, void *stream);

/*
 * One Deviation Maximization step (Algorithm 1) on the trailing block
 * [A]_{ns:m, ns:n} given its partial norms vn1 (device, n entries, entries
 * >= ns are read), exactly as the factorization performs it.  Host outputs:
 * L[kmax] candidate list (norm desc, position asc), *nL, theta[kmax*kmax]
 * (row-major nL x nL cosine matrix, may be NULL), J[kmax] accepted columns,
 * *ks.  A is not modified.
 */
int qrdm_dm_step(const double *A, int64_t m, int64_t n, int64_t lda, int64_t ns, const double *vn1,
                 double tau, double delta, int32_t kmax, int32_t *L, int32_t *nL, double *theta,
                 int32_t *J, int32_t *ks, void *stream);

/*
 * Least squares on top of a factorization: the basic solution of
 * min_x ||A_in x - b|| (Section 1: column pivoting singles out the solution
 * with `rank` nonzeros).  With r = min(rank, min(m,n)), y = Q_r^T b where
 * Q_r = H_0 ... H_{r-1} (the first r reflectors), R11 x1 = y[0:r) (R11 the
 * leading r x r block of R), x[perm[j]] = x1[j] for j < r and 0 for j >= r.
 *   A, tau_house, perm  [in] the output of qrdm_factor* / qrp_factor* (A and
 *              lda as passed to it); perm must be a permutation of 0..n-1
 *              (entries outside [0, n) are skipped).
 *   rank       [in, host] the rank to solve with (normally the factorization's);
 *              rank < 0: X and resid are set to NaN, B is unchanged.
 *   B          [in/out] m x nrhs, ldb >= max(1,m): on return rows [0, r) hold x1
 *              (the solution in pivoted order) and rows [r, m) hold y[r:m)
 *              (as LAPACK xgels leaves them).
 *   X          [out] n x nrhs, ldx >= max(1,n): the basic solution.
 *   resid      [out] nrhs doubles or NULL: ||y[r:m)|| = ||A_in x - b|| per column
 *              (exact in exact arithmetic, since x vanishes on the columns of R12, R22).
 * If some r_ii = 0 with i < r the solution holds Inf/NaN (no test is made).
 * One workgroup per 4 right-hand sides; nothing is synchronized.
 */
int qrdm_lstsq(const double *A, int64_t m, int64_t n, int64_t lda, const double *tau_house, const int32_t *perm,
               int64_t rank, double *B, int64_t ldb, int64_t nrhs, double *X, int64_t ldx, double *resid,
               void *stream);

/*
 * Post-hoc rank truncation (Section 5: where the stopping criterion
 * overestimates the numerical rank, the diagonal of R still shows the gap of
 * the singular values, and R can be truncated afterwards).  With
 * eps_1 = eps1_scale * 2^-52 (eps1_scale <= 0 selects n, the choice of eq.
 * (practical stopping criterion_choice1)), *rank_out = the first i < r with
 * |r_ii| <= eps_1 |r_00| (a NaN entry counts as small), or r if there is none,
 * where r = min(rank, m, n); rank <= 0 is passed through.  The result is a
 * prefix, so R11 stays the leading block that qrdm_lstsq solves with.
 *   A          [in] the output of a factorization (only the diagonal is read).
 *   rank_out   [out] one int64 in DEVICE memory (not synchronized).
 */
int qrdm_truncate_rank(const double *A, int64_t m, int64_t n, int64_t lda, int64_t rank, double eps1_scale,
                       int64_t *rank_out, void *stream);

/* Frees the workspace cached for the current device. */
void qrdm_release(void);

/* Text for a return code (static storage). */
const char *qrdm_strerror(int code);

/* ------------------------------------------------------------------------
 * Batched QRDM: many independent small matrices, each factored exactly as
 * qrdm_factor does (Algorithm 4 with Algorithm 1, FP64), by persistent
 * kernels that hold one matrix per workgroup and take matrices from an atomic
 * queue, longest first.  Matrices are grouped in size classes by m; each class
 * runs its own launch variant (the autotuner's choice per class).
 *
 * Limits: 0 <= n <= QRDM_BATCH_NMAX, any m >= 0, lda >= max(1, m), and
 * k_DM <= QRDM_BATCH_KMAX (larger per-matrix values are clamped to it).
 * ------------------------------------------------------------------------ */
#define QRDM_BATCH_NMAX 512
#define QRDM_BATCH_KMAX 64
#define QRDM_BATCH_CLASSES 4 /* size classes: m <= 64, <= 128, <= 256, > 256 */

/* Per-matrix method parameters (device array, optional): tau, delta and k_DM
 * as in qrdm_params; used by the learned parameter predictor.  k_DM = 0 leaves
 * the matrix as it is (A, tau_house, perm, rank, status and info untouched), so
 * that some matrices of a plan can be factored again without a new plan. */
typedef struct {
    double tau;
    double delta;
    int32_t kmax;
    int32_t pad;
} qrdm_batch_params;

/* Launch choice of one size class.  variant (256-thread workgroups): 0 = 16
 * columns per wavefront in the trailing update, panel rows held in registers;
 * 1 = the same with 32 columns; 2 = 16 columns, panel read from memory each
 * step.  Every variant computes the same factorization (variant 2 sums in
 * another order).  wgs_per_cu = workgroups per compute unit (0 = the
 * occupancy limit). */
typedef struct {
    int32_t variant;
    int32_t wgs_per_cu;
} qrdm_batch_tune;

typedef struct qrdm_batch_plan qrdm_batch_plan;

/* Plans a batch of `batch` matrices with HOST arrays m[batch], n[batch],
 * lda[batch] and default parameters *p (tau, delta, kmax, stop_rule,
 * eps1_scale, certified; precision must be FP64).  The batched path keeps
 * no per-step log: in certified mode every block meets Lemma 1 by
 * construction, and the bound itself is reported by qrdm_factor_ex only.  tune[QRDM_BATCH_CLASSES] (host, may be
 * NULL = built-in defaults).  Allocates the plan's device arrays (sizes, order,
 * queue counters) on the current device.  Returns 0, -i for an invalid
 * argument, QRDM_ERR_UNSUPPORTED if some n exceeds QRDM_BATCH_NMAX or
 * p->kmax exceeds QRDM_BATCH_KMAX, or QRDM_ERR_HIP + error. */
int qrdm_batch_plan_create(const int32_t *m, const int32_t *n, const int32_t *lda, int32_t batch,
                           const qrdm_params *p, const qrdm_batch_tune *tune, qrdm_batch_plan **plan);

/* Factors every matrix of the plan in place.  A, tau_house, perm: DEVICE arrays
 * of `batch` device pointers (matrix i is m[i] x n[i] with lda[i]; tau_house[i]
 * holds min(m,n) entries, perm[i] n entries; same output layout as
 * qrdm_factor).  rank, status: DEVICE arrays of `batch` entries; status 0 = ok,
 * 1 = NaN/Inf in the matrix (nothing written, rank -1).  pm: DEVICE array of
 * per-matrix parameters or NULL.  info: DEVICE array of 4 * batch entries or
 * NULL; per matrix: outer steps, steps whose panel stopped early (the length
 * check of eq. lenght_check), scalar-pivoting steps, and GPU wall-clock ticks
 * (100 MHz) the workgroup spent on it.  use_graph = 1 captures the launches in a
 * hipGraph on the first call with these arguments (captured on a stream of
 * the plan's own) and replays it on `stream` afterwards (the pointer arrays'
 * contents may change between calls; new array addresses get a new capture,
 * which happens automatically).
 * Work is enqueued on `stream`; nothing is synchronized.  Calls with one plan
 * must not overlap. */
int qrdm_batch_factor(qrdm_batch_plan *plan, double *const *A, double *const *tau_house, int32_t *const *perm,
                      int64_t *rank, int32_t *status, const qrdm_batch_params *pm, int64_t *info,
                      int32_t use_graph, void *stream);

/* qrdm_batch_factor with per-matrix parameters pm (required) and the online
 * check of qrdm_batch_check (Section 5's factor-10 rule, band = 0.1) taken in
 * the same launch: a matrix whose factorization fails the check is restored
 * from its pristine copy and factored again with the plan's parameters by the
 * workgroup that factored it, while the other workgroups keep working.
 * pristine: DEVICE array of `batch` device pointers, matrix i an unmodified
 * copy of A[i] with the same leading dimension (read only).  ok: DEVICE array
 * of `batch` int32: 1 = factored with pm[i] and kept, 0 = factored again with
 * the plan's parameters.  Other arguments and the stream as in
 * qrdm_batch_factor (no graph capture).  Returns -2 for a missing array, -9
 * for band < 0 or NaN. */
int qrdm_batch_factor_checked(qrdm_batch_plan *plan, double *const *A, double *const *tau_house,
                              int32_t *const *perm, int64_t *rank, int32_t *status, const qrdm_batch_params *pm,
                              const double *const *pristine, double band, int32_t *ok, int64_t *info,
                              void *stream);

/* Frees the plan, its device arrays and graphs (synchronizes the device). */
void qrdm_batch_plan_destroy(qrdm_batch_plan *plan);

/* Least squares for every matrix of the plan after qrdm_batch_factor: per
 * matrix i exactly what qrdm_lstsq computes, with rank[i] (DEVICE array, the
 * factorization's output; < 0 gives NaN solutions).  A, tau_house, perm as
 * passed to qrdm_batch_factor; B, X: DEVICE arrays of `batch` device pointers,
 * B[i] m[i] x nrhs with leading dimension max(1, m[i]) (in/out as in
 * qrdm_lstsq), X[i] n[i] x nrhs with leading dimension max(1, n[i]).
 * resid: DEVICE array of batch * nrhs doubles (matrix i at i * nrhs) or NULL.
 * One workgroup per matrix and 4 right-hand sides; nothing is synchronized. */
int qrdm_batch_lstsq(qrdm_batch_plan *plan, double *const *A, double *const *tau_house, int32_t *const *perm,
                     const int64_t *rank, double *const *B, double *const *X, int32_t nrhs, double *resid,
                     void *stream);

/* qrdm_truncate_rank for every matrix of the plan: rank_in, rank_out DEVICE
 * arrays of `batch` entries (they may be the same array). */
int qrdm_batch_truncate_rank(qrdm_batch_plan *plan, double *const *A, const int64_t *rank_in, double eps1_scale,
                             int64_t *rank_out, void *stream);

/* ------------------------------------------------------------------------
 * Learned (tau, delta, k_DM) per matrix.  The paper chooses the parameters by
 * a grid study and checks quality with the factor-10 rule on d_i / sigma_i
 * (Section 5); here a multilayer perceptron 16 -> 64 -> 64 -> 3 (tanh, tanh,
 * linear; FP32; 5443 parameters in the order W1[64][16], b1, W2[64][64], b2,
 * W3[3][64], b3) maps per-matrix features to the grid
 * tau in {0.05, 0.15, 0.3, 0.5, 0.7, 0.9}, delta in {0.5, 0.7, 0.9, 0.95},
 * k_DM in {32, 64}, and an incremental condition estimate of R11 decides
 * whether each prediction is kept.  All arrays are DEVICE arrays; work is
 * enqueued on `stream` and nothing is synchronized.
 * ------------------------------------------------------------------------ */
#define QRDM_NFEAT 16
#define QRDM_MLP_HIDDEN 64
#define QRDM_MLP_OUT 3
#define QRDM_MLP_NPARAM 5443
#define QRDM_MLP_NDELTA 131 /* per-sample work of the gradient: 3 + 2 * 64 */

/* features[16 * batch] (FP64) of the plan's matrices: [0..9) the order
 * statistics floor(q (n-1)), q = 0.1..0.9, of log10(||a_j|| / max ||a_j||)
 * (floored at -30); [9] log2 m; [10] log2 n; [11] n / m; over the columns
 * floor(k n / s), k < s = min(64, n), with theta_ij = G_ij / sqrt(G_ii G_jj)
 * (Algorithm 1's cosine; 0 if a column is zero): [12] mean |theta_ij|,
 * [13] the order statistic floor(0.95 (P-1)) of the P = s(s-1)/2 values,
 * [14] max, [15] fraction above 0.5.  A matrix that is empty or zero keeps
 * zeros except [9..12). */
int qrdm_batch_features(qrdm_batch_plan *plan, double *const *A, double *features, void *stream);

/* Forward pass for `batch` samples: x = (features - norm[0..16)) * norm[16..32)
 * (norm may be NULL: x = features); h1, h2 [batch * 64] (may be NULL when
 * only y is wanted), y [batch * 3]. */
int qrdm_mlp_forward(const float *params, const float *norm, const double *features, int32_t batch, float *h1,
                     float *h2, float *y, void *stream);

/* Gradient of L = 1/(2 batch) sum_b sum_o (y_bo - target_bo)^2 with respect
 * to params, after qrdm_mlp_forward filled h1, h2, y: grad[5443];
 * work[131 * batch] scratch; sqerr[batch] (may be NULL) the per-sample
 * squared errors.  Each gradient entry is a fixed-order sum over samples. */
int qrdm_mlp_gradient(const float *params, const float *norm, const double *features, const float *h1,
                      const float *h2, const float *y, const float *target, int32_t batch, float *work, float *grad,
                      float *sqerr, void *stream);

/* Adam step t >= 1 (Kingma & Ba) on params with moments m, v (5443 each). */
int qrdm_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t t, float lr, float beta1,
                  float beta2, float eps, void *stream);

/* MLP outputs y[3 * batch] -> per-matrix parameters: tau and delta are the
 * nearest grid values to y0 and y1, k_DM = 64 if y2 >= 0.5 else 32. */
int qrdm_mlp_to_params(const float *y, int32_t batch, qrdm_batch_params *out, void *stream);

/* Online quality check after a factorization of the plan's matrices: with
 * r = rank[i], an incremental condition estimate (Bischof) est of
 * sigma_min(R11) (R11 = leading r x r of R); ok[i] = 1 iff
 * est >= band * min_{j<r} |r_jj| (band = 0.1 for the factor-10 rule).
 * est may be NULL. */
int qrdm_batch_check(qrdm_batch_plan *plan, double *const *A, const int64_t *rank, double band, double *est,
                     int32_t *ok, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* QRDM_H */
