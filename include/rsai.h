/*
 * rsai.h -- C ABI of the MI355X (gfx950) implementation of RSAI(tol), the residual
 * based sparse approximate inverse of Jia & Kang (arXiv:1503.04500).
 *
 * What it computes. For a real nonsingular n x n sparse matrix A (Section 1, eq. (1.1))
 * the library builds M = (m_1, ..., m_n) column by column (eqs. (2.1)-(2.2)): each
 * m_k minimises ||A m_k - e_k||_2 over an adaptively grown pattern J_k, solved as the
 * reduced LS problem (2.3) on the rows I_k = nonzero rows of A(:, J_k). The pattern
 * grows by Algorithm 1 (Section 3): start from J_k = {k}; while ||r_k|| > eps and
 * fewer than lmax loops were done, take the c largest |r_k(i)| among the rows not used
 * before (ties: smaller row index), add the columns of those rows of A that are not
 * yet in J_k, and re-solve. After every solve, entries with |m_jk| <= tol (fixed
 * tolerance) or <= eps / (nnz(m_k) ||A||_1) (adaptive tolerance, eq. (4.3)) leave
 * J_k and the LS problem is solved again on the kept pattern (Section 4). The
 * result is used as a right preconditioner, A M y = b, x = M y (eq. (1.2)).
 *
 * Conventions.
 *   - Every pointer named in a function is a DEVICE pointer unless stated otherwise.
 *   - CSC: int64 colptr[n+1] (colptr[0] = 0, non-decreasing), int32 rowidx[nnz]
 *     (strictly ascending inside each column, in [0, n)), float64 val[nnz]. Every
 *     column must hold at least one entry. Explicitly stored zeros are structural
 *     nonzeros.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream). All device
 *     work is ordered on that stream; only the functions marked "synchronises" wait
 *     for it.
 *   - Errors: every function returns an rsai_status (negative on failure) and never
 *     throws; rsai_last_error() gives a thread-local message. On failure no output
 *     handle is created and nothing leaks.
 *   - A is borrowed: it must stay alive and unchanged until rsai_destroy when
 *     rsai_backward will be called (the adjoint re-reads A).
 */
#ifndef RSAI_H
#define RSAI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RSAI_OK = 0,
    RSAI_E_ARG = -1,      /* bad argument or parameter */
    RSAI_E_CSC = -2,      /* malformed CSC input */
    RSAI_E_SINGULAR = -3, /* a column's LS problem (2.3) is rank deficient */
    RSAI_E_NOMEM = -4,    /* allocation failed */
    RSAI_E_HIP = -5,      /* HIP runtime error */
    RSAI_E_CAP = -6,      /* a column outgrew the largest LS size the build supports, or
                             the spill queues (rsai_params.spill_capacity) were full */
    RSAI_E_STATE = -7     /* call not valid in the plan's state */
} rsai_status;

/* Borrowed view of one square CSC matrix (device pointers). */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int64_t *colptr;
    const int32_t *rowidx;
    const double *val;
} rsai_csc;

typedef enum {
    RSAI_DROP_NONE = 0,     /* basic RSAI, Algorithm 1 */
    RSAI_DROP_FIXED = 1,    /* drop |m_jk| <= tol */
    RSAI_DROP_ADAPTIVE = 2  /* drop |m_jk| <= eps / (nnz(m_k) ||A||_1), eq. (4.3) */
} rsai_drop_mode;

typedef enum {
    RSAI_SCHED_BATCHED = 0, /* size-bucketed persistent kernels, whole loop fused; columns
                               that outgrow the register tiers finish in a large class (one
                               256-thread workgroup per column, |I_k| <= 8192, |J_k| <= 128) */
    RSAI_SCHED_PLAIN = 1    /* one register class (16 lanes per column), one launch per
                               loop, state in HBM; columns that outgrow the class finish in
                               the same workgroup classes as in the batched schedule */
} rsai_sched;

/* One entry of a tuning table (rsai_params.tune_table): for a matrix with n in
   [n_lo, n_hi), mean column length nnz/n in [len_lo, len_hi) and longest column in
   [maxlen_lo, maxlen_hi), built with eps in [eps_lo, eps_hi), the schedule choices
   below (as timed by rsai_autotune; the first matching entry wins; -1 leaves a field
   to the default). */
typedef struct {
    double len_lo, len_hi;
    double eps_lo, eps_hi;   /* the build's eps in [eps_lo, eps_hi) */
    int64_t maxlen_lo, maxlen_hi;
    int64_t n_lo, n_hi;
    int32_t tier0, refill, route, t0_hash, last_tier, reserved;
} rsai_tune_entry;

typedef struct {
    int32_t c;        /* dominant rows taken per loop (Algorithm 1, step 4), 1..8 */
    int32_t lmax;     /* maximum number of loops, 0..64 */
    double eps;       /* stop when ||A m_k - e_k||_2 <= eps */
    int32_t drop;     /* rsai_drop_mode */
    double tol;       /* fixed drop tolerance (RSAI_DROP_FIXED) */
    int32_t sched;    /* rsai_sched */
    int32_t validate; /* CSC contract check: 0 none (input trusted), 1 checked with one
                         host wait, after the build's kernels are queued (RSAI_E_CSC from
                         rsai_build; the queued kernels do nothing on a malformed input),
                         2 checked on the device without synchronising (the build's kernels
                         then do nothing and rsai_plan_nnz reports RSAI_E_CSC) */
    int32_t tier0;    /* first size tier for the batched schedule: -1 default (0), else a
                         register tier index (rsai_tier_info) */
    int32_t timing;   /* 1: record per-kernel HIP event times (rsai_plan_timing) */
    int32_t refill;   /* first tier: -1 default (1), 0 a finished column's lanes take the next
                         column at once, 1 the lanes of a wave take new columns together */
    int32_t route;    /* spilled columns: -1 default (1), 0 to the next size class, 1 to the
                         first class that holds their estimated |I_k|, |J_k| */
    int32_t keep_factors;        /* 1: keep the R factor of every column's final solve for
                                    rsai_backward (R^T R = A(I,J)^T A(I,J)) */
    int64_t factor_budget_bytes; /* size of the factor store (0: 2 GB); columns that do not
                                    fit get their factor recomputed by rsai_backward */
    int32_t deterministic;       /* 1: rsai_backward adds every entry's contributions in a
                                    fixed order (sorted by column), so dA is bitwise
                                    repeatable; 0: FP64 atomics (faster) */
    int32_t tune_count;          /* entries of tune_table (0: none) */
    const rsai_tune_entry *tune_table; /* host array, read during rsai_build*: the schedule
                                    fields left at -1 (tier0, refill, route, t0_hash,
                                    last_tier) take the first entry matching the matrix
                                    and eps (for a batch: the smallest tier0, the largest
                                    route and last_tier, refill and t0_hash of the
                                    largest matrix's entry); no match keeps the
                                    defaults */
    int32_t t0_hash;  /* hash tables of the first register tier: -1 default (2), 2 or 4 times
                         its row and column capacity (a tile choice; results unchanged) */
    int32_t last_tier; /* last register tier: -1 default (2), 1 sends the columns that
                          outgrow tier 1 straight to the sparse-block class (a class edge;
                          results agree to rounding) */
    const int64_t *col_len_max; /* host array, one per matrix: its longest column, for the
                          tuning table (NULL: read on the device, one host
                          synchronisation per build) */
    int64_t spill_capacity; /* records each queue of the workgroup-per-column classes (the
                          sparse-block levels and the dense class) can hold: 0 default
                          (a quarter, 1/64 and 1/256 of the columns, at least 16384),
                          else this many, at most the number of columns. A build whose
                          spilled columns overflow a queue ends with RSAI_E_CAP and a
                          message that names this field; the number of columns makes
                          every column fit (small eps on large grids) at the cost of
                          the queues' memory (up to about 55 KB per column) */
} rsai_params;

typedef struct rsai_plan rsai_plan; /* opaque host handle */

typedef void *(*rsai_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*rsai_free_fn)(void *ptr, void *stream, void *ctx);

/* Defaults: c = 3, lmax = 10, eps = 0.4, FIXED, tol = 1e-3, batched, validate = 1
   (the parameter ranges the paper suggests, Section 3 and Section 5). */
rsai_status rsai_params_default(rsai_params *p);

/* Route every device allocation of the library through (alloc, dealloc, ctx).
   Passing NULLs restores hipMalloc/hipFree. Process-wide; not thread-safe against
   concurrent builds. Frees are stream-ordered: dealloc(p, stream, ctx) may be called
   while work queued on that stream still uses p, so the allocator must not hand p to
   other work before that work completes (as PyTorch's caching allocator and
   hipFreeAsync guarantee for work on the same stream). */
rsai_status rsai_set_allocator(rsai_alloc_fn alloc, rsai_free_fn dealloc, void *ctx);

/* Result of one autotuning candidate. */
typedef struct {
    int32_t tier0, refill, route, t0_hash, last_tier, reserved;
    double ms; /* median build time over the repetitions (HIP events) */
} rsai_tune_choice;

/* Time the batched build of A for every combination of the schedule choices, which
   change the speed and never the results: tier0 (each register tier), refill (0, 1),
   route (0, 1), the first tier's hash tables t0_hash (2, 4; with tier0 = 0 only) and
   the last register tier last_tier (1, 2; not below tier0): 28 combinations, reps
   builds each after one warm-up build (p gives the method parameters). Writes up to
   cap results to out (host array), their number to *count and the index of the
   fastest to *best. Synchronises the stream. */
rsai_status rsai_autotune(const rsai_csc *A, const rsai_params *p, int32_t reps, void *stream,
                          rsai_tune_choice *out, int32_t cap, int32_t *count, int32_t *best);

/* Build M for one matrix: every column m_k minimises ||A m_k - e_k||_2 (eqs. (2.1)-(2.2))
   over its pattern J_k, solved as the reduced LS problem (2.3) on the rows I_k, with J_k
   grown by Algorithm 1 (Section 3) and pruned by the dropping of Section 4 (fixed tol, or
   the adaptive tolerance of eq. (4.3)). Queues all work on stream; with p->validate = 1
   it then waits for the CSC contract check, which runs first on the stream (RSAI_E_CSC
   on violation); with p->validate = 0 or 2 it does not synchronise at all. On success
   *out owns every device buffer of the build (released by rsai_destroy); A stays
   borrowed. */
rsai_status rsai_build(const rsai_csc *A, const rsai_params *p, void *stream, rsai_plan **out);

/* Build M for count matrices in one pass: the columns of all matrices share the
   same size-bucketed persistent kernels (the method treats every column
   independently, eq. (2.2)). Matrix i of the plan is A[i] (A is a host array). */
rsai_status rsai_build_batched(int32_t count, const rsai_csc *A, const rsai_params *p, void *stream,
                               rsai_plan **out);

/* Run the build again on the plan's buffers: Algorithm 1 for every column of every
   matrix, with the values the plan's matrices hold now (same pointers, same pattern;
   e.g. the next step of a time-dependent problem). Stream-ordered on stream; results
   of the previous build (M, statistics, cached nnz) are replaced. use_graph = 1 runs
   the build's kernel sequence as a HIP graph, captured on first use (no host
   synchronisation, no allocation; the CSC contract check of validate = 1 is not
   repeated, validate = 2 stays on the device). Returns RSAI_E_HIP if capture or
   launch fails. */
rsai_status rsai_rebuild(rsai_plan *P, int32_t use_graph, void *stream);

/* The schedule a plan was built with, after defaults and the tuning table (host
   outputs, any may be NULL): first register tier, refill mode, routing, hash factor of
   the first tier (2 or 4) and last register tier. */
rsai_status rsai_plan_schedule(const rsai_plan *P, int32_t *tier0, int32_t *refill, int32_t *route, int32_t *t0_hash,
                               int32_t *last_tier);

/* Number of matrices in a plan. */
rsai_status rsai_plan_count(const rsai_plan *P, int32_t *count);

/* nnz(M) = sum_k |J_k| of matrix mat (host output; M = (m_1, ..., m_n), eq. (2.2)).
   Synchronises the build stream. Returns RSAI_E_SINGULAR (a column's LS problem (2.3)
   is rank deficient) / RSAI_E_CAP (a column outgrew the supported LS sizes) if any
   column of the plan failed, RSAI_E_CSC with validate = 2 on a malformed input. */
rsai_status rsai_plan_nnz(const rsai_plan *P, int32_t mat, int64_t *nnzM);

/* Write M = (m_1, ..., m_n) of matrix mat (eq. (2.2)) as CSC into caller device
   buffers: int64 colptr[n+1], int32 rowidx[nnzM] (row indices of column k = J_k,
   ascending), float64 val[nnzM] (the LS solution of (2.3) on that pattern). nnzM comes
   from rsai_plan_nnz; the same errors. Stream-ordered copies on stream. */
rsai_status rsai_export_M(const rsai_plan *P, int32_t mat, int64_t *colptr, int32_t *rowidx, double *val,
                          void *stream);

/* Per-column statistics of matrix mat, each a device array of n entries (any may
   be NULL): loops used, final ||A m_k - e_k||_2, |I_k|, |J_k|, the column's
   algorithmic flop count (Householder update model), and a status code
   (0 ok, RSAI_E_SINGULAR, RSAI_E_CAP). */
rsai_status rsai_export_stats(const rsai_plan *P, int32_t mat, int32_t *loops, double *resnorm, int32_t *nI,
                              int32_t *nJ, double *flops, int32_t *status, void *stream);

/* y = M x for matrix mat: the application of the right preconditioner of eq. (1.2)
   (A M y = b, x = M y). x, y: device arrays of n doubles, distinct. The rows of M are
   formed once per build (one host synchronisation on the first call after a build);
   each row is summed in ascending column order. Errors of rsai_plan_nnz,
   RSAI_E_ARG on NULL vectors, RSAI_E_NOMEM. */
rsai_status rsai_apply(const rsai_plan *P, int32_t mat, const double *x, double *y, void *stream);

/* Adjoint of the fixed-pattern LS map A -> M (pattern of M fixed, values from (2.3)):
   dA_val += d/dA [ <dM_val, M> + w_frob * sum_k ||A m_k - e_k||^2 ] restricted to
   the structural nonzeros of A. dM_val (nnzM entries, CSC order of rsai_export_M)
   may be NULL. dA_val has nnz(A) entries and is accumulated into. Columns whose R
   factor the build kept (keep_factors) are solved on it; the others have it
   recomputed: A(I_k, J_k) re-gathered and refactorised in registers when |J_k| <= 32
   and |I_k| <= 64, else R from A_k^T A_k (dot products of the sparse columns,
   Cholesky) into a temporary store allocated for the call. Limit: |J_k| <= 128, the
   build's own; beyond it RSAI_E_CAP (checked before any accumulation, one host
   synchronisation on the first call of a plan). */
rsai_status rsai_backward(rsai_plan *P, int32_t mat, const double *dM_val, double w_frob, double *dA_val,
                          void *stream);

/* Solve A x = b by BiCGStab, right-preconditioned with M of matrix mat (use_M = 1;
   use_M = 0 runs it unpreconditioned), as in the experiments of Section 5: the
   iteration runs on A M y = b with x = M y carried directly, x0 = 0, shadow residual
   b, and it stops as soon as the true relative residual ||b - A x||_2 / ||b||_2 falls
   below tol, tested after the half step and after the full step of each iteration
   (the right-preconditioned form of (1.2)).
   b (input) and x (output) are device arrays of n doubles, distinct; A is the matrix
   the plan was built from (its values as they are now). The scalars of the recurrence
   stay on the device; the host reads them once per chunk of 16 iterations, and with
   use_graph = 1 the chunk is captured once as a HIP graph and replayed. Work buffers
   (9 n doubles plus a row-sorted copy of A) come from the allocator and are released
   before return. Host-synchronising.
   On return *iters is the iteration in which the test passed (0 if b = 0 or
   tol > 1), -1 on a breakdown (rho, r^.v or t.t exactly zero, or omega = 0), or
   maxit + 1 if it did not converge; *relres is the last tested relative residual.
   Errors: RSAI_E_ARG (NULL pointer, tol < 0, maxit < 0), the errors of
   rsai_plan_nnz when use_M = 1, RSAI_E_NOMEM, RSAI_E_HIP. */
rsai_status rsai_bicgstab(rsai_plan *P, int32_t mat, const double *b, double *x, double tol, int32_t maxit,
                          int32_t use_M, int32_t use_graph, int32_t *iters, double *relres, void *stream);

/* The left form of (1.2): solve M A x = M b by BiCGStab, where the left
   preconditioner is M = N^T for N the RSAI(tol) factor of A^T (columns of N
   minimise ||A^T n_k - e_k||, so the rows of M minimise ||e_k^T - m_k^T A||).
   PT is a plan built on A^T (see rsai_transpose) and A the matrix itself (device
   CSC, same n and nnz). x0 = 0, shadow residual M b, and the stopping test of
   Section 5 on the true residual ||b - A x|| / ||b|| < tol after each half and full
   step. Arguments, results, buffers and errors otherwise as rsai_bicgstab; also
   RSAI_E_ARG if A does not match the plan's matrix in n and nnz. */
rsai_status rsai_bicgstab_left(const rsai_csc *A, rsai_plan *PT, int32_t mat, const double *b, double *x,
                               double tol, int32_t maxit, int32_t use_graph, int32_t *iters, double *relres,
                               void *stream);

/* A^T of a CSC matrix, as CSC (rows ascending in each column), into caller device
   buffers colptrT[n+1], rowidxT[nnz], valT[nnz]. Deterministic. Work buffers come
   from the allocator. Host-synchronising. Errors: RSAI_E_ARG (NULL pointer,
   n < 1 or nnz < n), RSAI_E_NOMEM, RSAI_E_HIP. */
rsai_status rsai_transpose(const rsai_csc *A, int64_t *colptrT, int32_t *rowidxT, double *valT, void *stream);

/* Maximum transversal of the pattern of A: the preprocessing Section 5 applies to its
   matrices with zero diagonal entries, a row permutation to a zero-free diagonal.
   Writes p[k] = the row matched to column k (A(p[k], k) is a stored entry), -1 for a
   column left unmatched, into the caller's device array p[n], and the size of the
   matching (the structural rank of A) to *size (host). *size == n means p is a
   permutation with a zero-free diagonal; a smaller size means A is structurally
   singular (no row permutation makes the diagonal zero-free). Any maximum matching
   may be returned (the device search is not ordered), its size is unique. Greedy
   claims, then phases of breadth-first searches along alternating paths from all
   unmatched columns. Host-synchronising (a few reads per phase); work buffers
   (9 n int32) come from the allocator. The CSC contract is checked first.
   Errors: RSAI_E_ARG (NULL pointer, bad sizes), RSAI_E_CSC, RSAI_E_NOMEM, RSAI_E_HIP. */
rsai_status rsai_transversal(const rsai_csc *A, int32_t *p, int64_t *size, void *stream);

/* B = P A for the row permutation p (device int32[n], a permutation of 0..n-1, e.g.
   from rsai_transversal): row p[k] of A becomes row k of B, B(k, j) = A(p[k], j).
   Written as CSC into caller device buffers colptrB[n+1], rowidxB[nnz] (rows
   ascending in every column), valB[nnz]. With p from rsai_transversal, B has a
   zero-free diagonal; RSAI of B gives the right preconditioner of (P A) x = P b.
   Host-synchronising (p is checked to be a permutation: RSAI_E_ARG if not; the CSC
   contract of A is checked too). Errors: RSAI_E_ARG, RSAI_E_CSC, RSAI_E_NOMEM,
   RSAI_E_HIP. */
rsai_status rsai_permute_rows(const rsai_csc *A, const int32_t *p, int64_t *colptrB, int32_t *rowidxB, double *valB,
                              void *stream);

/* y = A x (transpose = 0) or y = A^T x (transpose = 1) for a CSC matrix; x, y device
   arrays of n doubles. Stream-ordered, no host synchronisation. A x sums each row in
   ascending column order (the rows are formed in allocator work buffers per call). */
rsai_status rsai_spmv(const rsai_csc *A, const double *x, double *y, int32_t transpose, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops,
   harnesses that forbid allocation): rsai_spmv without any allocation. Same kernels,
   results and summation order as rsai_spmv. The work buffers of the row formation
   (transpose = 0) live in one static device array of RSAI_SPMV_NOALLOC_MAX_BYTES
   (64 MiB) that every device the library runs on holds until the process ends; a
   matrix that needs more (8n + 8(n + 1) + 12 nnz bytes plus the scan's partial sums,
   each part rounded up to 256 bytes; the 512 x 512 and 64^3 stencils fit, n = 10^6
   with 7 nnz per column does not) is rejected with RSAI_E_ARG before any work is
   queued. transpose = 1 needs no work buffers. All calls on one device share the
   array: calls that overlap on a device (different streams or threads) race and must
   be serialised by the caller; calls on one stream are ordered. Stream-ordered, no host
   synchronisation. The first call on a device looks up the array's device address
   (a host-side runtime query): make it once outside any graph capture.
   Errors: RSAI_E_ARG (NULL pointer, bad sizes, matrix too large), RSAI_E_HIP. */
#define RSAI_SPMV_NOALLOC_MAX_BYTES ((size_t)64 << 20)
rsai_status rsai_spmv_noalloc(const rsai_csc *A, const double *x, double *y, int32_t transpose, void *stream);

/* Gradient of y = A x with respect to the values of A: dval[e] += dy[i] * x[j] for
   every stored entry e = (i, j) of A (dval has nnz entries). */
rsai_status rsai_spmv_vjp(const rsai_csc *A, const double *dy, const double *x, double *dval, void *stream);

/* Kernel times of the last build/backward when p->timing = 1 (host array of up to
   n doubles, milliseconds): [0] preprocessing, [1] tier-0 kernel, [2] later tiers,
   [3] assembly, [4] whole build, [5] backward. Synchronises. */
rsai_status rsai_plan_timing(const rsai_plan *P, double *ms, int32_t n);

/* Describe size tier t (host outputs): lanes per column, max |I|, max |J|. The
   register tiers come first; the index after them describes the large class of the
   batched schedule. Returns RSAI_E_ARG past that. */
rsai_status rsai_tier_info(int32_t t, int32_t *lanes, int32_t *max_rows, int32_t *max_cols);

/* Measurement support, not part of the method: the FP64 vector FMA rate of the current
   device, for pricing the build's arithmetic against a measured peak beside the
   published one. Runs a kernel of 16 waves per CU in which every lane performs
   8 independent chains of iters fused multiply-adds (2 flops each), times it with HIP
   events on stream and writes TFLOP/s to *tflops (host). Synchronises the stream;
   one small work buffer from the allocator. Errors: RSAI_E_ARG (tflops NULL or
   iters < 16), RSAI_E_NOMEM, RSAI_E_HIP. */
rsai_status rsai_peak_fp64(int64_t iters, double *tflops, void *stream);

/* Destroy a plan (NULL is allowed). Synchronises the build stream. */
rsai_status rsai_destroy(rsai_plan *P);

/* Thread-local message for the last error (never NULL). */
const char *rsai_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RSAI_H */
