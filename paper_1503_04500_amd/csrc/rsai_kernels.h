// Internal launch interface between the kernel files and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rsai.h"
#include "rsai_tier.h"

namespace rsai {

// Set the thread-local message rsai_last_error() returns and return st.
rsai_status report(rsai_status st, const char *fmt, ...);

struct TierInfo {
    int G, MMAX, QMAX, REC;
    int WPS;  // waves per SIMD the tier's register budget allows
};
extern const TierInfo kTiers[];
extern const int kNumTiers;
extern const int kPlainTier;  // the one size class of the plain schedule

void launch_tier_kernel(int tier, int hash4, const TierArgs &a, int waves, hipStream_t s);

// ---- sparse-block size class (rsai_wide.hip): one workgroup per column, LS solved
// on the compressed block (shared rows + one row per column)
constexpr int WIDE_LEVELS = 4;   // instances: |I| <= 1024, 2048, 1024 (a larger compressed block), 8192
constexpr int WIDE_QMAX = 63;    // columns of J
constexpr int WIDE_RCAP = 8 * 64 + 1;  // dominant rows in a record: c * lmax + 1
struct WideArgs {
    const MatDev *mats;
    BuildParams P;
    ColOut out;
    int64_t arena_base;       // slot of a column: arena_base + ucol * 64
    const int32_t *rec_in;
    int rec_in_stride;
    const int32_t *rec_in_count;
    int64_t rec_in_cap;
    int32_t *rec_out;         // records for the next class
    int rec_out_stride;
    int32_t *rec_out_count;
    int64_t rec_out_cap;
    // Columns whose compressed block does not fit: [0] the first later level with a
    // larger block (when the next level's block is no larger), [1] the dense class
    // (when most of the block's rows are shared, so that compressing gains little);
    // nullptr where absent (the next class then takes them).
    int32_t *rec_alt[2];
    int rec_alt_stride[2];
    int32_t *rec_alt_count[2];
    int64_t rec_alt_cap[2];
    int32_t *err;
};
int wide_max_rows(int level);
int wide_rec_stride(int level);  // ints per record of up to that instance's rows
// Record queues after the register tiers, in launch order of their readers: queue 0
// feeds level 1 (rows over level 0's cap), queue 1 level 2 (level 0's blocks that do
// not fit), queue 2 level 3 (from levels 1 and 2), queue 3 the dense class.
int wide_queue_stride(int queue);
int wide_blocks_per_cu(int level);
void launch_wide_kernel(int level, const WideArgs &a, int blocks, hipStream_t s);

// ---- large size class (rsai_big.hip): one workgroup per column
constexpr int BMMAX_BIG = 8192;  // rows of the LS block
constexpr int BQMAX_BIG = 128;   // columns of the LS block
struct BigArgs {
    const MatDev *mats;
    BuildParams P;
    ColOut out;
    int64_t arena_base;       // slot of the record at queue position pos: arena_base + pos * BQMAX_BIG
    const int32_t *rec_in;
    int rec_in_stride;
    const int32_t *rec_in_count;
    int64_t rec_in_cap;
    double *scratch;          // per-workgroup slabs
    int64_t scratch_stride;   // doubles per slab
    int64_t ld;               // rows per block column in the slab: min(BMMAX_BIG, largest n)
    int32_t *err;
};
int big_max_rows();
int big_max_cols();
// doubles of one workgroup's slab for blocks of ld rows (ld <= BMMAX_BIG)
int64_t big_scratch_stride(int64_t ld);
void launch_big_kernel(const BigArgs &a, int blocks, hipStream_t s);

// ---- preprocessing (rsai_prep.hip)
// err bits: 1 colptr, 2 rows out of range / unsorted / duplicate, 4 empty column
void launch_validate(int64_t n, int64_t nnz, const int64_t *colptr, const int32_t *rowidx, int32_t *err,
                     hipStream_t s);
// the check fused with the row counts of the row pattern (cnt zeroed by the caller)
void launch_validate_counts(int64_t n, int64_t nnz, const int64_t *colptr, const int32_t *rowidx, int32_t *cnt,
                            int32_t *err, hipStream_t s);
void launch_fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t s);
void launch_fill_i64(int64_t *p, int64_t v, int64_t count, hipStream_t s);
void launch_fill_f64(double *p, double v, int64_t count, hipStream_t s);
// row pattern of A: counts -> rowptr (exclusive scan) -> colidx (unordered inside a row);
// g (max row count) and ||A||_1 as bit patterns in stats[0], stats[1]
void launch_row_counts(int64_t nnz, const int32_t *rowidx, int32_t *cnt, const int32_t *err, hipStream_t s);
void launch_row_fill(int64_t n, const int64_t *colptr, const int32_t *rowidx, const int64_t *rowptr,
                     int32_t *fillpos, int32_t *colidx, const int32_t *err, hipStream_t s);
void launch_mat_stats(int64_t n, const int64_t *colptr, const double *val, const int32_t *rowcnt,
                      unsigned long long *stats, const int32_t *err, hipStream_t s);
// up to FILL_SLOTS int32 fills in one launch; with 0 < ntab <= FILL_TAB the same launch
// writes the matrix table tab[0..ntab) to dtab and colbase[0..ntab] to dcolbase
constexpr int FILL_SLOTS = 8;
constexpr int FILL_TAB = 4;
void launch_fill_many(int32_t *const *p, const int64_t *count, const int32_t *v, int k, const MatDev *tab,
                      const int64_t *colbase, int ntab, MatDev *dtab, int64_t *dcolbase, hipStream_t s);
// longest column of a CSC matrix into *out (atomic max; *out zeroed by the caller)
void launch_max_collen(int64_t n, const int64_t *colptr, int32_t *out, hipStream_t s);

// exclusive scan of n int32 counts into out[0..n] (out[n] = total); tmp needs
// scan_tmp_elems(n) int64 elements
int64_t scan_tmp_elems(int64_t n);
void launch_scan_i32(const int32_t *in, int64_t n, int64_t *out, int64_t *tmp, hipStream_t s);
// the same in one launch (decoupled look-back): state holds scan1_state_elems(n) words,
// zero before the launch; err bit 64 reports a state that was not. With host_flags
// (device-visible host memory) the error flags as they stand at the launch are copied
// there.
int64_t scan1_state_elems(int64_t n);
void launch_scan1_i32(const int32_t *in, int64_t n, int64_t *out, unsigned long long *state, int32_t *err,
                      int32_t *host_flags, hipStream_t s);

// ---- assembly: per-column results in the arena -> CSC (rows ascending)
void launch_assemble(int64_t n, int qcap, const int64_t *off, const int32_t *nJ, const int64_t *colptrM,
                     const int32_t *arenaJ, const double *arenaV, int32_t *rowidxM, double *valM,
                     const int32_t *status, const int32_t *err, int64_t *summary, hipStream_t s);

// ---- SpMV
void launch_csc_transpose_fill(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *val,
                               const int64_t *rowptr, int32_t *fillpos, int32_t *colidxT, double *valT,
                               hipStream_t s);
void launch_sort_rows(int64_t n, const int64_t *rowptr, int32_t *colidx, double *val, hipStream_t s);
// rows of a CSC matrix (n, nnz, colptr, rowidx, val) with values, each row sorted by
// column so that row sums have a fixed order. Work buffers: cnt, fill (n each), stmp
// (scan_tmp_elems(n + 1)), zerr (4); every one is cleared by a kernel first.
void enqueue_rows(int64_t n, int64_t nnz, const int64_t *colptr, const int32_t *rowidx, const double *val,
                  int64_t *rp, int32_t *ci, double *vv, int32_t *cnt, int32_t *fill, int64_t *stmp, int32_t *zerr,
                  hipStream_t s);
// ---- maximum transversal and row permutation (rsai_match.hip)
void launch_match_greedy(int64_t n, const int64_t *colptr, const int32_t *rowidx, int32_t *match_col,
                         int32_t *match_row, hipStream_t s);
void launch_match_roots(int64_t n, const int32_t *match_col, int32_t *root, int32_t *found, int32_t *roots,
                        int32_t *nroots, hipStream_t s);
void launch_match_expand(int64_t n, const int64_t *colptr, const int32_t *rowidx, int32_t stamp, int32_t *visited,
                         int32_t *parent, int32_t *root, int32_t *found, const int32_t *match_row, const int32_t *fin,
                         const int32_t *nin, int32_t *fout, int32_t *nout, int64_t nin_host, hipStream_t s);
void launch_match_augment(const int32_t *roots, const int32_t *nroots, int64_t nroots_host, const int32_t *found,
                          const int32_t *parent, int32_t *match_col, int32_t *match_row, int32_t *naug,
                          hipStream_t s);
void launch_match_count(int64_t n, const int32_t *match_col, unsigned long long *size, hipStream_t s);
void launch_perm_invert(int64_t n, const int32_t *p, int32_t *inv, int32_t *err, hipStream_t s);
void launch_perm_rows(int64_t n, int64_t nnz, const int64_t *colptr, const int32_t *rowidx, const double *val,
                      const int32_t *inv, int64_t *colptrB, int32_t *rowidxB, double *valB, hipStream_t s);
// ---- right-preconditioned BiCGStab (rsai_krylov.hip)
struct BicgState {
    double rho, rho1, rho1n, alpha, omega, rel, nb, tol;
    int32_t done;   // 0 running, 1 converged, 2 breakdown, 3 iteration limit
    int32_t ret;    // iterations (0: b itself passed), -1 breakdown, maxit + 1
    int32_t it;     // current iteration, from 1
    int32_t half;   // converged after a half step: the solution is xh
    int32_t maxit, pad;
};
constexpr int BICG_MAXGRID = 1024;  // workgroups of a vector kernel (partial sums per value)
struct BicgArgs {
    int64_t n;
    // A and M in SELL-64: per slice of 64 rows its first entry and width; entry k of
    // row i at sp[i / 64] + k * 64 + i % 64 (column, value), zero-valued padding
    const int64_t *asp;
    const int32_t *aw, *aci;
    const double *ava;
    const int64_t *msp;
    const int32_t *mw, *mci;
    const double *mva;
    const double *b;
    // iterate and recurrence vectors; fr, fp, fs = F r, F p, F s for the operator F
    // applied first (right: M, left: A), unused without a preconditioner
    double *x, *r, *rh, *p, *w, *v, *s, *t, *xh, *res, *fr, *fp, *fs;
    double *part;        // 2 buffers of 2 * BICG_MAXGRID partial sums
    BicgState *st;       // 2 copies of the state
};
struct BicgStep {
    int stage;             // partial sums to fold in first (0: none)
    int np;                // partial sums per value (the producer's grid)
    const double *pin;     // partial sums to fold in
    double *pout;          // partial sums this kernel writes
    const BicgState *sin;  // state to read
    BicgState *sout;       // state to write (workgroup 0)
};
// host-side launch sequence: which state copy and partial-sum buffer each kernel uses
struct BicgSeq {
    BicgArgs a{};
    int grid = 1;
    int mode = 1;  // 0 no preconditioner, 1 right (A M y = b), 2 left (M A x = M b)
    int sp = 0, pb = 0, pending = 0;
    void step(int stage, bool produces, BicgStep &q);
    void init(hipStream_t s);                    // x0 = 0 and the initial test; state in copy 0
    void iterations(int count, hipStream_t s);   // count iterations (no-ops once ended)
    void settle(hipStream_t s);                  // fold pending sums; both copies equal
};
int bicg_grid(int64_t n);
int64_t sell_slices(int64_t n);
void launch_sell_widths(int64_t n, const int64_t *rp, int32_t *cnt, int32_t *sw, hipStream_t s);
void launch_sell_fill(int64_t n, const int64_t *rp, const int32_t *ci, const double *va, const int64_t *sp,
                      const int32_t *sw, int32_t *sci, double *sva, hipStream_t s);

void launch_csr_spmv(int64_t n, const int64_t *rowptr, const int32_t *colidx, const double *val, const double *x,
                     double *y, hipStream_t s);
void launch_csc_spmv_t(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *val,
                       const double *x, double *y, hipStream_t s);

void launch_spmv_vjp(int64_t n, const int64_t *colptr, const int32_t *rowidx, const double *dy, const double *x,
                     double *dval, hipStream_t s);

// ---- adjoint (rsai_backward.hip)
struct BwdArgs {
    const MatDev *mats;
    int mat;
    int64_t n;
    const int64_t *Mcolptr;
    const int32_t *Mrowidx;
    const double *Mval;
    const double *gM;   // nullable
    double w_frob;
    double *dA;
    int32_t *err;
    const double *fac;      // kept R factors (nullable)
    const int64_t *foff;    // per column of this matrix: record offset or -1 (nullable)
    // fixed-order mode (ckey != nullptr): every contribution to dA is appended as
    // (key = entry << 32 | column, value) at a slot reserved per column instead of
    // being added with an atomic, and r, A_k z are summed over J_k in ascending order
    unsigned long long *ckey;
    double *cval;
    unsigned long long *ccur;  // slots handed out
    int64_t ccap;
};
// contributions the adjoint of matrix mat would append: sum over the entries (j, k)
// of M of the length of column j of A (into *total, one atomic per workgroup)
void launch_contrib_count(const MatDev *mats, int mat, int64_t n, const int64_t *Mcolptr, const int32_t *Mrowidx,
                          unsigned long long *total, hipStream_t s);
// sort the appended contributions by (entry, column) and add each entry's sum, taken in
// column order, into dA; temp: device bytes returned by det_reduce_bytes
size_t det_reduce_bytes(int64_t count);
hipError_t det_reduce(unsigned long long *key, double *val, unsigned long long *key2, double *val2, int64_t count,
                      void *temp, size_t temp_bytes, double *dA, hipStream_t s);
int backward_max_cols();
int backward_max_rows();
int backward_factored_max_cols();
// out2[0] = max a; out2[1] = max b over the entries with mask < 0 (all if mask is null);
// out2[2] = number of those entries
// the adjoint's size maxima: outc holds MAX2_COPIES copies of five int32 (zeroed by the
// caller); max2_combine folds a host copy of them into the five values
constexpr int MAX2_COPIES = 32;
void launch_max2(int64_t n, const int32_t *a, const int32_t *b, const int64_t *mask, int32_t *outc, hipStream_t s);
void max2_combine(const int32_t *h, int32_t *out5);
// FP64 FMA throughput probe (256-thread blocks, fma_probe_chains() chains per lane)
int fma_probe_chains();
void launch_fma_probe(int blocks, int64_t iters, double *out, hipStream_t s);
void launch_backward(const BwdArgs &a, int waves, hipStream_t s);
// recomputed factors for the adjoint: columns without a kept factor and beyond the
// refactorising kernel's block (|J_k| > small_cols or |I_k| > small_rows), |J_k| <= 128
struct RefArgs {
    const MatDev *mats;
    int mat;
    int64_t n;
    const int64_t *Mcolptr;
    const int32_t *Mrowidx;
    const int32_t *nI;        // |I_k| of the matrix's columns
    const int64_t *foff;      // kept factors (nullable)
    int small_cols, small_rows;
    double *fac;              // temporary store
    int64_t cap;              // its size in doubles
    unsigned long long *cur;  // doubles handed out
    int64_t *tfoff;           // record offset per column in the temporary store, -1 none
    int32_t *err;             // bit 32: rank-deficient A_k, bit 64: store too small
};
int refactor_max_cols();
void launch_refactor_size(const RefArgs &r, unsigned long long *total, hipStream_t s);
void launch_refactor(const RefArgs &r, int cus, hipStream_t s);
void launch_merge_masks(int64_t n, const int64_t *a, const int64_t *b, int64_t *out, hipStream_t s);
// 16 lanes per column for |J_k| <= 32; with large also a wavefront per column for
// 32 < |J_k| <= 128. Persistent grids of as many workgroups as fit on cus CUs.
void launch_backward_factored(const BwdArgs &a, int cus, bool large, hipStream_t s);

}  // namespace rsai
