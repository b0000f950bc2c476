// C ABI of the RSAI(tol) library: plan object, device memory, launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/rsai.h"
#include "rsai_kernels.h"

using namespace rsai;

namespace {

thread_local std::string g_err = "";

struct Alloc {
    rsai_alloc_fn alloc = nullptr;
    rsai_free_fn dealloc = nullptr;
    void *ctx = nullptr;
} g_alloc;

rsai_status fail(rsai_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(RSAI_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

void *dev_alloc(size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 8;
    if (g_alloc.alloc) return g_alloc.alloc(bytes, (void *)s, g_alloc.ctx);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}
void dev_free(void *p, hipStream_t s) {
    if (!p) return;
    if (g_alloc.dealloc) g_alloc.dealloc(p, (void *)s, g_alloc.ctx);
    else (void)hipFree(p);
}

// The synchronous CSC check of a build: the kernel after the check copies the flags to
// a pinned host word (one per thread, with one event per device, both kept until the
// process ends), and the host waits for them only once the rest of the sequence is
// queued, so that the queue never runs dry on the host's wait.
struct ValCheck {
    bool active = false;
    int32_t *host = nullptr;   // the word (host address)
    int32_t *dev = nullptr;    // its device address
    hipEvent_t ev = nullptr;
};
constexpr int32_t kValUnset = -1;
bool val_check_prepare(ValCheck &vc) {
    constexpr int kMaxDev = 64;
    thread_local int32_t *word = nullptr;
    thread_local hipEvent_t evs[kMaxDev] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return false;
    if (!word && hipHostMalloc((void **)&word, 64, hipHostMallocPortable | hipHostMallocMapped) != hipSuccess) {
        word = nullptr;
        return false;
    }
    void *dp = nullptr;
    if (hipHostGetDevicePointer(&dp, word, 0) != hipSuccess || !dp) return false;
    if (!evs[dev] && hipEventCreateWithFlags(&evs[dev], hipEventDisableTiming) != hipSuccess) {
        evs[dev] = nullptr;
        return false;
    }
    *(volatile int32_t *)word = kValUnset;
    vc.host = word;
    vc.dev = (int32_t *)dp;
    vc.ev = evs[dev];
    return true;
}
bool val_check_finish(const ValCheck &vc, const int32_t *err, hipStream_t s, int32_t &herr) {
    if (hipEventSynchronize(vc.ev) != hipSuccess) return false;
    herr = *(volatile int32_t *)vc.host;
    if (herr == kValUnset) {
        // (not written: read the flags themselves)
        if (hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return false;
    }
    return true;
}

}  // namespace

rsai_status rsai::report(rsai_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

struct MatPlan {
    rsai_csc A{};
    int64_t col_base = 0;
    int64_t *rowptr = nullptr;
    int32_t *colidx = nullptr;
    int32_t *rowcnt = nullptr;
    int64_t *colptrM = nullptr;
    int32_t *rowidxM = nullptr;
    double *valM = nullptr;
    int64_t capM = 0;
    int64_t nnzM = -1;
    bool sizes_clear = false;  // the build's first launch zeroed the size maxima, not used since
    unsigned long long *scan_state = nullptr;  // the build's two single-pass scan states
    int64_t *summary = nullptr;  // device: nnz(M), error flags, failed-column counts; from [8] the
                                 // copies of the adjoint's size maxima (int32) when factors are kept
    int32_t maxq = -1, maxm = -1;  // largest final |J_k| and |I_k| (first backward)
    int32_t nofac = -1;            // columns without a kept factor
    int32_t maxq_nofac = -1;       // their largest |J_k|
    int32_t nlarge = -1;           // columns with a kept factor and |J_k| > 32
    // transpose of M (rows) for y = M x
    int64_t *rowptrT = nullptr;
    int32_t *rowcntT = nullptr;  // 2n: row counts and fill positions
    int64_t capT = 0;        // entries the transpose buffers hold
    bool t_valid = false;    // transpose matches the current M
    int32_t *colidxT = nullptr;
    double *valT = nullptr;
};

struct rsai_plan {
    rsai_params p{};
    hipStream_t stream = nullptr;
    std::vector<MatPlan> mats;
    std::vector<MatDev> hmats;
    std::vector<int64_t> hcolbase;
    int64_t ncols = 0;
    MatDev *d_mats = nullptr;
    int64_t *d_colbase = nullptr;
    ColOut out{};
    int64_t arena_cap = 0;
    int32_t *rec[8] = {};
    double *big_scratch = nullptr;   // per-workgroup slabs of the large size class
    int32_t *rec_count = nullptr;
    int32_t *err = nullptr;
    unsigned long long *stats = nullptr;
    int64_t *scan_tmp = nullptr;
    std::vector<void *> owned;
    hipEvent_t ev[8] = {};
    bool recorded[8] = {};
    bool have_events = false;
    void record(int i, hipStream_t s) {
        if (have_events && !capturing && hipEventRecord(ev[i], s) == hipSuccess) recorded[i] = true;
    }
    int ntiers_used = 0;
    int sched_t0 = 0, sched_refill = 1, sched_route = 1, sched_hash = 2, sched_last = 2;  // as resolved
    // the build's kernel sequence (everything after allocation and table upload), kept
    // for rsai_rebuild; first = the initial build (may check the CSC contract on the host)
    std::function<rsai_status(hipStream_t, bool)> enqueue;
    bool capturing = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;

    template <class T>
    T *alloc(int64_t count, rsai_status &st) {
        if (st != RSAI_OK) return nullptr;
        void *q = dev_alloc(sizeof(T) * (size_t)std::max<int64_t>(count, 1), stream);
        if (!q) {
            st = fail(RSAI_E_NOMEM, "device allocation of %lld bytes failed", (long long)(sizeof(T) * count));
            return nullptr;
        }
        owned.push_back(q);
        return (T *)q;
    }
    void release() {
        if (stream) (void)hipStreamSynchronize(stream);
        else (void)hipDeviceSynchronize();
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        gexec = nullptr;
        graph = nullptr;
        cap_stream = nullptr;
        for (void *q : owned) dev_free(q, stream);
        owned.clear();
        if (have_events)
            for (auto &e : ev) (void)hipEventDestroy(e);
        have_events = false;
    }
};

static rsai_status check_params(const rsai_params *p) {
    if (!p) return fail(RSAI_E_ARG, "params is NULL");
    if (p->c < 1 || p->c > CMAX) return fail(RSAI_E_ARG, "c must be in 1..%d", CMAX);
    if (p->lmax < 0 || p->lmax > 64) return fail(RSAI_E_ARG, "lmax must be in 0..64");
    if (!(p->eps >= 0.0)) return fail(RSAI_E_ARG, "eps must be >= 0");
    if (p->drop < 0 || p->drop > 2) return fail(RSAI_E_ARG, "drop mode must be 0, 1 or 2");
    if (p->drop == 1 && !(p->tol >= 0.0)) return fail(RSAI_E_ARG, "tol must be >= 0");
    if (p->sched < 0 || p->sched > 1) return fail(RSAI_E_ARG, "sched must be 0 or 1");
    if (p->validate < 0 || p->validate > 2) return fail(RSAI_E_ARG, "validate must be 0, 1 or 2");
    if (p->tier0 < -1 || p->tier0 >= kNumTiers) return fail(RSAI_E_ARG, "tier0 out of range");
    if (p->refill < -1 || p->refill > 1) return fail(RSAI_E_ARG, "refill must be -1, 0 or 1");
    if (p->route < -1 || p->route > 1) return fail(RSAI_E_ARG, "route must be -1, 0 or 1");
    if (p->deterministic < 0 || p->deterministic > 1) return fail(RSAI_E_ARG, "deterministic must be 0 or 1");
    if (p->tune_count < 0 || (p->tune_count > 0 && !p->tune_table))
        return fail(RSAI_E_ARG, "tune_count must be >= 0, with a table when > 0");
    if (p->t0_hash != -1 && p->t0_hash != 2 && p->t0_hash != 4) return fail(RSAI_E_ARG, "t0_hash must be -1, 2 or 4");
    if (p->last_tier < -1 || p->last_tier == 0 || p->last_tier >= kNumTiers)
        return fail(RSAI_E_ARG, "last_tier must be -1 or a register tier from 1 to %d", kNumTiers - 1);
    if (p->last_tier > 0 && p->tier0 > p->last_tier) return fail(RSAI_E_ARG, "tier0 is past last_tier");
    if (p->spill_capacity < 0) return fail(RSAI_E_ARG, "spill_capacity must be >= 0");
    return RSAI_OK;
}

// Bump layout over one device allocation: a first pass measures, a second assigns.
struct Layout {
    char *base = nullptr;
    size_t off = 0;
    template <class T>
    T *take(int64_t count) {
        const size_t a = (off + 255) & ~(size_t)255;
        off = a + sizeof(T) * (size_t)std::max<int64_t>(count, 1);
        return base ? reinterpret_cast<T *>(base + a) : nullptr;
    }
};

// rows of a CSC matrix with values, each row sorted by column so that row sums have a
// fixed order
namespace rsai {
void enqueue_rows(int64_t n, int64_t nnz, const int64_t *colptr, const int32_t *rowidx, const double *val,
                  int64_t *rp, int32_t *ci, double *vv, int32_t *cnt, int32_t *fill, int64_t *stmp, int32_t *zerr,
                  hipStream_t s) {
    launch_fill_i32(zerr, 0, 4, s);
    launch_fill_i32(cnt, 0, n, s);
    launch_fill_i32(fill, 0, n, s);
    launch_row_counts(nnz, rowidx, cnt, zerr, s);
    launch_scan_i32(cnt, n, rp, stmp, s);
    launch_csc_transpose_fill(n, colptr, rowidx, val, rp, fill, ci, vv, s);
    launch_sort_rows(n, rp, ci, vv, s);
}
}  // namespace rsai

extern "C" {

rsai_status rsai_params_default(rsai_params *p) {
    if (!p) return fail(RSAI_E_ARG, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->c = 3;
    p->lmax = 10;
    p->eps = 0.4;
    p->drop = RSAI_DROP_FIXED;
    p->tol = 1e-3;
    p->sched = RSAI_SCHED_BATCHED;
    p->validate = 1;
    p->tier0 = -1;
    p->timing = 0;
    p->refill = -1;
    p->route = -1;
    p->keep_factors = 0;
    p->factor_budget_bytes = 0;
    p->deterministic = 0;
    p->tune_count = 0;
    p->tune_table = nullptr;
    p->t0_hash = -1;
    p->last_tier = -1;
    p->col_len_max = nullptr;
    p->spill_capacity = 0;
    return RSAI_OK;
}

rsai_status rsai_set_allocator(rsai_alloc_fn alloc, rsai_free_fn dealloc, void *ctx) {
    if ((alloc == nullptr) != (dealloc == nullptr)) return fail(RSAI_E_ARG, "alloc and dealloc must both be set");
    g_alloc.alloc = alloc;
    g_alloc.dealloc = dealloc;
    g_alloc.ctx = ctx;
    return RSAI_OK;
}

const char *rsai_last_error(void) { return g_err.c_str(); }

rsai_status rsai_tier_info(int32_t t, int32_t *lanes, int32_t *max_rows, int32_t *max_cols) {
    if (t < 0 || t > kNumTiers + WIDE_LEVELS) return fail(RSAI_E_ARG, "no tier %d", t);
    if (t >= kNumTiers && t < kNumTiers + WIDE_LEVELS) {  // sparse-block classes: 256 lanes per column
        if (lanes) *lanes = 256;
        if (max_rows) *max_rows = wide_max_rows(t - kNumTiers);
        if (max_cols) *max_cols = WIDE_QMAX;
        return RSAI_OK;
    }
    if (t == kNumTiers + WIDE_LEVELS) {  // the dense large class: one 256-lane workgroup per column
        if (lanes) *lanes = 256;
        if (max_rows) *max_rows = big_max_rows();
        if (max_cols) *max_cols = big_max_cols();
        return RSAI_OK;
    }
    if (lanes) *lanes = kTiers[t].G;
    if (max_rows) *max_rows = kTiers[t].MMAX;
    if (max_cols) *max_cols = kTiers[t].QMAX;
    return RSAI_OK;
}

static int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

static int sync_refill_default(int requested) {
    if (requested == 0 || requested == 1) return requested;
    const char *e = getenv("RSAI_SYNC_REFILL");
    if (e && (e[0] == '0' || e[0] == '1')) return e[0] - '0';
    return 1;
}

// spill routing by size estimate (1, default) or always to the next class (0);
// RSAI_ROUTE overrides
static int route_default(int requested) {
    if (requested == 0 || requested == 1) return requested;
    const char *e = getenv("RSAI_ROUTE");
    if (e && (e[0] == '0' || e[0] == '1')) return e[0] - '0';
    return 1;
}

// Schedule fields left at -1 take the first tuning-table entry whose ranges hold the
// matrix (n, mean column length, longest column); for a batch the smallest tier0, the
// largest route and last_tier, and refill and t0_hash of the largest matrix's entry.
static rsai_status apply_tune_table(int32_t count, const rsai_csc *As, rsai_params &p, hipStream_t s) {
    if (p.tune_count <= 0 || p.sched == RSAI_SCHED_PLAIN) return RSAI_OK;
    if (p.tier0 >= 0 && p.refill >= 0 && p.route >= 0 && p.t0_hash >= 0 && p.last_tier >= 0) return RSAI_OK;
    std::vector<int64_t> maxlen(count, 0);
    if (p.col_len_max) {
        for (int i = 0; i < count; ++i) maxlen[i] = p.col_len_max[i];
    } else {
        std::vector<int32_t> ml(count, 0);
        int32_t *d = (int32_t *)dev_alloc(4 * (size_t)count, s);
        if (!d) return fail(RSAI_E_NOMEM, "tuning: longest-column buffer");
        launch_fill_i32(d, 0, count, s);
        for (int i = 0; i < count; ++i) launch_max_collen(As[i].n, As[i].colptr, d + i, s);
        const bool ok = hipMemcpyAsync(ml.data(), d, 4 * (size_t)count, hipMemcpyDeviceToHost, s) == hipSuccess &&
                        hipStreamSynchronize(s) == hipSuccess;
        dev_free(d, s);
        if (!ok) return fail(RSAI_E_HIP, "tuning: longest-column readback failed");
        for (int i = 0; i < count; ++i) maxlen[i] = ml[i];
    }
    int big = 0;
    for (int i = 1; i < count; ++i)
        if (As[i].n > As[big].n) big = i;
    int t0 = -1, rf = -1, rt = -1, hh = -1, lt = -1;
    for (int i = 0; i < count; ++i) {
        const double mean = (double)As[i].nnz / (double)As[i].n;
        for (int e = 0; e < p.tune_count; ++e) {
            const rsai_tune_entry &E = p.tune_table[e];
            if (E.len_lo <= mean && mean < E.len_hi && E.maxlen_lo <= maxlen[i] && maxlen[i] < E.maxlen_hi &&
                E.n_lo <= As[i].n && As[i].n < E.n_hi && E.eps_lo <= p.eps && p.eps < E.eps_hi) {
                t0 = (t0 < 0) ? E.tier0 : std::min(t0, E.tier0);
                rt = std::max(rt, E.route);
                lt = std::max(lt, E.last_tier);
                if (i == big) {
                    rf = E.refill;
                    hh = E.t0_hash;
                }
                break;
            }
        }
    }
    if (p.tier0 < 0 && t0 >= 0 && t0 < kNumTiers) p.tier0 = t0;
    if (p.refill < 0 && (rf == 0 || rf == 1)) p.refill = rf;
    if (p.route < 0 && (rt == 0 || rt == 1)) p.route = rt;
    if (p.t0_hash < 0 && (hh == 2 || hh == 4)) p.t0_hash = hh;
    if (p.last_tier < 0 && lt >= 1 && lt < kNumTiers && lt >= p.tier0) p.last_tier = lt;
    return RSAI_OK;
}

static rsai_status build_impl(int32_t count, const rsai_csc *As, const rsai_params *prm, void *stream,
                              rsai_plan **out) {
    if (!out) return fail(RSAI_E_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1 || !As) return fail(RSAI_E_ARG, "need at least one matrix");
    rsai_status st = check_params(prm);
    if (st != RSAI_OK) return st;
    int64_t ncols = 0;
    for (int i = 0; i < count; ++i) {
        const rsai_csc &A = As[i];
        if (A.n < 1 || A.n > INT32_MAX - 1 || A.nnz < A.n || A.nnz > INT32_MAX || !A.colptr || !A.rowidx || !A.val)
            return fail(RSAI_E_ARG, "matrix %d: bad sizes or NULL pointers", i);
        ncols += A.n;
    }
    if (ncols > INT32_MAX - 1) return fail(RSAI_E_ARG, "too many columns in one build");
    (void)hipGetLastError();  // clear an error left by an unrelated earlier call
    rsai_params pp = *prm;
    st = apply_tune_table(count, As, pp, (hipStream_t)stream);
    if (st != RSAI_OK) return st;
    rsai_plan *P = new rsai_plan();
    P->p = pp;

    P->stream = (hipStream_t)stream;
    hipStream_t s = P->stream;
    auto bail = [&](rsai_status code) {
        P->release();
        delete P;
        return code;
    };
    if (P->p.timing) {
        for (auto &e : P->ev)
            if (hipEventCreate(&e) != hipSuccess) return bail(fail(RSAI_E_HIP, "hipEventCreate failed"));
        P->have_events = true;
        P->record(0, s);
    }
    P->mats.resize(count);
    P->hcolbase.resize(count + 1);
    for (int i = 0, acc = 0; i < count; ++i) {
        P->mats[i].A = As[i];
        P->mats[i].col_base = acc;
        P->hcolbase[i] = acc;
        acc += (int)As[i].n;
    }
    P->hcolbase[count] = ncols;
    P->ncols = ncols;
    int64_t maxn = 0;
    for (int i = 0; i < count; ++i) maxn = std::max(maxn, As[i].n);

    // ---- size classes and the result arena: one slot of QMAX entries per column
    // for every size class that may finish it
    const bool plain = (P->p.sched == RSAI_SCHED_PLAIN);
    const int t0 = plain ? kPlainTier : ((P->p.tier0 >= 0) ? P->p.tier0 : 0);
    const int tlast = plain ? kPlainTier : ((P->p.last_tier > 0) ? P->p.last_tier : kNumTiers - 1);
    const int hash4 = (P->p.t0_hash == 4) ? 1 : 0;
    if (t0 > tlast) return bail(fail(RSAI_E_ARG, "tier0 is past the last register tier"));
    P->sched_t0 = t0;
    P->sched_refill = sync_refill_default(P->p.refill);
    P->sched_route = route_default(P->p.route);
    P->sched_hash = hash4 ? 4 : 2;
    P->sched_last = tlast;
    int64_t slot_base[8] = {};
    int64_t acap = 0;
    for (int t = t0; t <= tlast; ++t) {
        slot_base[t] = acap;
        acap += ncols * (int64_t)kTiers[t].QMAX;
    }
    // capacity of the record queues after the register tiers (queue w feeds level w + 1
    // of the sparse-block class, queue WIDE_LEVELS - 1 the dense class): few columns
    // need the later classes; more than this many end with RSAI_E_CAP
    int64_t wide_rec_cap[WIDE_LEVELS];
    // (every column of a build of up to 16384 columns fits every queue, so a small eps,
    // which sends most columns of a grid to the workgroup classes, still completes)
    wide_rec_cap[0] = std::min<int64_t>(ncols, std::max<int64_t>(16384, ncols / 4));
    wide_rec_cap[1] = std::min<int64_t>(ncols, std::max<int64_t>(16384, ncols / 64));
    wide_rec_cap[2] = std::min<int64_t>(ncols, std::max<int64_t>(16384, ncols / 64));
    wide_rec_cap[3] = std::min<int64_t>(ncols, std::max<int64_t>(16384, ncols / 256));
    if (P->p.spill_capacity > 0)
        for (int w = 0; w < WIDE_LEVELS; ++w) wide_rec_cap[w] = std::min<int64_t>(ncols, P->p.spill_capacity);
    // both schedules end with the workgroup-per-column classes (the plain schedule hands
    // them the columns that outgrow its one register class): the sparse-block class (an
    // arena slot of 64 per column) and the dense large class, whose columns (at most its
    // record capacity) get a slot of BQMAX_BIG per record
    const bool big = true;
    const int64_t big_cap = big ? wide_rec_cap[WIDE_LEVELS - 1] : 0;
    const int64_t wide_base = acap;
    if (big) acap += ncols * (int64_t)(WIDE_QMAX + 1);
    const int64_t big_base = acap;
    if (big) acap += big_cap * (int64_t)BQMAX_BIG;
    P->arena_cap = acap;
    // record queues and their counters. Batched: the register tiers' queues (counter k
    // feeds class t0 + 1 + k), then the workgroup classes' queues. Plain: two queues
    // used in turn by the loop launches (counter L is written by launch L), the queue of
    // the columns that outgrow the register class, then the workgroup classes' queues.
    const int nlaunch = plain ? P->p.lmax + 2 + WIDE_LEVELS : (tlast - t0 + 1 + (big ? 1 + WIDE_LEVELS : 0));
    const int q_in0 = plain ? 2 : tlast;                      // rec[] of sparse-block level 0's input
    const int c_in0 = plain ? P->p.lmax + 1 : tlast - t0;     // its counter
    const int q_wide = q_in0 + 1;                             // rec[] of the workgroup queue 0
    const int c_wide = c_in0 + 1;                             // its counter
    const int64_t qlast = big ? std::max<int64_t>(kTiers[tlast].QMAX, BQMAX_BIG) : kTiers[tlast].QMAX;
    const int64_t qmid = big ? std::max<int64_t>(kTiers[tlast].QMAX, WIDE_QMAX + 1) : qlast;
    const int big_blocks = device_cus();
    // slab rows of the dense class: no LS block has more rows than the matrix
    const int64_t big_ld = std::min<int64_t>(BMMAX_BIG, (maxn + 63) / 64 * 64);

    // R factors kept for the adjoint: an arena of the requested size (default 2 GB,
    // against 288 GB of HBM: the 64-matrix batch's factors fit); columns that do not fit
    // get their factor recomputed by the adjoint
    const int64_t fac_cap = P->p.keep_factors
                                ? std::max<int64_t>(1, (P->p.factor_budget_bytes > 0 ? P->p.factor_budget_bytes
                                                                                     : (int64_t)2 << 30) / 8)
                                : 0;

    // ---- every device buffer of the build, from one allocation
    std::vector<int32_t *> fillpos(count);
    auto layout = [&](Layout &L) {
        P->err = L.take<int32_t>(4);  // [0] error flags
        P->stats = L.take<unsigned long long>(2 * (int64_t)count);
        P->scan_tmp = L.take<int64_t>(scan_tmp_elems(maxn + 1));
        P->d_mats = L.take<MatDev>(count);
        P->d_colbase = L.take<int64_t>(count + 1);
        for (int i = 0; i < count; ++i) {
            MatPlan &M = P->mats[i];
            const int64_t n = As[i].n, nnz = As[i].nnz;
            M.rowptr = L.take<int64_t>(n + 1);
            M.colidx = L.take<int32_t>(nnz);
            M.rowcnt = L.take<int32_t>(n);
            fillpos[i] = L.take<int32_t>(n);
            // entries of M: at most qmid per column, and up to qlast for the columns the
            // dense class finishes (no more than its record capacity)
            M.capM = n * qmid + std::min<int64_t>(n, big_cap) * (qlast - qmid);
            // the summary, then the states of the build's two single-pass scans (row
            // pattern, colptr of M), all zeroed by the first launch
            M.summary = L.take<int64_t>(8 + 5 * MAX2_COPIES / 2 + 2 * scan1_state_elems(n));
            M.scan_state = (unsigned long long *)(M.summary + 8 + 5 * MAX2_COPIES / 2);
            M.colptrM = L.take<int64_t>(n + 1);
            M.rowidxM = L.take<int32_t>(M.capM);
            M.valM = L.take<double>(M.capM);
        }
        P->out.off = L.take<int64_t>(ncols);
        P->out.nJ = L.take<int32_t>(ncols);
        P->out.nI = L.take<int32_t>(ncols);
        P->out.loops = L.take<int32_t>(ncols);
        P->out.status = L.take<int32_t>(ncols);
        P->out.resnorm = L.take<double>(ncols);
        P->out.flops = L.take<double>(ncols);
        P->out.arenaJ = L.take<int32_t>(acap);
        P->out.arenaV = L.take<double>(acap);
        if (fac_cap > 0) {
            P->out.fac = L.take<double>(fac_cap);
            P->out.fac_cur = L.take<unsigned long long>(1);
            P->out.foff = L.take<int64_t>(ncols);
            P->out.fac_cap = fac_cap;
            // a wave's chunk: large enough that few finishing columns wait on the
            // store's atomic, small enough that the chunks left partly unused at the
            // end of a launch (at most one per wave) stay a small share of the store
            P->out.fac_chunk = (int32_t)std::min<int64_t>(2048, std::max<int64_t>(128, fac_cap / (64 * (int64_t)device_cus())));
        } else {
            P->out.fac = nullptr;
            P->out.fac_cur = nullptr;
            P->out.foff = nullptr;
            P->out.fac_cap = 0;
            P->out.fac_chunk = 0;
        }
        P->rec_count = L.take<int32_t>(nlaunch + 1);
        for (int t = 0; t < 8; ++t) P->rec[t] = nullptr;
        if (plain) {
            for (int r = 0; r < 3; ++r) P->rec[r] = L.take<int32_t>(ncols * (int64_t)kTiers[kPlainTier].REC);
        } else {
            for (int t = t0; t < tlast + (big ? 1 : 0); ++t)
                P->rec[t] = L.take<int32_t>(ncols * (int64_t)kTiers[t].REC);
        }
        if (big)
            for (int w = 0; w < WIDE_LEVELS; ++w)
                P->rec[q_wide + w] = L.take<int32_t>(wide_rec_cap[w] * (int64_t)wide_queue_stride(w));
        P->big_scratch = big ? L.take<double>((int64_t)big_blocks * big_scratch_stride(big_ld)) : nullptr;
    };
    Layout L0;
    layout(L0);
    Layout L1;
    L1.base = P->alloc<char>((int64_t)L0.off, st);
    if (st != RSAI_OK) return bail(st);
    layout(L1);

    // ---- the matrix table (device pointers only: no kernel result is needed)
    P->hmats.resize(count);
    for (int i = 0; i < count; ++i) {
        MatPlan &M = P->mats[i];
        MatDev &D = P->hmats[i];
        D.n = As[i].n;
        D.colptr = As[i].colptr;
        D.rowidx = As[i].rowidx;
        D.val = As[i].val;
        D.rowptr = M.rowptr;
        D.colidx = M.colidx;
        D.norm1_bits = P->stats + 2 * i + 1;
        D.col_base = M.col_base;
    }
    // (a table of up to FILL_TAB matrices travels in the arguments of the build's first
    // fill launch instead)
    if (count > FILL_TAB &&
        (hipMemcpyAsync(P->d_mats, P->hmats.data(), sizeof(MatDev) * count, hipMemcpyHostToDevice, s) != hipSuccess ||
         hipMemcpyAsync(P->d_colbase, P->hcolbase.data(), sizeof(int64_t) * (count + 1), hipMemcpyHostToDevice, s) !=
             hipSuccess))
        return bail(fail(RSAI_E_HIP, "matrix table upload failed"));

    // ---- the kernel sequence: CSC contract, row pattern, ||A||_1, the size classes,
    // assembly of M (stream-ordered; kept for rsai_rebuild)
    std::vector<rsai_csc> Av(As, As + count);
    P->enqueue = [=](hipStream_t s, bool first) -> rsai_status {
        const rsai_csc *As = Av.data();
        // ---- preprocessing: CSC contract, row pattern, ||A||_1 (all on the stream).
        // Every initial fill of the build (and the matrix table) in as few launches as
        // their number allows: the host's launches, not the GPU, set the pace before
        // the first size class starts
        {
            std::vector<int32_t *> fp;
            std::vector<int64_t> fc;
            std::vector<int32_t> fv;
            auto add = [&](void *p, int64_t words, int32_t v) {
                fp.push_back((int32_t *)p);
                fc.push_back(words);
                fv.push_back(v);
            };
            add(P->err, 4, 0);
            add(P->stats, 4 * (int64_t)count, 0);
            add(P->rec_count, nlaunch + 1, 0);
            add(P->out.status, ncols, ST_INTERNAL);  // every column's status must be written
            add(P->out.nJ, ncols, 0);
            if (P->out.fac) {
                // no factor record yet: foff = -1 (two int32 -1 words), cursor = 0
                add(P->out.foff, 2 * ncols, -1);
                add(P->out.fac_cur, 2, 0);
            }
            for (int i = 0; i < count; ++i) {
                MatPlan &M = P->mats[i];
                add(M.rowcnt, As[i].n, 0);
                add(fillpos[i], As[i].n, 0);
                // the summary (counts the assembly adds up; the adjoint's size maxima,
                // which rsai_plan_nnz gathers) and the two single-pass scan states
                add(M.summary, 2 * (8 + 5 * MAX2_COPIES / 2 + 2 * scan1_state_elems(As[i].n)), 0);
            }
            const int ntab = count <= FILL_TAB ? count : 0;
            for (size_t a = 0; a < fp.size(); a += FILL_SLOTS) {
                const int k = (int)std::min<size_t>(FILL_SLOTS, fp.size() - a);
                launch_fill_many(fp.data() + a, fc.data() + a, fv.data() + a, k, P->hmats.data(),
                                 P->hcolbase.data(), a == 0 ? ntab : 0, P->d_mats, P->d_colbase, s);
            }
        }
        // the CSC check and the row counts of the row pattern in one pass. Synchronous
        // check (validate = 1): RSAI_E_CSC is returned by this call, once the sequence
        // is queued (its kernels skip their work on a malformed matrix); the first scan
        // after the checks leaves the flags in host memory. With validate = 2 the error
        // is reported by rsai_plan_nnz.
        ValCheck vc;
        if (P->p.validate == 1 && first && !val_check_prepare(vc))
            return fail(RSAI_E_HIP, "validation readback failed");
        if (P->p.validate)
            for (int i = 0; i < count; ++i)
                launch_validate_counts(As[i].n, As[i].nnz, As[i].colptr, As[i].rowidx, P->mats[i].rowcnt, P->err, s);
        for (int i = 0; i < count; ++i) {
            MatPlan &M = P->mats[i];
            const int64_t n = As[i].n, nnz = As[i].nnz;
            if (!P->p.validate) launch_row_counts(nnz, As[i].rowidx, M.rowcnt, P->err, s);
            launch_scan1_i32(M.rowcnt, n, M.rowptr, M.scan_state, P->err, i == 0 ? vc.dev : nullptr, s);
            if (i == 0 && vc.dev) {
                if (hipEventRecord(vc.ev, s) != hipSuccess) return fail(RSAI_E_HIP, "validation readback failed");
                vc.active = true;
            }
            launch_row_fill(n, As[i].colptr, As[i].rowidx, M.rowptr, fillpos[i], M.colidx, P->err, s);
            if (P->p.drop == RSAI_DROP_ADAPTIVE)
                launch_mat_stats(n, As[i].colptr, As[i].val, M.rowcnt, P->stats + 2 * i, P->err, s);
        }
        P->record(1, s);

        TierArgs base{};
        base.mats = P->d_mats;
        base.nmat = count;
        base.col_base = P->d_colbase;
        base.P.c = P->p.c;
        base.P.lmax = P->p.lmax;
        base.P.drop = P->p.drop;
        base.P.eps = P->p.eps;
        base.P.tol = P->p.tol;
        base.out = P->out;
        base.qlen = ncols;
        base.err = P->err;
        base.sync_refill = sync_refill_default(P->p.refill);
        const int cus = device_cus();
        if (plain) {
            // ---- plain schedule: one size class, one launch per loop of Algorithm 1;
            // the state of every unfinished column goes through HBM between launches
            const int t = kPlainTier;
            const int gpw = 64 / kTiers[t].G;
            for (int L = 0; L <= P->p.lmax; ++L) {
                TierArgs a = base;
                a.arena_base = slot_base[t];
                a.one_loop = 1;
                a.sync_refill = 0;
                if (L == 0) {
                    a.rec_in = nullptr;
                } else {
                    a.rec_in = P->rec[(L - 1) % 2];
                    a.rec_in_stride = kTiers[t].REC;
                    a.rec_in_count = P->rec_count + (L - 1);
                    a.rec_in_cap = ncols;
                }
                // queue 0: the columns parked after this loop; queue 1: those that
                // outgrew the register class (to the workgroup classes)
                a.nq = 2;
                a.q_rec[0] = P->rec[L % 2];
                a.q_stride[0] = kTiers[t].REC;
                a.q_count[0] = P->rec_count + L;
                a.q_cap[0] = ncols;
                a.q_mmax[0] = kTiers[t].MMAX;
                a.q_qmax[0] = kTiers[t].QMAX;
                a.q_rec[1] = P->rec[q_in0];
                a.q_stride[1] = kTiers[t].REC;
                a.q_count[1] = P->rec_count + c_in0;
                a.q_cap[1] = ncols;
                a.q_mmax[1] = wide_max_rows(0);
                a.q_qmax[1] = WIDE_QMAX;
                int64_t want = (L == 0) ? (ncols + gpw - 1) / gpw : (int64_t)cus * 8;
                int waves = (int)std::max<int64_t>(8, std::min<int64_t>(want, (int64_t)cus * 16));
                waves = (waves + 7) / 8 * 8;
                launch_tier_kernel(t, 0, a, waves, s);
            }
            P->record(2, s);
        } else {
            for (int t = t0; t <= tlast; ++t) {
                TierArgs a = base;
                a.arena_base = slot_base[t];
                a.one_loop = 0;
                if (t != t0) a.sync_refill = 0;
                if (t == t0) {
                    a.rec_in = nullptr;
                } else {
                    a.rec_in = P->rec[t - 1];
                    a.rec_in_stride = kTiers[t - 1].REC;
                    a.rec_in_count = P->rec_count + (t - t0 - 1);
                    a.rec_in_cap = ncols;
                }
                // queues of the later classes: queue i feeds class t + 1 + i (the register
                // tiers, then the first two sparse-block levels); records use the stride
                // their reader expects
                a.nq = 0;
                const int nq_max = route_default(P->p.route) ? TierArgs::MAXQ : 1;
                for (int c = t + 1; c <= tlast + (big ? 2 : 0) && a.nq < nq_max; ++c) {
                    const int i = a.nq++;
                    a.q_rec[i] = P->rec[c - 1];
                    a.q_stride[i] = c <= tlast + 1 ? kTiers[c - 1].REC : wide_queue_stride(0);
                    a.q_count[i] = P->rec_count + (c - 1 - t0);
                    a.q_cap[i] = c <= tlast + 1 ? ncols : wide_rec_cap[0];
                    a.q_mmax[i] = c <= tlast ? kTiers[c].MMAX : wide_max_rows(c - tlast - 1);
                    a.q_qmax[i] = c <= tlast ? kTiers[c].QMAX : WIDE_QMAX;
                }
                const int gpw = 64 / kTiers[t].G;
                // a later tier gets as many persistent waves as its register budget lets
                // every SIMD hold (4 SIMDs per CU): when most columns outgrow the first
                // tier (small eps), the later tier carries the build
                int64_t want = (t == t0) ? (ncols + gpw - 1) / gpw : (int64_t)cus * 4 * kTiers[t].WPS;
                int waves = (int)std::max<int64_t>(8, std::min<int64_t>(want, (int64_t)cus * 16));
                waves = (waves + 7) / 8 * 8;
                launch_tier_kernel(t, hash4, a, waves, s);
                if (t == t0) P->record(2, s);
            }
        }
        if (big) {
            // columns that outgrew the register classes: one workgroup per column,
            // first on the compressed block, then (rarely) on the dense block.
            // Queue w (rec[q_wide + w], counter c_wide + w) feeds level w + 1; the
            // last one the dense class
            auto queue = [&](int w, int32_t *&buf, int &stride, int32_t *&count, int64_t &cap) {
                buf = P->rec[q_wide + w];
                stride = wide_queue_stride(w);
                count = P->rec_count + (c_wide + w);
                cap = wide_rec_cap[w];
            };
            // where each level sends its columns: rows over its cap (and, for levels
            // 1 to 3, blocks that do not fit) to out_q; level 0's blocks that do not
            // fit to level 2, which has a larger block; mostly shared blocks of levels
            // 0 to 2 to the dense class
            static const int out_q[WIDE_LEVELS] = {0, 2, 2, 3};
            for (int lv = 0; lv < WIDE_LEVELS; ++lv) {
                WideArgs w{};
                w.mats = P->d_mats;
                w.P = base.P;
                w.out = P->out;
                w.arena_base = wide_base;
                if (lv == 0) {
                    w.rec_in = P->rec[q_in0];
                    w.rec_in_stride = kTiers[plain ? kPlainTier : tlast].REC;
                    w.rec_in_count = P->rec_count + c_in0;
                    w.rec_in_cap = ncols;
                } else {
                    int32_t *buf, *cnt;
                    int st;
                    int64_t cap;
                    queue(lv - 1, buf, st, cnt, cap);
                    w.rec_in = buf;
                    w.rec_in_stride = st;
                    w.rec_in_count = cnt;
                    w.rec_in_cap = cap;
                }
                queue(out_q[lv], w.rec_out, w.rec_out_stride, w.rec_out_count, w.rec_out_cap);
                for (int a = 0; a < 2; ++a) {
                    w.rec_alt[a] = nullptr;
                    w.rec_alt_count[a] = nullptr;
                    w.rec_alt_stride[a] = 0;
                    w.rec_alt_cap[a] = 0;
                }
                if (lv == 0) queue(1, w.rec_alt[0], w.rec_alt_stride[0], w.rec_alt_count[0], w.rec_alt_cap[0]);
                if (lv < WIDE_LEVELS - 1)
                    queue(WIDE_LEVELS - 1, w.rec_alt[1], w.rec_alt_stride[1], w.rec_alt_count[1],
                          w.rec_alt_cap[1]);
                w.err = P->err;
                launch_wide_kernel(lv, w, device_cus() * wide_blocks_per_cu(lv), s);
            }
            BigArgs b{};
            b.mats = P->d_mats;
            b.P = base.P;
            b.out = P->out;
            b.arena_base = big_base;
            b.rec_in = P->rec[q_wide + WIDE_LEVELS - 1];
            b.rec_in_stride = wide_queue_stride(WIDE_LEVELS - 1);
            b.rec_in_count = P->rec_count + (c_wide + WIDE_LEVELS - 1);
            b.rec_in_cap = wide_rec_cap[WIDE_LEVELS - 1];
            b.scratch = P->big_scratch;
            b.scratch_stride = big_scratch_stride(big_ld);
            b.ld = big_ld;
            b.err = P->err;
            launch_big_kernel(b, big_blocks, s);
        }
        P->ntiers_used = tlast - t0 + 1 + (big ? 1 + WIDE_LEVELS : 0);
        P->record(3, s);

        // ---- assembly of M per matrix: colptr = scan(nJ), then compaction
        for (int i = 0; i < count; ++i) {
            MatPlan &M = P->mats[i];
            const int64_t n = As[i].n;
            launch_scan1_i32(P->out.nJ + M.col_base, n, M.colptrM, M.scan_state + scan1_state_elems(n), P->err,
                             nullptr, s);
            launch_assemble(n, (int)qlast, P->out.off + M.col_base, P->out.nJ + M.col_base, M.colptrM, P->out.arenaJ,
                            P->out.arenaV, M.rowidxM, M.valM, P->out.status + M.col_base, P->err, M.summary, s);
        }
        P->record(4, s);
        hipError_t le = hipGetLastError();
        if (le != hipSuccess) return fail(RSAI_E_HIP, "launch failed: %s", hipGetErrorString(le));
        if (vc.active) {
            int32_t herr = 0;
            if (!val_check_finish(vc, P->err, s, herr)) return fail(RSAI_E_HIP, "validation readback failed");
            if (herr) {
                (void)hipStreamSynchronize(s);
                return fail(RSAI_E_CSC, "malformed CSC (flags %d: 1 colptr, 2 row indices, 4 empty column)", herr);
            }
        }
        return RSAI_OK;

    };
    st = P->enqueue(s, true);
    if (st != RSAI_OK) return bail(st);
    for (MatPlan &M : P->mats) M.sizes_clear = true;
    *out = P;
    return RSAI_OK;
}

rsai_status rsai_build(const rsai_csc *A, const rsai_params *p, void *stream, rsai_plan **out) {
    return build_impl(1, A, p, stream, out);
}

rsai_status rsai_build_batched(int32_t count, const rsai_csc *A, const rsai_params *p, void *stream,
                               rsai_plan **out) {
    return build_impl(count, A, p, stream, out);
}

// later plan calls run on the plan's stream: order it after work queued on s
static rsai_status order_after(rsai_plan *P, hipStream_t s) {
    if (s == P->stream) return RSAI_OK;
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(RSAI_E_HIP, "event creation failed");
    const bool ok = hipEventRecord(e, s) == hipSuccess && hipStreamWaitEvent(P->stream, e, 0) == hipSuccess;
    (void)hipEventDestroy(e);
    return ok ? RSAI_OK : fail(RSAI_E_HIP, "stream ordering failed");
}

rsai_status rsai_rebuild(rsai_plan *P, int32_t use_graph, void *stream) {
    if (!P || !P->enqueue) return fail(RSAI_E_ARG, "plan is NULL");
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    // results of the previous build are out of date
    for (MatPlan &M : P->mats) {
        M.nnzM = -1;
        M.sizes_clear = false;
        M.maxq = M.maxm = M.maxq_nofac = M.nlarge = -1;
        M.t_valid = false;
    }
    for (bool &r : P->recorded) r = false;
    // the sequence starts by zeroing every matrix's summary and scan states
    auto cleared = [P]() {
        for (MatPlan &M : P->mats) M.sizes_clear = true;
    };
    if (!use_graph) {
        const rsai_status st = P->enqueue(s, false);
        if (st != RSAI_OK) return st;
        cleared();
        return order_after(P, s);
    }
    if (!P->gexec) {
        // capture the sequence once on a private stream, then replay it on any stream
        if (!P->cap_stream && hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return fail(RSAI_E_HIP, "stream creation failed");
        if (hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(RSAI_E_HIP, "graph capture could not start");
        P->capturing = true;
        rsai_status st = P->enqueue(P->cap_stream, false);
        P->capturing = false;
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(P->cap_stream, &g);
        if (st != RSAI_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (ec != hipSuccess || !g) return fail(RSAI_E_HIP, "graph capture failed: %s", hipGetErrorString(ec));
        P->graph = g;
        if (hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
            P->gexec = nullptr;
            return fail(RSAI_E_HIP, "graph instantiation failed");
        }
    }
    if (hipGraphLaunch(P->gexec, s) != hipSuccess) return fail(RSAI_E_HIP, "graph launch failed");
    cleared();
    return order_after(P, s);
}

rsai_status rsai_autotune(const rsai_csc *A, const rsai_params *p, int32_t reps, void *stream,
                          rsai_tune_choice *out, int32_t cap, int32_t *count, int32_t *best) {
    if (!A || !p || !out || !count || !best || cap < 1 || reps < 1) return fail(RSAI_E_ARG, "NULL or bad argument");
    rsai_status st = check_params(p);
    if (st != RSAI_OK) return st;
    int32_t nout = 0, ib = -1;
    for (int t0 = 0; t0 < kNumTiers; ++t0)
        for (int lt = 1; lt < kNumTiers; ++lt)
            for (int hh = 2; hh <= 4; hh += 2)
                for (int rf = 0; rf <= 1; ++rf)
                    for (int rt = 0; rt <= 1; ++rt) {
                        if (lt < t0 || (hh == 4 && t0 != 0)) continue;  // no such schedule
                        rsai_params q = *p;
                        q.sched = RSAI_SCHED_BATCHED;
                        q.tier0 = t0;
                        q.refill = rf;
                        q.route = rt;
                        q.t0_hash = hh;
                        q.last_tier = lt;
                        q.tune_count = 0;
                        q.tune_table = nullptr;
                        q.col_len_max = nullptr;
                        q.timing = 1;
                        std::vector<double> ms;
                        for (int r = 0; r < reps + 1; ++r) {
                            rsai_plan *P = nullptr;
                            st = rsai_build(A, &q, stream, &P);
                            if (st != RSAI_OK) return st;
                            int64_t nz = 0;
                            st = rsai_plan_nnz(P, 0, &nz);
                            double tm[6] = {};
                            if (st == RSAI_OK) st = rsai_plan_timing(P, tm, 6);
                            rsai_destroy(P);
                            if (st != RSAI_OK) return st;
                            if (r > 0) ms.push_back(tm[4]);  // the first build warms the allocator
                        }
                        std::sort(ms.begin(), ms.end());
                        if (nout < cap) {
                            rsai_tune_choice &c = out[nout];
                            c.tier0 = t0;
                            c.refill = rf;
                            c.route = rt;
                            c.t0_hash = hh;
                            c.last_tier = lt;
                            c.reserved = 0;
                            c.ms = ms[ms.size() / 2];
                            if (ib < 0 || c.ms < out[ib].ms) ib = nout;
                            ++nout;
                        }
                    }
    *count = nout;
    *best = ib;
    return RSAI_OK;
}

rsai_status rsai_plan_schedule(const rsai_plan *P, int32_t *tier0, int32_t *refill, int32_t *route, int32_t *t0_hash,
                               int32_t *last_tier) {
    if (!P) return fail(RSAI_E_ARG, "plan is NULL");
    if (tier0) *tier0 = P->sched_t0;
    if (refill) *refill = P->sched_refill;
    if (route) *route = P->sched_route;
    if (t0_hash) *t0_hash = P->sched_hash;
    if (last_tier) *last_tier = P->sched_last;
    return RSAI_OK;
}

rsai_status rsai_plan_count(const rsai_plan *P, int32_t *count) {
    if (!P || !count) return fail(RSAI_E_ARG, "NULL argument");
    *count = (int32_t)P->mats.size();
    return RSAI_OK;
}

static rsai_status check_mat(const rsai_plan *P, int32_t mat) {
    if (!P) return fail(RSAI_E_ARG, "plan is NULL");
    if (mat < 0 || mat >= (int32_t)P->mats.size()) return fail(RSAI_E_ARG, "matrix index %d out of range", mat);
    return RSAI_OK;
}

rsai_status rsai_plan_nnz(const rsai_plan *Pc, int32_t mat, int64_t *nnzM) {
    rsai_status st = check_mat(Pc, mat);
    if (st != RSAI_OK) return st;
    if (!nnzM) return fail(RSAI_E_ARG, "nnzM is NULL");
    rsai_plan *P = const_cast<rsai_plan *>(Pc);
    MatPlan &M = P->mats[mat];
    if (M.nnzM < 0) {
        const int64_t n = M.A.n;
        int64_t h[8 + 5 * MAX2_COPIES / 2] = {};
        // (the first words were written by the assembly at the end of the build); with
        // kept factors the adjoint's size maxima come back in the same copy
        const bool sizes = P->out.foff != nullptr && M.maxq < 0;
        if (sizes && !M.sizes_clear) launch_fill_i64(M.summary + 8, 0, 5 * MAX2_COPIES / 2, P->stream);
        M.sizes_clear = false;
        if (sizes)
            launch_max2(n, P->out.nJ + M.col_base, P->out.nI + M.col_base, P->out.foff + M.col_base,
                        (int32_t *)(M.summary + 8), P->stream);
        HIPCHK(hipMemcpyAsync(h, M.summary, sizeof(h), hipMemcpyDeviceToHost, P->stream));
        HIPCHK(hipStreamSynchronize(P->stream));
        if (sizes) {
            int32_t hc[5 * MAX2_COPIES], h2[5];
            std::memcpy(hc, h + 8, sizeof(hc));
            max2_combine(hc, h2);
            M.maxq = h2[0];
            M.maxm = h2[1];
            M.nofac = h2[2];
            M.maxq_nofac = h2[3];
            M.nlarge = h2[4];
        }
        const int64_t herr = h[1];
        if (herr & 7) return fail(RSAI_E_CSC, "malformed CSC (flags %lld: 1 colptr, 2 row indices, 4 empty column)",
                                  (long long)herr);
        if (herr & ~32LL) return fail(RSAI_E_STATE, "internal index error (flags %lld)", (long long)herr);
        if (herr & 32)
            return fail(RSAI_E_CAP,
                        "%lld columns did not fit the spill queues of the workgroup-per-column classes "
                        "(rsai_params.spill_capacity: %lld; the number of columns makes every column fit)",
                        (long long)h[3], (long long)P->p.spill_capacity);
        if (h[4]) return fail(RSAI_E_STATE, "%lld columns were not processed", (long long)h[4]);
        if (h[2]) return fail(RSAI_E_SINGULAR, "%lld columns have a rank-deficient LS problem", (long long)h[2]);
        if (h[3]) return fail(RSAI_E_CAP, "%lld columns outgrew the largest supported LS size", (long long)h[3]);
        M.nnzM = h[0];
    }
    *nnzM = M.nnzM;
    return RSAI_OK;
}

rsai_status rsai_export_M(const rsai_plan *P, int32_t mat, int64_t *colptr, int32_t *rowidx, double *val,
                          void *stream) {
    int64_t nz = 0;
    rsai_status st = rsai_plan_nnz(P, mat, &nz);
    if (st != RSAI_OK) return st;
    const MatPlan &M = P->mats[mat];
    hipStream_t s = (hipStream_t)stream;
    if (colptr) HIPCHK(hipMemcpyAsync(colptr, M.colptrM, sizeof(int64_t) * (M.A.n + 1), hipMemcpyDeviceToDevice, s));
    if (rowidx && nz) HIPCHK(hipMemcpyAsync(rowidx, M.rowidxM, sizeof(int32_t) * nz, hipMemcpyDeviceToDevice, s));
    if (val && nz) HIPCHK(hipMemcpyAsync(val, M.valM, sizeof(double) * nz, hipMemcpyDeviceToDevice, s));
    return RSAI_OK;
}

rsai_status rsai_export_stats(const rsai_plan *P, int32_t mat, int32_t *loops, double *resnorm, int32_t *nI,
                              int32_t *nJ, double *flops, int32_t *status, void *stream) {
    rsai_status st = check_mat(P, mat);
    if (st != RSAI_OK) return st;
    const MatPlan &M = P->mats[mat];
    const int64_t n = M.A.n, b = M.col_base;
    hipStream_t s = (hipStream_t)stream;
    if (s != P->stream) HIPCHK(hipStreamSynchronize(P->stream));
    if (loops) HIPCHK(hipMemcpyAsync(loops, P->out.loops + b, 4 * n, hipMemcpyDeviceToDevice, s));
    if (resnorm) HIPCHK(hipMemcpyAsync(resnorm, P->out.resnorm + b, 8 * n, hipMemcpyDeviceToDevice, s));
    if (nI) HIPCHK(hipMemcpyAsync(nI, P->out.nI + b, 4 * n, hipMemcpyDeviceToDevice, s));
    if (nJ) HIPCHK(hipMemcpyAsync(nJ, P->out.nJ + b, 4 * n, hipMemcpyDeviceToDevice, s));
    if (flops) HIPCHK(hipMemcpyAsync(flops, P->out.flops + b, 8 * n, hipMemcpyDeviceToDevice, s));
    if (status) HIPCHK(hipMemcpyAsync(status, P->out.status + b, 4 * n, hipMemcpyDeviceToDevice, s));
    return RSAI_OK;
}

// rows of M (row-sorted CSR), built once per build; needs a finished build
static rsai_status rows_of_M(rsai_plan *P, int32_t mat) {
    int64_t nz = 0;
    rsai_status st = rsai_plan_nnz(P, mat, &nz);
    if (st != RSAI_OK) return st;
    MatPlan &M = P->mats[mat];
    const int64_t n = M.A.n;
    if (!M.t_valid) {
        // rows of M once per build: counts, scan, fill, sort each row by column
        if (!M.rowptrT || nz > M.capT) {
            M.rowcntT = P->alloc<int32_t>(2 * n, st);
            M.rowptrT = P->alloc<int64_t>(n + 1, st);
            M.colidxT = P->alloc<int32_t>(nz, st);
            M.valT = P->alloc<double>(nz, st);
            if (st != RSAI_OK) {
                M.rowptrT = nullptr;
                return st;
            }
            M.capT = nz;
        }
        int32_t *cnt = M.rowcntT, *fill = M.rowcntT + n;
        launch_fill_i32(cnt, 0, 2 * n, P->stream);
        launch_row_counts(nz, M.rowidxM, cnt, P->err, P->stream);
        launch_scan_i32(cnt, n, M.rowptrT, P->scan_tmp, P->stream);
        launch_csc_transpose_fill(n, M.colptrM, M.rowidxM, M.valM, M.rowptrT, fill, M.colidxT, M.valT, P->stream);
        launch_sort_rows(n, M.rowptrT, M.colidxT, M.valT, P->stream);
        HIPCHK(hipStreamSynchronize(P->stream));
        M.t_valid = true;
    }
    return RSAI_OK;
}

rsai_status rsai_apply(const rsai_plan *Pc, int32_t mat, const double *x, double *y, void *stream) {
    rsai_plan *P = const_cast<rsai_plan *>(Pc);
    rsai_status st = rows_of_M(P, mat);
    if (st != RSAI_OK) return st;
    if (!x || !y) return fail(RSAI_E_ARG, "NULL vector");
    MatPlan &M = P->mats[mat];
    const int64_t n = M.A.n;
    hipStream_t s = (hipStream_t)stream;
    launch_csr_spmv(n, M.rowptrT, M.colidxT, M.valT, x, y, s);
    HIPCHK(hipGetLastError());
    return RSAI_OK;
}


static void enqueue_rows(const rsai_csc *A, int64_t *rp, int32_t *ci, double *vv, int32_t *cnt, int32_t *fill,
                         int64_t *stmp, int32_t *zerr, hipStream_t s) {
    rsai::enqueue_rows(A->n, A->nnz, A->colptr, A->rowidx, A->val, rp, ci, vv, cnt, fill, stmp, zerr, s);
}

rsai_status rsai_spmv(const rsai_csc *A, const double *x, double *y, int32_t transpose, void *stream) {
    if (!A || !x || !y) return fail(RSAI_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (transpose) {
        launch_csc_spmv_t(A->n, A->colptr, A->rowidx, A->val, x, y, s);
        HIPCHK(hipGetLastError());
        return RSAI_OK;
    }
    // y = A x through the rows of A (deterministic summation order); the work buffers
    // come from one allocation (each allocator call may cross into the host runtime
    // that owns the memory)
    rsai_status st = RSAI_OK;
    const int64_t n = A->n, nnz = A->nnz;
    int32_t *cnt = nullptr, *fill = nullptr, *ci = nullptr, *zerr = nullptr;
    int64_t *rp = nullptr, *stmp = nullptr;
    double *vv = nullptr;
    auto layout = [&](Layout &L) {
        cnt = L.take<int32_t>(n);
        fill = L.take<int32_t>(n);
        rp = L.take<int64_t>(n + 1);
        ci = L.take<int32_t>(nnz);
        vv = L.take<double>(nnz);
        stmp = L.take<int64_t>(scan_tmp_elems(n + 1));
        zerr = L.take<int32_t>(4);
    };
    Layout L0;
    layout(L0);
    Layout L1;
    L1.base = (char *)dev_alloc(L0.off, s);
    if (!L1.base) return fail(RSAI_E_NOMEM, "spmv work buffers (%zu bytes)", L0.off);
    layout(L1);
    enqueue_rows(A, rp, ci, vv, cnt, fill, stmp, zerr, s);
    launch_csr_spmv(n, rp, ci, vv, x, y, s);
    if (hipGetLastError() != hipSuccess) st = fail(RSAI_E_HIP, "spmv launch failed");
    // stream-ordered release: the work queued on s above still uses the block
    dev_free(L1.base, s);
    return st;
}

rsai_status rsai_spmv_vjp(const rsai_csc *A, const double *dy, const double *x, double *dval, void *stream) {
    if (!A || !dy || !x || !dval) return fail(RSAI_E_ARG, "NULL argument");
    launch_spmv_vjp(A->n, A->colptr, A->rowidx, dy, x, dval, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return RSAI_OK;
}

// SELL-64 copy of a row-sorted CSR matrix (one host synchronisation for its size)
static rsai_status to_sell(int64_t n, const int64_t *rp, const int32_t *ci, const double *va, int64_t *stmp,
                           const std::function<void *(size_t)> &al, const int64_t *&sp, const int32_t *&sw,
                           const int32_t *&sci, const double *&sva, hipStream_t s) {
    const int64_t nsl = sell_slices(n);
    int32_t *cnt = (int32_t *)al(4 * (size_t)nsl);
    int32_t *w = (int32_t *)al(4 * (size_t)nsl);
    int64_t *p = (int64_t *)al(8 * (size_t)(nsl + 1));
    if (!cnt || !w || !p) return RSAI_E_NOMEM;
    launch_sell_widths(n, rp, cnt, w, s);
    launch_scan_i32(cnt, nsl, p, stmp, s);
    int64_t total = 0;
    HIPCHK(hipMemcpyAsync(&total, p + nsl, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int32_t *c2 = (int32_t *)al(4 * (size_t)total);
    double *v2 = (double *)al(8 * (size_t)total);
    if (!c2 || !v2) return RSAI_E_NOMEM;
    launch_sell_fill(n, rp, ci, va, p, w, c2, v2, s);
    sp = p;
    sw = w;
    sci = c2;
    sva = v2;
    return RSAI_OK;
}

// BiCGStab on A with the preconditioner given by its rows (mode 1 right, 2 left;
// mrp == nullptr and mode 0 without one)
static rsai_status bicg_solve(const rsai_csc &A, int mode, const int64_t *mrp, const int32_t *mci,
                              const double *mva, const double *b, double *x, double tol, int32_t maxit,
                              int32_t use_graph, int32_t *iters, double *relres, hipStream_t s) {
    rsai_status st = RSAI_OK;
    const int64_t n = A.n, nnz = A.nnz;
    std::vector<void *> tmp;
    std::function<void *(size_t)> al = [&](size_t bytes) -> void * {
        void *q = dev_alloc(std::max<size_t>(bytes, 8), s);
        if (!q) st = fail(RSAI_E_NOMEM, "allocation failed");
        tmp.push_back(q);
        return q;
    };
    auto cleanup = [&](rsai_status r) {
        (void)hipStreamSynchronize(s);
        for (void *q : tmp) dev_free(q, s);
        return r;
    };
    BicgSeq seq;
    BicgArgs &a = seq.a;
    a.n = n;
    {
        // rows of A (sorted), then both matrices in SELL-64
        int64_t *arp = (int64_t *)al(8 * (n + 1));
        int32_t *aci = (int32_t *)al(4 * nnz);
        double *ava = (double *)al(8 * nnz);
        int32_t *cnt = (int32_t *)al(4 * n), *fill = (int32_t *)al(4 * n), *zerr = (int32_t *)al(16);
        int64_t *stmp = (int64_t *)al(8 * scan_tmp_elems(n + 1));
        if (st != RSAI_OK) return cleanup(st);
        enqueue_rows(&A, arp, aci, ava, cnt, fill, stmp, zerr, s);
        rsai_status r2 = to_sell(n, arp, aci, ava, stmp, al, a.asp, a.aw, a.aci, a.ava, s);
        if (r2 == RSAI_OK && mode != 0) r2 = to_sell(n, mrp, mci, mva, stmp, al, a.msp, a.mw, a.mci, a.mva, s);
        if (st != RSAI_OK || r2 != RSAI_OK) return cleanup(st != RSAI_OK ? st : r2);
    }
    double *vec = (double *)al(8 * 12 * (size_t)n);
    a.part = (double *)al(8 * 4 * (size_t)BICG_MAXGRID);
    a.st = (BicgState *)al(2 * sizeof(BicgState));
    if (st != RSAI_OK) return cleanup(st);
    a.b = b;
    a.x = x;
    double *vp = vec;
    a.r = vp; vp += n;
    a.rh = vp; vp += n;
    a.p = vp; vp += n;
    a.w = vp; vp += n;
    a.v = vp; vp += n;
    a.s = vp; vp += n;
    a.t = vp; vp += n;
    a.fp = vp; vp += n;
    a.fs = vp; vp += n;
    a.res = vp; vp += n;
    a.fr = vp; vp += n;
    a.xh = vp;
    seq.grid = bicg_grid(n);
    seq.mode = mode;
    BicgState h[2] = {};
    h[0].tol = h[1].tol = tol;
    h[0].maxit = h[1].maxit = maxit;
    if (hipMemcpyAsync(a.st, h, sizeof(h), hipMemcpyHostToDevice, s) != hipSuccess)
        return cleanup(fail(RSAI_E_HIP, "state upload failed"));
    seq.init(s);
    // iterations are enqueued in chunks, each ending with a settle; the host reads the
    // state once per chunk
    constexpr int CHUNK = 16;
    hipGraphExec_t gx = nullptr;
    hipStream_t cs = nullptr;
    if (use_graph) {
        hipGraph_t g = nullptr;
        bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess &&
                  hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            seq.iterations(CHUNK, cs);
            seq.settle(cs);
            ok = hipStreamEndCapture(cs, &g) == hipSuccess && g;
        }
        if (ok) ok = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
        if (!ok) {
            if (cs) (void)hipStreamDestroy(cs);
            return cleanup(fail(RSAI_E_HIP, "graph capture of the iteration failed"));
        }
    }
    int done_iters = 0;
    int chunk = use_graph ? CHUNK : 4;
    hipError_t he = hipSuccess;
    bool stuck = false;
    BicgState hs{};
    for (;;) {
        he = hipMemcpyAsync(&hs, a.st, sizeof(hs), hipMemcpyDeviceToHost, s);
        if (he == hipSuccess) he = hipStreamSynchronize(s);
        if (he != hipSuccess || hs.done) break;
        if (use_graph) {
            he = hipGraphLaunch(gx, s);
        } else {
            seq.iterations(chunk, s);
            seq.settle(s);
            he = hipGetLastError();
        }
        if (he != hipSuccess) break;
        done_iters += chunk;
        if (!use_graph) chunk = std::min(chunk * 2, CHUNK);
        if (done_iters > maxit + 2 * CHUNK) {  // every iteration advances or ends the solve
            stuck = true;
            break;
        }
    }
    if (gx) (void)hipGraphExecDestroy(gx);
    if (cs) (void)hipStreamDestroy(cs);
    if (stuck) return cleanup(fail(RSAI_E_STATE, "BiCGStab state did not advance"));
    if (he != hipSuccess) return cleanup(fail(RSAI_E_HIP, "BiCGStab iteration failed: %s", hipGetErrorString(he)));
    if (hs.half && hipMemcpyAsync(x, a.xh, 8 * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return cleanup(fail(RSAI_E_HIP, "copy of the half-step solution failed"));
    *iters = hs.ret;
    *relres = hs.rel;
    return cleanup(RSAI_OK);
}

rsai_status rsai_bicgstab(rsai_plan *P, int32_t mat, const double *b, double *x, double tol, int32_t maxit,
                          int32_t use_M, int32_t use_graph, int32_t *iters, double *relres, void *stream) {
    rsai_status st = check_mat(P, mat);
    if (st != RSAI_OK) return st;
    if (!b || !x || !iters || !relres) return fail(RSAI_E_ARG, "NULL argument");
    if (!(tol >= 0.0) || maxit < 0) return fail(RSAI_E_ARG, "tol must be >= 0 and maxit >= 0");
    MatPlan &M = P->mats[mat];
    if (use_M) {
        st = rows_of_M(P, mat);
        if (st != RSAI_OK) return st;
        return bicg_solve(M.A, 1, M.rowptrT, M.colidxT, M.valT, b, x, tol, maxit, use_graph, iters, relres,
                          (hipStream_t)stream);
    }
    return bicg_solve(M.A, 0, nullptr, nullptr, nullptr, b, x, tol, maxit, use_graph, iters, relres,
                      (hipStream_t)stream);
}

rsai_status rsai_bicgstab_left(const rsai_csc *A, rsai_plan *PT, int32_t mat, const double *b, double *x, double tol,
                               int32_t maxit, int32_t use_graph, int32_t *iters, double *relres, void *stream) {
    rsai_status st = check_mat(PT, mat);
    if (st != RSAI_OK) return st;
    if (!A || !A->colptr || !A->rowidx || !A->val || !b || !x || !iters || !relres)
        return fail(RSAI_E_ARG, "NULL argument");
    if (!(tol >= 0.0) || maxit < 0) return fail(RSAI_E_ARG, "tol must be >= 0 and maxit >= 0");
    MatPlan &M = PT->mats[mat];
    if (A->n != M.A.n || A->nnz != M.A.nnz)
        return fail(RSAI_E_ARG, "A does not match the transposed matrix of the plan (n %lld vs %lld, nnz %lld vs %lld)",
                    (long long)A->n, (long long)M.A.n, (long long)A->nnz, (long long)M.A.nnz);
    int64_t nz = 0;
    st = rsai_plan_nnz(PT, mat, &nz);
    if (st != RSAI_OK) return st;
    // rows of the left preconditioner M^T are the columns of the plan's M (CSC, rows
    // ascending within each column)
    return bicg_solve(*A, 2, M.colptrM, M.rowidxM, M.valM, b, x, tol, maxit, use_graph, iters, relres,
                      (hipStream_t)stream);
}

rsai_status rsai_transpose(const rsai_csc *A, int64_t *colptrT, int32_t *rowidxT, double *valT, void *stream) {
    if (!A || !A->colptr || !A->rowidx || !A->val || !colptrT || !rowidxT || !valT)
        return fail(RSAI_E_ARG, "NULL argument");
    if (A->n < 1 || A->nnz < A->n) return fail(RSAI_E_ARG, "bad sizes");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = A->n;
    rsai_status st = RSAI_OK;
    std::vector<void *> tmp;
    auto al = [&](size_t bytes) -> void * {
        void *q = dev_alloc(std::max<size_t>(bytes, 8), s);
        if (!q) st = fail(RSAI_E_NOMEM, "allocation failed");
        tmp.push_back(q);
        return q;
    };
    int32_t *cnt = (int32_t *)al(4 * n), *fill = (int32_t *)al(4 * n), *zerr = (int32_t *)al(16);
    int64_t *stmp = (int64_t *)al(8 * scan_tmp_elems(n + 1));
    if (st == RSAI_OK) {
        // the rows of A, sorted by column, are the columns of A^T sorted by row
        enqueue_rows(A, colptrT, rowidxT, valT, cnt, fill, stmp, zerr, s);
        if (hipStreamSynchronize(s) != hipSuccess) st = fail(RSAI_E_HIP, "transpose failed");
    }
    for (void *q : tmp) dev_free(q, s);
    return st;
}

rsai_status rsai_transversal(const rsai_csc *A, int32_t *p, int64_t *size, void *stream) {
    if (!A || !A->colptr || !A->rowidx || !p || !size) return fail(RSAI_E_ARG, "NULL argument");
    if (A->n < 1 || A->n > INT32_MAX - 1 || A->nnz < 0 || A->nnz > INT32_MAX) return fail(RSAI_E_ARG, "bad sizes");
    *size = 0;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = A->n;
    rsai_status st = RSAI_OK;
    std::vector<void *> tmp;
    auto al = [&](size_t bytes) -> void * {
        void *q = dev_alloc(std::max<size_t>(bytes, 8), s);
        if (!q) st = fail(RSAI_E_NOMEM, "allocation failed");
        tmp.push_back(q);
        return q;
    };
    auto done = [&](rsai_status r) {
        (void)hipStreamSynchronize(s);
        for (void *q : tmp) dev_free(q, s);
        return r;
    };
    int32_t *match_row = (int32_t *)al(4 * n), *visited = (int32_t *)al(4 * n), *parent = (int32_t *)al(4 * n);
    int32_t *root = (int32_t *)al(4 * n), *found = (int32_t *)al(4 * n), *roots = (int32_t *)al(4 * n);
    int32_t *fa = (int32_t *)al(4 * n), *fb = (int32_t *)al(4 * n);
    int32_t *cnt = (int32_t *)al(4 * 64);  // [0] roots, [1] augmented, [2 + l % 2] frontier sizes
    if (st != RSAI_OK) return done(st);
    // the CSC contract first: the search indexes rows by the stored row indices
    {
        int32_t herr = 0;
        launch_fill_i32(cnt, 0, 64, s);
        launch_validate(n, A->nnz, A->colptr, A->rowidx, cnt, s);
        if (hipMemcpyAsync(&herr, cnt, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return done(fail(RSAI_E_HIP, "transversal: validation readback failed"));
        if (herr) return done(fail(RSAI_E_CSC, "malformed CSC (flags %d: 1 colptr, 2 row indices, 4 empty column)", herr));
    }
    launch_fill_i32(p, -1, n, s);
    launch_fill_i32(match_row, -1, n, s);
    launch_fill_i32(visited, 0, n, s);
    launch_match_greedy(n, A->colptr, A->rowidx, p, match_row, s);
    // phases of augmentation; each flips at least one path or ends the search
    for (int32_t phase = 1; phase <= n + 1; ++phase) {
        launch_fill_i32(cnt, 0, 64, s);
        launch_match_roots(n, p, root, found, roots, cnt, s);
        int32_t h[2] = {0, 0};
        if (hipMemcpyAsync(h, cnt, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            return done(fail(RSAI_E_HIP, "transversal: root count readback failed"));
        const int64_t nroots = h[0];
        if (nroots == 0) break;  // every column is matched
        // level-synchronous search: level 0 is the list of roots
        const int32_t *fin = roots;
        const int32_t *nin = cnt;
        int64_t nin_h = nroots;
        for (int lev = 0; nin_h > 0; ++lev) {
            int32_t *fout = (lev % 2 == 0) ? fa : fb;
            int32_t *nout = cnt + 2 + (lev % 2);
            launch_fill_i32(nout, 0, 1, s);
            launch_match_expand(n, A->colptr, A->rowidx, phase, visited, parent, root, found, match_row, fin, nin,
                                fout, nout, nin_h, s);
            int32_t hn = 0;
            if (hipMemcpyAsync(&hn, nout, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return done(fail(RSAI_E_HIP, "transversal: frontier readback failed"));
            fin = fout;
            nin = nout;
            nin_h = hn;
        }
        launch_match_augment(roots, cnt, nroots, found, parent, p, match_row, cnt + 1, s);
        if (hipMemcpyAsync(h, cnt, 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            return done(fail(RSAI_E_HIP, "transversal: augmentation readback failed"));
        if (h[1] == 0) break;  // no augmenting path left: the matching is maximum
    }
    unsigned long long *sz = (unsigned long long *)al(8);
    if (st != RSAI_OK) return done(st);
    launch_fill_i64((int64_t *)sz, 0, 1, s);
    launch_match_count(n, p, sz, s);
    unsigned long long hs = 0;
    if (hipMemcpyAsync(&hs, sz, 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return done(fail(RSAI_E_HIP, "transversal: size readback failed"));
    if (hipGetLastError() != hipSuccess) return done(fail(RSAI_E_HIP, "transversal: launch failed"));
    *size = (int64_t)hs;
    return done(RSAI_OK);
}

rsai_status rsai_permute_rows(const rsai_csc *A, const int32_t *p, int64_t *colptrB, int32_t *rowidxB, double *valB,
                              void *stream) {
    if (!A || !A->colptr || !A->rowidx || !A->val || !p || !colptrB || !rowidxB || !valB)
        return fail(RSAI_E_ARG, "NULL argument");
    if (A->n < 1 || A->n > INT32_MAX - 1 || A->nnz < 0 || A->nnz > INT32_MAX) return fail(RSAI_E_ARG, "bad sizes");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = A->n;
    int32_t *inv = (int32_t *)dev_alloc(4 * (size_t)n + 256, s);
    if (!inv) return fail(RSAI_E_NOMEM, "allocation failed");
    int32_t *err = inv + ((n + 63) / 64) * 64;
    int32_t herr[2] = {0, 0};
    launch_fill_i32(inv, -1, n, s);
    launch_fill_i32(err, 0, 2, s);
    launch_validate(n, A->nnz, A->colptr, A->rowidx, err + 1, s);
    launch_perm_invert(n, p, inv, err, s);
    rsai_status st = RSAI_OK;
    if (hipMemcpyAsync(herr, err, 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        st = fail(RSAI_E_HIP, "permutation check readback failed");
    else if (herr[1])
        st = fail(RSAI_E_CSC, "malformed CSC (flags %d: 1 colptr, 2 row indices, 4 empty column)", herr[1]);
    else if (herr[0])
        st = fail(RSAI_E_ARG, "p is not a permutation of 0..n-1 (the transversal was not of full size?)");
    if (st == RSAI_OK) {
        launch_perm_rows(n, A->nnz, A->colptr, A->rowidx, A->val, inv, colptrB, rowidxB, valB, s);
        // rows ascending in every column: the segment sort of the row formation
        launch_sort_rows(n, colptrB, rowidxB, valB, s);
        if (hipGetLastError() != hipSuccess) st = fail(RSAI_E_HIP, "permutation launch failed");
    }
    dev_free(inv, s);
    return st;
}

rsai_status rsai_backward(rsai_plan *P, int32_t mat, const double *dM_val, double w_frob, double *dA_val,
                          void *stream) {
    int64_t nz = 0;
    rsai_status st = rsai_plan_nnz(P, mat, &nz);
    if (st != RSAI_OK) return st;
    if (!dA_val) return fail(RSAI_E_ARG, "dA_val is NULL");
    MatPlan &M = P->mats[mat];
    hipStream_t s = (hipStream_t)stream;
    const int64_t *foff = P->out.foff ? P->out.foff + M.col_base : nullptr;
    if (M.maxq < 0) {
        // largest |J_k|; for the columns without a kept factor their largest |I_k|,
        // count and largest |J_k|; columns with a factor and |J_k| > 32
        int32_t *d2 = P->alloc<int32_t>(5 * MAX2_COPIES, st);
        if (st != RSAI_OK) return st;
        int32_t hc[5 * MAX2_COPIES] = {}, h2[5];
        launch_fill_i32(d2, 0, 5 * MAX2_COPIES, P->stream);
        launch_max2(M.A.n, P->out.nJ + M.col_base, P->out.nI + M.col_base, foff, d2, P->stream);
        HIPCHK(hipMemcpyAsync(hc, d2, sizeof(hc), hipMemcpyDeviceToHost, P->stream));
        HIPCHK(hipStreamSynchronize(P->stream));
        max2_combine(hc, h2);
        M.maxq = h2[0];
        M.maxm = h2[1];
        M.nofac = h2[2];
        M.maxq_nofac = h2[3];
        M.nlarge = h2[4];
    }
    // columns on a kept factor: |J_k| <= 128 (every column the build can produce)
    if (M.maxq > backward_factored_max_cols())
        return fail(RSAI_E_CAP, "adjoint supports |J_k| <= %d; this M has %d", backward_factored_max_cols(), M.maxq);
    BwdArgs a{};
    a.mats = P->d_mats;
    a.mat = mat;
    a.n = M.A.n;
    a.Mcolptr = M.colptrM;
    a.Mrowidx = M.rowidxM;
    a.Mval = M.valM;
    a.gM = dM_val;
    a.w_frob = w_frob;
    a.dA = dA_val;
    a.err = P->err;
    a.fac = P->out.fac;
    a.foff = foff;
    // columns without a kept factor beyond the refactorising kernel's block: their
    // factor is recomputed into a temporary store (one host read for its size)
    const bool recompute = M.nofac > 0 && (M.maxq_nofac > backward_max_cols() || M.maxm > backward_max_rows());
    std::vector<void *> tmp;
    auto release = [&]() {
        for (void *q : tmp) dev_free(q, s);
        tmp.clear();
    };
    int64_t *tfoff = nullptr, *mask = nullptr;
    double *tfac = nullptr;
    if (recompute) {
        const int64_t n = M.A.n;
        auto al = [&](size_t bytes) -> void * {
            void *q = dev_alloc(std::max<size_t>(bytes, 8), s);
            if (q) tmp.push_back(q);
            return q;
        };
        unsigned long long *cur = (unsigned long long *)al(32);  // cursor, size, error flags
        tfoff = (int64_t *)al(8 * (size_t)n);
        mask = (int64_t *)al(8 * (size_t)n);
        if (!cur || !tfoff || !mask) {
            release();
            return fail(RSAI_E_NOMEM, "adjoint work buffers");
        }
        RefArgs r{};
        r.mats = P->d_mats;
        r.mat = mat;
        r.n = n;
        r.Mcolptr = M.colptrM;
        r.Mrowidx = M.rowidxM;
        r.nI = P->out.nI + M.col_base;
        r.foff = foff;
        r.small_cols = backward_max_cols();
        r.small_rows = backward_max_rows();
        r.cur = cur;
        r.tfoff = tfoff;
        r.err = (int32_t *)(cur + 2);
        launch_fill_i64((int64_t *)cur, 0, 4, s);
        launch_refactor_size(r, cur + 1, s);
        unsigned long long need = 0;
        if (hipMemcpyAsync(&need, cur + 1, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            release();
            return fail(RSAI_E_HIP, "adjoint: size readback failed");
        }
        tfac = (double *)al(8 * (size_t)std::max<unsigned long long>(need, 1));
        if (!tfac) {
            release();
            return fail(RSAI_E_NOMEM, "recomputed factor store (%llu doubles)", need);
        }
        r.fac = tfac;
        r.cap = (int64_t)need;
        launch_fill_i64(tfoff, -1, n, s);
        launch_refactor(r, device_cus(), s);
        launch_merge_masks(n, foff, tfoff, mask, s);
        int32_t ferr = 0;
        if (hipMemcpyAsync(&ferr, r.err, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            release();
            return fail(RSAI_E_HIP, "adjoint: factor recomputation failed");
        }
        if (ferr) {
            release();
            return fail(ferr & 32 ? RSAI_E_SINGULAR : RSAI_E_STATE,
                        "adjoint: recomputing a column's factor failed (flags %d: 32 A_k^T A_k not positive "
                        "definite, 64 store too small); nothing was accumulated", ferr);
        }
    }
    // fixed-order mode: a slot per contribution (one host read for their number)
    unsigned long long *ccur = nullptr;
    unsigned long long *ck2 = nullptr;
    double *cv2 = nullptr;
    void *ctemp = nullptr;
    size_t ctemp_bytes = 0;
    if (P->p.deterministic) {
        auto al = [&](size_t bytes) -> void * {
            void *q = dev_alloc(std::max<size_t>(bytes, 8), s);
            if (q) tmp.push_back(q);
            return q;
        };
        ccur = (unsigned long long *)al(16);
        if (!ccur) {
            release();
            return fail(RSAI_E_NOMEM, "adjoint work buffers");
        }
        launch_fill_i64((int64_t *)ccur, 0, 2, s);
        launch_contrib_count(P->d_mats, mat, M.A.n, M.colptrM, M.rowidxM, ccur + 1, s);
        unsigned long long cnt = 0;
        if (hipMemcpyAsync(&cnt, ccur + 1, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            release();
            return fail(RSAI_E_HIP, "adjoint: contribution count readback failed");
        }
        if (cnt > (unsigned long long)INT32_MAX) {
            release();
            return fail(RSAI_E_CAP, "fixed-order adjoint: %llu contributions exceed 2^31", cnt);
        }
        ctemp_bytes = det_reduce_bytes((int64_t)cnt);
        a.ckey = (unsigned long long *)al(8 * (size_t)cnt);
        a.cval = (double *)al(8 * (size_t)cnt);
        ck2 = (unsigned long long *)al(8 * (size_t)cnt);
        cv2 = (double *)al(8 * (size_t)cnt);
        ctemp = al(ctemp_bytes);
        if (!a.ckey || !a.cval || !ck2 || !cv2 || !ctemp) {
            release();
            return fail(RSAI_E_NOMEM, "fixed-order adjoint buffers (%llu contributions)", cnt);
        }
        a.ccur = ccur;
        a.ccap = (int64_t)cnt;
    }
    P->record(5, s);
    if (foff) launch_backward_factored(a, device_cus(), M.nlarge > 0, s);
    if (recompute) {
        BwdArgs b = a;
        b.fac = tfac;
        b.foff = tfoff;
        launch_backward_factored(b, device_cus(), M.maxq_nofac > backward_max_cols(), s);
        b.foff = mask;  // the rest of the columns without a kept factor
        launch_backward(b, device_cus() * 8, s);
    } else if (!foff || M.nofac > 0) {
        launch_backward(a, device_cus() * 8, s);
    }
    if (P->p.deterministic) {
        // the appended contributions, sorted by (entry, column), summed per entry
        unsigned long long used = 0;
        if (hipMemcpyAsync(&used, ccur, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            release();
            return fail(RSAI_E_HIP, "adjoint: contribution readback failed");
        }
        if (used > (unsigned long long)a.ccap) {
            release();
            return fail(RSAI_E_STATE, "fixed-order adjoint: %llu contributions for %lld slots", used,
                        (long long)a.ccap);
        }
        if (det_reduce(a.ckey, a.cval, ck2, cv2, (int64_t)used, ctemp, ctemp_bytes, dA_val, s) != hipSuccess) {
            release();
            return fail(RSAI_E_HIP, "fixed-order adjoint: sort or sum failed");
        }
    }
    P->record(6, s);
    const hipError_t le = hipGetLastError();
    // stream-ordered release: the kernels queued on s still read these buffers
    for (void *q : tmp) dev_free(q, s);
    tmp.clear();
    if (le != hipSuccess) return fail(RSAI_E_HIP, "adjoint launch failed: %s", hipGetErrorString(le));
    return RSAI_OK;
}

rsai_status rsai_plan_timing(const rsai_plan *P, double *ms, int32_t n) {
    if (!P || !ms) return fail(RSAI_E_ARG, "NULL argument");
    if (!P->have_events) return fail(RSAI_E_STATE, "plan was built without timing");
    HIPCHK(hipStreamSynchronize(P->stream));
    auto el = [&](int a, int b) {
        float t = 0.f;
        if (!P->recorded[a] || !P->recorded[b]) return -1.0;
        if (hipEventElapsedTime(&t, P->ev[a], P->ev[b]) != hipSuccess) return -1.0;
        return (double)t;
    };
    double v[6] = {el(0, 1), el(1, 2), el(2, 3), el(3, 4), el(0, 4), el(5, 6)};
    for (int i = 0; i < n && i < 6; ++i) ms[i] = v[i];
    return RSAI_OK;
}

rsai_status rsai_peak_fp64(int64_t iters, double *tflops, void *stream) {
    if (!tflops || iters < 16) return fail(RSAI_E_ARG, "tflops must be non-NULL and iters >= 16");
    *tflops = 0.0;
    hipStream_t s = (hipStream_t)stream;
    const int blocks = device_cus() * 16;  // 16 waves per CU
    double *out = (double *)dev_alloc(sizeof(double) * (size_t)blocks, s);
    if (!out) return fail(RSAI_E_NOMEM, "probe output (%d doubles)", blocks);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rsai_status st = RSAI_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        st = fail(RSAI_E_HIP, "hipEventCreate failed");
    } else {
        launch_fma_probe(blocks, iters / 16, out, s);  // warm-up
        float ms = 0.f;
        if (hipEventRecord(e0, s) != hipSuccess) st = fail(RSAI_E_HIP, "hipEventRecord failed");
        if (st == RSAI_OK) {
            launch_fma_probe(blocks, iters, out, s);
            if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.f)
                st = fail(RSAI_E_HIP, "FMA probe launch or timing failed");
        }
        if (st == RSAI_OK) {
            const double flops = 2.0 * fma_probe_chains() * (double)iters * (double)blocks * 256.0;
            *tflops = flops / ((double)ms * 1e-3) / 1e12;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dev_free(out, s);
    return st;
}

rsai_status rsai_destroy(rsai_plan *P) {
    if (!P) return RSAI_OK;
    P->release();
    delete P;
    return RSAI_OK;
}

}  // extern "C"
