// Device-side shared definitions of the RSAI(tol) kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsai {

// ----------------------------------------------------------------- per-build data

struct MatDev {              // one matrix of a (possibly batched) build
    int64_t n;
    const int64_t *colptr;   // CSC of A (borrowed)
    const int32_t *rowidx;
    const double *val;
    const int64_t *rowptr;   // row pattern of A (transpose), built by the library
    const int32_t *colidx;
    const unsigned long long *norm1_bits;  // ||A||_1 (max column absolute sum, eq. (4.3)) as bits
    int64_t col_base;        // global id of the matrix's first column in the batch
};

struct BuildParams {
    int c, lmax, drop;
    double eps, tol;
};

enum : int { DROP_NONE = 0, DROP_FIXED = 1, DROP_ADAPTIVE = 2 };
enum : int { ST_OK = 0, ST_SINGULAR = 3, ST_CAP = 6, ST_INTERNAL = 7 };
// error flags on which the size-class kernels process nothing: the CSC contract failed
// (1, 2, 4) or a single-pass scan found its state not zeroed (64)
constexpr int ERR_SKIP = 7 | 64;

constexpr int CMAX = 8;      // largest c supported (dominant rows per loop)

struct ColOut {              // per global column
    int64_t *off;            // arena offset of the column's result
    int32_t *nJ, *nI, *loops, *status;
    double *resnorm, *flops;
    int32_t *arenaJ;         // arena of J lists (global column ids, solve order)
    double *arenaV;          // arena of values
    // R factors of the final solves, kept for the adjoint (fac == nullptr: not kept).
    // Record of a column at foff[col] (-1: not stored): J in solve order (q values),
    // then the upper triangle of R row by row (row i: R(i, i..q-1)).
    double *fac;
    unsigned long long *fac_cur;  // doubles handed out so far
    int64_t fac_cap;
    int64_t *foff;
    int32_t fac_chunk;            // doubles a wave takes from the store at a time
};

// Reserve a factor record of q columns; -1 when the arena is full (the adjoint then
// refactorises that column).
__device__ __forceinline__ long long fac_reserve(const ColOut &o, int q) {
    const unsigned long long need = (unsigned long long)(q + q * (q + 1) / 2);
    const unsigned long long at = atomicAdd(o.fac_cur, need);
    return (at + need <= (unsigned long long)o.fac_cap) ? (long long)at : -1LL;
}
// A wave's current chunk of the factor store (LDS).
struct FacChunk {
    long long base;  // store offset of the chunk, -1: none
    int used, len;   // doubles handed out from it, its length
};
__device__ __forceinline__ void fac_chunk_init(FacChunk &W) {
    if (threadIdx.x == 0) {
        W.base = -1;
        W.used = 0;
        W.len = 0;
    }
}
__host__ __device__ inline int64_t fac_row(int q, int i) { return q + (int64_t)i * q - (int64_t)i * (i - 1) / 2; }

// ----------------------------------------------------------------- DPP helpers
// Data-parallel-primitive lane moves within a 16-lane row. Patterns used:
//   0xB1 quad_perm [1,0,3,2] (xor 1), 0x4E quad_perm [2,3,0,1] (xor 2),
//   0x141 row_half_mirror (i <-> 7-i in each 8), 0x140 row_mirror (i <-> 15-i).
// Each pairs lane i with a lane of the other half of its aligned 2/4/8/16-group,
// so applying them in order all-reduces over aligned groups of G <= 16 lanes, and
// every lane of a group ends with the bitwise-identical result (a+b == b+a).

// Every lane reads a lane of its own row under these patterns and all rows and banks
// are enabled, so no lane keeps its old value: the move needs no initialised
// destination (one instruction per 32-bit word instead of two).
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int x) {
    return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    long long b = __double_as_longlong(x);
    int lo = (int)(b & 0xffffffffLL);
    int hi = (int)(b >> 32);
    lo = dpp_i32<CTRL>(lo);
    hi = dpp_i32<CTRL>(hi);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Groups of 32 and 64 lanes add one and two cross-row steps: v_permlane16_swap
// (gfx950) called with the same register as both operands leaves, in every lane of an
// aligned pair of 16-lane rows, the value of the even row in the first result and the
// value of the odd row in the second; v_permlane32_swap does the same for the two
// 32-lane halves. Adding the two results in that order gives every lane of the group
// the bitwise-identical sum.
__device__ __forceinline__ void xrow16_i32(int x, int &a, int &b) {
    const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    a = (int)p[0];
    b = (int)p[1];
}
__device__ __forceinline__ void xrow32_i32(int x, int &a, int &b) {
    const auto p = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    a = (int)p[0];
    b = (int)p[1];
}
template <int W>
__device__ __forceinline__ void xrow_f64(double x, double &a, double &b) {
    const long long v = __double_as_longlong(x);
    int alo, ahi, blo, bhi;
    if constexpr (W == 16) {
        xrow16_i32((int)(v & 0xffffffffLL), alo, blo);
        xrow16_i32((int)(v >> 32), ahi, bhi);
    } else {
        xrow32_i32((int)(v & 0xffffffffLL), alo, blo);
        xrow32_i32((int)(v >> 32), ahi, bhi);
    }
    a = __longlong_as_double(((long long)ahi << 32) | (long long)(unsigned)alo);
    b = __longlong_as_double(((long long)bhi << 32) | (long long)(unsigned)blo);
}

template <int G>
__device__ __forceinline__ double gsum(double x) {
    static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16 || G == 32 || G == 64, "group size");
    if constexpr (G >= 2) x = x + dpp_f64<0xB1>(x);
    if constexpr (G >= 4) x = x + dpp_f64<0x4E>(x);
    if constexpr (G >= 8) x = x + dpp_f64<0x141>(x);
    if constexpr (G >= 16) x = x + dpp_f64<0x140>(x);
    if constexpr (G >= 32) {
        double a, b;
        xrow_f64<16>(x, a, b);
        x = a + b;
    }
    if constexpr (G >= 64) {
        double a, b;
        xrow_f64<32>(x, a, b);
        x = a + b;
    }
    return x;
}

template <int G>
__device__ __forceinline__ int gsum_i(int x) {
    if constexpr (G >= 2) x = x + dpp_i32<0xB1>(x);
    if constexpr (G >= 4) x = x + dpp_i32<0x4E>(x);
    if constexpr (G >= 8) x = x + dpp_i32<0x141>(x);
    if constexpr (G >= 16) x = x + dpp_i32<0x140>(x);
    if constexpr (G >= 32) {
        int a, b;
        xrow16_i32(x, a, b);
        x = a + b;
    }
    if constexpr (G >= 64) {
        int a, b;
        xrow32_i32(x, a, b);
        x = a + b;
    }
    return x;
}

template <int G>
__device__ __forceinline__ int gmax_i(int x) {
    if constexpr (G >= 2) x = max(x, dpp_i32<0xB1>(x));
    if constexpr (G >= 4) x = max(x, dpp_i32<0x4E>(x));
    if constexpr (G >= 8) x = max(x, dpp_i32<0x141>(x));
    if constexpr (G >= 16) x = max(x, dpp_i32<0x140>(x));
    if constexpr (G >= 32) {
        int a, b;
        xrow16_i32(x, a, b);
        x = max(a, b);
    }
    if constexpr (G >= 64) {
        int a, b;
        xrow32_i32(x, a, b);
        x = max(a, b);
    }
    return x;
}

template <int CTRL>
__device__ __forceinline__ void amax_step(double &a, int &g) {
    double a2 = dpp_f64<CTRL>(a);
    int g2 = dpp_i32<CTRL>(g);
    bool take = (a2 > a) || (a2 == a && g2 < g);
    a = take ? a2 : a;
    g = take ? g2 : g;
}
template <int W>
__device__ __forceinline__ void amax_xrow(double &a, int &g) {
    double a0, a1;
    int g0, g1;
    xrow_f64<W>(a, a0, a1);
    if constexpr (W == 16) xrow16_i32(g, g0, g1); else xrow32_i32(g, g0, g1);
    const bool take1 = (a1 > a0) || (a1 == a0 && g1 < g0);
    a = take1 ? a1 : a0;
    g = take1 ? g1 : g0;
}

// Group arg-max with key (a descending, g ascending): the dominant-row order with
// ties going to the smaller global row index.
template <int G>
__device__ __forceinline__ void gargmax(double &a, int &g) {
    if constexpr (G >= 2) amax_step<0xB1>(a, g);
    if constexpr (G >= 4) amax_step<0x4E>(a, g);
    if constexpr (G >= 8) amax_step<0x141>(a, g);
    if constexpr (G >= 16) amax_step<0x140>(a, g);
    if constexpr (G >= 32) amax_xrow<16>(a, g);
    if constexpr (G >= 64) amax_xrow<32>(a, g);
}

// Value of x held by group lane `src` (others contribute exact zeros).
template <int G>
__device__ __forceinline__ double gbcast(double x, bool is_src) {
    return gsum<G>(is_src ? x : 0.0);
}
template <int G>
__device__ __forceinline__ int gbcast_i(int x, bool is_src) {
    return gsum_i<G>(is_src ? x : 0);
}

// Wave-wide max of an int (all 64 lanes): row reduction then 4 lane reads.
__device__ __forceinline__ int wave_max_i(int x) {
    x = gmax_i<16>(x);
    int a = __builtin_amdgcn_readlane(x, 0);
    int b = __builtin_amdgcn_readlane(x, 16);
    int c = __builtin_amdgcn_readlane(x, 32);
    int d = __builtin_amdgcn_readlane(x, 48);
    return max(max(a, b), max(c, d));
}

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0; }

// Synchronisation point of a single-wave workgroup. The LDS executes one wave's
// instructions in order, so lanes see each other's earlier LDS writes; the fences
// only stop the compiler from moving memory accesses across this point. Unlike
// __syncthreads() it does not wait for outstanding global loads.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ bool wave_all(bool p) { return __ballot(!p) == 0; }

// Factor records for the active lanes of a wave: every lane with need > 0 gets need
// consecutive doubles of the wave's chunk (lanes in ascending order). A chunk that
// cannot hold them all is replaced by a fresh one, taken from the store with a single
// atomic (the rest of the old one stays unused), so the finishing columns of a wave
// do not each wait on a contended device-wide atomic. -1 when the store is full.
template <class O>  // ColOut, in any address space
__device__ __forceinline__ long long fac_take(const O &o, FacChunk &W, int need) {
    const int lane = (int)__lane_id();
    const unsigned long long lm = __ballot(need > 0);
    if (lm == 0ull) return -1LL;
    int pre = 0, total = 0;
    for (unsigned long long mm = lm; mm != 0ull; mm &= mm - 1ull) {
        const int src = __builtin_ctzll(mm);
        const int nl = __shfl(need, src);
        if (src < lane) pre += nl;
        total += nl;
    }
    const int first = __builtin_ctzll(__ballot(1));
    wave_sync();
    long long base = W.base;
    int used = W.used, len = W.len;
    if (used + total > len) {
        int blo = -1, bhi = -1, nl = 0;
        if (lane == first) {
            const int want = o.fac_chunk > total ? o.fac_chunk : total;
            const unsigned long long at = atomicAdd(o.fac_cur, (unsigned long long)want);
            const unsigned long long cap = (unsigned long long)o.fac_cap;
            if (at < cap) {
                blo = (int)(at & 0xffffffffull);
                bhi = (int)(at >> 32);
                nl = (int)((cap - at) < (unsigned long long)want ? (cap - at) : (unsigned long long)want);
            }
        }
        blo = __shfl(blo, first);
        bhi = __shfl(bhi, first);
        len = __shfl(nl, first);
        base = (bhi < 0) ? -1LL : (((long long)bhi << 32) | (long long)(unsigned)blo);
        used = 0;
    }
    const long long fo = (need > 0 && base >= 0 && used + pre + need <= len) ? base + used + pre : -1LL;
    wave_sync();
    if (lane == first) {
        W.base = base;
        W.used = (used + total < len) ? used + total : len;
        W.len = len;
    }
    wave_sync();
    return fo;
}

// ----------------------------------------------------------------- LDS hash sets
// Open addressing with linear probing, keys are global indices (>= 0), EMPTY = -1.
// Callers keep the load below the table size so that probing always ends.

constexpr int HEMPTY = -1;

template <int LOGHS>
__device__ __forceinline__ unsigned hslot(int key) {
    return ((unsigned)key * 0x9E3779B1u) >> (32 - LOGHS);
}

// Insert key; returns true if it was not present. slot receives its position.
template <int LOGHS>
__device__ __forceinline__ bool hinsert(int *hk, int key, int &slot) {
    constexpr unsigned MASK = (1u << LOGHS) - 1u;
    unsigned h = hslot<LOGHS>(key);
    // first probe straight-line (the usual case at the load factors used here), the
    // probing loop only after a collision
    int old = atomicCAS(&hk[h], HEMPTY, key);
    if (old == HEMPTY || old == key) {
        slot = (int)h;
        return old == HEMPTY;
    }
    for (int probe = 1; probe < (1 << LOGHS); ++probe) {
        h = (h + 1u) & MASK;
        old = atomicCAS(&hk[h], HEMPTY, key);
        if (old == HEMPTY) { slot = (int)h; return true; }
        if (old == key) { slot = (int)h; return false; }
    }
    slot = -1;  // table full: callers size tables so this cannot happen
    return false;
}

// Slot of key, or -1.
template <int LOGHS>
__device__ __forceinline__ int hfind(const int *hk, int key) {
    constexpr unsigned MASK = (1u << LOGHS) - 1u;
    unsigned h = hslot<LOGHS>(key);
    int v = hk[h];  // first probe straight-line, as in hinsert
    if (v == key) return (int)h;
    if (v == HEMPTY) return -1;
    for (int probe = 1; probe < (1 << LOGHS); ++probe) {
        h = (h + 1u) & MASK;
        v = hk[h];
        if (v == key) return (int)h;
        if (v == HEMPTY) return -1;
    }
    return -1;
}

constexpr int ilog2ceil(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

// Algorithmic flops of one Householder-update LS solve (Algorithm 1, step 7): the
// factor of the first qlo columns was formed on m0 rows and is kept; the block now
// has m rows and qn columns. The rows added since are zero in the old columns, so
// stored reflector j < qlo updates the qn - qlo new columns over rows j..m0-1 only
// (4 (m0 - j) per column); reflectors qlo..qn-1 cost their norm 2 (m - j) and
// 4 (m - j) for each later column and for Q^T e; then back substitution (qn^2) and
// the residual norm ||(Q^T e)(qn:m)|| (2 (m - qn)). qlo = 0: from scratch.
__host__ __device__ inline double solve_flops(int m0, int m, int qlo, int qn) {
    double f = 0.0;
    double p = (double)(qn - qlo);
    // sum_{j<qlo} 4 (m0-j) p
    f += 4.0 * p * ((double)qlo * m0 - 0.5 * (double)qlo * (qlo - 1));
    for (int j = qlo; j < qn; ++j) {
        double mj = (double)(m - j);
        f += mj * (2.0 + 4.0 * (double)(qn - j - 1) + 4.0);
    }
    f += (double)qn * qn + 2.0 * (double)(m - qn);
    return f;
}

}  // namespace rsai
