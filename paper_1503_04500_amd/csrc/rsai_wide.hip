// Sparse-block size class of the RSAI(tol) build: one 256-thread workgroup per
// column, for LS blocks A(I_k, J_k) that outgrow the register tiers but are mostly
// structurally empty (long sparse columns with few rows in common, as in matrices
// with power-law column lengths). Up to 8192 rows and WIDE_QMAX columns.
//
// The LS problem (2.3) is solved on an orthogonally equivalent compressed block.
// A row of I_k met by exactly one column j of J_k (a private row of j) adds to
// column j only; an orthogonal transformation of the private rows of j turns them
// into one row holding their 2-norm s_j, and the part of e_k on them into
// a_kj / s_j on that row (when k is one of them) plus a constant part
// (s_j^2 - a_kj^2) / s_j^2 of ||r||^2 that no choice of m_k can reduce. The rows
// met by two or more columns (shared rows) stay as they are. Householder QR of the
// (shared + |J_k|) x |J_k| block then gives m_k and ||A m_k - e_k||.
//
// Everything else follows the register tiers step for step (Algorithm 1 with the
// dropping of Section 4): I_k is an LDS hash set whose entries carry the number of
// columns of J_k that hold the row and a flag for rows already used as dominant
// rows; the residual for step 4 is formed from the sparse columns with the columns
// taken in ascending global order, so exact ties reach the smaller-index rule.
// Columns arrive as spill records of the previous class. A column whose |I_k| or
// compressed block outgrows this class moves on to the next one.
#include <climits>
#include <type_traits>

#include "rsai_kernels.h"

namespace rsai {

namespace {
constexpr int NT = 256;                 // threads per column
constexpr int NW = NT / 64;             // waves
constexpr int QM = WIDE_QMAX;
constexpr int LOGHJ = 8;                // column hash: 256 slots
constexpr int HJ = 1 << LOGHJ;

// Three instances: rows of I up to 1024 (2048-slot row hash, four workgroups per CU),
// up to 2048 (three per CU) and up to 8192 (one per CU, larger compressed blocks).
//   BLK  doubles of the compressed block, (S + q) x (q + 1), row-major
//   SHV  doubles of the shared rows' values, S x q
//   SMAX shared rows
template <int LOGH, int BLK, int SHV, int SMAX>
struct WLds {
    static constexpr int HS = 1 << LOGH;
    int hk[HS];             // row keys
    unsigned hv[HS / 4];    // one byte per slot: bits 0-6 columns of J holding the row, bit 7 row in R
    int hJ[HJ];             // J as a set
    double blk[BLK];
    double shv[SHV];
    double s2[64];          // private rows of each column: sum of squares
    double mt[64], rd[64];  // solution by slot, diagonal of R
    int64_t cb[64];         // first entry of each column of J
    int clen[64];
    int Jl[64];             // J, slot order
    int ord[64];            // slots in ascending column order
    int srow[SMAX];         // shared rows, ascending
    unsigned long long shm[SMAX];  // columns (slots) of J holding each shared row
    int stmp[SMAX];
    int slist[SMAX];        // rows whose holder count reached 2 since the last scan, plus
                            // the shared rows of that scan (slovf: the list overflowed)
    int newc[64];           // columns of J-hat
    int Rh[CMAX];           // pending dominant rows
    double cva[NW];
    int cvg[NW];
    double akv;             // a_kj when k is a private row of column slot kcol
    int kcol;
    int cnt, nsh, flag, nsl, slovf, nsh2;
    double rn;
};

template <class L>
__device__ __forceinline__ unsigned hget(const L &S, int sl) {
    return (S.hv[sl >> 2] >> ((sl & 3) * 8)) & 0xFFu;
}
// one more column holds the row of slot sl; a row that becomes shared (two holders)
// joins the candidate list of the next shared-row scan
template <class L>
__device__ __forceinline__ void hinc(L &S, int sl, int row) {
    const unsigned old = atomicAdd(&S.hv[sl >> 2], 1u << ((sl & 3) * 8));
    if (((old >> ((sl & 3) * 8)) & 0x7Fu) == 1u) {
        const int ps = atomicAdd(&S.nsl, 1);
        if (ps < (int)(sizeof(S.slist) / sizeof(int))) S.slist[ps] = row; else S.slovf = 1;
    }
}
template <class L>
__device__ __forceinline__ void hdec(L &S, int sl) { atomicSub(&S.hv[sl >> 2], 1u << ((sl & 3) * 8)); }
template <class L>
__device__ __forceinline__ void hsetR(L &S, int sl) { atomicOr(&S.hv[sl >> 2], 0x80u << ((sl & 3) * 8)); }

// wave-wide sum; every lane gets the bitwise-same value
__device__ __forceinline__ double wsum(double x) {
    x = gsum<16>(x);
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    return x;
}

__device__ __forceinline__ double readlane_f64(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// (a desc, g asc) order of dominant-row candidates
__device__ __forceinline__ bool better(double a, int g, double b, int h) { return a > b || (a == b && g < h); }

// index of row in the ascending shared-row list, or -1
__device__ __forceinline__ int sfind(const int *srow, int nsh, int row) {
    int lo = 0, hi = nsh - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = srow[mid];
        if (v == row) return mid;
        if (v < row) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}
// Visit every entry of the columns c0 + wid + NW*s (below c1) of J with the lanes of
// one wave, one column after another: f(c, row, val) for each entry, then done(c).
// The first 64 entries of the next HB columns are loaded together ahead of use; the
// loop over columns stays rolled to keep the code small.
// Columns for which want(c) is false are skipped without loading their entries.
template <bool VAL, class L, class F, class D, class W>
__device__ __forceinline__ void wave_cols_if(const L &S, const MatDev &A, int c0, int c1, int wid, int lane, F &&f,
                                             D &&done, W &&want) {
    constexpr int HB = 8;
    for (int cb0 = c0 + wid; cb0 < c1; cb0 += NW * HB) {
        int rr[HB];
        double vv[HB];
#pragma unroll
        for (int s = 0; s < HB; ++s) {
            const int c = cb0 + NW * s;
            rr[s] = -1;
            vv[s] = 0.0;
            if (c < c1 && lane < S.clen[c] && want(c)) {
                const int64_t e = S.cb[c] + lane;
                rr[s] = A.rowidx[e];
                if (VAL) vv[s] = A.val[e];
            }
        }
#pragma unroll 1
        for (int s = 0; s < HB; ++s) {
            const int c = cb0 + NW * s;
            if (c >= c1) break;
            const int r0 = rr[0];
            const double v0 = vv[0];
#pragma unroll
            for (int t = 0; t < HB - 1; ++t) {
                rr[t] = rr[t + 1];
                vv[t] = vv[t + 1];
            }
            if (r0 >= 0) f(c, r0, v0);
            const int len = S.clen[c];
            if (len > 64 && want(c)) {
                const int64_t e0 = S.cb[c];
                for (int t = 64 + lane; t < len; t += 64) f(c, A.rowidx[e0 + t], VAL ? A.val[e0 + t] : 0.0);
            }
            done(c);
        }
    }
}
template <bool VAL, class L, class F, class D>
__device__ __forceinline__ void wave_cols(const L &S, const MatDev &A, int c0, int c1, int wid, int lane, F &&f,
                                          D &&done) {
    wave_cols_if<VAL>(S, A, c0, c1, wid, lane, f, done, [](int) { return true; });
}
}  // namespace

template <int LOGH, int BLK, int SHV, int SMAX, int WPC>
__global__ __launch_bounds__(NT, WPC) void wide_kernel(WideArgs args) {
    constexpr int HS = 1 << LOGH;
    constexpr int MM = HS / 2;  // row hash load at most one half
    __shared__ WLds<LOGH, BLK, SHV, SMAX> S;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (*args.err & ERR_SKIP) return;
    const BuildParams P = args.P;
    const int64_t Q = min((int64_t)(*args.rec_in_count), args.rec_in_cap);

    for (int64_t pos = blockIdx.x; pos < Q; pos += gridDim.x) {
        const int32_t *rec = args.rec_in + pos * (int64_t)args.rec_in_stride;
        const int ucol = rec[0], mat = rec[1], k = rec[2];
        int l = rec[3], q = rec[4], m = rec[5];
        const int nR0 = rec[6];
        int nRh = rec[7];
        double fl = __longlong_as_double(((long long)rec[9] << 32) | (long long)(unsigned)rec[8]);
        bool linc = (rec[10] & 1) != 0;
        const MatDev A = args.mats[mat];
        const int32_t *RJ = rec + RHDR, *RI = RJ + q, *RR = RI + m, *RHp = RR + nR0;
        int status = ST_OK;
        bool spill = false, pend = false, pend_drop = false;
        int pend_qmod = -1, pend_mmod = 0;
        int blk_nsh = -1;         // shared rows when the compressed block did not fit
        bool lookup_fail = false;
        double rn = 0.0;

        // ---------------------------------------------------------- state from the record
        for (int t = tid; t < HS; t += NT) S.hk[t] = HEMPTY;
        for (int t = tid; t < HS / 4; t += NT) S.hv[t] = 0u;
        for (int t = tid; t < HJ; t += NT) S.hJ[t] = HEMPTY;
        if (tid == 0) { S.flag = 0; S.nsl = 0; S.slovf = 0; }
        __syncthreads();
        if (q > QM || m > MM || nRh > CMAX) status = ST_CAP;  // larger than any register tier
        if (status == ST_OK) {
            for (int t = tid; t < q; t += NT) {
                const int col = RJ[t];
                S.Jl[t] = col;
                S.cb[t] = A.colptr[col];
                S.clen[t] = (int)(A.colptr[col + 1] - S.cb[t]);
                int sl;
                hinsert<LOGHJ>(S.hJ, col, sl);
            }
            for (int t = tid; t < m; t += NT) {
                int sl;
                hinsert<LOGH>(S.hk, RI[t], sl);
            }
            if (tid < nRh) S.Rh[tid] = RHp[tid];
        }
        __syncthreads();
        if (status == ST_OK) {
            // how many columns of J hold each row (every row of a column of J is in I)
            wave_cols<false>(
                S, A, 0, q, wid, lane,
                [&](int, int row, double) {
                    const int sl = hfind<LOGH>(S.hk, row);
                    if (sl >= 0) hinc(S, sl, row); else lookup_fail = true;
                },
                [](int) {});
            for (int t = tid; t < nR0; t += NT) {
                const int row = RR[t];
                const int sl = hfind<LOGH>(S.hk, row);
                if (sl >= 0) hsetR(S, sl);
                else if (row == k) S.flag = 1;  // k used as a dominant row while k is not in I
            }
        }
        __syncthreads();
        bool kR = S.flag != 0;
        __syncthreads();

        bool first = true, need_solve = true, dropok = false;
        int qmod = -1, mmod = 0;
        int p = 0;
        if (rec[10] & 2) {
            // augmented pattern handed over before its solve
            dropok = (rec[10] & 4) != 0;
            qmod = rec[11];
            mmod = rec[12];
        }
        if (status == ST_OK && q == 0 && nRh == 0) {
            // a column whose own rows exceed the register tiers: J = {k}, loop 0
            if (tid == 0) {
                S.Jl[0] = k;
                S.cb[0] = A.colptr[k];
                S.clen[0] = (int)(A.colptr[k + 1] - A.colptr[k]);
                int sl;
                hinsert<LOGHJ>(S.hJ, k, sl);
            }
            __syncthreads();
            p = 1;
            dropok = true;
            qmod = 0;
        }

        while (status == ST_OK && !spill) {
            // ================= J-hat: columns of the pending dominant rows not in J (step 5)
            if (nRh > 0) {
                if (linc) ++l;  // step 6
                linc = false;
                int64_t sb[CMAX];
                int sp[CMAX + 1];
                sp[0] = 0;
#pragma unroll
                for (int t = 0; t < CMAX; ++t) {
                    int64_t b0 = 0, e0 = 0;
                    if (t < nRh) {
                        const int rt = S.Rh[t];
                        b0 = A.rowptr[rt];
                        e0 = A.rowptr[rt + 1];
                    }
                    sb[t] = b0;
                    sp[t + 1] = sp[t] + (int)(e0 - b0);
                }
                if (tid == 0) S.cnt = 0;
                __syncthreads();
                bool ovf = false;
                for (int u = tid; u < sp[CMAX]; u += NT) {
                    int64_t b0 = sb[0];
                    int o0 = 0;
#pragma unroll
                    for (int t = 1; t < CMAX; ++t)
                        if (u >= sp[t]) { b0 = sb[t]; o0 = sp[t]; }
                    const int col = A.colidx[b0 + (u - o0)];
                    int sl;
                    if (hinsert<LOGHJ>(S.hJ, col, sl)) {
                        const int ps = atomicAdd(&S.cnt, 1);
                        if (q + ps < QM) S.newc[ps] = col; else ovf = true;
                    } else if (sl < 0) {
                        ovf = true;  // table full
                    }
                }
                if (__syncthreads_or(ovf)) { spill = true; break; }
                p = S.cnt;
                if (tid < p) {
                    const int key = S.newc[tid];
                    int rank = 0;
                    for (int t = 0; t < p; ++t) rank += (S.newc[t] < key) ? 1 : 0;
                    S.Jl[q + rank] = key;
                    S.cb[q + rank] = A.colptr[key];
                    S.clen[q + rank] = (int)(A.colptr[key + 1] - A.colptr[key]);
                }
                need_solve = !(p == 0 && !first);  // empty J-hat: the loop ends without a solve
                dropok = (p > 0);
                qmod = (p > 0) ? q : (first ? -1 : q);
                mmod = m;
                __syncthreads();
            }
            // ================= I-hat: rows of the new columns not in I (step 5)
            if (need_solve && p > 0) {
                int total = 0;
                for (int t = 0; t < p; ++t) total += S.clen[q + t];
                if (m + total > MM) { spill = true; break; }  // may outgrow the row hash
                if (tid == 0) S.cnt = 0;
                __syncthreads();
                int added = 0;
                wave_cols<false>(
                    S, A, q, q + p, wid, lane,
                    [&](int, int row, double) {
                        int sl;
                        if (hinsert<LOGH>(S.hk, row, sl)) ++added;
                        if (sl >= 0) hinc(S, sl, row); else lookup_fail = true;
                    },
                    [](int) {});
                if (added) atomicAdd(&S.cnt, added);
                __syncthreads();
                m += S.cnt;
                if (kR) {
                    // k entered I: its flag moves into the hash entry
                    const int sl = hfind<LOGH>(S.hk, k);
                    if (sl >= 0) {
                        if (tid == 0) hsetR(S, sl);
                        kR = false;
                    }
                }
                q += p;
                p = 0;
            }
            nRh = 0;  // pending rows consumed
            first = false;

            // ================= LS solve(s) on (I, J) (2.3): pass 0 the augmented pattern,
            // pass 1 the pattern kept after dropping (Section 4)
            // (after a drop, the drop step leaves the kept columns' compressed data in
            // LDS: shared rows, their values, private sums and the row of k; the re-solve
            // forms its block from them instead of gathering every column again)
            bool reuse_next = false;
            for (int pass = 0; pass < 2 && need_solve && status == ST_OK; ++pass) {
                const bool reuse = reuse_next;
                reuse_next = false;
                // ---- shared rows (held by two or more columns of J), ascending
                if (tid == 0) {
                    if (!reuse) { S.nsh = 0; S.kcol = -1; S.akv = 0.0; }
                    S.flag = 0;
                }
                __syncthreads();
                const bool slovf = S.slovf != 0;
                if (reuse) {
                    // (shared rows already known)
                } else if (slovf) {
                    for (int t = tid; t < HS; t += NT) {
                        const int key = S.hk[t];
                        if (key != HEMPTY && (hget(S, t) & 0x7Fu) >= 2u) {
                            const int ps = atomicAdd(&S.nsh, 1);
                            if (ps < SMAX) S.stmp[ps] = key;
                        }
                    }
                } else {
                    // every row with two or more holders is in the candidate list: it
                    // was shared at the last scan or reached two holders since
                    const int nl = S.nsl;
                    for (int t = tid; t < nl; t += NT) {
                        const int key = S.slist[t];
                        const int sl = hfind<LOGH>(S.hk, key);
                        if (sl >= 0 && (hget(S, sl) & 0x7Fu) >= 2u) {
                            const int ps = atomicAdd(&S.nsh, 1);
                            if (ps < SMAX) S.stmp[ps] = key;
                        }
                    }
                }
                __syncthreads();
                const int nsh = S.nsh;
                if (!reuse && !slovf && nsh <= SMAX) {
                    // the list keeps the shared rows only (no row enters it twice)
                    for (int t = tid; t < nsh; t += NT) S.slist[t] = S.stmp[t];
                    if (tid == 0) S.nsl = nsh;
                }
                const int ld = q + 1, mp = nsh + q;
                if (nsh > SMAX || nsh * q > SHV || mp * ld > BLK) {
                    // the compressed block does not fit: hand the unsolved pattern over
                    spill = true;
                    blk_nsh = nsh;
                    pend = true;
                    pend_drop = dropok && pass == 0;
                    pend_qmod = qmod;
                    pend_mmod = mmod;
                    break;
                }
                if (!reuse && tid < nsh) {
                    const int key = S.stmp[tid];
                    int rank = 0;
                    for (int t = 0; t < nsh; ++t) rank += (S.stmp[t] < key) ? 1 : 0;
                    S.srow[rank] = key;
                }
                for (int t = tid; t < mp * ld; t += NT) S.blk[t] = 0.0;
                if (!reuse) {
                    for (int t = tid; t < nsh * q; t += NT) S.shv[t] = 0.0;
                    for (int t = tid; t < nsh; t += NT) S.shm[t] = 0ull;
                }
                __syncthreads();
                if (reuse) {
                    // the kept shared values into the block
                    for (int t = tid; t < nsh * q; t += NT) {
                        const int si = t / q, c = t - si * q;
                        S.blk[(q + si) * ld + c] = S.shv[t];
                    }
                } else
                // ---- gather: shared entries into the block, private rows into column sums
                {
                    auto visit = [&](int c, int row, double v, double &a2) {
                        const int sl = hfind<LOGH>(S.hk, row);
                        const unsigned cn = sl >= 0 ? (hget(S, sl) & 0x7Fu) : 0u;
                        if (cn == 1u) {
                            a2 += v * v;
                            if (row == k) { S.kcol = c; S.akv = v; }
                        } else if (cn >= 2u) {
                            const int si = sfind(S.srow, nsh, row);
                            if (si >= 0) {
                                S.blk[(q + si) * ld + c] = v;
                                S.shv[si * q + c] = v;
                                atomicOr(&S.shm[si], 1ull << c);
                            } else {
                                lookup_fail = true;
                            }
                        } else {
                            lookup_fail = true;
                        }
                    };
                    // HB columns per wave at a time: entries loaded together, then the
                    // private rows' sums of squares of the HB columns reduced together
                    constexpr int HB = 8;
                    for (int cb0 = wid; cb0 < q; cb0 += NW * HB) {
                        int rr[HB];
                        double vv[HB], a2[HB];
#pragma unroll
                        for (int t = 0; t < HB; ++t) {
                            const int c = cb0 + NW * t;
                            rr[t] = -1;
                            vv[t] = 0.0;
                            if (c < q && lane < S.clen[c]) {
                                const int64_t e = S.cb[c] + lane;
                                rr[t] = A.rowidx[e];
                                vv[t] = A.val[e];
                            }
                        }
#pragma unroll
                        for (int t = 0; t < HB; ++t) {
                            const int c = cb0 + NW * t;
                            a2[t] = 0.0;
                            if (c < q) {
                                if (rr[t] >= 0) visit(c, rr[t], vv[t], a2[t]);
                                const int len = S.clen[c];
                                if (len > 64) {
                                    const int64_t e0 = S.cb[c];
                                    for (int u = 64 + lane; u < len; u += 64) visit(c, A.rowidx[e0 + u], A.val[e0 + u], a2[t]);
                                }
                            }
                        }
#pragma unroll
                        for (int t = 0; t < HB; ++t) {
                            const int c = cb0 + NW * t;
                            if (c < q) {
                                const double x = wsum(a2[t]);
                                if (lane == 0) S.s2[c] = x;
                            }
                        }
                    }
                }
                __syncthreads();
                // ---- the row of row k: shared (right-hand side 1), private (compressed), or
                // outside the pattern (a constant 1 in ||r||^2). Private in column j: the
                // collapsed row carries beta = a_kj / s_j and ||r||^2 gains 1 - beta^2.
                const int ksl = hfind<LOGH>(S.hk, k);
                const int kcn = ksl >= 0 ? (int)(hget(S, ksl) & 0x7Fu) : -1;
                double kconst = (kcn <= 0) ? 1.0 : 0.0;
                if (kcn == 1 && S.kcol >= 0) {
                    const double sk = sqrt(S.s2[S.kcol]);
                    const double bk = sk > 0.0 ? S.akv / sk : 0.0;
                    kconst = fmax(0.0, 1.0 - bk * bk);
                }
                // rows 0..q-1: the collapsed private rows (diagonal), rows q..q+S-1: shared
                if (tid < q) {
                    const double sj = sqrt(S.s2[tid]);
                    S.blk[tid * ld + tid] = sj;
                    if (kcn == 1 && S.kcol == tid && sj > 0.0) S.blk[tid * ld + q] = S.akv / sj;
                }
                if (kcn >= 2 && tid == 0) {
                    const int si = sfind(S.srow, nsh, k);
                    if (si >= 0) S.blk[(q + si) * ld + q] = 1.0;
                }
                __syncthreads();
                // ---- Householder QR of the compressed block and Q^T e (wave 0: lane c
                // holds column c, lane q the right-hand side). Column j has nonzeros only
                // in row j and the shared rows (the reflectors of earlier columns touch
                // exactly those rows), so each reflector has 1 + S entries.
                if (wid == 0) {
                    bool singular = false;
                    constexpr int SU = 8;
                    // Few shared rows: lane c keeps the shared-row entries of column c in
                    // registers; the reflector of step j is read from lane j. Row j of
                    // column c > j is zero before step j, except the right-hand side of
                    // the collapsed row of the column where k is private. SU slots: 4 when
                    // the column set has at most 4 shared rows (the common case), else 8.
                    // The slots past nsh hold zeros, but the two instances fuse their
                    // sums of products differently, so their results agree only to
                    // rounding level, not bit for bit.
                    auto qr_regs = [&](auto ns) {
                        constexpr int SU = decltype(ns)::value;
                        double b[SU];
#pragma unroll
                        for (int t = 0; t < SU; ++t) b[t] = (lane <= q && t < nsh) ? S.blk[(q + t) * ld + lane] : 0.0;
                        const double sjl = (lane < q) ? S.blk[lane * ld + lane] : 0.0;
                        const int kc = (kcn == 1) ? S.kcol : -1;
                        const double rk = (kc >= 0) ? S.blk[kc * ld + q] : 0.0;
                        for (int j = 0; j < q; ++j) {
                            double u[SU];
#pragma unroll
                            for (int t = 0; t < SU; ++t) u[t] = readlane_f64(b[t], j);
                            const double x0 = readlane_f64(sjl, j);
                            double s0 = x0 * x0, s1 = 0.0;
#pragma unroll
                            for (int t = 0; t < SU; t += 2) {
                                s0 += u[t] * u[t];
                                s1 += u[t + 1] * u[t + 1];
                            }
                            const double nx = sqrt(s0 + s1);
                            const double alpha = (x0 >= 0.0) ? -nx : nx;
                            const double be = (nx > 0.0) ? 1.0 / (nx * (nx + fabs(x0))) : 0.0;
                            const double v0 = x0 - alpha;
                            if (!(nx > 0.0)) singular = true;
                            if (lane > j && lane <= q) {
                                const double bj = (lane == q && j == kc) ? rk : 0.0;
                                double w0 = v0 * bj, w1 = 0.0;
#pragma unroll
                                for (int t = 0; t < SU; t += 2) {
                                    w0 += u[t] * b[t];
                                    w1 += u[t + 1] * b[t + 1];
                                }
                                const double w = (w0 + w1) * be;
                                S.blk[j * ld + lane] = bj - w * v0;
#pragma unroll
                                for (int t = 0; t < SU; ++t) b[t] -= w * u[t];
                            }
                            if (lane == 0) S.rd[j] = alpha;
                        }
                        // the right-hand side left in the shared rows (lane q)
                        double r2 = 0.0;
#pragma unroll
                        for (int t = 0; t < SU; ++t) r2 += b[t] * b[t];
                        r2 = readlane_f64(r2, q);
                        if (lane == 0) S.rn = sqrt(r2 + kconst);
                    };
                    if (nsh <= 4) {
                        qr_regs(std::integral_constant<int, 4>{});
                    } else if (nsh <= SU) {
                        qr_regs(std::integral_constant<int, SU>{});
                    } else {
                    for (int j = 0; j < q; ++j) {
                        // the reflector's entries (row j and the first shared rows) and this
                        // lane's column, loaded together
                        double u[SU], b[SU];
                        const bool act = lane > j && lane <= q;
                        const double x0 = S.blk[j * ld + j];
                        const double bj = act ? S.blk[j * ld + lane] : 0.0;
#pragma unroll
                        for (int t = 0; t < SU; ++t) {
                            u[t] = (t < nsh) ? S.blk[(q + t) * ld + j] : 0.0;
                            b[t] = (act && t < nsh) ? S.blk[(q + t) * ld + lane] : 0.0;
                        }
                        double s0 = x0 * x0, s1 = 0.0;
#pragma unroll
                        for (int t = 0; t < SU; t += 2) {
                            s0 += u[t] * u[t];
                            s1 += u[t + 1] * u[t + 1];
                        }
                        double s = s0 + s1;
                        if (nsh > SU) {
                            double r = 0.0;
                            for (int t = SU + lane; t < nsh; t += 64) {
                                const double x = S.blk[(q + t) * ld + j];
                                r += x * x;
                            }
                            s += wsum(r);
                        }
                        const double nx = sqrt(s);
                        const double alpha = (x0 >= 0.0) ? -nx : nx;
                        const double be = (nx > 0.0) ? 1.0 / (nx * (nx + fabs(x0))) : 0.0;
                        const double v0 = x0 - alpha;
                        if (!(nx > 0.0)) singular = true;
                        if (act) {
                            double w0 = v0 * bj, w1 = 0.0;
#pragma unroll
                            for (int t = 0; t < SU; t += 2) {
                                w0 += u[t] * b[t];
                                w1 += u[t + 1] * b[t + 1];
                            }
                            for (int t = SU; t < nsh; ++t) w0 += S.blk[(q + t) * ld + j] * S.blk[(q + t) * ld + lane];
                            const double w = (w0 + w1) * be;
                            S.blk[j * ld + lane] = bj - w * v0;
#pragma unroll
                            for (int t = 0; t < SU; ++t)
                                if (t < nsh) S.blk[(q + t) * ld + lane] = b[t] - w * u[t];
                            for (int t = SU; t < nsh; ++t) S.blk[(q + t) * ld + lane] -= w * S.blk[(q + t) * ld + j];
                        }
                        if (lane == 0) S.rd[j] = alpha;
                        wave_sync();
                    }
                    // the right-hand side left in the shared rows
                    double r2 = 0.0;
                    for (int t = lane; t < nsh; t += 64) {
                        const double x = S.blk[(q + t) * ld + q];
                        r2 += x * x;
                    }
                    r2 = wsum(r2);
                    if (lane == 0) S.rn = sqrt(r2 + kconst);
                    }
                    wave_sync();
                    if (!singular) {
                        // back substitution: lane i holds (Q^T e)_i; m_j broadcast by readlane
                        double y = (lane < q) ? S.blk[lane * ld + q] : 0.0;
                        for (int j = q - 1; j >= 0; --j) {
                            const long long yb = __double_as_longlong(y);
                            const int lo = __builtin_amdgcn_readlane((int)(yb & 0xffffffffLL), j);
                            const int hi = __builtin_amdgcn_readlane((int)(yb >> 32), j);
                            const double yj = __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
                            const double mj = yj / S.rd[j];
                            if (lane == 0) S.mt[j] = mj;
                            if (lane < j) y -= S.blk[lane * ld + j] * mj;
                        }
                    } else if (lane == 0) {
                        S.flag = 1;
                    }
                }
                __syncthreads();
                if (S.flag) { status = ST_SINGULAR; break; }
                rn = S.rn;
                if (qmod >= 0) fl += solve_flops(mmod, m, qmod, q);
                // ---- dropping (Section 4), after the augment solve only
                if (pass == 0 && dropok && P.drop != DROP_NONE) {
                    const double th = (P.drop == DROP_FIXED)
                                          ? P.tol
                                          : P.eps / ((double)q * __longlong_as_double((long long)*A.norm1_bits));
                    // kept columns as a lane mask (q <= 63: one lane per column, each wave
                    // forms the same mask); with none above the threshold, the largest |m_j|
                    // stays (the smaller column index on ties)
                    const bool inq = lane < q;
                    const double am = inq ? fabs(S.mt[lane]) : -1.0;
                    const int jg = inq ? S.Jl[lane] : INT_MAX;
                    unsigned long long keepm = __ballot(inq && am > th);
                    const int nk = __popcll(keepm);
                    if (nk == 0) {
                        double ba = am;
                        int bg = jg;
#pragma unroll
                        for (int off = 32; off >= 1; off >>= 1) {
                            const double a2 = __shfl_xor(ba, off);
                            const int g2 = __shfl_xor(bg, off);
                            if (a2 > ba || (a2 == ba && g2 < bg)) { ba = a2; bg = g2; }
                        }
                        keepm = __ballot(inq && jg == bg);
                    }
                    if (nk < q) {
                        // rows of the dropped columns lose one holder
                        wave_cols_if<false>(
                            S, A, 0, q, wid, lane,
                            [&](int, int row, double) {
                                const int sl = hfind<LOGH>(S.hk, row);
                                if (sl >= 0) hdec(S, sl); else lookup_fail = true;
                            },
                            [](int) {}, [&](int c) { return ((keepm >> c) & 1ull) == 0ull; });
                        __syncthreads();
                        // the kept columns' compressed data for the re-solve (old slots
                        // here): a shared row keeps its place among the rows still held by
                        // two or more kept columns; a row held by one kept column joins that
                        // column's private sum (after the sum it had, rows ascending); the
                        // row of k is private, shared or gone as its holders are
                        {
                            const int qo = q, nso = nsh;
                            const int qn = __popcll(keepm);
                            auto slot = [&](int c) { return __popcll(keepm & ((1ull << c) - 1ull)); };
                            if (wid == 0) {
                                int base = 0;
                                for (int s0 = 0; s0 < nso; s0 += 64) {
                                    const int si = s0 + lane;
                                    const bool kr = si < nso && __popcll(S.shm[si] & keepm) >= 2;
                                    const unsigned long long bal = __ballot(kr);
                                    if (si < nso) S.stmp[si] = kr ? base + __popcll(bal & ((1ull << lane) - 1ull)) : -1;
                                    base += __popcll(bal);
                                }
                                if (lane == 0) S.nsh2 = base;
                            }
                            int kc = -1;
                            double ka = 0.0;
                            if (tid == 0) {
                                const int ksl2 = hfind<LOGH>(S.hk, k);
                                const unsigned kcn2 = ksl2 >= 0 ? (hget(S, ksl2) & 0x7Fu) : 0u;
                                if (kcn2 == 1u) {
                                    if (S.kcol >= 0 && ((keepm >> S.kcol) & 1ull)) {
                                        kc = slot(S.kcol);
                                        ka = S.akv;
                                    } else {
                                        const int si = sfind(S.srow, nso, k);
                                        if (si >= 0) {
                                            const unsigned long long hm = S.shm[si] & keepm;
                                            if (__popcll(hm) == 1) {
                                                const int c = __ffsll((long long)hm) - 1;
                                                kc = slot(c);
                                                ka = S.shv[si * qo + c];
                                            }
                                        }
                                    }
                                }
                            }
                            __syncthreads();
                            // kept shared values (staged in blk, free until the re-solve
                            // forms its block) and the kept columns' private sums (in rd)
                            for (int t = tid; t < nso * qo; t += NT) {
                                const int si = t / qo, c = t - si * qo;
                                const int ns = S.stmp[si];
                                if (ns >= 0 && ((keepm >> c) & 1ull)) S.blk[ns * qn + slot(c)] = S.shv[t];
                            }
                            if (tid < qo && ((keepm >> tid) & 1ull)) {
                                double acc = S.s2[tid];
                                const unsigned long long me = 1ull << tid;
                                for (int si = 0; si < nso; ++si)
                                    if ((S.shm[si] & keepm) == me) {
                                        const double v = S.shv[si * qo + tid];
                                        acc += v * v;
                                    }
                                S.rd[slot(tid)] = acc;
                            }
                            const int myrow = tid < nso ? S.srow[tid] : 0;
                            const int mynew = tid < nso ? S.stmp[tid] : -1;
                            __syncthreads();
                            const int nsn = S.nsh2;
                            if (mynew >= 0) S.srow[mynew] = myrow;
                            for (int t = tid; t < nsn * qn; t += NT) S.shv[t] = S.blk[t];
                            if (tid < qn) S.s2[tid] = S.rd[tid];
                            if (tid == 0) {
                                S.kcol = kc;
                                S.akv = ka;
                                S.nsh = nsn;
                            }
                            __syncthreads();
                            if (S.slovf == 0) {
                                // the candidate list keeps the shared rows only
                                for (int t = tid; t < nsn; t += NT) S.slist[t] = S.srow[t];
                                if (tid == 0) S.nsl = nsn;
                            }
                        }
                        if (wid == 0) {
                            // compaction of the slots in order: lane c moves to the number of
                            // kept slots below it
                            const bool kc = inq && ((keepm >> lane) & 1ull);
                            int jl = 0, cl = 0;
                            int64_t cbv = 0;
                            if (kc) {
                                jl = S.Jl[lane];
                                cbv = S.cb[lane];
                                cl = S.clen[lane];
                            }
                            const int d = __popcll(keepm & ((1ull << lane) - 1ull));
                            wave_sync();
                            if (kc) {
                                S.Jl[d] = jl;
                                S.cb[d] = cbv;
                                S.clen[d] = cl;
                            }
                            if (lane == 0) S.cnt = __popcll(keepm);
                        }
                        for (int t = tid; t < HJ; t += NT) S.hJ[t] = HEMPTY;
                        __syncthreads();
                        q = S.cnt;
                        for (int c = tid; c < q; c += NT) {
                            int sl;
                            hinsert<LOGHJ>(S.hJ, S.Jl[c], sl);
                        }
                        qmod = 0;
                        reuse_next = true;
                        __syncthreads();
                        continue;  // solve on the kept pattern
                    }
                }
                break;
            }
            if (status != ST_OK || spill) break;
            need_solve = false;

            // ================= stop test (step 3)
            if (rn <= P.eps || l >= P.lmax) break;

            // ================= dominant rows of r = A(I,J) m - e_k (step 4)
            const int nsh = S.nsh;
            if (tid < q) {
                const int jc = S.Jl[tid];
                int rank = 0;
                for (int t = 0; t < q; ++t) rank += (S.Jl[t] < jc) ? 1 : 0;
                S.ord[rank] = tid;
            }
            __syncthreads();
            double ta[CMAX];
            int tg[CMAX];
#pragma unroll
            for (int s = 0; s < CMAX; ++s) { ta[s] = -1.0; tg[s] = INT_MAX; }
            auto offer = [&](double a, int g) {
#pragma unroll
                for (int s = 0; s < CMAX; ++s) {
                    if (better(a, g, ta[s], tg[s])) {
                        const double a1 = ta[s];
                        const int g1 = tg[s];
                        ta[s] = a;
                        tg[s] = g;
                        a = a1;
                        g = g1;
                    }
                }
            };
            // shared rows: the columns in ascending global order, fused multiply-adds
            if (tid < nsh) {
                double acc = 0.0;
                for (int t = 0; t < q; ++t) {
                    const int c = S.ord[t];
                    const double a = S.shv[tid * q + c];
                    if (a != 0.0) acc = __fma_rn(a, S.mt[c], acc);
                }
                const int row = S.srow[tid];
                const double ri = acc - ((row == k) ? 1.0 : 0.0);
                const int sl = hfind<LOGH>(S.hk, row);
                if (ri != 0.0 && sl >= 0 && !(hget(S, sl) & 0x80u)) offer(fabs(ri), row);
            }
            // private rows: one product each
            wave_cols<true>(
                S, A, 0, q, wid, lane,
                [&](int c, int row, double v) {
                    const int sl = hfind<LOGH>(S.hk, row);
                    const unsigned hvv = sl >= 0 ? hget(S, sl) : 0u;
                    if ((hvv & 0x7Fu) == 1u && !(hvv & 0x80u)) {
                        const double ri = __fma_rn(v, S.mt[c], 0.0) - ((row == k) ? 1.0 : 0.0);
                        if (ri != 0.0) offer(fabs(ri), row);
                    }
                },
                [](int) {});
            // row k outside the columns of J: r(k) = -1
            if (tid == 0) {
                const int ksl = hfind<LOGH>(S.hk, k);
                if (ksl >= 0) {
                    const unsigned hvv = hget(S, ksl);
                    if ((hvv & 0x7Fu) == 0u && !(hvv & 0x80u)) offer(1.0, k);
                } else if (!kR) {
                    offer(1.0, k);
                }
            }
            int nsel = 0;
            for (int t = 0; t < P.c; ++t) {
                double a = ta[0];
                int g = tg[0];
                gargmax<16>(a, g);
#pragma unroll
                for (int off = 16; off <= 32; off <<= 1) {
                    const double a2 = __shfl_xor(a, off);
                    const int g2 = __shfl_xor(g, off);
                    if (better(a2, g2, a, g)) { a = a2; g = g2; }
                }
                if (lane == 0) { S.cva[wid] = a; S.cvg[wid] = g; }
                __syncthreads();
                a = S.cva[0];
                g = S.cvg[0];
#pragma unroll
                for (int w = 1; w < NW; ++w)
                    if (better(S.cva[w], S.cvg[w], a, g)) { a = S.cva[w]; g = S.cvg[w]; }
                __syncthreads();
                if (a < 0.0) break;
                // the holder of the winner drops it from its list
                if (tg[0] == g && ta[0] == a) {
#pragma unroll
                    for (int s = 0; s < CMAX - 1; ++s) { ta[s] = ta[s + 1]; tg[s] = tg[s + 1]; }
                    ta[CMAX - 1] = -1.0;
                    tg[CMAX - 1] = INT_MAX;
                }
                if (tid == 0) {
                    S.Rh[t] = g;
                    const int sl = hfind<LOGH>(S.hk, g);
                    if (sl >= 0) hsetR(S, sl);
                }
                if (g == k && hfind<LOGH>(S.hk, k) < 0) kR = true;
                nsel = t + 1;
            }
            __syncthreads();
            if (nsel == 0) break;  // no candidate row left: r = 0 (Section 3)
            nRh = nsel;
            linc = true;
        }
        if (lookup_fail) atomicOr(args.err, 16);

        if (spill) {
            // ---- hand the column over to a later class: the next one, or for a block
            // that did not fit, the first level with a larger block, or the dense class
            // when most of its rows are shared
            int32_t *qo = args.rec_out, *qc = args.rec_out_count;
            int qs = args.rec_out_stride;
            int64_t qcap = args.rec_out_cap;
            if (blk_nsh >= 0) {
                const int d = (args.rec_alt[1] != nullptr && 2 * blk_nsh >= m) ? 1 : (args.rec_alt[0] != nullptr ? 0 : -1);
                if (d >= 0) {
                    qo = args.rec_alt[d];
                    qc = args.rec_alt_count[d];
                    qs = args.rec_alt_stride[d];
                    qcap = args.rec_alt_cap[d];
                }
            }
            if (tid == 0) {
                int ps = INT_MAX;
                if (qo) ps = atomicAdd(qc, 1);
                S.cnt = ps;
                S.nsh = 0;  // R rows written
                S.flag = 0; // I rows written
            }
            __syncthreads();
            const int ps = S.cnt;
            if (qo != nullptr && (int64_t)ps < qcap) {
                int32_t *R = qo + (int64_t)ps * qs;
                int32_t *RJo = R + RHDR, *RIo = RJo + q, *RRo = RIo + m;
                for (int t = tid; t < q; t += NT) RJo[t] = S.Jl[t];
                // I (hash order; the receiver numbers its rows in ascending order) and R
                for (int t = tid; t < HS; t += NT) {
                    const int key = S.hk[t];
                    if (key != HEMPTY) {
                        RIo[atomicAdd(&S.flag, 1)] = key;
                        if (hget(S, t) & 0x80u) {
                            const int r = atomicAdd(&S.nsh, 1);
                            if (r < WIDE_RCAP) RRo[r] = key;
                        }
                    }
                }
                __syncthreads();
                int nR = S.nsh;
                if (tid == 0 && kR && nR < WIDE_RCAP) RRo[nR] = k;
                nR += kR ? 1 : 0;
                nR = min(nR, WIDE_RCAP);
                if (tid < nRh) RRo[nR + tid] = S.Rh[tid];
                if (tid == 0) {
                    R[0] = ucol; R[1] = mat; R[2] = k; R[3] = l;
                    R[4] = q; R[5] = m; R[6] = nR; R[7] = nRh;
                    const long long fb = __double_as_longlong(fl);
                    R[8] = (int32_t)(fb & 0xffffffffLL);
                    R[9] = (int32_t)(fb >> 32);
                    R[10] = (linc ? 1 : 0) | (pend ? 2 : 0) | (pend_drop ? 4 : 0);
                    R[11] = pend_qmod;
                    R[12] = pend_mmod;
                }
                __syncthreads();
                continue;
            }
            status = ST_CAP;  // no room in the next class
            if (tid == 0 && qo != nullptr) atomicOr(args.err, 32);  // queue full
        }

        // ---------------------------------------------------------- output (rows ascending)
        const int qq = (status == ST_OK) ? q : 0;
        const int64_t slot = args.arena_base + (int64_t)ucol * 64;
        for (int c = tid; c < qq; c += NT) {
            const int jc = S.Jl[c];
            int rank = 0;
            for (int t = 0; t < qq; ++t) rank += (S.Jl[t] < jc) ? 1 : 0;
            args.out.arenaJ[slot + rank] = jc;
            args.out.arenaV[slot + rank] = S.mt[c];
        }
        if (tid == 0) {
            args.out.off[ucol] = slot;
            args.out.nJ[ucol] = qq;
            args.out.nI[ucol] = m;
            args.out.loops[ucol] = l;
            args.out.status[ucol] = status;
            args.out.resnorm[ucol] = rn;
            args.out.flops[ucol] = fl;
        }
        if (args.out.fac != nullptr) {
            // R of the final (compressed) solve: R^T R = A(I,J)^T A(I,J); rows 0..q-1 of
            // the block hold its strict upper part, rd the diagonal
            if (tid == 0) {
                const long long fo = (qq > 0) ? fac_reserve(args.out, qq) : -1LL;
                args.out.foff[ucol] = fo;
                S.cnt = (int)(fo & 0xffffffffLL);
                S.nsh = (int)(fo >> 32);
            }
            __syncthreads();
            const long long fo = ((long long)S.nsh << 32) | (long long)(unsigned)S.cnt;
            if (fo >= 0) {
                double *F = args.out.fac + fo;
                const int ld = qq + 1;
                for (int c = tid; c < qq; c += NT) F[c] = (double)S.Jl[c];
                for (int t = tid; t < qq * qq; t += NT) {
                    const int i = t / qq, c = t % qq;
                    if (c >= i) F[fac_row(qq, i) + (c - i)] = (c == i) ? S.rd[i] : S.blk[i * ld + c];
                }
            }
        }
        __syncthreads();
    }
}

namespace {
// Level 2 takes level 0's columns whose compressed block does not fit (many shared
// rows, as in the columns that pick a relatively dense row) at two workgroups per CU
// instead of sending them to the one-per-CU level 3.
constexpr int kWideLogH[WIDE_LEVELS] = {11, 12, 11, 14};
constexpr int kWidePerCU[WIDE_LEVELS] = {4, 3, 2, 1};
#define RSAI_WIDE0 kWideLogH[0], 2048, 768, 128, kWidePerCU[0]
#define RSAI_WIDE1 kWideLogH[1], 2048, 768, 128, kWidePerCU[1]
#define RSAI_WIDE2 kWideLogH[2], 4096, 1536, 128, kWidePerCU[2]
#define RSAI_WIDE3 kWideLogH[3], 6144, 1536, 256, kWidePerCU[3]
}  // namespace

int wide_max_rows(int level) { return (1 << kWideLogH[level]) / 2; }
int wide_rec_stride(int level) { return RHDR + 64 + wide_max_rows(level) + WIDE_RCAP + CMAX; }
int wide_queue_stride(int queue) {
    // rows of the largest record a writer of the queue can hand over
    static const int writer_level[WIDE_LEVELS] = {0, 0, 1, 3};
    return wide_rec_stride(writer_level[queue]);
}
int wide_blocks_per_cu(int level) { return kWidePerCU[level]; }

void launch_wide_kernel(int level, const WideArgs &a, int blocks, hipStream_t s) {
    if (level == 0)
        hipLaunchKernelGGL((wide_kernel<RSAI_WIDE0>), dim3(blocks), dim3(NT), 0, s, a);
    else if (level == 1)
        hipLaunchKernelGGL((wide_kernel<RSAI_WIDE1>), dim3(blocks), dim3(NT), 0, s, a);
    else if (level == 2)
        hipLaunchKernelGGL((wide_kernel<RSAI_WIDE2>), dim3(blocks), dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((wide_kernel<RSAI_WIDE3>), dim3(blocks), dim3(NT), 0, s, a);
}

}  // namespace rsai
