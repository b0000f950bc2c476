// Large size class of the RSAI(tol) build: one 256-thread workgroup per column,
// for the columns that outgrow the register tiers (tall LS blocks A(I_k, J_k) of up
// to BMMAX rows and BQMAX columns, e.g. the power-law matrices whose long columns
// bring hundreds to thousands of rows into I_k).
//
// Same steps as the register tiers (Algorithm 1 with the dropping of Section 4):
//   * index sets are LDS hash sets; new rows are numbered in ascending global order
//     (bitonic sort in LDS), so results do not depend on thread timing;
//   * the dense block lives in a per-workgroup slab of global memory (column-major,
//     leading dimension BMMAX) and holds the Householder factor between loops: a
//     solve applies the stored reflectors to the new columns and forms theirs
//     (blocked, FP64 MFMA compact WY); the solve after a drop refactors the kept
//     columns;
//   * the residual for step 4 is A(I,J) m - e_k(I) accumulated from the sparse
//     columns in ascending column order (eq. (2.4)), so exact ties reach the
//     smaller-index rule.
// Columns arrive as spill records of the previous class; a column that outgrows this
// class ends with status RSAI_E_CAP.
#include <climits>
#include <utility>

#include "rsai_kernels.h"

namespace rsai {

namespace {
constexpr int NT = 256;                    // threads per workgroup
constexpr int NW = NT / 64;                // waves
constexpr int BLOGH = 14;                  // row hash: 16384 slots
constexpr int BH = 1 << BLOGH;
constexpr int BLOGHJ = 8;                  // column hash: 256 slots
constexpr int BHJ = 1 << BLOGHJ;
constexpr int SORTN = 8192;                // bitonic buffer for new rows
constexpr int NB = 16;                     // panel width of the blocked QR
constexpr int NCTMAX = (BQMAX_BIG + 1 - NB + 15) / 16;  // column tiles after a panel (+ Q^T e)
constexpr int REDN = NW * (NCTMAX + 1) * 256;            // doubles of per-wave MFMA partials

struct BigLds {
    int hI[BH];
    unsigned short hIv[BH];
    int hJ[BHJ];
    int skey[SORTN];
    int Jlist[BQMAX_BIG];
    double mt[BQMAX_BIG];
    double rd[BQMAX_BIG];
    double bt[BQMAX_BIG];
    double red[NW * 8];
    double redp[NW * (NB + 1)];    // per-wave partials of the register-panel reductions
    double Tm[16 * 16];            // T of the compact WY form of a panel
    double Wp[16 * NCTMAX * 16];   // T^T V^T C of a panel
    int ired[NW * 2];
    double dred[NW];
    int Rh[CMAX];
    int cnt, misc;
};
}  // namespace

int big_max_rows() { return BMMAX_BIG; }
int big_max_cols() { return BQMAX_BIG; }

// block-wide sum (every thread gets the result)
__device__ __forceinline__ double bsum(double x, BigLds &S) {
    x = gsum<16>(x);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    __syncthreads();
    if (lane == 0) S.dred[w] = x;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) t += S.dred[i];
    __syncthreads();
    return t;
}
__device__ __forceinline__ int bsum_i(int x, BigLds &S) {
    x = gsum_i<16>(x);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    __syncthreads();
    if (lane == 0) S.ired[w] = x;
    __syncthreads();
    int t = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) t += S.ired[i];
    __syncthreads();
    return t;
}
// block arg-max of (a desc, g asc); every thread gets the winner
__device__ __forceinline__ void bargmax(double &a, int &g, BigLds &S) {
    gargmax<16>(a, g);
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) {
        double a2 = __shfl_xor(a, off);
        int g2 = __shfl_xor(g, off);
        if (a2 > a || (a2 == a && g2 < g)) { a = a2; g = g2; }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) { S.red[w] = a; S.ired[w] = g; }
    __syncthreads();
    a = S.red[0];
    g = S.ired[0];
#pragma unroll
    for (int i = 1; i < NW; ++i)
        if (S.red[i] > a || (S.red[i] == a && S.ired[i] < g)) { a = S.red[i]; g = S.ired[i]; }
    __syncthreads();
}

typedef double mfma_d4 __attribute__((ext_vector_type(4)));

// V(r, i) of the current panel: reflector i (column p0 + i) below its diagonal,
// its head on the diagonal, zero above and outside the panel or the block
__device__ __forceinline__ double vget(const double *B, int64_t ld, int m, int p0, int pw, int r, int i) {
    if (i >= pw || r >= m || r < p0 + i) return 0.0;
    return B[(int64_t)(p0 + i) * ld + r];
}
// column c of the trailing part: a column of the block, or Q^T e for c == qn
__device__ __forceinline__ double *colp(double *B, int64_t ld, double *y, int qn, int c) {
    return (c < qn) ? B + (int64_t)c * ld : y;
}

// Apply Q_p^T = I - V T^T V^T of the panel (columns p0 .. p0+pw-1, pw <= 16) to the
// ntr columns c_lo .. c_lo+ntr-1 (the last one is Q^T e). W = V^T C and the Gram
// matrix V^T V are FP64 MFMA reductions over the rows, split across the waves;
// C -= V (T^T W) is an MFMA per 16x16 tile of C.
// MFMA 16x16x4 f64 operands (lane l): A(l % 16, l / 16), B(l / 16, l % 16); result
// element t of lane l is D(l / 16 + 4 t, l % 16).
__device__ void panel_update(double *B, int64_t ld, double *y, int m, int qn, int p0, int pw, int c_lo, int ntr,
                             BigLds &S, double *red) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nct = (ntr + 15) / 16;  // column tiles of the trailing part (<= 5)
    // red: [NW][NCTMAX + 1][64][4] partials in the workgroup's slab
    // ---- G = V^T V (tile 0) and W = V^T C (tiles 1..nct), K = rows p0..m-1
    mfma_d4 acc[NCTMAX + 1];
#pragma unroll
    for (int t = 0; t <= NCTMAX; ++t) acc[t] = mfma_d4{0.0, 0.0, 0.0, 0.0};
    for (int r0 = p0 + 4 * w; r0 < m; r0 += 4 * NW) {
        const int r = r0 + lk;
        const double a = vget(B, ld, m, p0, pw, r, li);
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, acc[0], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < NCTMAX; ++t) {
            if (t < nct) {
                const int c = c_lo + 16 * t + li;
                const double bv = (c < c_lo + ntr && r < m) ? colp(B, ld, y, qn, c)[r] : 0.0;
                acc[t + 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[t + 1], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t <= NCTMAX; ++t)
        if (t <= nct)
#pragma unroll
            for (int e = 0; e < 4; ++e) red[((w * (NCTMAX + 1) + t) * 64 + lane) * 4 + e] = acc[t][e];
    __syncthreads();
    // sum over the waves into wave 0's slots; element (row, col) of tile t sits in
    // lane col + 16 * (row % 4), entry row / 4
    for (int x = tid; x < (nct + 1) * 256; x += NT) {
        double v = 0.0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) v += red[(ww * (NCTMAX + 1)) * 256 + x];
        red[x] = v;
    }
    __syncthreads();
    auto tile = [&](int t, int row, int col) -> double {
        return red[(t * 64 + col + 16 * (row & 3)) * 4 + (row >> 2)];
    };
    // ---- T (upper triangular): T(j,j) = beta_j, T(0:j, j) = -beta_j T(0:j,0:j) G(0:j, j)
    double *T = S.Tm;  // [16][16], row-major
    if (tid < 64) {
        for (int j = 0; j < pw; ++j) {
            double v = 0.0;
            if (lane < j) {
                for (int t = lane; t < j; ++t) v += T[lane * 16 + t] * tile(0, t, j);
                v *= -S.bt[p0 + j];
            }
            if (lane < j) T[lane * 16 + j] = v;
            if (lane == j) T[j * 16 + j] = S.bt[p0 + j];
            if (lane > j && lane < 16) T[lane * 16 + j] = 0.0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    __syncthreads();
    // ---- W' = T^T W (16 x ntr), stored as Wp[i][c]
    double *Wp = S.Wp;  // [16][NCTMAX * 16]
    for (int x = tid; x < 16 * nct * 16; x += NT) {
        const int i = x / (nct * 16), c = x % (nct * 16);
        double v = 0.0;
        if (i < pw)
            for (int t = 0; t <= i; ++t) v += T[t * 16 + i] * tile(1 + c / 16, t, c % 16);
        Wp[i * (NCTMAX * 16) + c] = v;
    }
    __syncthreads();
    // ---- C -= V W': 16-row tiles of rows p0..m-1 times the column tiles
    const int nrt = (m - p0 + 15) / 16;
    for (int x = w; x < nrt * nct; x += NW) {
        const int rt = x / nct, ct = x % nct;
        const int r0 = p0 + 16 * rt;
        const int c = c_lo + 16 * ct + li;
        const bool cok = c < c_lo + ntr;
        double *cp = cok ? colp(B, ld, y, qn, c) : nullptr;
        mfma_d4 d;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = r0 + lk + 4 * e;
            d[e] = (cok && r < m) ? cp[r] : 0.0;
        }
#pragma unroll
        for (int k0 = 0; k0 < 16; k0 += 4) {
            const double a = -vget(B, ld, m, p0, pw, r0 + li, k0 + lk);
            const double bv = Wp[(k0 + lk) * (NCTMAX * 16) + 16 * ct + li];
            d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, d, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = r0 + lk + 4 * e;
            if (cok && r < m) cp[r] = d[e];
        }
    }
    __syncthreads();
}

// Block-wide sums of x[LO..HI) (up to NB + 1 values): a wave-level tree per value,
// then the four waves' partials through LDS. Every thread gets the totals.
template <int LO, int HI>
__device__ __forceinline__ void bsum_many(double (&x)[NB + 1], BigLds &S) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int u = LO; u < HI; ++u) {
        x[u] = gsum<16>(x[u]);
        x[u] += __shfl_xor(x[u], 16);
        x[u] += __shfl_xor(x[u], 32);
    }
    if (lane == 0)
#pragma unroll
        for (int u = LO; u < HI; ++u) S.redp[w * (NB + 1) + u] = x[u];
    __syncthreads();
#pragma unroll
    for (int u = LO; u < HI; ++u) {
        double t = 0.0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) t += S.redp[ww * (NB + 1) + u];
        x[u] = t;
    }
    __syncthreads();
}

// One step of the register panel: the reflector of panel column UJ (block column
// p0 + UJ) and its application to the panel's later columns.
template <int RPT, int UJ>
__device__ __forceinline__ void panel_step(double (&pv)[RPT][NB], int m, int p0, int pw, BigLds &S,
                                           bool &singular) {
    if (UJ >= pw) return;
    const int tid = threadIdx.x;
    const int j = p0 + UJ;
    double x[NB + 1];
    x[0] = 0.0;  // ||column j from its diagonal down||^2
    x[1] = 0.0;  // its diagonal entry (held by one thread)
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int r = tid + NT * i;
        if (r >= j && r < m) x[0] += pv[i][UJ] * pv[i][UJ];
        if (r == j) x[1] = pv[i][UJ];
    }
    bsum_many<0, 2>(x, S);
    const double x0 = x[1];
    const double nx = sqrt(x[0]);
    const double alpha = (x0 >= 0.0) ? -nx : nx;
    const double vj = x0 - alpha;
    const double be = (nx > 0.0) ? 1.0 / (nx * (nx + fabs(x0))) : 0.0;
    if (!(nx > 0.0)) singular = true;
    double v[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int r = tid + NT * i;
        v[i] = (r > j && r < m) ? pv[i][UJ] : 0.0;
        if (r == j) {
            v[i] = vj;
            pv[i][UJ] = vj;
        }
    }
    if constexpr (UJ + 1 < NB) {
        if (UJ + 1 < pw) {
            double d[NB + 1];
#pragma unroll
            for (int u = UJ + 1; u < NB; ++u) {
                d[u] = 0.0;
#pragma unroll
                for (int i = 0; i < RPT; ++i) d[u] += v[i] * pv[i][u];
            }
            bsum_many<UJ + 1, NB>(d, S);
#pragma unroll
            for (int u = UJ + 1; u < NB; ++u) {
                const double f = d[u] * be;
#pragma unroll
                for (int i = 0; i < RPT; ++i) pv[i][u] -= f * v[i];
            }
        }
    }
    if (tid == 0) {
        S.rd[j] = alpha;
        S.bt[j] = be;
    }
}

template <int RPT, int... UJ>
__device__ __forceinline__ void panel_steps(double (&pv)[RPT][NB], int m, int p0, int pw, BigLds &S, bool &singular,
                                            std::integer_sequence<int, UJ...>) {
    (panel_step<RPT, UJ>(pv, m, p0, pw, S, singular), ...);
}

// Factor the panel columns p0 .. p0+pw-1 (pw <= NB) of an m-row block, m <= NT * RPT,
// with the panel held in registers (thread t holds rows t + NT * i of every panel
// column): each step takes the norm of column j from its diagonal down and the diagonal
// entry in one block reduction, forms the reflector, and applies it to the panel's
// later columns with one more reduction of all their products. The panel is written
// back (reflector heads on the diagonal, R above it); alpha and beta go to S.rd, S.bt.
// Returns true if a column has zero norm from its diagonal down (rank deficiency).
template <int RPT>
__device__ bool panel_factor_regs(double *B, int64_t ld, int m, int p0, int pw, BigLds &S) {
    const int tid = threadIdx.x;
    double pv[RPT][NB];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int r = tid + NT * i;
#pragma unroll
        for (int u = 0; u < NB; ++u) pv[i][u] = (r < m && u < pw) ? B[(int64_t)(p0 + u) * ld + r] : 0.0;
    }
    bool singular = false;
    panel_steps<RPT>(pv, m, p0, pw, S, singular, std::make_integer_sequence<int, NB>{});
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int r = tid + NT * i;
        if (r < m)
#pragma unroll
            for (int u = 0; u < NB; ++u)
                if (u < pw) B[(int64_t)(p0 + u) * ld + r] = pv[i][u];
    }
    __syncthreads();
    return singular;
}

__global__ __launch_bounds__(NT) void big_kernel(BigArgs args) {
    __shared__ BigLds S;
    const int tid = threadIdx.x;
    if (*args.err & ERR_SKIP) return;
    const BuildParams P = args.P;
    const int64_t Q = min((int64_t)(*args.rec_in_count), args.rec_in_cap);
    double *B = args.scratch + (int64_t)blockIdx.x * args.scratch_stride;  // [BQMAX][BMMAX]
    const int64_t ld = args.ld;                                            // rows per block column
    double *y = B + (int64_t)BQMAX_BIG * ld;                               // Q^T e
    double *racc = y + ld;                                                 // residual
    int *Il = reinterpret_cast<int *>(racc + ld);                          // rows of I
    unsigned char *rfl = reinterpret_cast<unsigned char *>(Il + ld);       // row in R
    double *gred = racc + ld + (ld * 5 + 7) / 8 + 8;                       // panel partials

    for (int64_t pos = blockIdx.x; pos < Q; pos += gridDim.x) {
        const int32_t *rec = args.rec_in + pos * (int64_t)args.rec_in_stride;
        const int ucol = rec[0], mat = rec[1], k = rec[2];
        int l = rec[3], q = rec[4], m = rec[5];
        const int nR = rec[6];
        int nRh = rec[7];
        double fl = __longlong_as_double(((long long)rec[9] << 32) | (long long)(unsigned)rec[8]);
        const bool linc0 = (rec[10] & 1) != 0;
        const MatDev A = args.mats[mat];
        const int32_t *RJ = rec + RHDR, *RI = RJ + q, *RR = RI + m, *RHp = RR + nR;
        int status = ST_OK;
        double rn = 0.0;
        bool kR = false;
        int kidx = -1;

        // ---- state from the record
        for (int t = tid; t < BH; t += NT) S.hI[t] = HEMPTY;
        for (int t = tid; t < BHJ; t += NT) S.hJ[t] = HEMPTY;
        __syncthreads();
        if (q > BQMAX_BIG || m > ld) status = ST_CAP;
        int np2 = 1;
        while (np2 < m) np2 <<= 1;
        if (status == ST_OK) {
            for (int t = tid; t < q; t += NT) {
                S.Jlist[t] = RJ[t];
                int sl;
                hinsert<BLOGHJ>(S.hJ, RJ[t], sl);
            }
            // rows of I numbered in ascending order (records may list them in any order)
            for (int t = tid; t < np2; t += NT) S.skey[t] = (t < m) ? RI[t] : INT_MAX;
            if (tid < nRh) S.Rh[tid] = RHp[tid];
        }
        __syncthreads();
        if (status == ST_OK) {
            for (int kk = 2; kk <= np2; kk <<= 1) {
                for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                    for (int i = tid; i < np2; i += NT) {
                        const int ixj = i ^ jj;
                        if (ixj > i) {
                            const int a = S.skey[i], b = S.skey[ixj];
                            const bool up = (i & kk) == 0;
                            if ((a > b) == up) { S.skey[i] = b; S.skey[ixj] = a; }
                        }
                    }
                    __syncthreads();
                }
            }
            for (int t = tid; t < m; t += NT) {
                const int row = S.skey[t];
                Il[t] = row;
                rfl[t] = 0;
                int sl;
                hinsert<BLOGH>(S.hI, row, sl);
                if (sl >= 0) S.hIv[sl] = (unsigned short)t;
            }
        }
        __syncthreads();
        if (status == ST_OK) {
            for (int t = tid; t < nR; t += NT) {
                const int row = RR[t];
                const int sl = hfind<BLOGH>(S.hI, row);
                if (sl >= 0) rfl[S.hIv[sl]] = 1;
            }
            if (tid == 0) {
                const int sl = hfind<BLOGH>(S.hI, k);
                S.misc = sl >= 0 ? S.hIv[sl] : -1;
                int kr = 0;
                for (int t = 0; t < nR; ++t) kr |= (RR[t] == k);
                S.cnt = kr;
            }
        }
        __syncthreads();
        kidx = S.misc;
        kR = (kidx < 0) && S.cnt;
        __syncthreads();

        int fq = 0, fm = 0;      // columns and rows of the factor held in the block
        bool linc = linc0;       // advance l when J-hat is formed
        bool first = true;       // the stored pattern has no factor here yet
        bool need_solve = true;
        bool dropok = false;
        int qmod = -1, mmod = 0;
        int p_fresh = 0;
        if (rec[10] & 2) {
            // augmented pattern handed over before its solve
            dropok = (rec[10] & 4) != 0;
            qmod = rec[11];
            mmod = rec[12];
        }
        if (status == ST_OK && q == 0 && nRh == 0) {
            // a column whose own rows exceed the register tiers: J = {k}, loop 0
            if (tid == 0) {
                S.Jlist[0] = k;
                int sl;
                hinsert<BLOGHJ>(S.hJ, k, sl);
            }
            __syncthreads();
            p_fresh = 1;
            linc = true;
            dropok = true;
            qmod = 0;
        }
        while (status == ST_OK) {
            // ================= J-hat from the pending dominant rows (step 5)
            int p = p_fresh;
            p_fresh = 0;
            if (nRh > 0) {
                if (tid == 0) S.cnt = 0;
                __syncthreads();
                bool ovf = false;
                for (int t = 0; t < nRh; ++t) {
                    const int row = S.Rh[t];
                    for (int64_t e = A.rowptr[row] + tid; e < A.rowptr[row + 1]; e += NT) {
                        const int col = A.colidx[e];
                        int sl;
                        if (hinsert<BLOGHJ>(S.hJ, col, sl)) {
                            const int ps = atomicAdd(&S.cnt, 1);
                            if (q + ps < BQMAX_BIG) S.skey[ps] = col; else ovf = true;
                        } else if (sl < 0) {
                            ovf = true;  // table full
                        }
                    }
                    if (__syncthreads_or(ovf)) { ovf = true; break; }
                }
                if (ovf) { status = ST_CAP; break; }
                p = S.cnt;
                // ascending order of the new columns (p < BQMAX_BIG: rank sort)
                if (tid < p) {
                    const int key = S.skey[tid];
                    int rank = 0;
                    for (int t = 0; t < p; ++t) rank += (S.skey[t] < key) ? 1 : 0;
                    S.Jlist[q + rank] = key;
                }
                __syncthreads();
                if (linc) ++l;
                nRh = 0;
                if (p == 0 && !first) need_solve = false;   // empty J-hat: no solve (step 6)
                else need_solve = true;
                dropok = (p > 0);
                qmod = (p > 0) ? q : (first ? -1 : q);
                mmod = m;
            }
            // ================= I-hat: rows of the new columns (step 5)
            if (need_solve && p > 0) {
                if (tid == 0) S.cnt = 0;
                __syncthreads();
                bool ovf = false;
                for (int t = 0; t < p; ++t) {
                    const int j = S.Jlist[q + t];
                    for (int64_t e = A.colptr[j] + tid; e < A.colptr[j + 1]; e += NT) {
                        const int row = A.rowidx[e];
                        int sl;
                        if (hinsert<BLOGH>(S.hI, row, sl)) {
                            const int ps = atomicAdd(&S.cnt, 1);
                            if (m + ps < ld && ps < SORTN) S.skey[ps] = row; else ovf = true;
                        } else if (sl < 0) {
                            ovf = true;  // table full
                        }
                    }
                    if (__syncthreads_or(ovf)) { ovf = true; break; }
                }
                if (ovf) { status = ST_CAP; break; }
                const int nn = S.cnt;
                // bitonic sort of the new rows (ascending), padded with INT_MAX
                int np2 = 1;
                while (np2 < nn) np2 <<= 1;
                for (int t = nn + tid; t < np2; t += NT) S.skey[t] = INT_MAX;
                if (tid == 0) S.misc = -1;
                __syncthreads();
                for (int kk = 2; kk <= np2; kk <<= 1) {
                    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                        for (int i = tid; i < np2; i += NT) {
                            const int ixj = i ^ jj;
                            if (ixj > i) {
                                const int a = S.skey[i], b = S.skey[ixj];
                                const bool up = (i & kk) == 0;
                                if ((a > b) == up) { S.skey[i] = b; S.skey[ixj] = a; }
                            }
                        }
                        __syncthreads();
                    }
                }
                for (int t = tid; t < nn; t += NT) {
                    const int row = S.skey[t];
                    const int li = m + t;
                    Il[li] = row;
                    rfl[li] = 0;
                    const int sl = hfind<BLOGH>(S.hI, row);
                    if (sl >= 0) S.hIv[sl] = (unsigned short)li;
                    if (row == k) {
                        S.misc = li;
                    }
                }
                __syncthreads();
                if (S.misc >= 0) {
                    kidx = S.misc;
                    if (kR) {
                        if (tid == 0) rfl[kidx] = 1;
                        kR = false;
                    }
                }
                m += nn;
                q += p;
                __syncthreads();
            } else if (p > 0) {
                q += p;
            }
            first = false;

            // ================= LS solve(s) on (I, J): gather, QR, back substitution
            int pass_drop = 0;
            while (need_solve && status == ST_OK) {
                const int qn = q;
                // The factor of the previous solve (columns 0..fq-1 on rows 0..fm-1) is
                // updated in place (Algorithm 1, step 7): the old columns are zero in the
                // new rows (every row of a column of J is already in I), so their
                // reflectors are unchanged; they are applied to the new columns, whose
                // own reflectors are then formed. The solve after a drop starts afresh.
                const int q0 = (pass_drop == 0 && fq <= qn) ? fq : 0;
                const int m0 = (q0 > 0) ? fm : 0;
                // gather: zero the new part of the block, scatter the new columns'
                // entries, Q^T e = e_k on the new rows
                for (int c = 0; c < q0; ++c)
                    for (int i = m0 + tid; i < m; i += NT) B[(int64_t)c * ld + i] = 0.0;
                for (int c = q0; c < qn; ++c)
                    for (int i = tid; i < m; i += NT) B[(int64_t)c * ld + i] = 0.0;
                for (int i = m0 + tid; i < m; i += NT) y[i] = (i == kidx) ? 1.0 : 0.0;
                __syncthreads();
                for (int c = q0; c < qn; ++c) {
                    const int j = S.Jlist[c];
                    for (int64_t e = A.colptr[j] + tid; e < A.colptr[j + 1]; e += NT) {
                        const int sl = hfind<BLOGH>(S.hI, A.rowidx[e]);
                        if (sl >= 0) B[(int64_t)c * ld + S.hIv[sl]] = A.val[e];
                    }
                }
                __syncthreads();
                // the stored reflectors, a panel of NB at a time, on the new columns
                for (int p0 = 0; p0 < q0; p0 += NB)
                    for (int c_lo = q0; c_lo < qn; c_lo += NCTMAX * 16)
                        panel_update(B, ld, y, m, qn, p0, min(NB, q0 - p0), c_lo, min(NCTMAX * 16, qn - c_lo), S,
                                     gred);
                bool singular = false;
                // Blocked Householder QR: panels of NB columns are factored column by
                // column; the rest of the block (and Q^T e) is updated once per panel
                // with the compact WY form Q_p = I - V T V^T (FP64 MFMA 16x16x4).
                for (int p0 = q0; p0 < qn; p0 += NB) {
                    const int pw = min(NB, qn - p0);
                    // blocks of up to 1024 rows: the panel in registers; taller: in the slab
                    if (m <= NT * 2) {
                        if (panel_factor_regs<2>(B, ld, m, p0, pw, S)) singular = true;
                    } else if (m <= NT * 4) {
                        if (panel_factor_regs<4>(B, ld, m, p0, pw, S)) singular = true;
                    } else
                    for (int j = p0; j < p0 + pw; ++j) {
                        double *bj = B + (int64_t)j * ld;
                        double s2 = 0.0;
                        for (int i = j + tid; i < m; i += NT) s2 += bj[i] * bj[i];
                        s2 = bsum(s2, S);
                        const double x0 = bj[j];
                        const double nx = sqrt(s2);
                        const double alpha = (x0 >= 0.0) ? -nx : nx;
                        const double vj = x0 - alpha;
                        const double be = (nx > 0.0) ? 1.0 / (nx * (nx + fabs(x0))) : 0.0;
                        if (!(nx > 0.0)) singular = true;
                        __syncthreads();
                        if (tid == 0) {
                            bj[j] = vj;
                            S.rd[j] = alpha;
                            S.bt[j] = be;
                        }
                        __syncthreads();
                        // the remaining columns of the panel, eight at a time
                        for (int c0 = j + 1; c0 < p0 + pw; c0 += 8) {
                            double part[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) part[u] = 0.0;
                            for (int i = j + tid; i < m; i += NT) {
                                const double vi = bj[i];
#pragma unroll
                                for (int u = 0; u < 8; ++u) {
                                    const int c = c0 + u;
                                    if (c < p0 + pw) part[u] += vi * B[(int64_t)c * ld + i];
                                }
                            }
#pragma unroll
                            for (int u = 0; u < 8; ++u) part[u] = gsum<16>(part[u]);
                            const int lane = tid & 63, w = tid >> 6;
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                part[u] += __shfl_xor(part[u], 16);
                                part[u] += __shfl_xor(part[u], 32);
                            }
                            if (lane == 0)
#pragma unroll
                                for (int u = 0; u < 8; ++u) S.red[w * 8 + u] = part[u];
                            __syncthreads();
                            double wv[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                double t = 0.0;
#pragma unroll
                                for (int ww = 0; ww < NW; ++ww) t += S.red[ww * 8 + u];
                                wv[u] = t * be;
                            }
                            __syncthreads();
                            for (int i = j + tid; i < m; i += NT) {
                                const double vi = bj[i];
#pragma unroll
                                for (int u = 0; u < 8; ++u) {
                                    const int c = c0 + u;
                                    if (c < p0 + pw) B[(int64_t)c * ld + i] -= wv[u] * vi;
                                }
                            }
                            __syncthreads();
                        }
                    }
                    // columns after the panel plus the right-hand side (column qn)
                    const int c_lo = p0 + pw, ntr = qn + 1 - c_lo;
                    if (ntr > 0) panel_update(B, ld, y, m, qn, p0, pw, c_lo, ntr, S, gred);
                }
                if (singular) { status = ST_SINGULAR; break; }
                fq = qn;
                fm = m;
                // back substitution by wave 0: lane c holds m_c
                if (tid < 64) {
                    double mc_lane = 0.0;
                    for (int j = qn - 1; j >= 0; --j) {
                        double part = 0.0;
                        for (int c = j + 1 + tid; c < qn; c += 64)
                            part += B[(int64_t)c * ld + j] * S.mt[c];
                        part = gsum<16>(part);
                        part += __shfl_xor(part, 16);
                        part += __shfl_xor(part, 32);
                        const double mj = (y[j] - part) / S.rd[j];
                        if (tid == 0) S.mt[j] = mj;
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        (void)mc_lane;
                    }
                }
                __syncthreads();
                double s = 0.0;
                for (int i = qn + tid; i < m; i += NT) s += y[i] * y[i];
                s = bsum(s, S);
                rn = sqrt(s + (kidx < 0 ? 1.0 : 0.0));
                if (qmod >= 0) fl += solve_flops(mmod, m, qmod, qn);
                // ---- dropping (Section 4), after the augment solve only
                if (pass_drop == 0 && dropok && P.drop != DROP_NONE) {
                    const double t = (P.drop == DROP_FIXED)
                                         ? P.tol
                                         : P.eps / ((double)qn * __longlong_as_double((long long)*A.norm1_bits));
                    int nk = 0;
                    for (int c = 0; c < qn; ++c) nk += (fabs(S.mt[c]) > t) ? 1 : 0;
                    if (nk < qn) {
                        __syncthreads();
                        if (tid == 0) {
                            if (nk == 0) {
                                int bc = 0;
                                for (int c = 1; c < qn; ++c) {
                                    const double a = fabs(S.mt[c]), b = fabs(S.mt[bc]);
                                    if (a > b || (a == b && S.Jlist[c] < S.Jlist[bc])) bc = c;
                                }
                                S.Jlist[0] = S.Jlist[bc];
                                nk = 1;
                            } else {
                                int w = 0;
                                for (int c = 0; c < qn; ++c)
                                    if (fabs(S.mt[c]) > t) S.Jlist[w++] = S.Jlist[c];
                            }
                            S.cnt = nk;
                        }
                        for (int t2 = tid; t2 < BHJ; t2 += NT) S.hJ[t2] = HEMPTY;
                        __syncthreads();
                        nk = S.cnt;
                        for (int c = tid; c < nk; c += NT) {
                            int sl;
                            hinsert<BLOGHJ>(S.hJ, S.Jlist[c], sl);
                        }
                        __syncthreads();
                        q = nk;
                        qmod = 0;
                        pass_drop = 1;
                        continue;  // solve on the kept pattern
                    }
                }
                break;
            }
            if (status != ST_OK) break;
            need_solve = false;

            // ================= stop test (step 3)
            if (rn <= P.eps || l >= P.lmax) break;

            // ================= dominant rows of r (step 4), r from the sparse columns
            if (tid == 0) {
                // ascending column order, kept in skey
                for (int c = 0; c < q; ++c) {
                    int rank = 0;
                    for (int t = 0; t < q; ++t) rank += (S.Jlist[t] < S.Jlist[c]) ? 1 : 0;
                    S.skey[rank] = c;
                }
            }
            for (int i = tid; i < m; i += NT) racc[i] = 0.0;
            __syncthreads();
            for (int t = 0; t < q; ++t) {
                const int c = S.skey[t];
                const int j = S.Jlist[c];
                const double mc = S.mt[c];
                for (int64_t e = A.colptr[j] + tid; e < A.colptr[j + 1]; e += NT) {
                    const int sl = hfind<BLOGH>(S.hI, A.rowidx[e]);
                    if (sl >= 0) {
                        const int li = S.hIv[sl];
                        racc[li] = __fma_rn(A.val[e], mc, racc[li]);
                    }
                }
                __syncthreads();
            }
            bool kcand = (kidx < 0) && !kR;
            int nsel = 0;
            for (int t = 0; t < P.c; ++t) {
                double a = -1.0;
                int g = INT_MAX;
                for (int i = tid; i < m; i += NT) {
                    if (rfl[i]) continue;
                    const double ri = racc[i] - ((i == kidx) ? 1.0 : 0.0);
                    if (ri == 0.0) continue;
                    const double ar = fabs(ri);
                    const int gi = Il[i];
                    if (ar > a || (ar == a && gi < g)) { a = ar; g = gi; }
                }
                bargmax(a, g, S);
                if (kcand && (1.0 > a || (1.0 == a && k < g))) { a = 1.0; g = k; }
                if (a < 0.0) break;
                if (tid == 0) S.Rh[t] = g;
                nsel = t + 1;
                if (kcand && g == k) {
                    kcand = false;
                    kR = true;
                } else {
                    const int sl = hfind<BLOGH>(S.hI, g);
                    if (tid == 0 && sl >= 0) rfl[S.hIv[sl]] = 1;
                }
                __syncthreads();
            }
            if (nsel == 0) break;  // no candidate row left: r = 0 (Section 3)
            nRh = nsel;
            linc = true;
            __syncthreads();
        }

        // ================= output (rows of m_k ascending)
        const int qq = (status == ST_OK) ? q : 0;
        const int64_t slot = args.arena_base + pos * BQMAX_BIG;  // one slot per record
        for (int c = tid; c < qq; c += NT) {
            const int jc = S.Jlist[c];
            int rank = 0;
            for (int t = 0; t < qq; ++t) rank += (S.Jlist[t] < jc) ? 1 : 0;
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
            // R of the final solve: strict upper part in the block, diagonal in rd
            if (tid == 0) {
                const long long fo = (qq > 0) ? fac_reserve(args.out, qq) : -1LL;
                args.out.foff[ucol] = fo;
                S.cnt = (int)(fo & 0xffffffffLL);
                S.misc = (int)(fo >> 32);
            }
            __syncthreads();
            const long long fo = ((long long)S.misc << 32) | (long long)(unsigned)S.cnt;
            if (fo >= 0) {
                double *F = args.out.fac + fo;
                for (int c = tid; c < qq; c += NT) F[c] = (double)S.Jlist[c];
                for (int t = tid; t < qq * qq; t += NT) {
                    const int i = t / qq, c = t % qq;
                    if (c >= i) F[fac_row(qq, i) + (c - i)] = (c == i) ? S.rd[i] : B[(int64_t)c * ld + i];
                }
            }
        }
        __syncthreads();
    }
}

int64_t big_scratch_stride(int64_t ld) {
    // doubles per workgroup: block, Q^T e, residual, then rows (int) and flags (byte)
    return (int64_t)BQMAX_BIG * ld + 2 * ld + (ld * 5 + 7) / 8 + 8 + REDN;
}

void launch_big_kernel(const BigArgs &a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(big_kernel, dim3(blocks), dim3(NT), 0, s, a);
}

}  // namespace rsai
