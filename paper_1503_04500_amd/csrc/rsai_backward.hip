// Adjoint of the fixed-pattern LS map A -> M (pattern of M fixed, each m_k the
// solution of (2.3) on I_k = nonzero rows of A(:, J_k)).
//
// From the normal equations A_k^T (A_k m - e) = 0 of (2.3):
//   dm = -(A_k^T A_k)^{-1} (dA_k^T r + A_k^T dA_k m),   r = A_k m - e_k(I_k),
// so for an upstream gradient g = dL/dm and z = (A_k^T A_k)^{-1} g = R^{-1} R^{-T} g:
//   dL/dA_k = -(r z^T + (A_k z) m^T).
// The Frobenius term w * sum_k ||A m_k - e_k||^2 adds 2 w r m^T (its part through M
// vanishes because A_k^T r = 0). Contributions land on the structural nonzeros of
// A(I_k, J_k) and are accumulated with atomics into dA.
//
// One group of 16 lanes per column: the block A(I_k, J_k) is re-gathered and
// factorised by Householder QR in registers (row i in lane i mod 16), then
// A_k z = Q [R z; 0] = Q [u; 0] with R^T u = g, and r = -Q [0; (Q^T e)(q:m)].
#include <climits>

#include <algorithm>

#include "rsai_kernels.h"

namespace rsai {

namespace {
constexpr int BG = 16, BRPL = 4, BQMAX = 32, BSTAGE = 4;
constexpr int BMMAX = BG * BRPL;
constexpr int BGPW = 64 / BG;
constexpr int BLOGHSI = ilog2ceil(2 * BMMAX);
constexpr int BHSI = 1 << BLOGHSI;

struct BLds {
    double stage[BSTAGE * BMMAX];
    double rdiag[BQMAX];
    double beta[BQMAX];
    double zS[BQMAX];
    int Jl[BQMAX];
    int Il[BMMAX];
    int hI[BHSI];
    int hIv[BHSI];
    int newk[BMMAX];
    int news[BMMAX];
    int cnt;
    int pad;
    long long cbase;  // fixed-order mode: first slot of the column's contributions
};
}  // namespace

int backward_max_cols() { return BQMAX; }
int backward_max_rows() { return BMMAX; }

// Five values: largest |J_k|; over the columns without a kept factor (mask[k] < 0,
// or all columns without a mask) the largest |I_k|, their count and their largest
// |J_k|; the number of columns with a factor and |J_k| > 32. Reduced per workgroup
// first, then one atomic per workgroup and value into one of MAX2_COPIES copies of
// the five words (out[copy * 5 + value], copy = workgroup % MAX2_COPIES), so that
// fewer workgroups meet on one address; max2_combine folds the copies on the host.
__global__ __launch_bounds__(256) void k_max2(int64_t n, const int32_t *a, const int32_t *b, const int64_t *mask,
                                              int32_t *outc) {
    __shared__ int red[5][4];
    int v[5] = {0, 0, 0, 0, 0};  // max a, max b, count, max a (no factor), count large
    // U columns per thread with their loads in flight together
    constexpr int U = 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i0 < n; i0 += U * stride) {
        int av[U], bv[U];
        bool nf[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * stride;
            av[u] = -1;
            bv[u] = 0;
            nf[u] = false;
            if (i < n) {
                av[u] = a[i];
                bv[u] = b[i];
                nf[u] = !mask || mask[i] < 0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (av[u] < 0) continue;
            v[0] = max(v[0], av[u]);
            if (nf[u]) {
                v[1] = max(v[1], bv[u]);
                v[3] = max(v[3], av[u]);
                ++v[2];
            } else if (av[u] > 32) {
                ++v[4];
            }
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        v[0] = max(v[0], __shfl_xor(v[0], off));
        v[1] = max(v[1], __shfl_xor(v[1], off));
        v[2] += __shfl_xor(v[2], off);
        v[3] = max(v[3], __shfl_xor(v[3], off));
        v[4] += __shfl_xor(v[4], off);
    }
    if (lane == 0)
        for (int t = 0; t < 5; ++t) red[t][w] = v[t];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < 4; ++q) {
            v[0] = max(v[0], red[0][q]);
            v[1] = max(v[1], red[1][q]);
            v[2] += red[2][q];
            v[3] = max(v[3], red[3][q]);
            v[4] += red[4][q];
        }
        int32_t *out5 = outc + (blockIdx.x % MAX2_COPIES) * 5;
        atomicMax(&out5[0], v[0]);
        atomicMax(&out5[1], v[1]);
        atomicAdd(&out5[2], v[2]);
        atomicMax(&out5[3], v[3]);
        atomicAdd(&out5[4], v[4]);
    }
}
void max2_combine(const int32_t *h, int32_t *out5) {
    for (int t = 0; t < 5; ++t) out5[t] = h[t];
    for (int c = 1; c < MAX2_COPIES; ++c) {
        const int32_t *q = h + c * 5;
        out5[0] = std::max(out5[0], q[0]);
        out5[1] = std::max(out5[1], q[1]);
        out5[2] += q[2];
        out5[3] = std::max(out5[3], q[3]);
        out5[4] += q[4];
    }
}

void launch_max2(int64_t n, const int32_t *a, const int32_t *b, const int64_t *mask, int32_t *outc, hipStream_t s) {
    // few blocks: each ends with five atomics on the same five words
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 256));
    hipLaunchKernelGGL(k_max2, dim3((unsigned)blocks), dim3(256), 0, s, n, a, b, mask, outc);
}

__global__ __launch_bounds__(64) void backward_kernel(BwdArgs a) {
    constexpr int G = BG, RPL = BRPL, QMAX = BQMAX, MMAX = BMMAX;
    __shared__ BLds lds[BGPW];
    const int gl = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    BLds &S = lds[grp];
    const MatDev A = a.mats[a.mat];
    const int64_t n = a.n;
    const int64_t gstride = (int64_t)gridDim.x * BGPW;
    // uniform trip count over the wave so every barrier is reached by all lanes
    const int64_t iters = (n + gstride - 1) / gstride;

    for (int64_t itk = 0; itk < iters; ++itk) {
        const int64_t k = itk * gstride + (int64_t)blockIdx.x * BGPW + grp;
        bool act = k < n;
        int q = 0, m = 0;
        int64_t mb = 0;
        if (act) {
            mb = a.Mcolptr[k];
            q = (int)(a.Mcolptr[k + 1] - mb);
            if (q > QMAX || q < 1) {
                if (q > QMAX && gl == 0 && !(a.foff && a.foff[k] >= 0)) atomicOr(a.err, 8);
                act = false;
            }
            if (a.foff && a.foff[k] >= 0) act = false;  // kept factor: the factored kernel
        }
        bool any_g = false;
        if (act && a.gM)
            for (int c = 0; c < q; ++c) any_g |= (a.gM[mb + c] != 0.0);
        if (act && !any_g && a.w_frob == 0.0) act = false;
        for (int t = gl; t < BHSI; t += G) S.hI[t] = HEMPTY;
        if (act) {
            for (int t = gl; t < q; t += G) S.Jl[t] = a.Mrowidx[mb + t];
            if (gl == 0) S.cnt = 0;
        }
        __syncthreads();
        // ---- I_k: rows of A(:, J_k)
        bool ovf = false;
        if (act) {
            for (int c = 0; c < q; ++c) {
                const int j = S.Jl[c];
                for (int64_t e = A.colptr[j] + gl; e < A.colptr[j + 1]; e += G) {
                    int sl;
                    if (hinsert<BLOGHSI>(S.hI, A.rowidx[e], sl)) {
                        int ps = atomicAdd(&S.cnt, 1);
                        if (ps < MMAX) { S.newk[ps] = A.rowidx[e]; S.news[ps] = sl; }
                    }
                }
                // keep the table below MMAX + one column: checked after each column
                if (S.cnt > MMAX) { ovf = true; break; }
            }
        }
        __syncthreads();
        if (act) {
            m = S.cnt;
            if (m > MMAX || ovf) {
                if (gl == 0) atomicOr(a.err, 8);
                act = false;
            }
        }
        int kidx = -1;
        if (act) {
            for (int s = 0; s < (MMAX + G - 1) / G; ++s) {
                const int idx = s * G + gl;
                if (idx < m) {
                    const int key = S.newk[idx];
                    int rank = 0;
                    for (int t = 0; t < m; ++t) rank += (S.newk[t] < key) ? 1 : 0;
                    S.Il[rank] = key;
                    S.hIv[S.news[idx]] = rank;
                    if (key == (int)k) kidx = rank;
                }
            }
        }
        kidx = gmax_i<G>(kidx);
        __syncthreads();
        // ---- gather A(I, J) into registers
        double b[RPL][QMAX];
        double y[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            y[r] = (act && r * G + gl == kidx) ? 1.0 : 0.0;
#pragma unroll
            for (int c = 0; c < QMAX; ++c) b[r][c] = 0.0;
        }
        const int qmaxw = wave_max_i(act ? q : 0);
        for (int c0 = 0; c0 < qmaxw; c0 += BSTAGE) {
#pragma unroll
            for (int s = 0; s < BSTAGE; ++s)
#pragma unroll
                for (int r = 0; r < RPL; ++r) S.stage[s * MMAX + r * G + gl] = 0.0;
            __syncthreads();
            if (act) {
#pragma unroll
                for (int s = 0; s < BSTAGE; ++s) {
                    const int c = c0 + s;
                    if (c < q) {
                        const int j = S.Jl[c];
                        for (int64_t e = A.colptr[j] + gl; e < A.colptr[j + 1]; e += G) {
                            const int sl = hfind<BLOGHSI>(S.hI, A.rowidx[e]);
                            const int li = sl >= 0 ? S.hIv[sl] : -1;
                            if (li >= 0 && li < MMAX) S.stage[s * MMAX + li] = A.val[e];
                        }
                    }
                }
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int c = 0; c < QMAX; ++c) {
                    const int s = c - c0;
                    if (s >= 0 && s < BSTAGE && c < q)
#pragma unroll
                        for (int r = 0; r < RPL; ++r) b[r][c] = S.stage[s * MMAX + r * G + gl];
                }
            }
            __syncthreads();
        }
        // ---- Householder QR of A(I, J) and Q^T e
#pragma unroll
        for (int j = 0; j < QMAX; ++j) {
            if (j >= qmaxw) continue;
            const bool ja = act && j < q;
            double s2 = 0.0, x0p = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = r * G + gl;
                if (i >= j) s2 += b[r][j] * b[r][j];
                if (i == j) x0p = b[r][j];
            }
            s2 = gsum<G>(s2);
            const double x0 = gsum<G>(x0p);
            const double nx = sqrt(s2);
            const double alpha = (x0 >= 0.0) ? -nx : nx;
            const double vj = x0 - alpha;
            const double bj = (nx > 0.0) ? 1.0 / (nx * (nx + fabs(x0))) : 0.0;
            if (ja) {
#pragma unroll
                for (int r = 0; r < RPL; ++r)
                    if (r * G + gl == j) b[r][j] = vj;
                if (gl == j % G) { S.rdiag[j] = alpha; S.beta[j] = bj; }
            }
#pragma unroll
            for (int c = 0; c < QMAX; ++c) {
                    if (c <= j) continue;
                if (c >= qmaxw) continue;
                double w = 0.0;
#pragma unroll
                for (int r = 0; r < RPL; ++r)
                    if (r * G + gl >= j) w += b[r][j] * b[r][c];
                w = gsum<G>(w);
                if (ja && c < q) {
#pragma unroll
                    for (int r = 0; r < RPL; ++r)
                        if (r * G + gl >= j) b[r][c] -= bj * w * b[r][j];
                }
            }
            double w = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r)
                if (r * G + gl >= j) w += b[r][j] * y[r];
            w = gsum<G>(w);
            if (ja) {
#pragma unroll
                for (int r = 0; r < RPL; ++r)
                    if (r * G + gl >= j) y[r] -= bj * w * b[r][j];
            }
        }
        __syncthreads();  // rdiag / beta visible to every lane of the group
        // ---- u = R^{-T} g (forward substitution over the rows of R); lane keeps
        // u_i for its own rows in ul
        double ul[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) ul[r] = 0.0;
#pragma unroll
        for (int j = 0; j < QMAX; ++j) {
            if (j >= qmaxw) continue;
            double part = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r)
                if (r * G + gl < j) part += b[r][j] * ul[r];
            part = gsum<G>(part);
            double uj = 0.0;
            if (act && j < q) uj = ((a.gM ? a.gM[mb + j] : 0.0) - part) / S.rdiag[j];
            if (gl == j % G) ul[j / G] = uj;
        }
        // ---- z = R^{-1} u (back substitution); z_j goes to LDS
        {
            double t[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) t[r] = ul[r];
#pragma unroll
            for (int j = QMAX - 1; j >= 0; --j) {
                if (j >= qmaxw) continue;
                double val = 0.0;
                if (gl == j % G && act && j < q) val = t[j / G] / S.rdiag[j];
                const double zj = gsum<G>(val);
                if (act && j < q) {
                    if (gl == 0) S.zS[j] = zj;
#pragma unroll
                    for (int r = 0; r < RPL; ++r)
                        if (r * G + gl < j) t[r] -= b[r][j] * zj;
                }
            }
        }
        // ---- A_k z = Q [u; 0] and r = -Q [0; (Q^T e)(q:m)]: reflectors in reverse
        double az[RPL], rr[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = r * G + gl;
            az[r] = (i < q) ? ul[r] : 0.0;
            rr[r] = (i >= q && i < m) ? y[r] : 0.0;
        }
#pragma unroll
        for (int j = QMAX - 1; j >= 0; --j) {
            if (j >= qmaxw) continue;
            double w1 = 0.0, w2 = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r)
                if (r * G + gl >= j) {
                    w1 += b[r][j] * az[r];
                    w2 += b[r][j] * rr[r];
                }
            w1 = gsum<G>(w1);
            w2 = gsum<G>(w2);
            if (act && j < q) {
                const double bj = S.beta[j];
#pragma unroll
                for (int r = 0; r < RPL; ++r)
                    if (r * G + gl >= j) {
                        az[r] -= bj * w1 * b[r][j];
                        rr[r] -= bj * w2 * b[r][j];
                    }
            }
        }
        // stage r (negated: r = -z) and A_k z per local row
        if (act) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = r * G + gl;
                S.stage[i] = -rr[r];
                S.stage[MMAX + i] = az[r];
            }
        }
        __syncthreads();
        // ---- scatter onto the nonzeros of A(:, J_k) (the fixed-order mode appends
        // the contributions at the column's reserved slots instead)
        const bool det = a.ckey != nullptr;
        if (det && act && gl == 0) {
            int tot = 0;
            for (int c = 0; c < q; ++c) tot += (int)(A.colptr[S.Jl[c] + 1] - A.colptr[S.Jl[c]]);
            S.cbase = (long long)atomicAdd(a.ccur, (unsigned long long)tot);
        }
        __syncthreads();
        if (act) {
            const double w2 = 2.0 * a.w_frob;
            long long slot0 = det ? S.cbase : 0;
#pragma unroll
            for (int c = 0; c < QMAX; ++c) {
                if (c < q) {
                    const int j = S.Jl[c];
                    const double zc = S.zS[c], mc = a.Mval[mb + c];
                    const int64_t c0 = A.colptr[j], c1 = A.colptr[j + 1];
                    for (int64_t e = c0 + gl; e < c1; e += G) {
                        const int sl = hfind<BLOGHSI>(S.hI, A.rowidx[e]);
                        const int li = sl >= 0 ? S.hIv[sl] : -1;
                        double g = 0.0;
                        if (li >= 0) {
                            const double ri = S.stage[li], azi = S.stage[MMAX + li];
                            g = -(ri * zc + azi * mc) + w2 * ri * mc;
                        }
                        if (det) {
                            const long long slot = slot0 + (e - c0);
                            a.ckey[slot] = ((unsigned long long)e << 32) | (unsigned long long)(unsigned)k;
                            a.cval[slot] = g;
                        } else if (li >= 0) {
                            atomicAdd(&a.dA[e], g);
                        }
                    }
                    slot0 += c1 - c0;
                }
            }
        }
        __syncthreads();
    }
}

void launch_backward(const BwdArgs &a, int waves, hipStream_t s) {
    hipLaunchKernelGGL(backward_kernel, dim3(waves), dim3(64), 0, s, a);
}

// ---------------------------------------------------------------- kept factors
// The same adjoint for the columns whose R factor the build kept: z = R^{-1} R^{-T} g
// by two triangular solves on the stored R (R^T R = A_k^T A_k for any QR of A_k,
// compressed or not), then r = A_k m - e_k and A_k z. For small column sets the
// entries of the columns of J sit in registers and r, A_k z are accumulated per row
// in LDS; otherwise row by row from the sparse data: the columns of row i (row
// pattern of A) that belong to J_k, each value a_ij found by binary search in
// column j (rows ascending). No dense block, so |I_k| is not limited here.
//
// The kernel is bound by the latency of each column's dependent steps, so its
// throughput is the number of columns resident per CU: the LDS record of a column
// is split by phase (the solves, then the accumulation) and the two halves share
// storage.
namespace {
// sum over a group of G lanes (G up to 64), every lane of the group gets it
template <int G>
__device__ __forceinline__ double group_sum(double x) {
    if constexpr (G <= 16) {
        return gsum<G>(x);
    } else {
        x = gsum<16>(x);
        x += __shfl_xor(x, 16);
        if constexpr (G == 64) x += __shfl_xor(x, 32);
        return x;
    }
}
// inclusive prefix sum over a group of G lanes (lane gl of the group)
template <int G>
__device__ __forceinline__ int group_scan(int x, int gl) {
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        const int y = __shfl_up(x, d, G);
        if (gl >= d) x += y;
    }
    return x;
}
// entries of the columns of J held in registers (small path), distinct rows
// accumulated in LDS and the row hash
constexpr int FM = 128, FR = 64, FLOGHI = 7, FHI = 1 << FLOGHI;
template <int FQ>
struct FLds {
    // R is staged here for the two triangular solves when |J_k| <= RQ, so that their
    // q dependent steps read LDS instead of waiting on global memory; larger
    // records are read in place
    static constexpr int RQ = FQ <= 32 ? 20 : 0;
    static constexpr int RSZ = RQ > 0 ? RQ * (RQ + 1) / 2 : 1;
    double z[FQ];  // g (ascending order) until the back substitution writes z over it
    int js[FQ];    // J ascending (the order of M's column)
    int cnt;
    long long cbase;  // fixed-order mode: first slot of the column's contributions
    union {
        struct {             // the triangular solves
            double R[RSZ];   // R row by row
            double u[FQ];    // g in solve order, then R^{-T} g
            int rk[FQ];      // ascending position of each solve-order column
        } sv;
        struct {             // r and A_k z
            int64_t cb[FQ];  // first entry of each column of J
            int pre[FQ + 1]; // prefix of the column lengths
            double racc[FR]; // r_i and (A_k z)_i by local row
            double aacc[FR];
            int hI[FHI];     // row -> local row
            unsigned char hIv[FHI];
        } acc;
    } w;
};
// position of column key in the ascending J (q entries), or -1
__device__ __forceinline__ int jpos(const int *js, int q, int key) {
    int lo = 0, hi = q - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = js[mid];
        if (v == key) return mid;
        if (v < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}
// value of A(i, j), or 0 if not stored (rows of a column ascending)
__device__ __forceinline__ double aval(const MatDev &A, int j, int i) {
    int64_t lo = A.colptr[j], hi = A.colptr[j + 1] - 1;
    while (lo <= hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int v = A.rowidx[mid];
        if (v == i) return A.val[mid];
        if (v < i) lo = mid + 1; else hi = mid - 1;
    }
    return 0.0;
}
// offset of row i of R (upper triangle stored row by row, q columns)
__device__ __forceinline__ int rrow(int q, int i) { return i * q - i * (i - 1) / 2; }
}  // namespace

int backward_factored_max_cols() { return 128; }

// (at least four waves per SIMD: the register budget is cut to 128 per lane, which the
// small instance, R staged in LDS, needs to keep four waves; one register more cost it a
// wave and a fifth of its speed)
template <int FG, int FQ, int QLO>
__global__ __launch_bounds__(64, 4) void backward_factored_kernel(BwdArgs a) {
    constexpr int G = FG, FGPW = 64 / FG, CPL = FQ / G;
    using LT = FLds<FQ>;
    static_assert(FQ % G == 0 && FM % G == 0, "columns and entries split evenly over the lanes");
    __shared__ LT lds[FGPW];
    const int gl = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    LT &S = lds[grp];
    const MatDev A = a.mats[a.mat];
    const int64_t n = a.n;
    // each XCD takes a contiguous eighth of the columns (block b runs on XCD b % 8):
    // neighbouring columns add into the same entries of A, and their atomics then
    // meet in one L2. The trip count is uniform within a block.
    int64_t hi = n, k = (int64_t)blockIdx.x * FGPW + grp, gstride = (int64_t)gridDim.x * FGPW, lo = 0;
    if (gridDim.x >= 8) {
        const int x = blockIdx.x % 8, w = blockIdx.x / 8, nwx = (gridDim.x - x + 7) / 8;
        const int64_t chunk = (n + 7) / 8;
        lo = (int64_t)x * chunk;
        hi = lo + chunk < n ? lo + chunk : n;
        k = lo + (int64_t)w * FGPW + grp;
        gstride = (int64_t)nwx * FGPW;
    }
    const int64_t iters = hi > lo ? (hi - lo + gstride - 1) / gstride : 0;
    uint64_t gmask = ~0ull;
    if constexpr (G < 64) gmask = (1ull << G) - 1;
    // the header of the group's first column; each iteration loads the next one's
    int64_t nfo = -1, nmb = 0, nme = 0;
    if (k < hi) {
        nfo = a.foff[k];
        nmb = a.Mcolptr[k];
        nme = a.Mcolptr[k + 1];
    }
    for (int64_t itk = 0; itk < iters; ++itk, k += gstride) {
        const int64_t fo = nfo, mb = nmb;
        const int q = (int)(nme - nmb);
        bool act = k < hi && fo >= 0 && q >= QLO && q <= FQ;
        {
            const int64_t kn = k + gstride;
            nfo = -1;
            nmb = nme = 0;
            if (kn < hi) {
                nfo = a.foff[kn];
                nmb = a.Mcolptr[kn];
                nme = a.Mcolptr[kn + 1];
            }
        }
        const double *F = a.fac + (act ? fo : 0);
        const bool staged = act && q <= LT::RQ;
        // the pattern, the record's solve order, the incoming gradient and the column
        // extents of J, loaded by the group's lanes together; R staged in LDS
        int fj[CPL], clen[CPL];
        int64_t cbr[CPL];
        bool nzg = false;
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            const int c = gl + t * G;
            fj[t] = -1;
            clen[t] = 0;
            cbr[t] = 0;
            if (act && c < q) {
                const int j = a.Mrowidx[mb + c];
                S.js[c] = j;
                fj[t] = (int)F[c];
                const double gc = a.gM ? a.gM[mb + c] : 0.0;
                S.z[c] = gc;
                nzg |= gc != 0.0;
                cbr[t] = A.colptr[j];
                clen[t] = (int)(A.colptr[j + 1] - cbr[t]);
            }
        }
        if (staged)
            for (int t = gl; t < q * (q + 1) / 2; t += G) S.w.sv.R[t] = F[q + t];
        if (act && !(((__ballot(nzg) >> (grp * G)) & gmask) != 0) && a.w_frob == 0.0) act = false;
        wave_sync();
        const double *Fr = staged ? S.w.sv.R : F + q;
        // solve-order column -> ascending position; g in solve order
        if (act) {
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                const int c = gl + t * G;
                if (c < q) {
                    const int p = jpos(S.js, q, fj[t]);
                    S.w.sv.rk[c] = p;
                    S.w.sv.u[c] = p >= 0 ? S.z[p] : 0.0;
                }
            }
        }
        wave_sync();
        // u = R^{-T} g (forward substitution)
        for (int j = 0; j < FQ; ++j) {
            if (!wave_any(act && j < q)) break;
            double part = 0.0;
            if (act && j < q)
                for (int i = gl; i < j; i += G) part += Fr[rrow(q, i) + (j - i)] * S.w.sv.u[i];
            part = group_sum<G>(part);
            if (act && j < q && gl == 0) S.w.sv.u[j] = (S.w.sv.u[j] - part) / Fr[rrow(q, j)];
            wave_sync();
        }
        // z = R^{-1} u (back substitution), stored by ascending position
        for (int j = FQ - 1; j >= 0; --j) {
            if (!wave_any(act && j < q)) continue;
            double part = 0.0;
            if (act && j < q)
                for (int c = j + 1 + gl; c < q; c += G) {
                    const int rc = S.w.sv.rk[c];
                    part += Fr[rrow(q, j) + (c - j)] * (rc >= 0 ? S.z[rc] : 0.0);
                }
            part = group_sum<G>(part);
            if (act && j < q && gl == 0) {
                const int rj = S.w.sv.rk[j];
                if (rj >= 0) S.z[rj] = (S.w.sv.u[j] - part) / Fr[rrow(q, j)];
            }
            wave_sync();
        }
        // the columns of J: first entries and the prefix of their lengths
        {
            int base = 0;
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                const int c = gl + t * G;
                const int inc = group_scan<G>(clen[t], gl);
                if (act && c < q) {
                    S.w.acc.cb[c] = cbr[t];
                    S.w.acc.pre[c + 1] = base + inc;
                }
                base += __shfl(inc, G - 1, G);
            }
        }
        for (int t = gl; t < FHI; t += G) S.w.acc.hI[t] = HEMPTY;
        if (gl == 0) {
            S.w.acc.pre[0] = 0;
            S.cnt = 0;
        }
        wave_sync();
        const int tot = act ? S.w.acc.pre[q] : 0;
        const bool det = a.ckey != nullptr;
        if (det && act && gl == 0) S.cbase = (long long)atomicAdd(a.ccur, (unsigned long long)tot);
        wave_sync();
        // small I_k: r and A_k z accumulated once per row in LDS (atomics: not in the
        // fixed-order mode)
        bool small = act && tot <= FM && !det;
        if (wave_any(small)) {
            // entries u = gl + t G of the flattened columns, loaded once (all loads in
            // flight together) and used by the three passes
            constexpr int EPL = FM / G;
            int erow[EPL], ecol[EPL], eli[EPL];
            int64_t eidx[EPL];
            double ev[EPL], em[EPL];
#pragma unroll
            for (int t = 0; t < EPL; ++t) {
                const int u = gl + t * G;
                erow[t] = -1;
                ecol[t] = 0;
                eli[t] = 0;
                eidx[t] = 0;
                ev[t] = 0.0;
                em[t] = 0.0;
                if (small && u < tot) {
                    int lo = 0, hi = q - 1;  // the column holding entry u
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (S.w.acc.pre[mid] <= u) lo = mid; else hi = mid - 1;
                    }
                    const int64_t e = S.w.acc.cb[lo] + (u - S.w.acc.pre[lo]);
                    ecol[t] = lo;
                    eidx[t] = e;
                    erow[t] = A.rowidx[e];
                    ev[t] = A.val[e];
                    em[t] = a.Mval[mb + lo];
                }
            }
            // the distinct rows; more than FR of them send the column to the row path
#pragma unroll
            for (int t = 0; t < EPL; ++t) {
                if (erow[t] >= 0) {
                    int sl;
                    if (hinsert<FLOGHI>(S.w.acc.hI, erow[t], sl)) {
                        const int li = atomicAdd(&S.cnt, 1);
                        S.w.acc.hIv[sl] = (unsigned char)li;
                        if (li < FR) {
                            S.w.acc.racc[li] = 0.0;
                            S.w.acc.aacc[li] = 0.0;
                        }
                    } else if (sl < 0) {
                        atomicMax(&S.cnt, FR + 1);
                    }
                }
            }
            wave_sync();
            small = small && S.cnt <= FR;
            if (small) {
#pragma unroll
                for (int t = 0; t < EPL; ++t) {
                    if (erow[t] >= 0) {
                        const int li = S.w.acc.hIv[hfind<FLOGHI>(S.w.acc.hI, erow[t])];
                        eli[t] = li;
                        atomicAdd(&S.w.acc.racc[li], ev[t] * em[t]);
                        atomicAdd(&S.w.acc.aacc[li], ev[t] * S.z[ecol[t]]);
                    }
                }
            }
            wave_sync();
            if (small) {
                const double w2 = 2.0 * a.w_frob;
#pragma unroll
                for (int t = 0; t < EPL; ++t) {
                    if (erow[t] >= 0) {
                        const int li = eli[t];
                        const double ri = S.w.acc.racc[li] - ((erow[t] == (int)k) ? 1.0 : 0.0);
                        const double azi = S.w.acc.aacc[li];
                        const double zc = S.z[ecol[t]], mc = em[t];
                        atomicAdd(&a.dA[eidx[t]], -(ri * zc + azi * mc) + w2 * ri * mc);
                    }
                }
            }
            wave_sync();
        }
        // larger I_k: r_i and (A_k z)_i from row i's pattern, per entry; in the
        // fixed-order mode over J_k in ascending order (the row pattern's order is
        // not fixed) and appended instead of added
        if (act && !small) {
            const double w2 = 2.0 * a.w_frob;
            const long long cbase = det ? S.cbase : 0;
            for (int c = 0; c < q; ++c) {
                const int j = S.js[c];
                const double zc = S.z[c], mc = a.Mval[mb + c];
                const int64_t c0 = A.colptr[j];
                for (int64_t e = c0 + gl; e < A.colptr[j + 1]; e += G) {
                    const int i = A.rowidx[e];
                    double ri = (i == (int)k) ? -1.0 : 0.0, azi = 0.0;
                    if (det) {
                        for (int t = 0; t < q; ++t) {
                            const int jj = S.js[t];
                            const double aij = (jj == j) ? A.val[e] : aval(A, jj, i);
                            ri += aij * a.Mval[mb + t];
                            azi += aij * S.z[t];
                        }
                    } else {
                        for (int64_t f = A.rowptr[i]; f < A.rowptr[i + 1]; ++f) {
                            const int jj = A.colidx[f];
                            const int t = jpos(S.js, q, jj);
                            if (t < 0) continue;
                            const double aij = (jj == j) ? A.val[e] : aval(A, jj, i);
                            ri += aij * a.Mval[mb + t];
                            azi += aij * S.z[t];
                        }
                    }
                    const double gv = -(ri * zc + azi * mc) + w2 * ri * mc;
                    if (det) {
                        const long long slot = cbase + S.w.acc.pre[c] + (e - c0);
                        a.ckey[slot] = ((unsigned long long)e << 32) | (unsigned long long)(unsigned)k;
                        a.cval[slot] = gv;
                    } else {
                        atomicAdd(&a.dA[e], gv);
                    }
                }
            }
        }
        wave_sync();
    }
}

// ---------------------------------------------------------------- recomputed factors
// Columns without a kept factor that are larger than the refactorising kernel's
// register block (|J_k| > 32 or |I_k| > 64) get a factor recomputed here, into a
// temporary store, and are then differentiated by the factored kernel. The factor is
// the Cholesky factor L of the normal-equation matrix A_k^T A_k (R = L^T satisfies
// R^T R = A_k^T A_k, all the factored kernel needs), so the dense block A(I_k, J_k)
// is never formed: entry (a, b) is the dot product of the sparse columns J_a and J_b,
// merged along their ascending row lists, and |I_k| is not limited.
namespace {
constexpr int RNT = 256;
constexpr int RQMAX = 128;
constexpr int RPACK = RQMAX * (RQMAX + 1) / 2;
struct RLds {
    double G[RPACK];   // lower triangle of A_k^T A_k, then of L, row by row
    int64_t cb[RQMAX];
    int cl[RQMAX];
    int js[RQMAX];
    int flag;
};
__device__ __forceinline__ int tri(int a, int b) { return a * (a + 1) / 2 + b; }  // a >= b
// (a, b) with a >= b of packed lower-triangle position p
__device__ __forceinline__ void untri(int p, int &a, int &b) {
    int x = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
    while ((x + 1) * (x + 2) / 2 <= p) ++x;
    while (x * (x + 1) / 2 > p) --x;
    a = x;
    b = p - x * (x + 1) / 2;
}
__device__ __forceinline__ bool needs_refactor(const RefArgs &r, int64_t k, int q) {
    if (q < 1 || q > RQMAX) return false;
    if (r.foff && r.foff[k] >= 0) return false;
    return q > r.small_cols || r.nI[k] > r.small_rows;
}
}  // namespace

int refactor_max_cols() { return RQMAX; }

// doubles of the records to recompute (one atomic per workgroup)
__global__ __launch_bounds__(256) void k_refactor_size(RefArgs r, unsigned long long *total) {
    unsigned long long t = 0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < r.n; k += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(r.Mcolptr[k + 1] - r.Mcolptr[k]);
        if (needs_refactor(r, k, q)) t += (unsigned long long)(q + q * (q + 1) / 2);
    }
    for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off);
    if ((threadIdx.x & 63) == 0 && t) atomicAdd(total, t);
}

__global__ __launch_bounds__(RNT) void k_refactor(RefArgs r) {
    __shared__ RLds S;
    const int tid = threadIdx.x;
    const MatDev A = r.mats[r.mat];
    for (int64_t k = blockIdx.x; k < r.n; k += gridDim.x) {
        const int64_t mb = r.Mcolptr[k];
        const int q = (int)(r.Mcolptr[k + 1] - mb);
        if (!needs_refactor(r, k, q)) continue;  // uniform over the workgroup
        if (tid < q) {
            const int j = r.Mrowidx[mb + tid];
            S.js[tid] = j;
            S.cb[tid] = A.colptr[j];
            S.cl[tid] = (int)(A.colptr[j + 1] - S.cb[tid]);
        }
        if (tid == 0) S.flag = 0;
        __syncthreads();
        // A_k^T A_k: sparse column dot products, rows merged in ascending order
        const int np = q * (q + 1) / 2;
        for (int p = tid; p < np; p += RNT) {
            int a, b;
            untri(p, a, b);
            const int64_t ea = S.cb[a] + S.cl[a], eb = S.cb[b] + S.cl[b];
            int64_t ia = S.cb[a], ib = S.cb[b];
            double sum = 0.0;
            while (ia < ea && ib < eb) {
                const int ra = A.rowidx[ia], rb = A.rowidx[ib];
                if (ra == rb) {
                    sum += A.val[ia] * A.val[ib];
                    ++ia;
                    ++ib;
                } else if (ra < rb) {
                    ++ia;
                } else {
                    ++ib;
                }
            }
            S.G[p] = sum;
        }
        __syncthreads();
        // Cholesky A_k^T A_k = L L^T, right-looking, in place
        for (int j = 0; j < q; ++j) {
            if (tid == 0) {
                const double d = S.G[tri(j, j)];
                if (d > 0.0) S.G[tri(j, j)] = sqrt(d); else S.flag = 1;
            }
            __syncthreads();
            if (S.flag) break;
            const double dj = S.G[tri(j, j)];
            for (int a = j + 1 + tid; a < q; a += RNT) S.G[tri(a, j)] /= dj;
            __syncthreads();
            const int w = q - j - 1;
            for (int t = tid; t < w * (w + 1) / 2; t += RNT) {
                int a, b;
                untri(t, a, b);
                a += j + 1;
                b += j + 1;
                S.G[tri(a, b)] -= S.G[tri(a, j)] * S.G[tri(b, j)];
            }
            __syncthreads();
        }
        if (S.flag) {
            if (tid == 0) atomicOr(r.err, 32);  // rank-deficient A_k: no factor
            __syncthreads();
            continue;
        }
        // record: J (ascending: the solve order of L), then R = L^T row by row
        if (tid == 0) {
            const unsigned long long need = (unsigned long long)(q + np);
            const unsigned long long at = atomicAdd(r.cur, need);
            S.cb[0] = (at + need <= (unsigned long long)r.cap) ? (int64_t)at : -1;
        }
        __syncthreads();
        const int64_t fo = S.cb[0];
        if (fo >= 0) {
            double *F = r.fac + fo;
            for (int t = tid; t < q; t += RNT) F[t] = (double)S.js[t];
            for (int p = tid; p < np; p += RNT) {
                int c, i;
                untri(p, c, i);  // L(c, i), c >= i, is R(i, c)
                F[q + i * q - i * (i - 1) / 2 + (c - i)] = S.G[p];
            }
            if (tid == 0) r.tfoff[k] = fo;
        } else if (tid == 0) {
            atomicOr(r.err, 64);  // store too small (sized exactly: internal error)
        }
        __syncthreads();
    }
}

// columns with a factor in either store (mask >= 0), for the refactorising kernel
__global__ void k_merge_masks(int64_t n, const int64_t *a, const int64_t *b, int64_t *out) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = ((a && a[k] >= 0) || b[k] >= 0) ? 0 : -1;
}

void launch_refactor_size(const RefArgs &r, unsigned long long *total, hipStream_t s) {
    const int64_t nb = std::min<int64_t>(std::max<int64_t>((r.n + 255) / 256, 1), 4096);
    hipLaunchKernelGGL(k_refactor_size, dim3(nb), dim3(256), 0, s, r, total);
}
void launch_refactor(const RefArgs &r, int cus, hipStream_t s) {
    hipLaunchKernelGGL(k_refactor, dim3(cus * 2), dim3(RNT), 0, s, r);
}
void launch_merge_masks(int64_t n, const int64_t *a, const int64_t *b, int64_t *out, hipStream_t s) {
    const int64_t nb = std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 4096);
    hipLaunchKernelGGL(k_merge_masks, dim3(nb), dim3(256), 0, s, n, a, b, out);
}

// resident workgroups per CU of each instance (the grids are persistent: a wave
// beyond what fits would start only after a resident one finishes)
static int factored_resident(const void *fn) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64, 0) != hipSuccess || nb < 1) nb = 1;
    return nb;
}

void launch_backward_factored(const BwdArgs &a, int cus, bool large, hipStream_t s) {
    static const int r_small = factored_resident(reinterpret_cast<const void *>(&backward_factored_kernel<16, 32, 1>));
    static const int r_large = factored_resident(reinterpret_cast<const void *>(&backward_factored_kernel<64, 128, 33>));
    hipLaunchKernelGGL((backward_factored_kernel<16, 32, 1>), dim3(cus * r_small), dim3(64), 0, s, a);
    if (large)
        hipLaunchKernelGGL((backward_factored_kernel<64, 128, 33>), dim3(cus * r_large), dim3(64), 0, s, a);
}

}  // namespace rsai
