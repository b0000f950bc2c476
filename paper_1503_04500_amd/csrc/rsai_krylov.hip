// Preconditioned BiCGStab on the device: the solve step of the paper's experiments
// (Section 5) with the RSAI(tol) factor M, in the right form A M y = b, x = M y, or
// the left form M A x = M b of (1.2) (M then comes from RSAI on A^T, transposed).
//
// x0 = 0; shadow residual r^ = r0 (b, or M b in the left form). The stopping test is
// the true relative residual ||b - A x|| / ||b|| < tol, evaluated after the half step
// and after the full step of every iteration (x = M y is carried directly in the
// right form).
//
// Device design:
//  * A and M are held in SELL-64 form (slices of 64 rows, one wavefront; a slice is
//    as wide as its longest row and stores entry k of its rows contiguously, padding
//    with zero values), so a thread's loads of its row need no row pointer and are
//    coalesced across the wavefront, and x is gathered right after them.
//  * Every scalar of the recurrence lives in device memory, double-buffered: each
//    kernel reads one copy and its workgroup 0 writes the other, so workgroups of the
//    same kernel never see a half-updated state. Kernels return at once after the
//    solve has ended (still passing the state on), so the host enqueues many
//    iterations between checks or replays them as a captured graph.
//  * Dot products and norms are reduced without atomics: the producing kernel writes
//    one partial sum per workgroup, and every workgroup of the next kernel adds all
//    partials in index order (the same order everywhere, so all workgroups agree to
//    the bit) before applying the scalar step. The kernel boundary orders the two.
//  * Products are split by linearity so that no kernel gathers more than needed and
//    no kernel exists for an elementwise update alone. With F the operator applied
//    first to a direction and G the second (right: F = M, G = A; left: F = A,
//    G = M), and w = p - omega v kept from the previous iteration:
//    F p = F r + beta F w; F s = F r - alpha F v; and the half-step residual
//    b - A (x + alpha d) = (b - A x) - alpha A d with A d = v (right, d = M p) or
//    A d = F p (left, d = p). Every residual is still formed from fresh products of
//    the current vectors (b - A x by an SpMV of x in each iteration), not carried by
//    a recurrence.
//
// Kernels of one iteration k (| the partial sums a kernel produces, [] the step it
// applies first from the previous kernel's partials):
//   pre   [r^.r of iteration k-1: beta] p = r + beta w, fp = F r + beta F w (F r
//         kept), res = b - A x | ||res||^2
//   av    [full-step test of x_k (for k = 1 the initial test), end tests] v = G fp
//         | r^.v
//   half  [alpha] s = r - alpha v, xh = x + alpha d, fs = F r - alpha F v
//         | ||res - alpha A d||^2
//   at    [half-step test] t = G fs | t.t, t.s
//   uf    [omega] x = xh + omega (M s right, s otherwise), r = s - omega t,
//         w = p - omega v | r^.r
// Without M, F = I and G = A. In the first iteration beta = 0 and w = 0, so p = r.
#include <algorithm>

#include "rsai_kernels.h"

namespace rsai {

namespace {
constexpr int KT = 256;  // threads per workgroup; rows per thread-pass = KT
constexpr int SL = 64;   // rows per SELL slice (one wavefront)

enum Stage { BS_NONE = 0, BS_INIT, BS_RES, BS_AV, BS_HALF, BS_AT, BS_UF };

// The scalar step of a stage, from the totals of its partial sums. S.it is the
// iteration that runs next (pre .. uf).
__device__ void apply_stage(BicgState &S, int stage, const double *tot) {
    switch (stage) {
    case BS_INIT: {  // ||b||^2, r^.r of the initial residual
        const double nb = sqrt(tot[0]);
        S.nb = (nb == 0.0) ? 1.0 : nb;
        S.rel = nb / S.nb;
        S.rho = S.alpha = S.omega = 1.0;
        S.rho1 = S.rho1n = tot[1];
        S.it = 1;
        S.half = 0;
        if (S.rel < S.tol) { S.done = 1; S.ret = 0; }
        else if (S.maxit < 1) { S.done = 3; S.ret = S.maxit + 1; }
        else if (S.rho1 == 0.0) { S.done = 2; S.ret = -1; }
        else S.done = 0;
        break;
    }
    case BS_UF:  // r^.r after the full step of iteration it; iteration it + 1 is next
        S.rho1n = tot[0];
        S.it += 1;
        break;
    case BS_RES:  // ||b - A x|| for the x of the last full step (the initial x when it == 1)
        S.rel = sqrt(tot[0]) / S.nb;
        if (S.rel < S.tol) { S.done = 1; S.ret = S.it - 1; }
        else if (S.it > 1) {
            if (S.omega == 0.0) { S.done = 2; S.ret = -1; }
            else {
                S.rho = S.rho1;
                S.rho1 = S.rho1n;
                if (S.it > S.maxit) { S.done = 3; S.ret = S.maxit + 1; }
                else if (S.rho1 == 0.0) { S.done = 2; S.ret = -1; }
            }
        }
        break;
    case BS_AV:
        if (tot[0] == 0.0) { S.done = 2; S.ret = -1; }
        else S.alpha = S.rho1 / tot[0];
        break;
    case BS_HALF:
        S.rel = sqrt(tot[0]) / S.nb;
        if (S.rel < S.tol) { S.done = 1; S.half = 1; S.ret = S.it; }
        break;
    case BS_AT:
        if (tot[0] == 0.0) { S.done = 2; S.ret = -1; }
        else S.omega = tot[1] / tot[0];
        break;
    default:
        break;
    }
}

__device__ __forceinline__ int stage_values(int stage) { return (stage == BS_AT || stage == BS_INIT) ? 2 : 1; }

// Read the state, fold in the pending partial sums, pass the state on (workgroup 0).
// Every thread of every workgroup ends with the same S. Returns false when the solve
// has ended.
__device__ bool take_state(const BicgStep &q, BicgState &S) {
    __shared__ double red[2][KT / 64];
    S = *q.sin;
    if (!S.done && q.stage != BS_NONE) {
        const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
        const int nv = stage_values(q.stage);
        double tot[2] = {0.0, 0.0};
        for (int k = 0; k < nv; ++k) {
            double t = 0.0;
            for (int i = tid; i < q.np; i += KT) t += q.pin[(int64_t)k * q.np + i];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off);
            if (lane == 0) red[k][w] = t;
        }
        __syncthreads();
        for (int k = 0; k < nv; ++k)
            for (int i = 0; i < KT / 64; ++i) tot[k] += red[k][i];
        apply_stage(S, q.stage, tot);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *q.sout = S;
    return S.done == 0;
}

// one partial sum per value per workgroup
template <int NV>
__device__ void write_partials(double (&x)[NV], double *pout) {
    __shared__ double red[NV][KT / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x[k] += __shfl_xor(x[k], off);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[k][w] = x[k];
    __syncthreads();
    if (tid == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double t = 0.0;
            for (int i = 0; i < KT / 64; ++i) t += red[k][i];
            pout[(int64_t)k * gridDim.x + blockIdx.x] = t;
        }
}

// row i of a SELL-64 matrix times x (entries in column order; padding adds 0 * x[i])
__device__ __forceinline__ double sell_row(const int64_t *sp, const int32_t *sw, const int32_t *ci,
                                           const double *va, const double *x, int64_t i) {
    const int64_t sl = i / SL;
    const int64_t e0 = sp[sl] + (i % SL);
    const int w = sw[sl];
    double q = 0.0;
#pragma unroll 4
    for (int k = 0; k < w; ++k) q += va[e0 + (int64_t)k * SL] * x[ci[e0 + (int64_t)k * SL]];
    return q;
}

// row i of a SELL-64 matrix times two vectors (one pass over the row)
__device__ __forceinline__ void sell_row2(const int64_t *sp, const int32_t *sw, const int32_t *ci, const double *va,
                                          const double *x, const double *y, int64_t i, double &qx, double &qy) {
    const int64_t sl = i / SL;
    const int64_t e0 = sp[sl] + (i % SL);
    const int w = sw[sl];
    qx = 0.0;
    qy = 0.0;
#pragma unroll 4
    for (int k = 0; k < w; ++k) {
        const int64_t e = e0 + (int64_t)k * SL;
        const int j = ci[e];
        const double m = va[e];
        qx += m * x[j];
        qy += m * y[j];
    }
}

#define ROWS(i, n) for (int64_t i = blockIdx.x * (int64_t)KT + threadIdx.x; i < (n); i += (int64_t)gridDim.x * KT)
}  // namespace

// Modes: 0 no preconditioner, 1 right (A M y = b, x = M y), 2 left (M A x = M b).
// F is the operator applied first to a direction and G the second: right F = M,
// G = A; left F = A, G = M; none F = I, G = A. fr = F r, fp = F p, fs = F s.
#define SELL_A a.asp, a.aw, a.aci, a.ava
#define SELL_M a.msp, a.mw, a.mci, a.mva

// x = 0, r = r^ = p = b (left: M b), w = v = 0 | ||b||^2, r^.r
template <int MODE>
__global__ __launch_bounds__(KT) void kb_init(BicgArgs a, BicgStep q) {
    double acc[2] = {0.0, 0.0};
    ROWS(i, a.n) {
        const double bi = a.b[i];
        const double ri = (MODE == 2) ? sell_row(SELL_M, a.b, i) : bi;
        a.x[i] = 0.0;
        a.r[i] = ri;
        a.rh[i] = ri;
        a.p[i] = ri;
        a.w[i] = 0.0;
        a.v[i] = 0.0;
        acc[0] += bi * bi;
        acc[1] += ri * ri;
    }
    write_partials<2>(acc, q.pout);
}

// one workgroup: fold in pending partial sums and write the state to both copies
__global__ __launch_bounds__(KT) void kb_settle(BicgArgs a, BicgStep q, BicgState *other) {
    BicgState S;
    take_state(q, S);
    if (threadIdx.x == 0) *other = S;
}

// [beta] p = r + beta w, fp = F r + beta F w (F r kept), res = b - A x | ||res||^2
template <int MODE>
__global__ __launch_bounds__(KT) void kb_pre(BicgArgs a, BicgStep q) {
    BicgState S;
    if (!take_state(q, S)) return;
    const double beta = (S.it == 1) ? 0.0 : (S.rho1n / S.rho1) * (S.alpha / S.omega);
    double acc[1] = {0.0};
    ROWS(i, a.n) {
        a.p[i] = a.r[i] + beta * a.w[i];
        double ax;
        if (MODE == 2) {
            // one pass over the rows of A for A r, A w and A x
            const int64_t sl = i / SL, e0 = a.asp[sl] + (i % SL);
            const int wd = a.aw[sl];
            double qr = 0.0, qw = 0.0, qx = 0.0;
#pragma unroll 4
            for (int k = 0; k < wd; ++k) {
                const int64_t e = e0 + (int64_t)k * SL;
                const int j = a.aci[e];
                const double m = a.ava[e];
                qr += m * a.r[j];
                qw += m * a.w[j];
                qx += m * a.x[j];
            }
            a.fr[i] = qr;
            a.fp[i] = qr + beta * qw;
            ax = qx;
        } else {
            if (MODE == 1) {
                double mr, mw;
                sell_row2(SELL_M, a.r, a.w, i, mr, mw);
                a.fr[i] = mr;
                a.fp[i] = mr + beta * mw;
            }
            ax = sell_row(SELL_A, a.x, i);
        }
        const double d = a.b[i] - ax;
        a.res[i] = d;
        acc[0] += d * d;
    }
    write_partials<1>(acc, q.pout);
}

// [full-step test] v = G fp | r^.v
template <int MODE>
__global__ __launch_bounds__(KT) void kb_av(BicgArgs a, BicgStep q) {
    BicgState S;
    if (!take_state(q, S)) return;
    const double *fp = (MODE == 0) ? a.p : a.fp;
    double acc[1] = {0.0};
    ROWS(i, a.n) {
        const double vi = (MODE == 2) ? sell_row(SELL_M, fp, i) : sell_row(SELL_A, fp, i);
        a.v[i] = vi;
        acc[0] += a.rh[i] * vi;
    }
    write_partials<1>(acc, q.pout);
}

// [alpha] s = r - alpha v, xh = x + alpha (M p or p), fs = F r - alpha F v
// | ||b - A xh||^2 = ||res - alpha A (M p or p)||^2 (A M p = v right, A p = v none,
// A p = fp left)
template <int MODE>
__global__ __launch_bounds__(KT) void kb_half(BicgArgs a, BicgStep q) {
    BicgState S;
    if (!take_state(q, S)) return;
    const double al = S.alpha;
    const double *step = (MODE == 1) ? a.fp : a.p;
    const double *astep = (MODE == 2) ? a.fp : a.v;
    double acc[1] = {0.0};
    ROWS(i, a.n) {
        const double vi = a.v[i];
        a.s[i] = a.r[i] - al * vi;
        a.xh[i] = a.x[i] + al * step[i];
        if (MODE == 1) a.fs[i] = a.fr[i] - al * sell_row(SELL_M, a.v, i);
        if (MODE == 2) a.fs[i] = a.fr[i] - al * sell_row(SELL_A, a.v, i);
        const double d = a.res[i] - al * astep[i];
        acc[0] += d * d;
    }
    write_partials<1>(acc, q.pout);
}

// [half-step test] t = G fs | t.t, t.s
template <int MODE>
__global__ __launch_bounds__(KT) void kb_at(BicgArgs a, BicgStep q) {
    BicgState S;
    if (!take_state(q, S)) return;
    const double *fs = (MODE == 0) ? a.s : a.fs;
    double acc[2] = {0.0, 0.0};
    ROWS(i, a.n) {
        const double ti = (MODE == 2) ? sell_row(SELL_M, fs, i) : sell_row(SELL_A, fs, i);
        a.t[i] = ti;
        acc[0] += ti * ti;
        acc[1] += ti * a.s[i];
    }
    write_partials<2>(acc, q.pout);
}

// [omega] x = xh + omega (M s or s), r = s - omega t, w = p - omega v | r^.r
template <int MODE>
__global__ __launch_bounds__(KT) void kb_uf(BicgArgs a, BicgStep q) {
    BicgState S;
    if (!take_state(q, S)) return;
    const double om = S.omega;
    const double *sstep = (MODE == 1) ? a.fs : a.s;
    double acc[1] = {0.0};
    ROWS(i, a.n) {
        a.x[i] = a.xh[i] + om * sstep[i];
        const double ri = a.s[i] - om * a.t[i];
        a.r[i] = ri;
        a.w[i] = a.p[i] - om * a.v[i];
        acc[0] += a.rh[i] * ri;
    }
    write_partials<1>(acc, q.pout);
}

// ---- SELL-64 construction from row-sorted CSR

// entries of each slice (64 x its longest row) and its width
__global__ void k_sell_widths(int64_t n, const int64_t *rp, int32_t *cnt, int32_t *sw) {
    const int64_t nsl = (n + SL - 1) / SL;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nsl; s += (int64_t)gridDim.x * blockDim.x) {
        int64_t w = 0;
        for (int64_t i = s * SL; i < min(n, (s + 1) * SL); ++i) w = max(w, rp[i + 1] - rp[i]);
        sw[s] = (int32_t)w;
        cnt[s] = (int32_t)(w * SL);
    }
}

__global__ void k_sell_fill(int64_t n, const int64_t *rp, const int32_t *ci, const double *va, const int64_t *sp,
                            const int32_t *sw, int32_t *sci, double *sva) {
    const int64_t nsl = (n + SL - 1) / SL;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nsl * SL;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t sl = i / SL, e0 = sp[sl] + (i % SL);
        const int64_t len = (i < n) ? rp[i + 1] - rp[i] : 0;
        for (int k = 0; k < sw[sl]; ++k) {
            const int64_t e = e0 + (int64_t)k * SL;
            if (k < len) {
                sci[e] = ci[rp[i] + k];
                sva[e] = va[rp[i] + k];
            } else {
                sci[e] = (int32_t)min(i, n - 1);  // any valid column: the value is zero
                sva[e] = 0.0;
            }
        }
    }
}

int64_t sell_slices(int64_t n) { return (n + SL - 1) / SL; }

void launch_sell_widths(int64_t n, const int64_t *rp, int32_t *cnt, int32_t *sw, hipStream_t s) {
    const int64_t nsl = sell_slices(n);
    hipLaunchKernelGGL(k_sell_widths, dim3((unsigned)std::max<int64_t>(1, (nsl + 255) / 256)), dim3(256), 0, s, n,
                       rp, cnt, sw);
}

void launch_sell_fill(int64_t n, const int64_t *rp, const int32_t *ci, const double *va, const int64_t *sp,
                      const int32_t *sw, int32_t *sci, double *sva, hipStream_t s) {
    const int64_t rows = sell_slices(n) * SL;
    hipLaunchKernelGGL(k_sell_fill, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((rows + 255) / 256, 65536))),
                       dim3(256), 0, s, n, rp, ci, va, sp, sw, sci, sva);
}

// ---- launch sequence

int bicg_grid(int64_t n) {
    const int64_t b = (n + KT - 1) / KT;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, BICG_MAXGRID));
}

void BicgSeq::step(int stage, bool produces, BicgStep &q) {
    q.stage = stage;
    q.np = grid;
    q.pin = a.part + (size_t)pb * 2 * BICG_MAXGRID;
    q.pout = a.part + (size_t)(pb ^ 1) * 2 * BICG_MAXGRID;
    q.sin = a.st + sp;
    q.sout = a.st + (sp ^ 1);
    sp ^= 1;
    if (produces) pb ^= 1;
}

namespace {
template <int MODE>
void launch_init(BicgSeq &z, const BicgStep &q, hipStream_t s) {
    hipLaunchKernelGGL(kb_init<MODE>, dim3(z.grid), dim3(KT), 0, s, z.a, q);
}

template <int MODE>
void one_iteration(BicgSeq &z, hipStream_t s) {
    BicgStep q{};
    z.step(z.pending, true, q);
    hipLaunchKernelGGL(kb_pre<MODE>, dim3(z.grid), dim3(KT), 0, s, z.a, q);
    z.step(BS_RES, true, q);
    hipLaunchKernelGGL(kb_av<MODE>, dim3(z.grid), dim3(KT), 0, s, z.a, q);
    z.step(BS_AV, true, q);
    hipLaunchKernelGGL(kb_half<MODE>, dim3(z.grid), dim3(KT), 0, s, z.a, q);
    z.step(BS_HALF, true, q);
    hipLaunchKernelGGL(kb_at<MODE>, dim3(z.grid), dim3(KT), 0, s, z.a, q);
    z.step(BS_AT, true, q);
    hipLaunchKernelGGL(kb_uf<MODE>, dim3(z.grid), dim3(KT), 0, s, z.a, q);
    z.pending = BS_UF;
}
}  // namespace

void BicgSeq::init(hipStream_t s) {
    BicgStep q{};
    step(BS_NONE, true, q);
    sp = 0;  // kb_init touches no state
    if (mode == 1) launch_init<1>(*this, q, s);
    else if (mode == 2) launch_init<2>(*this, q, s);
    else launch_init<0>(*this, q, s);
    pending = BS_INIT;
    settle(s);
}

void BicgSeq::settle(hipStream_t s) {
    BicgStep q{};
    step(pending, false, q);
    hipLaunchKernelGGL(kb_settle, dim3(1), dim3(KT), 0, s, a, q, a.st + (sp ^ 1));
    sp = 0;  // both copies now hold the state
    pending = BS_NONE;
}

void BicgSeq::iterations(int count, hipStream_t s) {
    for (int it = 0; it < count; ++it) {
        if (mode == 1) one_iteration<1>(*this, s);
        else if (mode == 2) one_iteration<2>(*this, s);
        else one_iteration<0>(*this, s);
    }
}

}  // namespace rsai
