// y = A x (or A^T x) without any allocation: the work buffers of the row formation
// live in one file-scope device array, so the call suits callers that cannot
// allocate (code under graph capture, serving loops, harnesses that forbid it).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>
#include <mutex>

#include "../../include/rsai.h"
#include "rsai_kernels.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // RSAI_SPMV_NOALLOC_MAX_BYTES
static_assert(kScratchBytes == RSAI_SPMV_NOALLOC_MAX_BYTES, "header and library agree on the limit");

// The work area. Its name is a host-side stand-in in host code: kernels get the
// device address taken below, never the name.
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char *g_ptr[kMaxDevices] = {};  // device address of scratch on each device

// device address of the work area on the current device, taken once per device
rsai_status scratch_ptr(char **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return rsai::report(RSAI_E_HIP, "rsai_spmv_noalloc: no usable current device (%d)", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return rsai::report(RSAI_E_HIP, "rsai_spmv_noalloc: hipGetSymbolAddress failed: %s",
                                hipGetErrorString(e));
        g_ptr[dev] = (char *)p;
    }
    *out = g_ptr[dev];
    return RSAI_OK;
}

// bytes of the row formation's work buffers for a matrix, with each buffer's offset
struct Parts {
    size_t cnt, fill, rp, ci, vv, stmp, zerr, total;
};
size_t up(size_t x) { return (x + 255) & ~(size_t)255; }
Parts parts(int64_t n, int64_t nnz) {
    Parts p{};
    size_t o = 0;
    p.cnt = o;  o = up(o + 4 * (size_t)n);
    p.fill = o; o = up(o + 4 * (size_t)n);
    p.rp = o;   o = up(o + 8 * (size_t)(n + 1));
    p.ci = o;   o = up(o + 4 * (size_t)nnz);
    p.vv = o;   o = up(o + 8 * (size_t)nnz);
    p.stmp = o; o = up(o + 8 * (size_t)rsai::scan_tmp_elems(n + 1));
    p.zerr = o; o = up(o + 16);
    p.total = o;
    return p;
}

}  // namespace

extern "C" rsai_status rsai_spmv_noalloc(const rsai_csc *A, const double *x, double *y, int32_t transpose,
                                         void *stream) {
    if (!A || !A->colptr || !A->rowidx || !A->val || !x || !y)
        return rsai::report(RSAI_E_ARG, "rsai_spmv_noalloc: NULL argument");
    if (A->n < 1 || A->n > INT32_MAX - 1 || A->nnz < 0 || A->nnz > INT32_MAX)
        return rsai::report(RSAI_E_ARG, "rsai_spmv_noalloc: bad sizes (n %lld, nnz %lld)", (long long)A->n,
                            (long long)A->nnz);
    hipStream_t s = (hipStream_t)stream;
    if (transpose) {  // column dot products: no work buffers
        rsai::launch_csc_spmv_t(A->n, A->colptr, A->rowidx, A->val, x, y, s);
        if (hipGetLastError() != hipSuccess) return rsai::report(RSAI_E_HIP, "rsai_spmv_noalloc: launch failed");
        return RSAI_OK;
    }
    const Parts pt = parts(A->n, A->nnz);
    if (pt.total > kScratchBytes)
        return rsai::report(RSAI_E_ARG,
                            "rsai_spmv_noalloc: n = %lld, nnz = %lld needs %zu bytes of work area; it holds %zu "
                            "(use rsai_spmv)",
                            (long long)A->n, (long long)A->nnz, pt.total, kScratchBytes);
    char *base = nullptr;
    const rsai_status st = scratch_ptr(&base);
    if (st != RSAI_OK) return st;
    int32_t *cnt = (int32_t *)(base + pt.cnt);
    int32_t *fill = (int32_t *)(base + pt.fill);
    int64_t *rp = (int64_t *)(base + pt.rp);
    int32_t *ci = (int32_t *)(base + pt.ci);
    double *vv = (double *)(base + pt.vv);
    int64_t *stmp = (int64_t *)(base + pt.stmp);
    int32_t *zerr = (int32_t *)(base + pt.zerr);
    // the same kernels and summation order as rsai_spmv; every buffer is cleared or
    // fully written by a kernel before it is read (no hipMemsetAsync)
    rsai::enqueue_rows(A->n, A->nnz, A->colptr, A->rowidx, A->val, rp, ci, vv, cnt, fill, stmp, zerr, s);
    rsai::launch_csr_spmv(A->n, rp, ci, vv, x, y, s);
    if (hipGetLastError() != hipSuccess) return rsai::report(RSAI_E_HIP, "rsai_spmv_noalloc: launch failed");
    return RSAI_OK;
}
