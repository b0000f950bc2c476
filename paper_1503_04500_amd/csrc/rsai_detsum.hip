// Fixed-order accumulation of the adjoint's contributions (the deterministic mode of
// rsai_backward): the contributions of all columns to the entries of A are sorted by
// (entry, column) and each entry's sum is taken in ascending column order, so the
// gradient is bitwise repeatable whatever the order the columns ran in.
#include <hipcub/hipcub.hpp>

#include "rsai_kernels.h"

namespace rsai {

namespace {
__global__ __launch_bounds__(256) void k_contrib_count(const MatDev *mats, int mat, int64_t n, const int64_t *Mcolptr,
                                                       const int32_t *Mrowidx, unsigned long long *total) {
    const MatDev A = mats[mat];
    unsigned long long t = 0;
    const int64_t nnzM = Mcolptr[n];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnzM; e += (int64_t)gridDim.x * blockDim.x) {
        const int j = Mrowidx[e];
        t += (unsigned long long)(A.colptr[j + 1] - A.colptr[j]);
    }
    for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off);
    if ((threadIdx.x & 63) == 0 && t) atomicAdd(total, t);
}

// one thread per sorted position: the first position of each entry adds the entry's
// contributions, in their (column) order, and writes dA[entry] once
__global__ __launch_bounds__(256) void k_segsum(const unsigned long long *key, const double *val, int64_t count,
                                                double *dA) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < count; p += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long e = key[p] >> 32;
        if (p > 0 && (key[p - 1] >> 32) == e) continue;
        double sum = 0.0;
        for (int64_t t = p; t < count && (key[t] >> 32) == e; ++t) sum += val[t];
        dA[e] += sum;
    }
}
}  // namespace

void launch_contrib_count(const MatDev *mats, int mat, int64_t n, const int64_t *Mcolptr, const int32_t *Mrowidx,
                          unsigned long long *total, hipStream_t s) {
    hipLaunchKernelGGL(k_contrib_count, dim3(2048), dim3(256), 0, s, mats, mat, n, Mcolptr, Mrowidx, total);
}

size_t det_reduce_bytes(int64_t count) {
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (unsigned long long *)nullptr,
                                             (unsigned long long *)nullptr, (double *)nullptr, (double *)nullptr,
                                             (int)count, 0, 64, (hipStream_t)0);
    return bytes;
}

hipError_t det_reduce(unsigned long long *key, double *val, unsigned long long *key2, double *val2, int64_t count,
                      void *temp, size_t temp_bytes, double *dA, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, key, key2, val, val2, (int)count, 0, 64, s);
    if (e != hipSuccess) return e;
    int64_t nb = (count + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_segsum, dim3((int)nb), dim3(256), 0, s, key2, val2, count, dA);
    return hipGetLastError();
}

}  // namespace rsai
