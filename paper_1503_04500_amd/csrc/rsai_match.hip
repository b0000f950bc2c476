// Maximum transversal of a sparse pattern and the row permutation it gives: the
// preprocessing that Section 5 applies to matrices with zero diagonal entries, so
// that A(p[k], k) != 0 for every column k.
//
// A transversal is a matching of columns to rows in the bipartite graph of the
// pattern. The device algorithm:
//   1. greedy: every column claims a free row of its own (its diagonal entry first,
//      then its rows in ascending order) with one compare-and-swap per try;
//   2. phases of augmentation: from all unmatched columns at once, a level-
//      synchronous breadth-first search along alternating paths (column -> any of
//      its rows -> the column matched to that row), every row claimed by the first
//      search that reaches it (an atomic max of the phase number), so the search
//      trees are vertex-disjoint; a tree that reaches an unmatched row records it
//      and stops growing. Each tree with an end row then flips its path (disjoint
//      paths, so in parallel). A phase that flips no path ends the algorithm: the
//      searches visited every row reachable along alternating paths from the
//      unmatched columns, and none was free, so no augmenting path exists and the
//      matching has the largest size.
// Which of several maximum transversals comes out depends on the order of the
// atomics; its size does not.
#include <climits>

#include "rsai_kernels.h"

namespace rsai {

namespace {
constexpr int MT = 256;
int blocks_for(int64_t work) {
    int64_t b = (work + MT - 1) / MT;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (int)b;
}
}  // namespace

// 1. greedy claims
__global__ void k_match_greedy(int64_t n, const int64_t *colptr, const int32_t *rowidx, int32_t *match_col,
                               int32_t *match_row) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = colptr[c], e = colptr[c + 1];
        int got = -1;
        // the diagonal entry, found by bisection (rows ascending)
        int64_t lo = s, hi = e - 1;
        while (lo <= hi) {
            const int64_t mid = (lo + hi) / 2;
            const int r = rowidx[mid];
            if (r == (int)c) { lo = mid; break; }
            if (r < (int)c) lo = mid + 1; else hi = mid - 1;
        }
        if (lo < e && rowidx[lo] == (int)c && atomicCAS(&match_row[c], -1, (int)c) == -1) got = (int)c;
        for (int64_t t = s; t < e && got < 0; ++t) {
            const int r = rowidx[t];
            if (r != (int)c && atomicCAS(&match_row[r], -1, (int)c) == -1) got = r;
        }
        match_col[c] = got;
    }
}

// 2a. the unmatched columns start the phase's search trees
__global__ void k_match_roots(int64_t n, const int32_t *match_col, int32_t *root, int32_t *found, int32_t *roots,
                              int32_t *nroots) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        if (match_col[c] < 0) {
            root[c] = (int)c;
            found[c] = -1;
            roots[atomicAdd(nroots, 1)] = (int)c;
        }
    }
}

// 2b. one level of the search: the rows of the frontier's columns
__global__ void k_match_expand(const int64_t *colptr, const int32_t *rowidx, int32_t stamp, int32_t *visited,
                               int32_t *parent, int32_t *root, int32_t *found, const int32_t *match_row,
                               const int32_t *fin, const int32_t *nin, int32_t *fout, int32_t *nout) {
    const int64_t cnt = *nin;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = fin[i];
        const int rt = root[c];
        if (found[rt] >= 0) continue;  // this tree already has a path
        for (int64_t t = colptr[c]; t < colptr[c + 1]; ++t) {
            const int r = rowidx[t];
            if (atomicMax(&visited[r], stamp) >= stamp) continue;  // another search has it
            parent[r] = c;
            const int c2 = match_row[r];
            if (c2 < 0) {
                atomicCAS(&found[rt], -1, r);
                break;
            }
            root[c2] = rt;
            fout[atomicAdd(nout, 1)] = c2;
        }
    }
}

// 2c. flip the path of every tree that reached a free row
__global__ void k_match_augment(const int32_t *roots, const int32_t *nroots, const int32_t *found,
                                const int32_t *parent, int32_t *match_col, int32_t *match_row, int32_t *naug) {
    const int64_t cnt = *nroots;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
        const int c0 = roots[i];
        int r = found[c0];
        if (r < 0) continue;
        for (;;) {
            const int cc = parent[r];
            const int prev = match_col[cc];
            match_col[cc] = r;
            match_row[r] = cc;
            if (cc == c0) break;
            r = prev;
        }
        atomicAdd(naug, 1);
    }
}

__global__ void k_match_count(int64_t n, const int32_t *match_col, unsigned long long *size) {
    unsigned long long m = 0;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        m += match_col[c] >= 0 ? 1ull : 0ull;
    for (int off = 32; off >= 1; off >>= 1) m += __shfl_xor(m, off);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(size, m);
}

// inverse of a permutation; err bit 1 for an entry out of range or repeated
__global__ void k_perm_invert(int64_t n, const int32_t *p, int32_t *inv, int32_t *err) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int r = p[k];
        if (r < 0 || r >= n) { atomicOr(err, 1); continue; }
        if (atomicExch(&inv[r], (int)k) != -1) atomicOr(err, 1);
    }
}

// B(k, j) = A(p[k], j): every stored entry of A gets row inv[row]
__global__ void k_perm_rows(int64_t n, int64_t nnz, const int64_t *colptr, const int32_t *rowidx, const double *val,
                            const int32_t *inv, int64_t *colptrB, int32_t *rowidxB, double *valB) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += stride) {
        rowidxB[e] = inv[rowidx[e]];
        valB[e] = val[e];
    }
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k <= n; k += stride) colptrB[k] = colptr[k];
}

void launch_match_greedy(int64_t n, const int64_t *colptr, const int32_t *rowidx, int32_t *match_col,
                         int32_t *match_row, hipStream_t s) {
    hipLaunchKernelGGL(k_match_greedy, dim3(blocks_for(n)), dim3(MT), 0, s, n, colptr, rowidx, match_col, match_row);
}
void launch_match_roots(int64_t n, const int32_t *match_col, int32_t *root, int32_t *found, int32_t *roots,
                        int32_t *nroots, hipStream_t s) {
    hipLaunchKernelGGL(k_match_roots, dim3(blocks_for(n)), dim3(MT), 0, s, n, match_col, root, found, roots, nroots);
}
void launch_match_expand(int64_t n, const int64_t *colptr, const int32_t *rowidx, int32_t stamp, int32_t *visited,
                         int32_t *parent, int32_t *root, int32_t *found, const int32_t *match_row, const int32_t *fin,
                         const int32_t *nin, int32_t *fout, int32_t *nout, int64_t nin_host, hipStream_t s) {
    (void)n;
    hipLaunchKernelGGL(k_match_expand, dim3(blocks_for(nin_host)), dim3(MT), 0, s, colptr, rowidx, stamp, visited,
                       parent, root, found, match_row, fin, nin, fout, nout);
}
void launch_match_augment(const int32_t *roots, const int32_t *nroots, int64_t nroots_host, const int32_t *found,
                          const int32_t *parent, int32_t *match_col, int32_t *match_row, int32_t *naug,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_match_augment, dim3(blocks_for(nroots_host)), dim3(MT), 0, s, roots, nroots, found, parent,
                       match_col, match_row, naug);
}
void launch_match_count(int64_t n, const int32_t *match_col, unsigned long long *size, hipStream_t s) {
    hipLaunchKernelGGL(k_match_count, dim3(blocks_for(n)), dim3(MT), 0, s, n, match_col, size);
}
void launch_perm_invert(int64_t n, const int32_t *p, int32_t *inv, int32_t *err, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_invert, dim3(blocks_for(n)), dim3(MT), 0, s, n, p, inv, err);
}
void launch_perm_rows(int64_t n, int64_t nnz, const int64_t *colptr, const int32_t *rowidx, const double *val,
                      const int32_t *inv, int64_t *colptrB, int32_t *rowidxB, double *valB, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_rows, dim3(blocks_for(nnz > n + 1 ? nnz : n + 1)), dim3(MT), 0, s, n, nnz, colptr,
                       rowidx, val, inv, colptrB, rowidxB, valB);
}

}  // namespace rsai
