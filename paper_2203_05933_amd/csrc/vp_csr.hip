// Plan-time transpose of the correction matrix (Section 4: the sparse matrix
// assembled from the local maps Pi_k).  The adjoint evaluation applies C^T
// as a CSR matrix of its own, so no atomics are needed and the result is
// deterministic.  The transpose is a stable sort of the non-zeros by column:
// within a column the rows stay in increasing order.

#include "vp_internal.hpp"

namespace vp {

__global__ void k_row_of(const int64_t *__restrict__ rowptr, int64_t m, int32_t *__restrict__ row_of) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) row_of[q] = (int32_t)i;
}

__global__ void k_col_keys(const int32_t *__restrict__ col, int64_t nnz, uint64_t *__restrict__ keys,
                           int32_t *__restrict__ idx) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnz) return;
    keys[q] = (uint64_t)(uint32_t)col[q];
    idx[q] = (int32_t)q;
}

__global__ void k_transpose_fill(const int32_t *__restrict__ perm, const int32_t *__restrict__ row_of,
                                 const double *__restrict__ val, int64_t nnz, int32_t *__restrict__ colT,
                                 double *__restrict__ valT) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    int32_t q = perm[k];
    colT[k] = row_of[q];
    valT[k] = val[q];
}

__global__ void k_col_ptr(const uint64_t *__restrict__ skeys, int64_t nnz, int64_t n,
                          int64_t *__restrict__ rowptrT) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > n) return;
    // first sorted position with key >= j
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (skeys[mid] < (uint64_t)j) lo = mid + 1;
        else hi = mid;
    }
    rowptrT[j] = lo;
}

void build_csr_transpose(vp_plan_s *P) {
    const int64_t nnz = P->nnz, n = P->nd, m = P->m;  // columns: the density values
    hipStream_t s = P->stream;
    P->rowptrT = P->mem.alloc<int64_t>(n + 1);
    P->colT = P->mem.alloc<int32_t>(nnz);
    P->valT = P->mem.alloc<double>(nnz + 2);  // padded like the values (aligned pair reads)
    fill_f64(P->valT + nnz, 0.0, 2, s);
    if (nnz == 0) {
        fill_f64(reinterpret_cast<double *>(P->rowptrT), 0.0, n + 1, s);  // all-zero int64
        return;
    }
    TempArena tmp;
    int32_t *row_of = tmp.alloc<int32_t>(nnz);
    uint64_t *keys = tmp.alloc<uint64_t>(nnz);
    int32_t *perm = tmp.alloc<int32_t>(nnz);
    auto g = [](int64_t x) { return dim3((unsigned)((x + 255) / 256)); };
    hipLaunchKernelGGL(k_row_of, g(m), dim3(256), 0, s, P->rowptr, m, row_of);
    hipLaunchKernelGGL(k_col_keys, g(nnz), dim3(256), 0, s, P->col, nnz, keys, perm);
    VP_LAUNCH_CHECK();
    int nbits = 1;
    while (nbits < 32 && ((int64_t)1 << nbits) < n) ++nbits;
    radix_sort_pairs_u64(keys, perm, (int)nnz, nbits, s);
    hipLaunchKernelGGL(k_transpose_fill, g(nnz), dim3(256), 0, s, perm, row_of, P->val, nnz, P->colT, P->valT);
    hipLaunchKernelGGL(k_col_ptr, g(n + 1), dim3(256), 0, s, keys, nnz, n, P->rowptrT);
    VP_LAUNCH_CHECK();
    VP_HIP(hipStreamSynchronize(s));
}

}  // namespace vp
