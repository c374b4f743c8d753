// Step 3 on the device: merge of each user's t partial lists (Section II-G,
// Algorithm 3).  A group of G >= t lanes serves one user; lane j holds the
// head of list j (each list is best first).  Each step the group picks the
// best head (exact Jaccard order; equal entries -- the same neighbour found in
// several lists -- resolved to the lowest lane), emits it unless it repeats
// the previous output, and that lane advances.  Similarities found in Step 2
// are reused; nothing is recomputed except U from the profile lengths.
#include "c2_internal.h"
#include "c2_kernels.h"

namespace c2 {

template <int G>
__global__ __launch_bounds__(256) void k_merge(const int64_t *__restrict__ indptr, uint64_t nnz,
                                               uint32_t n, uint32_t t, uint32_t k,
                                               const uint32_t *__restrict__ part_id,
                                               const uint32_t *__restrict__ part_I,
                                               uint32_t *__restrict__ knn_id,
                                               uint32_t *__restrict__ knn_I,
                                               uint32_t *__restrict__ knn_U) {
    const uint64_t gth = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t u = (uint32_t)(gth / G);
    const uint32_t j = threadIdx.x % G;
    if (u >= n) return;
    uint64_t a, e;
    row_range(indptr, u, nnz, a, e);
    const uint32_t Lu = (uint32_t)(e - a);
    const size_t lbase = ((size_t)u * t + j) * k;
    uint32_t ptr = 0, hv = kPad, hI = 0, hU = 0;
    auto load = [&]() {
        hv = kPad;
        if (j < t && ptr < k) {
            const uint32_t v = part_id[lbase + ptr];
            if (v != kPad && v < n) {
                uint64_t va, ve;
                row_range(indptr, v, nnz, va, ve);
                hv = v;
                hI = part_I[lbase + ptr];
                hU = Lu + (uint32_t)(ve - va) - hI;
            }
        }
    };
    load();
    uint32_t out = 0, last = kPad;
    uint32_t *oid = knn_id + (size_t)u * k, *oI = knn_I + (size_t)u * k, *oU = knn_U + (size_t)u * k;
    while (out < k) {
        bool ok = hv != kPad;
        uint32_t bI = hI, bU = hU, bv = hv, bj = j;
#pragma unroll
        for (int d = G / 2; d > 0; d >>= 1) {
            const bool ook = __shfl_xor((int)ok, d, G) != 0;
            const uint32_t oI2 = __shfl_xor(bI, d, G), oU2 = __shfl_xor(bU, d, G);
            const uint32_t ov = __shfl_xor(bv, d, G), oj = __shfl_xor(bj, d, G);
            bool take;
            if (ok != ook) take = ook;
            else if (!ok) take = oj < bj;
            else if (jbetter(oI2, oU2, ov, bI, bU, bv)) take = true;
            else if (jbetter(bI, bU, bv, oI2, oU2, ov)) take = false;
            else take = oj < bj;
            if (take) { ok = ook; bI = oI2; bU = oU2; bv = ov; bj = oj; }
        }
        if (!ok) break;
        if (bv != last) {
            if (j == 0) {
                oid[out] = bv;
                oI[out] = bI;
                oU[out] = bU;
            }
            ++out;
            last = bv;
        }
        if (j == bj) {
            ++ptr;
            load();
        }
    }
    for (uint32_t r = out + j; r < k; r += G) {
        oid[r] = kPad;
        oI[r] = 0;
        oU[r] = 0;
    }
}

hipError_t launch_merge(const int64_t *indptr, uint64_t nnz, uint32_t n, uint32_t t, uint32_t k,
                        const uint32_t *part_id, const uint32_t *part_I, uint32_t *knn_id,
                        uint32_t *knn_I, uint32_t *knn_U, hipStream_t s) {
    uint32_t G = 1;
    while (G < t) G <<= 1;
    const dim3 grid((uint32_t)div_up((uint64_t)n * G, 256));
#define C2_MERGE(GG)                                                                           \
    case GG:                                                                                   \
        hipLaunchKernelGGL(k_merge<GG>, grid, dim3(256), 0, s, indptr, nnz, n, t, k, part_id, \
                           part_I, knn_id, knn_I, knn_U);                                     \
        break;
    switch (G) {
        C2_MERGE(1) C2_MERGE(2) C2_MERGE(4) C2_MERGE(8) C2_MERGE(16) C2_MERGE(32) C2_MERGE(64)
        default: return hipErrorInvalidValue;
    }
#undef C2_MERGE
    return hipGetLastError();
}

}  // namespace c2
