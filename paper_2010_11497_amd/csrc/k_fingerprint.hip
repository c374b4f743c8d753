// GoldFinger fingerprints (Section II-F: local similarities estimated on a
// compact bit vector per user; 1024 bits in the evaluation, Section IV-C).
// A user's fingerprint is the set of positions g(i) in [0, B) of its items;
// the Jaccard index of two fingerprints is the estimate of the users'
// similarity.  The fingerprint is emitted as a CSR profile over B "items" so
// that the exact local-KNN and merge kernels run on it unchanged.
//
// Two passes, one wave per user.  Pass 1 sets the bits in an LDS bit vector,
// stores it (B/32 words per user) and the popcount; an exclusive scan of the
// popcounts is the fingerprint row pointer.  Pass 2 reads the stored words
// and writes each row's set positions in ascending order.
#include "c2_internal.h"
#include "c2_kernels.h"

namespace c2 {

constexpr int kFpWaves = 4;

size_t fp_words(uint32_t B) { return div_up(B, 32); }

// err bits: 1 = an item >= m in a row (the row's other items still count),
// 2 = a position g(i) >= B.
__global__ __launch_bounds__(64 * kFpWaves) void k_fp_bits(
    const int64_t *__restrict__ indptr, const uint32_t *__restrict__ indices, uint64_t nnz,
    uint32_t n, uint32_t m, const uint32_t *__restrict__ g, uint32_t B, uint32_t W,
    uint32_t *__restrict__ bits, uint64_t *__restrict__ cnt, uint32_t *err) {
    __shared__ uint32_t bm[kFpWaves][kFpMaxBits / 32];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t u = blockIdx.x * kFpWaves + wid;
    const bool live = u < n;
    for (uint32_t w = lane; w < W; w += 64) bm[wid][w] = 0;
    __syncthreads();
    uint32_t bad = 0;
    if (live) {
        uint64_t a, e;
        row_range(indptr, u, nnz, a, e);
        for (uint64_t p = a + lane; p < e; p += 64) {
            const uint32_t i = indices[p];
            if (i >= m) { bad |= 1u; continue; }
            const uint32_t x = g[i];
            if (x >= B) { bad |= 2u; continue; }
            atomicOr(&bm[wid][x >> 5], 1u << (x & 31));
        }
    }
    __syncthreads();
    if (!live) return;
    uint32_t c = 0;
    uint32_t *dst = bits + (size_t)u * W;
    for (uint32_t w = lane; w < W; w += 64) {
        const uint32_t v = bm[wid][w];
        c += __popc(v);
        dst[w] = v;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d);
    if (lane == 0) cnt[u] = c;
    if (bad) atomicOr(err, bad);
}

__global__ __launch_bounds__(64 * kFpWaves) void k_fp_write(const uint32_t *__restrict__ bits,
                                                            uint32_t W, uint32_t n,
                                                            const int64_t *__restrict__ fp_indptr,
                                                            uint32_t *__restrict__ fp_indices,
                                                            uint64_t cap) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t u = blockIdx.x * kFpWaves + wid;
    if (u >= n) return;
    const uint32_t *src = bits + (size_t)u * W;
    uint64_t base = (uint64_t)fp_indptr[u];
    for (uint32_t w0 = 0; w0 < W; w0 += 64) {
        const uint32_t w = w0 + lane;
        uint32_t v = w < W ? src[w] : 0u;
        const uint32_t c = __popc(v);
        uint32_t incl = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d);
            if (lane >= d) incl += y;
        }
        uint64_t pos = base + (incl - c);
        while (v) {
            const uint32_t b = __builtin_ctz(v);
            v &= v - 1;
            if (pos < cap) fp_indices[pos] = w * 32 + b;
            ++pos;
        }
        base += __shfl(incl, 63);
    }
}

size_t fingerprint_ws_bytes(uint32_t n, uint32_t B) {
    const size_t words = (size_t)n * fp_words(B);
    return ((4 * words + 255) & ~(size_t)255) + 8 * scan_tmp_elems(n);
}

hipError_t launch_fingerprint(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                              uint32_t n, uint32_t m, const uint32_t *g, uint32_t B,
                              int64_t *fp_indptr, uint32_t *fp_indices, void *ws, uint32_t *err,
                              hipStream_t s) {
    const uint32_t W = (uint32_t)fp_words(B);
    uint32_t *bits = reinterpret_cast<uint32_t *>(ws);
    uint64_t *tmp = reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(ws) +
                                                 (((size_t)4 * n * W + 255) & ~(size_t)255));
    uint64_t *cnt = reinterpret_cast<uint64_t *>(fp_indptr);
    const uint32_t blocks = (uint32_t)div_up(n, kFpWaves);
    hipLaunchKernelGGL(k_fp_bits, dim3(blocks), dim3(64 * kFpWaves), 0, s, indptr, indices, nnz,
                       n, m, g, B, W, bits, cnt, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // counts -> row pointer in place (fp_indptr[n] = total)
    e = scan_u64(cnt, cnt, n, tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fp_write, dim3(blocks), dim3(64 * kFpWaves), 0, s, bits, W, n, fp_indptr,
                       fp_indices, nnz);
    return hipGetLastError();
}

}  // namespace c2
