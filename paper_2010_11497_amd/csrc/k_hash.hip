// Item hashing (the generative hash functions h_j of Section II-D), the
// FastRandomHash user keys (Eq. 3), and the profile validation check.
#include "c2_internal.h"
#include "c2_kernels.h"

namespace c2 {

// One thread per (j, i): simple tabulation over the 4 bytes of i with the
// 64-bit tables of configuration j, reduced to [0, b) by the high word of x*b.
__global__ __launch_bounds__(256) void k_hash_items(const uint64_t *__restrict__ tab, uint32_t t,
                                                    uint32_t b, uint32_t m,
                                                    uint32_t *__restrict__ bucket) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (uint64_t)t * m) return;
    const uint32_t j = (uint32_t)(g / m), i = (uint32_t)(g % m);
    const uint64_t *T = tab + (size_t)j * 1024;
    const uint64_t x = T[i & 255u] ^ T[256 + ((i >> 8) & 255u)] ^ T[512 + ((i >> 16) & 255u)] ^
                       T[768 + (i >> 24)];
    bucket[g] = (uint32_t)__umul64hi(x, (uint64_t)b);
}

hipError_t launch_hash_items(const uint64_t *tab, uint32_t t, uint32_t b, uint32_t m,
                             uint32_t *bucket, hipStream_t s) {
    const uint64_t total = (uint64_t)t * m;
    hipLaunchKernelGGL(k_hash_items, dim3((uint32_t)div_up(total, 256)), dim3(256), 0, s, tab, t,
                       b, m, bucket);
    return hipGetLastError();
}

constexpr int kKeyLanes = 8;

// keys[j*n + u] = min over the profile of bucket[j*m + i]  (Eq. 3).
__global__ __launch_bounds__(256) void k_frh_keys(const int64_t *__restrict__ indptr,
                                                  const uint32_t *__restrict__ indices,
                                                  uint64_t nnz, uint32_t n, uint32_t m,
                                                  const uint32_t *__restrict__ bucket, uint32_t t,
                                                  uint32_t b, uint32_t *__restrict__ keys) {
    const uint64_t g = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kKeyLanes;
    const uint32_t gl = threadIdx.x % kKeyLanes;
    if (g >= (uint64_t)t * n) return;
    const uint32_t j = (uint32_t)(g / n), u = (uint32_t)(g % n);
    const uint32_t v = group_min_above<kKeyLanes>(indptr, indices, nnz, bucket + (size_t)j * m, m,
                                                  b, u, 0, gl);
    if (gl == 0) keys[g] = v;
}

hipError_t launch_frh_keys(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                           uint32_t n, uint32_t m, const uint32_t *bucket, uint32_t t, uint32_t b,
                           uint32_t *keys, hipStream_t s) {
    const uint64_t threads = (uint64_t)t * n * kKeyLanes;
    hipLaunchKernelGGL(k_frh_keys, dim3((uint32_t)div_up(threads, 256)), dim3(256), 0, s, indptr,
                       indices, nnz, n, m, bucket, t, b, keys);
    return hipGetLastError();
}

// Item-major copy of the bucket table: bt[i * t + j] = bucket[j * m + i], so
// that the t buckets of an item are one row (128 bytes at t = 32).
__global__ __launch_bounds__(256) void k_bucket_rows(const uint32_t *__restrict__ bucket,
                                                     uint32_t t, uint32_t m,
                                                     uint32_t *__restrict__ bt) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (uint64_t)t * m) return;
    const uint32_t i = (uint32_t)(g / t), j = (uint32_t)(g % t);
    bt[g] = bucket[(size_t)j * m + i];
}

constexpr int kRowLanes = 8;
constexpr uint32_t kRowConfigs = 32;

// Eq. 3 for configurations j0 .. j0 + nt - 1 (nt <= kRowConfigs) from the
// item-major table: a group of kRowLanes lanes per user reads the profile
// once, each lane folding the rows of every kRowLanes-th item (two in flight)
// into its nt running minima, then the group combines them.  VEC: t and j0
// multiples of 4, rows read 16 bytes at a time.
template <bool VEC>
__global__ __launch_bounds__(256) void k_frh_keys_rows(const int64_t *__restrict__ indptr,
                                                       const uint32_t *__restrict__ indices,
                                                       uint64_t nnz, uint32_t n, uint32_t m,
                                                       const uint32_t *__restrict__ bt, uint32_t t,
                                                       uint32_t b, uint32_t j0,
                                                       uint32_t *__restrict__ keys) {
    const uint32_t u = (uint32_t)(((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kRowLanes);
    const uint32_t gl = threadIdx.x % kRowLanes;
    if (u >= n) return;  // whole groups leave together
    const uint32_t nt = t - j0 < kRowConfigs ? t - j0 : kRowConfigs;
    uint32_t best[kRowConfigs];
#pragma unroll
    for (uint32_t q = 0; q < kRowConfigs; ++q) best[q] = b;
    auto fold = [&](uint32_t i) {
        const uint32_t *row = bt + (size_t)i * t + j0;
        if constexpr (VEC) {
#pragma unroll
            for (uint32_t q = 0; q < kRowConfigs; q += 4) {
                if (q < nt) {
                    const uint4 h = *reinterpret_cast<const uint4 *>(row + q);
                    best[q] = h.x < best[q] ? h.x : best[q];
                    best[q + 1] = h.y < best[q + 1] ? h.y : best[q + 1];
                    best[q + 2] = h.z < best[q + 2] ? h.z : best[q + 2];
                    best[q + 3] = h.w < best[q + 3] ? h.w : best[q + 3];
                }
            }
        } else {
#pragma unroll
            for (uint32_t q = 0; q < kRowConfigs; ++q)
                if (q < nt) best[q] = row[q] < best[q] ? row[q] : best[q];
        }
    };
    uint64_t a, e;
    row_range(indptr, u, nnz, a, e);
    uint64_t p = a + gl;
    for (; p + kRowLanes < e; p += 2 * kRowLanes) {
        const uint32_t i0 = indices[p], i1 = indices[p + kRowLanes];
        if (i0 < m) fold(i0);
        if (i1 < m) fold(i1);
    }
    if (p < e) {
        const uint32_t i = indices[p];
        if (i < m) fold(i);
    }
#pragma unroll
    for (uint32_t q = 0; q < kRowConfigs; ++q) {
#pragma unroll
        for (int d = kRowLanes / 2; d > 0; d >>= 1) {
            const uint32_t o = __shfl_xor(best[q], d, kRowLanes);
            best[q] = o < best[q] ? o : best[q];
        }
        if (q % kRowLanes == gl && q < nt) keys[(size_t)(j0 + q) * n + u] = best[q];
    }
}

hipError_t launch_frh_keys_rows(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                                uint32_t n, uint32_t m, const uint32_t *bucket, uint32_t t,
                                uint32_t b, uint32_t *bt, uint32_t *keys, hipStream_t s) {
    const uint64_t tm = (uint64_t)t * m;
    hipLaunchKernelGGL(k_bucket_rows, dim3((uint32_t)div_up(tm, 256)), dim3(256), 0, s, bucket, t,
                       m, bt);
    const dim3 grid((uint32_t)div_up((uint64_t)n * kRowLanes, 256));
    for (uint32_t j0 = 0; j0 < t; j0 += kRowConfigs) {
        if (t % 4 == 0)
            hipLaunchKernelGGL(k_frh_keys_rows<true>, grid, dim3(256), 0, s, indptr, indices, nnz,
                               n, m, bt, t, b, j0, keys);
        else
            hipLaunchKernelGGL(k_frh_keys_rows<false>, grid, dim3(256), 0, s, indptr, indices,
                               nnz, n, m, bt, t, b, j0, keys);
    }
    return hipGetLastError();
}

// Profile check; sets bit flags in *err: 1 = indptr[0] != 0 or indptr[n] != nnz,
// 2 = empty or reversed row, 4 = item >= m, 8 = items not strictly increasing.
__global__ __launch_bounds__(256) void k_validate(const int64_t *__restrict__ indptr,
                                                  const uint32_t *__restrict__ indices,
                                                  uint64_t nnz, uint32_t n, uint32_t m,
                                                  uint32_t *err) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0 && (indptr[0] != 0 || indptr[n] != (int64_t)nnz)) atomicOr(err, 1u);
    if (g >= n) return;
    const int64_t x = indptr[g], y = indptr[g + 1];
    if (!(y > x)) { atomicOr(err, 2u); return; }
    uint64_t a, e;
    row_range(indptr, (uint32_t)g, nnz, a, e);
    uint32_t flags = 0, prev = 0;
    for (uint64_t p = a; p < e; ++p) {
        const uint32_t i = indices[p];
        if (i >= m) flags |= 4u;
        if (p > a && i <= prev) flags |= 8u;
        prev = i;
    }
    if (flags) atomicOr(err, flags);
}

hipError_t launch_validate(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                           uint32_t n, uint32_t m, uint32_t *err, hipStream_t s) {
    hipLaunchKernelGGL(k_validate, dim3((uint32_t)div_up(n, 256)), dim3(256), 0, s, indptr,
                       indices, nnz, n, m, err);
    return hipGetLastError();
}

// Small utility: fill `n` u32 with `v` (used instead of memset nodes so the
// batched build can be captured in a graph).
__global__ void k_fill_u32(uint32_t *p, uint32_t v, uint32_t n) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) p[g] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)div_up(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

__global__ void k_iota(uint32_t *p, uint32_t n) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) p[g] = g;
}

hipError_t launch_iota(uint32_t *p, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3((uint32_t)div_up(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace c2
