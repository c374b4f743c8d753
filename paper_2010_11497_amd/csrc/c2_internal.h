// Internal declarations shared by the HIP translation units of libc2.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define C2_DEV __device__ __forceinline__

namespace c2 {

constexpr uint32_t kPad = 0xFFFFFFFFu;
constexpr uint32_t kMaxItems = 1u << 19;  // LDS dictionary bitmaps (two of m bits)
constexpr uint32_t kMaxK = 32;

// Cluster state stored at a segment's first position during splitting.
constexpr uint32_t kFinal = 0, kActive = 1, kRoot = 2;

// ------------------------------------------------------------ device helpers

// Row u of the CSR profiles, clamped to [0, nnz] so that malformed input can
// never address outside `indices`.
C2_DEV void row_range(const int64_t *indptr, uint32_t u, uint64_t nnz, uint64_t &a,
                      uint64_t &e) {
    int64_t x = indptr[u], y = indptr[u + 1];
    if (x < 0) x = 0;
    if (y > (int64_t)nnz) y = (int64_t)nnz;
    if (y < x) y = x;
    a = (uint64_t)x;
    e = (uint64_t)y;
}

// Workgroup barrier that waits only for this wave's LDS operations: global
// loads issued before it stay in flight (a plain __syncthreads() also drains
// them, which defeats software prefetching).
C2_DEV void lds_barrier() {
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// Exact Jaccard order: does (Ia, Ua, va) rank before (Ib, Ub, vb)?
C2_DEV bool jbetter(uint32_t Ia, uint32_t Ua, uint32_t va, uint32_t Ib, uint32_t Ub,
                    uint32_t vb) {
    uint64_t l = (uint64_t)Ia * Ub, r = (uint64_t)Ib * Ua;
    return l != r ? l > r : va < vb;
}

C2_DEV uint64_t shfl_up_u64(uint64_t v, int d) {
    uint32_t lo = __shfl_up((uint32_t)v, d), hi = __shfl_up((uint32_t)(v >> 32), d);
    return ((uint64_t)hi << 32) | lo;
}
C2_DEV uint64_t shfl_u64(uint64_t v, int src) {
    uint32_t lo = __shfl((uint32_t)v, src), hi = __shfl((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// Minimum bucket value >= thr over the items of row u in configuration j, by a
// group of G consecutive lanes (G divides 64); values >= b count as absent.
// Returns b when there is none.
template <int G>
C2_DEV uint32_t group_min_above(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                                const uint32_t *bucket_j, uint32_t m, uint32_t b, uint32_t u,
                                uint32_t thr, uint32_t gl) {
    uint64_t a, e;
    row_range(indptr, u, nnz, a, e);
    uint32_t best = b;
    // four independent index -> bucket gathers in flight per lane
    uint64_t p = a + gl;
    for (; p + 3 * G < e; p += 4 * G) {
        const uint32_t i0 = indices[p], i1 = indices[p + G], i2 = indices[p + 2 * G],
                       i3 = indices[p + 3 * G];
        const uint32_t h0 = i0 < m ? bucket_j[i0] : b, h1 = i1 < m ? bucket_j[i1] : b;
        const uint32_t h2 = i2 < m ? bucket_j[i2] : b, h3 = i3 < m ? bucket_j[i3] : b;
        if (h0 >= thr && h0 < best) best = h0;
        if (h1 >= thr && h1 < best) best = h1;
        if (h2 >= thr && h2 < best) best = h2;
        if (h3 >= thr && h3 < best) best = h3;
    }
    for (; p < e; p += G) {
        const uint32_t i = indices[p];
        if (i < m) {
            const uint32_t h = bucket_j[i];
            if (h >= thr && h < best) best = h;
        }
    }
#pragma unroll
    for (int d = G / 2; d > 0; d >>= 1) {
        const uint32_t o = __shfl_xor(best, d, G);
        best = o < best ? o : best;
    }
    return best;
}

// floor(I * (2^32 - 1) / U) for 0 <= I <= U < 2^16, U >= 1, without a
// division: an fp32 estimate from the reciprocal of U (within 2^10 of the
// quotient), one correction from the exact 32-bit remainder scaled by the
// same reciprocal (within 1), and a final step on the sign and size of the
// remainder.  Every remainder is below 2^31 in magnitude, so 32-bit integer
// arithmetic is exact.  Checked against 64-bit division for all (I, U) with
// the reciprocal exact, and on a sample with it 1 and 2 ulp off.
C2_DEV uint32_t jkey(uint32_t I, uint32_t U) {
    const float r = __builtin_amdgcn_rcpf((float)U);
    const float qf = (float)I * r * 4294967296.0f;
    const uint32_t q0 = qf >= 4294967295.0f ? 0xFFFFFFFFu : (uint32_t)qf;
    const int32_t rem = (int32_t)((0u - I) - q0 * U);  // I * 2^32 - I - q0 * U
    const int32_t c = (int32_t)floorf((float)rem * r);
    uint32_t q = q0 + (uint32_t)c;
    const int32_t rem1 = rem - c * (int32_t)U;
    if (rem1 < 0) q -= 1;
    else if (rem1 >= (int32_t)U) q += 1;
    return q;
}

C2_DEV uint32_t bit_width_dev(uint32_t x) { return x ? 32u - (uint32_t)__clz(x) : 0u; }

// Block-wide exclusive scan of one value per thread; returns the block total
// through *total.  NT threads (a multiple of 64), LDS for NT/64 wave sums.
template <typename T, int NT>
C2_DEV T block_excl_scan(T v, T *wsum, T *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y;
        if constexpr (sizeof(T) == 8) y = (T)shfl_up_u64((uint64_t)x, d);
        else y = (T)__shfl_up((uint32_t)x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    if (wid == 0) {
        T w = lane < NT / 64 ? wsum[lane] : (T)0;
        T z = w;
#pragma unroll
        for (int d = 1; d < NT / 64; d <<= 1) {
            T y;
            if constexpr (sizeof(T) == 8) y = (T)shfl_up_u64((uint64_t)z, d);
            else y = (T)__shfl_up((uint32_t)z, d);
            if (lane >= d) z += y;
        }
        if (lane < NT / 64) wsum[lane] = z - w;  // exclusive wave offsets
        if (lane == NT / 64 - 1) wsum[NT / 64] = z;
    }
    __syncthreads();
    T res = wsum[wid] + x - v;
    *total = wsum[NT / 64];
    __syncthreads();
    return res;
}

// ------------------------------------------------------------ host helpers

inline uint32_t bit_width(uint64_t x) {
    uint32_t w = 0;
    while (x) { ++w; x >>= 1; }
    return w;
}
inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Exclusive prefix sum of `in[0..N)` into `out[0..N]` (out[N] = total).
// `tmp` must hold scan_tmp_elems(N) elements.  `in` may alias `out`.
size_t scan_tmp_elems(uint32_t N);
hipError_t scan_u32(const uint32_t *in, uint32_t *out, uint32_t N, uint32_t *tmp, hipStream_t s);
hipError_t scan_u64(const uint64_t *in, uint64_t *out, uint32_t N, uint64_t *tmp, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the
// keys.  The element count is read on the device from *n_dev (<= n_max).
// Buffers: keys/vals (input), keys_alt/vals_alt (same size), hist holds
// radix_hist_elems(n_max) u32 and htmp scan_tmp_elems(256 * blocks) u32.
// Returns through *in_alt whether the sorted result ended in the alt buffers.
size_t radix_hist_elems(uint32_t n_max);
hipError_t radix_sort(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt,
                      const uint32_t *n_dev, uint32_t n_max, uint32_t bits, uint32_t *hist,
                      uint32_t *htmp, bool *in_alt, hipStream_t s);

}  // namespace c2
