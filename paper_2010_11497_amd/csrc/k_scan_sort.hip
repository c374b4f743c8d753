// Prefix sums and a stable LSD radix sort, used by the clustering step to
// regroup users by (parent cluster, next hash value) every split round.
#include "c2_internal.h"

namespace c2 {

// ------------------------------------------------------------------ scans

constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr uint32_t kScanChunk = kScanThreads * kScanPer;       // 4096
constexpr int kSingleThreads = 1024;
constexpr uint32_t kSingleChunk = kSingleThreads * kScanPer;  // 16384

// Scan of a chunk of NT*kScanPer elements starting at base, plus `offset`.
template <typename T, int NT>
C2_DEV void chunk_scan(const T *in, T *out, uint32_t N, uint32_t base, T offset, bool write_total,
                       T *wsum) {
    T loc[kScanPer];
    const uint32_t start = base + threadIdx.x * kScanPer;
    T sum = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        uint32_t idx = start + i;
        loc[i] = idx < N ? in[idx] : (T)0;
        sum += loc[i];
    }
    T total;
    T pre = block_excl_scan<T, NT>(sum, wsum, &total) + offset;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        uint32_t idx = start + i;
        if (idx < N) out[idx] = pre;
        pre += loc[i];
    }
    if (write_total && threadIdx.x == 0) out[N] = offset + total;
}

template <typename T>
__global__ __launch_bounds__(kSingleThreads) void k_scan_single(const T *in, T *out, uint32_t N) {
    __shared__ T wsum[kSingleThreads / 64 + 1];
    chunk_scan<T, kSingleThreads>(in, out, N, 0, (T)0, true, wsum);
}

// The chunk's total: the order of the sum does not matter, so the block reads
// its chunk in consecutive runs of kScanThreads elements (coalesced, all loads
// in flight before any is added).
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const T *in, T *part, uint32_t N) {
    __shared__ T wsum[kScanThreads / 64 + 1];
    const uint32_t start = blockIdx.x * kScanChunk + threadIdx.x;
    T v[kScanPer];
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        const uint32_t idx = start + i * kScanThreads;
        v[i] = idx < N ? in[idx] : (T)0;
    }
    T sum = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) sum += v[i];
    T total;
    block_excl_scan<T, kScanThreads>(sum, wsum, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// chunk_scan of one kScanChunk chunk staged through LDS: loads and stores in
// consecutive runs of kScanThreads elements (coalesced), each thread scanning
// kScanPer consecutive elements from the staging array.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const T *in, T *out, const T *part,
                                                            uint32_t N, uint32_t nb) {
    __shared__ T wsum[kScanThreads / 64 + 1];
    // element e of the chunk at e + e / kScanPer: a thread's kScanPer
    // consecutive elements then fall in different banks
    __shared__ T stage[kScanChunk + kScanChunk / kScanPer];
    auto at = [](uint32_t e) { return e + e / kScanPer; };
    const uint32_t base = blockIdx.x * kScanChunk, tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        const uint32_t idx = base + i * kScanThreads + tid;
        stage[at(i * kScanThreads + tid)] = idx < N ? in[idx] : (T)0;
    }
    __syncthreads();
    T loc[kScanPer];
    T sum = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        loc[i] = stage[at(tid * kScanPer + i)];
        sum += loc[i];
    }
    T total;
    T pre = block_excl_scan<T, kScanThreads>(sum, wsum, &total) + part[blockIdx.x];
    // (block_excl_scan's barriers order the reads above before these writes)
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        stage[at(tid * kScanPer + i)] = pre;
        pre += loc[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        const uint32_t idx = base + i * kScanThreads + tid;
        if (idx < N) out[idx] = stage[at(i * kScanThreads + tid)];
    }
    if (blockIdx.x == nb - 1 && tid == 0) out[N] = part[blockIdx.x] + total;
}

size_t scan_tmp_elems(uint32_t N) {
    size_t nb = div_up(N, kScanChunk);
    return nb + 1 + 64;
}

template <typename T>
static hipError_t scan_impl(const T *in, T *out, uint32_t N, T *tmp, hipStream_t s) {
    if (N <= kSingleChunk) {
        hipLaunchKernelGGL(k_scan_single<T>, dim3(1), dim3(kSingleThreads), 0, s, in, out, N);
        return hipGetLastError();
    }
    uint32_t nb = (uint32_t)div_up(N, kScanChunk);
    if (nb > kSingleChunk) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3(nb), dim3(kScanThreads), 0, s, in, tmp, N);
    hipLaunchKernelGGL(k_scan_single<T>, dim3(1), dim3(kSingleThreads), 0, s, tmp, tmp, nb);
    hipLaunchKernelGGL(k_scan_apply<T>, dim3(nb), dim3(kScanThreads), 0, s, in, out, tmp, N, nb);
    return hipGetLastError();
}

hipError_t scan_u32(const uint32_t *in, uint32_t *out, uint32_t N, uint32_t *tmp, hipStream_t s) {
    return scan_impl<uint32_t>(in, out, N, tmp, s);
}
hipError_t scan_u64(const uint64_t *in, uint64_t *out, uint32_t N, uint64_t *tmp, hipStream_t s) {
    return scan_impl<uint64_t>(in, out, N, tmp, s);
}

// ------------------------------------------------------------- radix sort
//
// One pass per 8-bit digit.  Pass = per-block digit histogram (digit-major so
// that one exclusive scan gives every block's output offset per digit), scan,
// then a stable scatter: inside a block, elements are ranked in index order
// using wave ballots to find equal digits and a per-wave count table in LDS.

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr uint32_t kSortTile = kSortThreads * kSortRounds;  // 2048
constexpr int kSortWaves = kSortThreads / 64;

size_t radix_hist_elems(uint32_t n_max) { return 256 * div_up(n_max ? n_max : 1, kSortTile) + 1; }

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t *keys,
                                                            const uint32_t *n_dev, uint32_t shift,
                                                            uint32_t *hist, uint32_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t n = *n_dev;
    const uint32_t base = blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        uint32_t idx = base + r * kSortThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint64_t *keys, const uint32_t *vals, uint64_t *okeys, uint32_t *ovals,
    const uint32_t *n_dev, uint32_t shift, const uint32_t *hist_scan, uint32_t nblocks) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kSortWaves][256];
    __shared__ uint32_t woff[kSortWaves][256];
    const uint32_t n = *n_dev;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    base[tid] = hist_scan[tid * nblocks + blockIdx.x];
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kSortRounds; ++r) {
        const uint32_t idx = blockIdx.x * kSortTile + r * kSortThreads + tid;
        const bool valid = idx < n;
        uint64_t key = 0;
        uint32_t val = 0, d = 0;
        if (valid) {
            key = keys[idx];
            val = vals[idx];
            d = (uint32_t)(key >> shift) & 255u;
        }
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1u;
            const uint64_t bb = __ballot(on);
            peers &= on ? bb : ~bb;
        }
        const uint32_t wrank = __popcll(peers & lt_mask);
        if (valid && wrank == 0) wcnt[wid][d] = __popcll(peers);
        __syncthreads();
        {   // digit tid: offsets of each wave's elements, in wave order
            uint32_t run = base[tid];
#pragma unroll
            for (int w = 0; w < kSortWaves; ++w) {
                woff[w][tid] = run;
                run += wcnt[w][tid];
                wcnt[w][tid] = 0;
            }
            base[tid] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = woff[wid][d] + wrank;
            okeys[pos] = key;
            ovals[pos] = val;
        }
    }
}

hipError_t radix_sort(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt,
                      const uint32_t *n_dev, uint32_t n_max, uint32_t bits, uint32_t *hist,
                      uint32_t *htmp, bool *in_alt, hipStream_t s) {
    *in_alt = false;
    if (n_max == 0 || bits == 0) return hipSuccess;
    const uint32_t nblocks = (uint32_t)div_up(n_max, kSortTile);
    uint64_t *ki = keys, *ko = keys_alt;
    uint32_t *vi = vals, *vo = vals_alt;
    for (uint32_t shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(kSortThreads), 0, s, ki, n_dev, shift,
                           hist, nblocks);
        hipError_t e = scan_u32(hist, hist, 256 * nblocks, htmp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(kSortThreads), 0, s, ki, vi, ko,
                           vo, n_dev, shift, hist, nblocks);
        uint64_t *tk = ki; ki = ko; ko = tk;
        uint32_t *tv = vi; vi = vo; vo = tv;
        *in_alt = !*in_alt;
    }
    return hipGetLastError();
}

}  // namespace c2
