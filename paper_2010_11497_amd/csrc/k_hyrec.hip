// Hyrec branch of Algorithm 2 (Section II-F; Hyrec as described in Section
// IV-B): the local KNN graph of a cluster of at least rho*k^2 members by
// greedy refinement instead of brute force.  Deterministic form:
//   - initial graph: member a draws k co-members uniformly with SplitMix64 at
//     counter (cluster << 40) | (a << 12) | q and keeps the k best distinct;
//   - iteration (synchronous): a's new list is the k best distinct of its own
//     list and its neighbours' lists (neighbours' neighbours), a excluded;
//   - the host stops after an iteration in which fewer than delta*k*s list
//     entries changed, or after max_iter iterations.
// Lists hold exact keys (jkey(I, U) << 32) | ~position, 0 = empty, so the
// order is the exact Jaccard order with ties to the lower id (positions
// follow ids inside a cluster).
#include "c2_internal.h"
#include "c2_kernels.h"

namespace c2 {

constexpr int kHyWaves = 4;
constexpr uint32_t kHyInvalid = 0xFFFFFFFFu;
constexpr int kHyGroup = 16;  // lanes per candidate when computing keys

// SplitMix64 (Steele, Lea and Flood, 2014): output number c + 1 of the
// generator whose state starts at `seed`.
C2_DEV uint64_t splitmix_at(uint64_t seed, uint64_t c) {
    uint64_t z = seed + 0x9e3779b97f4a7c15ull * (c + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

C2_DEV void hy_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave per member a.  NC: candidate slots (a power of two >= k + k*k).
template <int NC>
__global__ __launch_bounds__(64 * kHyWaves) void k_hyrec_step(
    const uint32_t *__restrict__ rows, const uint32_t *__restrict__ rlen, uint32_t W,
    const uint32_t *__restrict__ S, uint32_t s, uint32_t k, uint32_t cl, uint64_t seed,
    uint32_t init, const uint64_t *__restrict__ okey, uint64_t *__restrict__ nkey,
    uint32_t *__restrict__ nI, uint32_t *updates) {
    __shared__ uint32_t cpos_s[kHyWaves][NC];
    __shared__ uint64_t ckey_s[kHyWaves][NC];
    __shared__ uint32_t cI_s[kHyWaves][NC];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t a = blockIdx.x * kHyWaves + wid;
    if (a >= s) return;  // whole waves only: no block-wide barrier below
    uint32_t *cpos = cpos_s[wid];
    uint64_t *ckey = ckey_s[wid];
    uint32_t *cI = cI_s[wid];

    // candidate positions
    const uint32_t ncu = init ? k : k + k * k;
    for (uint32_t x = lane; x < NC; x += 64) {
        uint32_t pos = kHyInvalid;
        if (x < ncu) {
            if (init) {
                const uint64_t r = splitmix_at(seed, ((uint64_t)cl << 40) | ((uint64_t)a << 12) | x);
                pos = (uint32_t)(r % (uint64_t)(s - 1));
                pos += pos >= a ? 1u : 0u;
            } else if (x < k) {
                const uint64_t e = okey[(size_t)a * k + x];
                pos = e ? ~(uint32_t)e : kHyInvalid;
            } else {
                const uint32_t q = (x - k) / k, r = (x - k) % k;
                const uint64_t eq = okey[(size_t)a * k + q];
                if (eq) {
                    const uint32_t pq = ~(uint32_t)eq;
                    const uint64_t er = okey[(size_t)pq * k + r];
                    pos = er ? ~(uint32_t)er : kHyInvalid;
                    if (pos == a) pos = kHyInvalid;
                }
            }
        }
        cpos[x] = pos;
    }
    hy_wave_sync();

    // exact keys: 16 lanes per candidate, 4 candidates per step
    const uint32_t u = S[a];
    const uint32_t *ru = rows + (size_t)u * W;
    const uint32_t lu = rlen[u];
    const int sub = lane & (kHyGroup - 1), slot = lane / kHyGroup;
    for (uint32_t c0 = 0; c0 < (uint32_t)NC; c0 += 64 / kHyGroup) {
        const uint32_t c = c0 + slot;
        const uint32_t pos = cpos[c];
        uint32_t part = 0, lv = 0;
        if (pos != kHyInvalid) {
            const uint32_t v = S[pos];
            const uint32_t *rv = rows + (size_t)v * W;
            lv = rlen[v];
#pragma unroll 4
            for (uint32_t w = sub; w < W; w += kHyGroup) part += __popc(ru[w] & rv[w]);
        }
#pragma unroll
        for (int d = kHyGroup / 2; d >= 1; d >>= 1) part += __shfl_xor(part, d);
        if (sub == 0) {
            ckey[c] = pos != kHyInvalid
                          ? ((uint64_t)jkey(part, lu + lv - part) << 32) | (uint64_t)(~pos)
                          : 0ull;
            cI[c] = pos != kHyInvalid ? part : 0u;
        }
    }
    hy_wave_sync();

    // bitonic sort, descending by key, I carried along
    for (uint32_t size = 2; size <= (uint32_t)NC; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = lane; i < (uint32_t)NC / 2; i += 64) {
                const uint32_t lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
                const bool desc = (lo & size) == 0;
                const uint64_t x = ckey[lo], y = ckey[hi];
                if (desc ? x < y : x > y) {
                    ckey[lo] = y;
                    ckey[hi] = x;
                    const uint32_t t = cI[lo];
                    cI[lo] = cI[hi];
                    cI[hi] = t;
                }
            }
            hy_wave_sync();
        }
    }

    // the k best distinct (equal positions have equal keys, so they are adjacent)
    uint32_t found = 0;
    for (uint32_t base = 0; base < (uint32_t)NC && found < k; base += 64) {
        const uint32_t i = base + lane;
        const uint64_t key = ckey[i];
        // every 64-bit value is a possible key (J = 1 at position 0 is all
        // ones), so the first entry is compared with nothing
        const bool keep = key != 0 && (i == 0 || key != ckey[i - 1]);
        const uint64_t bal = __ballot(keep);
        const uint32_t rank = __popcll(bal & ((1ull << lane) - 1));
        if (keep && found + rank < k) {
            nkey[(size_t)a * k + found + rank] = key;
            nI[(size_t)a * k + found + rank] = cI[i];
        }
        found += (uint32_t)__popcll(bal);
        if (__ballot(key != 0) == 0) break;
    }
    if (found > k) found = k;
    for (uint32_t q = found + lane; q < k; q += 64) {
        nkey[(size_t)a * k + q] = 0;
        nI[(size_t)a * k + q] = 0;
    }
    if (init) return;
    // entries of the new list that were not in the old one
    uint32_t miss = 0;
    if ((uint32_t)lane < found) {
        const uint64_t e = nkey[(size_t)a * k + lane];
        bool in_old = false;
        for (uint32_t r = 0; r < k; ++r) in_old |= okey[(size_t)a * k + r] == e;
        miss = in_old ? 0u : 1u;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) miss += __shfl_xor(miss, d);
    if (lane == 0 && miss) atomicAdd(updates, miss);
}

__global__ __launch_bounds__(256) void k_hyrec_out(const uint32_t *__restrict__ S, uint32_t s,
                                                   uint32_t k, uint32_t j, uint32_t t,
                                                   const uint64_t *__restrict__ key,
                                                   const uint32_t *__restrict__ I,
                                                   uint32_t *__restrict__ part_id,
                                                   uint32_t *__restrict__ part_I) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (uint64_t)s * k) return;
    const uint32_t a = (uint32_t)(g / k), q = (uint32_t)(g % k);
    const uint32_t u = S[a];
    const uint64_t e = key[g];
    const size_t o = ((size_t)u * t + j) * k + q;
    part_id[o] = e ? S[~(uint32_t)e] : kPad;
    part_I[o] = e ? I[g] : 0u;
}

hipError_t launch_hyrec_step(const uint32_t *rows, const uint32_t *rlen, uint32_t W,
                             const uint32_t *S, uint32_t s, uint32_t k, uint32_t cl,
                             uint64_t seed, bool init, const uint64_t *okey, uint64_t *nkey,
                             uint32_t *nI, uint32_t *updates, hipStream_t st) {
    const dim3 grid((uint32_t)div_up(s, kHyWaves)), block(64 * kHyWaves);
    if (k + k * k <= 1024)
        hipLaunchKernelGGL(k_hyrec_step<1024>, grid, block, 0, st, rows, rlen, W, S, s, k, cl,
                           seed, init ? 1u : 0u, okey, nkey, nI, updates);
    else
        hipLaunchKernelGGL(k_hyrec_step<2048>, grid, block, 0, st, rows, rlen, W, S, s, k, cl,
                           seed, init ? 1u : 0u, okey, nkey, nI, updates);
    return hipGetLastError();
}

hipError_t launch_hyrec_out(const uint32_t *S, uint32_t s, uint32_t k, uint32_t j, uint32_t t,
                            const uint64_t *key, const uint32_t *I, uint32_t *part_id,
                            uint32_t *part_I, hipStream_t st) {
    hipLaunchKernelGGL(k_hyrec_out, dim3((uint32_t)div_up((uint64_t)s * k, 256)), dim3(256), 0,
                       st, S, s, k, j, t, key, I, part_id, part_I);
    return hipGetLastError();
}

}  // namespace c2
