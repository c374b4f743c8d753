// Step 3 on the device: merge of each user's t partial lists (Section II-G,
// Algorithm 3).  A group of G >= t lanes serves one user; lane j holds the
// head of list j (each list is best first).  Each step the group picks the
// best head in the exact Jaccard order and emits it, and every lane whose head
// is that neighbour advances: a neighbour found in several lists has the same
// I and U in all of them, and when it is the best head it is the head of every
// list that holds it (each list is sorted and holds a neighbour once), so each
// step emits a new neighbour and k steps suffice.  Similarities found in Step 2
// are reused; nothing is recomputed except U from the profile lengths.
#include "c2_internal.h"
#include "c2_kernels.h"

namespace c2 {

constexpr int kMergeThreads = 64;

// DPP controls of the group maximum: quad_perm [1,0,3,2] and [2,3,0,1]
// (partners at xor 1 and xor 2), then the half-row and row mirrors (which
// pair each 4- and 8-lane block with the other one of its 8 and 16 lanes).
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

// max(b, b of the partner lane under DPP control CTRL), u64.
template <int CTRL>
C2_DEV uint64_t max_dpp(uint64_t b) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, true);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, true);
    const uint64_t o = ((uint64_t)hi << 32) | lo;
    return o > b ? o : b;
}

// Maximum of b over the G lanes of the group (all of them end with it).
template <int G>
C2_DEV uint64_t group_max(uint64_t b) {
    if (G > 1) b = max_dpp<kDppXor1>(b);
    if (G > 2) b = max_dpp<kDppXor2>(b);
    if (G > 4) b = max_dpp<kDppHalfMirror>(b);
    if (G > 8) b = max_dpp<kDppMirror>(b);
#pragma unroll
    for (int d = 16; d < G; d <<= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)b, d, G), hi = __shfl_xor((uint32_t)(b >> 32), d, G);
        const uint64_t o = ((uint64_t)hi << 32) | lo;
        b = o > b ? o : b;
    }
    return b;
}

// One wave of 64 lanes serves 64/G users (one if G = 64): all 64 lanes copy
// the users' t lists (contiguous in part_*) into LDS with U computed,
// coalesced, in one pass of loads; the selection loop then runs from LDS.
// I and U share one word there (8 bytes per entry with the id, so that enough
// waves fit on a CU to hide the loads); a user with some U >= 2^16, which
// needs the exact comparison anyway, reads its heads from global memory.
// The profile lengths come from ulen when the caller has them (one gather per
// entry), else from indptr.
template <int G>
__global__ __launch_bounds__(kMergeThreads) void k_merge(const int64_t *__restrict__ indptr,
                                                         const uint32_t *__restrict__ ulen,
                                                         uint64_t nnz, uint32_t n, uint32_t t,
                                                         uint32_t k,
                                                         const uint32_t *__restrict__ part_id,
                                                         const uint32_t *__restrict__ part_I,
                                                         uint32_t *__restrict__ knn_id,
                                                         uint32_t *__restrict__ knn_I,
                                                         uint32_t *__restrict__ knn_U) {
    constexpr int UPW = G <= kMergeThreads ? kMergeThreads / G : 1;  // users per wave
    // per entry: the id, and I | U << 16 (exact when U < 2^16; a user with a
    // larger U is flagged wide and reads its lists from global memory instead)
    __shared__ uint32_t sv[UPW * G * kMaxK], sIU[UPW * G * kMaxK];
    const uint32_t lane = threadIdx.x;
    const uint64_t u0 = (uint64_t)blockIdx.x * UPW;
    // stage: entries of users u0 .. u0+UPW-1, list j, slot r at ((ul*G + j)*k + r).
    // The profile lengths of the block's users first; then, per lane, up to
    // 16 entries with all their loads (entry, then the neighbour's length)
    // in flight before any is used.  wide[ul]: some U of the user is >= 2^16.
    __shared__ uint32_t ulen_s[UPW], wide[UPW];
    const uint32_t nu = (uint32_t)(u0 + UPW <= n ? UPW : (u0 < n ? n - u0 : 0));
    if (lane < nu) {
        if (ulen) {
            ulen_s[lane] = ulen[u0 + lane];
        } else {
            uint64_t a0, a1;
            row_range(indptr, (uint32_t)(u0 + lane), nnz, a0, a1);
            ulen_s[lane] = (uint32_t)(a1 - a0);
        }
    }
    if (lane < UPW) wide[lane] = 0;
    __syncthreads();
    {
        const uint32_t tk = t * k;
        const uint32_t total = nu * tk;
        const size_t base = (size_t)u0 * tk;
        for (uint32_t e0 = 0; e0 < total; e0 += 16 * kMergeThreads) {
            uint32_t v[16], I[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const uint32_t e = e0 + q * kMergeThreads + lane;
                v[q] = e < total ? part_id[base + e] : kPad;
                I[q] = e < total ? part_I[base + e] : 0;
            }
            uint32_t lv[16];
            if (ulen) {
#pragma unroll
                for (int q = 0; q < 16; ++q) lv[q] = v[q] < n ? ulen[v[q]] : 0u;
            } else {
                int64_t b0[16], b1[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const bool ok = v[q] < n;
                    b0[q] = ok ? indptr[v[q]] : 0;
                    b1[q] = ok ? indptr[v[q] + 1] : 0;
                }
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    // the row bounds clamped as row_range does
                    const int64_t lb = b0[q] < 0 ? 0 : b0[q];
                    const int64_t hb = b1[q] < (int64_t)nnz ? b1[q] : (int64_t)nnz;
                    lv[q] = v[q] < n && hb > lb ? (uint32_t)(hb - lb) : 0u;
                }
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const uint32_t e = e0 + q * kMergeThreads + lane;
                if (e >= total) continue;
                // entry e = ul*tk + j*k + r goes to slot (ul*G + j)*k + r
                const uint32_t ul = e / tk;
                const uint32_t d = e + ul * (G - t) * k;
                const bool ok = v[q] < n;
                const uint32_t U = ulen_s[ul] + lv[q] - I[q];
                sv[d] = ok ? v[q] : kPad;
                sIU[d] = ok ? I[q] | U << 16 : 0u;
                if (ok && U >= 65536u) wide[ul] = 1;
            }
        }
    }
    __syncthreads();
    const uint32_t ul = lane / G, j = lane % G;
    const uint64_t u = u0 + ul;
    if (ul >= (uint32_t)UPW || u >= n) return;
    const uint32_t lb = (ul * G + j) * k;
    uint32_t ptr = 0, hv = kPad, hI = 0, hU = 0;
    auto load = [&]() {
        hv = kPad;
        if (j < t && ptr < k) {
            hv = sv[lb + ptr];
            const uint32_t iu = sIU[lb + ptr];
            hI = iu & 0xFFFFu;
            hU = iu >> 16;
        }
    };
    uint32_t out = 0;
    uint32_t *oid = knn_id + u * k, *oI = knn_I + u * k, *oU = knn_U + u * k;
    if (!wide[ul]) {
        // Every U < 2^16: the 32-bit key orders the similarities exactly
        // (distinct fractions get distinct keys, equal ones equal keys), so
        // (key, then the smaller id) is one 64-bit maximum over the group.
        // The lowest lane whose head is the maximum writes it.
        auto head_key = [&]() -> uint64_t {
            return hv == kPad ? 0ull : ((uint64_t)jkey(hI, hU) << 32) | (0xFFFFFFFFu - hv);
        };
        const uint64_t gmask = G == 64 ? ~0ull : ((1ull << G) - 1) << (ul * G);
        load();
        uint64_t my = head_key();
        while (out < k) {
            const uint64_t best = group_max<G>(my);
            if (best == 0) break;  // every list exhausted
            const uint64_t hit = __ballot(my == best) & gmask;
            if (my == best && lane == (uint32_t)__ffsll((long long)hit) - 1) {
                oid[out] = hv;
                oI[out] = hI;
                oU[out] = hU;
            }
            ++out;
            if (my == best) {
                ++ptr;
                load();
                my = head_key();
            }
        }
    } else {
        // the head of list j from global memory, U from the profile lengths as
        // in the staging above
        const size_t gb = ((size_t)u * t + j) * k;
        auto load_wide = [&]() {
            hv = kPad;
            if (j < t && ptr < k) {
                const uint32_t v = part_id[gb + ptr];
                if (v < n) {
                    uint32_t lv;
                    if (ulen) {
                        lv = ulen[v];
                    } else {
                        const int64_t b0 = indptr[v], b1 = indptr[v + 1];
                        const int64_t lo = b0 < 0 ? 0 : b0;
                        const int64_t hi = b1 < (int64_t)nnz ? b1 : (int64_t)nnz;
                        lv = hi > lo ? (uint32_t)(hi - lo) : 0u;
                    }
                    hv = v;
                    hI = part_I[gb + ptr];
                    hU = ulen_s[ul] + lv - hI;
                }
            }
        };
        load_wide();
        while (out < k) {
            // the group maximum of the heads (kPad: list exhausted), exact order
            bool ok = hv != kPad;
            uint32_t bI = hI, bU = hU, bv = hv;
#pragma unroll
            for (int d = G / 2; d > 0; d >>= 1) {
                const bool ook = __shfl_xor((int)ok, d, G) != 0;
                const uint32_t oI2 = __shfl_xor(bI, d, G), oU2 = __shfl_xor(bU, d, G);
                const uint32_t ov = __shfl_xor(bv, d, G);
                const bool take = ook && (!ok || jbetter(oI2, oU2, ov, bI, bU, bv));
                if (take) { ok = true; bI = oI2; bU = oU2; bv = ov; }
            }
            if (!ok) break;
            if (j == 0) {
                oid[out] = bv;
                oI[out] = bI;
                oU[out] = bU;
            }
            ++out;
            if (hv == bv) {
                ++ptr;
                load_wide();
            }
        }
    }
    for (uint32_t r = out + j; r < k; r += G) {
        oid[r] = kPad;
        oI[r] = 0;
        oU[r] = 0;
    }
}

hipError_t launch_merge(const int64_t *indptr, const uint32_t *ulen, uint64_t nnz, uint32_t n,
                        uint32_t t, uint32_t k, const uint32_t *part_id, const uint32_t *part_I,
                        uint32_t *knn_id, uint32_t *knn_I, uint32_t *knn_U, hipStream_t s) {
    uint32_t G = 1;
    while (G < t) G <<= 1;
    const uint32_t upw = G <= kMergeThreads ? kMergeThreads / G : 1;
    const dim3 grid((uint32_t)div_up((uint64_t)n, upw));
#define C2_MERGE(GG)                                                                           \
    case GG:                                                                                   \
        hipLaunchKernelGGL(k_merge<GG>, grid, dim3(kMergeThreads), 0, s, indptr, ulen, nnz, n, \
                           t, k, part_id, part_I, knn_id, knn_I, knn_U);                       \
        break;
    switch (G) {
        C2_MERGE(1) C2_MERGE(2) C2_MERGE(4) C2_MERGE(8) C2_MERGE(16) C2_MERGE(32) C2_MERGE(64)
        default: return hipErrorInvalidValue;
    }
#undef C2_MERGE
    return hipGetLastError();
}

}  // namespace c2
