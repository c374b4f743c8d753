// Step 1 for configurations of at most kWgMaxN users: all split rounds of one
// configuration run inside one workgroup, in LDS (Algorithm 1 and the
// recursive splitting of Section II-D, Fig. 3).
//
// The split of a cluster with index eta uses H\eta(u) = min{h(i) : i in P_u,
// h(i) > eta}.  At depth d a user's segment was formed by its d smallest
// distinct hash values, so the value that splits it next is its (d+1)-th
// smallest distinct value.  k_signature computes the kSigD smallest distinct
// values of every (configuration, user) in one pass over the profiles; deeper
// rounds fall back to a scan of the profile.
//
// The rounds follow the same rules, and produce the same layout, as the
// level-synchronous grid version: per round every active segment is
// regrouped in place, groups of at least two users in ascending new value
// first (users in their previous order), then the users that stay behind
// (no value above eta, or alone with theirs) in their previous order; the
// top level (the configuration) keeps every group, singletons included.
#include "c2_internal.h"
#include "c2_kernels.h"

namespace c2 {

constexpr int kSigLanes = 16;  // lanes per user: the longest profile sets the kernel's time
constexpr int kWgThreads = 1024;
constexpr int kWgWaves = kWgThreads / 64;
constexpr uint32_t kWgPer = kWgMaxN / kWgThreads;  // slots per thread in scans
constexpr uint32_t kNoValue = 0xFFFFFFFFu;
constexpr uint32_t kRankTab = kWgMaxN / 2;          // active segments hold >= 2 users
constexpr uint32_t kWideBits = 10;                  // keys this short sort in one pass
constexpr uint32_t kWideBins = 1u << kWideBits;

// Insert x into the ascending list s of distinct values (kNoValue = empty),
// keeping the kSigD smallest.
C2_DEV void sig_insert(uint32_t (&s)[kSigD], uint32_t x) {
    bool dup = false;
#pragma unroll
    for (int i = 0; i < kSigD; ++i) dup |= s[i] == x;
    if (dup || x >= s[kSigD - 1]) return;
#pragma unroll
    for (int i = kSigD - 1; i >= 1; --i) s[i] = x < s[i - 1] ? s[i - 1] : (x < s[i] ? x : s[i]);
    s[0] = x < s[0] ? x : s[0];
}

// sig[(j*n + u)*kSigD + r] = the (r+1)-th smallest distinct value of
// h_j over P_u, or kNoValue.  Block (x, j) takes kSigUsers users of
// configuration j, kSigLanes lanes per user; with STAGE the configuration's
// bucket table is first copied to LDS, so the per-item lookups are LDS reads.
// The first thread also clears the status word and the round counter of the
// workgroup pass.
constexpr uint32_t kSigUsers = 16;  // one user per lane group: many blocks in flight
static_assert(kSigD <= kSigLanes, "lane r < kSigD of a group writes signature value r");
constexpr uint32_t kSigTableMax = 8192;  // items whose bucket table is staged in LDS

template <bool STAGE>
__global__ __launch_bounds__(256) void k_signature(const int64_t *__restrict__ indptr,
                                                   const uint32_t *__restrict__ indices,
                                                   uint64_t nnz, uint32_t n, uint32_t m,
                                                   const uint32_t *__restrict__ bucket,
                                                   uint32_t *__restrict__ sig,
                                                   uint32_t *status, uint32_t *rctr) {
    extern __shared__ uint32_t tbl[];  // m entries when STAGE
    const uint32_t j = blockIdx.y;
    if (blockIdx.x == 0 && j == 0 && threadIdx.x == 0) {
        if (status) *status = 0;
        *rctr = 0;
    }
    const uint32_t *bj = bucket + (size_t)j * m;
    if (STAGE) {
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) tbl[i] = bj[i];
        __syncthreads();
    }
    const uint32_t *look = STAGE ? tbl : bj;
    const uint32_t gl = threadIdx.x % kSigLanes;
    const uint32_t u0 = blockIdx.x * kSigUsers;
    for (uint32_t ub = threadIdx.x / kSigLanes; ub < kSigUsers; ub += blockDim.x / kSigLanes) {
        const uint32_t u = u0 + ub;
        if (u >= n) break;  // whole groups leave together
        uint32_t s[kSigD];
#pragma unroll
        for (int i = 0; i < kSigD; ++i) s[i] = kNoValue;
        uint64_t a, e;
        row_range(indptr, u, nnz, a, e);
        // eight index -> bucket lookups in flight per lane
        for (uint64_t p = a + gl; p < e; p += 8 * kSigLanes) {
            uint32_t it[8], x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint64_t pq = p + (uint64_t)q * kSigLanes;
                it[q] = pq < e ? indices[pq] : m;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = it[q] < m ? look[it[q]] : kNoValue;
#pragma unroll
            for (int q = 0; q < 8; ++q) sig_insert(s, x[q]);
        }
        // merge the lanes' lists: kSigD times the group minimum of the heads;
        // lane r keeps the r-th value and the group writes them together
        uint32_t mine = kNoValue;
#pragma unroll
        for (int r = 0; r < kSigD; ++r) {
            uint32_t mn = s[0];
#pragma unroll
            for (int d = kSigLanes / 2; d > 0; d >>= 1) {
                const uint32_t o = __shfl_xor(mn, d, kSigLanes);
                mn = o < mn ? o : mn;
            }
            if ((uint32_t)r == gl) mine = mn;
            if (s[0] == mn && mn != kNoValue) {
#pragma unroll
                for (int i = 0; i + 1 < kSigD; ++i) s[i] = s[i + 1];
                s[kSigD - 1] = kNoValue;
            }
        }
        if (gl < (uint32_t)kSigD) sig[((size_t)j * n + u) * kSigD + gl] = mine;
    }
}

struct WgLds {
    uint32_t key[kWgMaxN];      // per slot: the value that formed its segment;
                                // during a round, the sort key (rank << bb | value)
    uint16_t uid[kWgMaxN];      // user at each slot
    uint16_t seg[kWgMaxN];      // first slot of each slot's segment
    uint16_t idx[2][kWgMaxN];   // active slots through the sort; then run starts
    uint8_t st[kWgMaxN];        // state of the segment starting at this slot
    uint8_t rflag[kWgMaxN];     // active slot that stays behind this round
    uint16_t tab[4][kRankTab];  // radix tables, then per-rank bookkeeping
    uint32_t hist[kWideBins];
    uint32_t base[kWideBins];
    uint32_t wsum[kWgWaves + 1];
};

// Block-wide exclusive scan of kWgPer consecutive values per thread (in
// place in v); returns the total.
C2_DEV uint32_t wg_scan(uint32_t (&v)[kWgPer], uint32_t *wsum) {
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t i = 0; i < kWgPer; ++i) {
        const uint32_t x = v[i];
        v[i] = sum;
        sum += x;
    }
    uint32_t total;
    const uint32_t pre = block_excl_scan<uint32_t, kWgThreads>(sum, wsum, &total);
#pragma unroll
    for (uint32_t i = 0; i < kWgPer; ++i) v[i] += pre;
    return total;
}

// Stable LSD radix sort of the A slot indices in L.idx[0] by L.key[slot] over
// nbits bits: one pass of up to kWideBits bits if the key is that short, else
// passes of 8 bits.  Each wave owns a contiguous range of the elements: it
// counts its digits into its own row of the table, one conversion turns the
// rows into output offsets (digit-major, waves in order), and the wave then
// places its range in index order with its row as running cursors.  Inside a
// wave, 64 elements at a time, equal digits are ranked by ballots.  Returns
// the buffer holding the result.
C2_DEV int wg_sort(WgLds &L, uint32_t A, uint32_t nbits) {
    const uint32_t tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint32_t width = nbits <= kWideBits ? kWideBits : 8;
    const uint32_t nbins = 1u << width;
    uint16_t *tab = &L.tab[0][0];  // [kWgWaves][nbins] over the whole bookkeeping area
    uint16_t *row = tab + wid * nbins;  // this wave's row
    static_assert(kWgWaves * kWideBins <= 4 * kRankTab, "radix table fits the bookkeeping area");
    const uint32_t per = (A + kWgWaves - 1) / kWgWaves;
    const uint32_t begin = wid * per < A ? wid * per : A;
    const uint32_t end = begin + per < A ? begin + per : A;
    int in = 0;
    for (uint32_t sh = 0; sh < nbits; sh += width) {
        const uint32_t dmask = nbins - 1;
        for (uint32_t d = lane; d < nbins; d += 64) row[d] = 0;
        // ranking of equal digits among the 64 elements at i0 .. i0+63
        auto rank = [&](uint32_t i0, uint32_t &s, uint32_t &d, uint64_t &peers, bool &valid) {
            const uint32_t i = i0 + lane;
            valid = i < end;
            s = valid ? L.idx[in][i] : 0u;
            d = valid ? (L.key[s] >> sh) & dmask : 0u;
            peers = __ballot(valid);
            for (uint32_t bit = 0; bit < width; ++bit) {
                const bool on = (d >> bit) & 1u;
                const uint64_t bb = __ballot(on);
                peers &= on ? bb : ~bb;
            }
        };
        for (uint32_t i0 = begin; i0 < end; i0 += 64) {
            uint32_t s, d;
            uint64_t peers;
            bool valid;
            rank(i0, s, d, peers, valid);
            if (valid && (peers & lt_mask) == 0) row[d] = (uint16_t)(row[d] + __popcll(peers));
        }
        __syncthreads();
        {   // digit tid: its total, the offsets of all digits before it, then
            // each wave's start inside the digit
            uint32_t tot = 0;
            if (tid < nbins)
                for (int w = 0; w < kWgWaves; ++w) tot += tab[w * nbins + tid];
            uint32_t all;
            uint32_t run = block_excl_scan<uint32_t, kWgThreads>(tid < nbins ? tot : 0u, L.wsum, &all);
            if (tid < nbins)
                for (int w = 0; w < kWgWaves; ++w) {
                    const uint32_t c = tab[w * nbins + tid];
                    tab[w * nbins + tid] = (uint16_t)run;
                    run += c;
                }
        }
        __syncthreads();
        for (uint32_t i0 = begin; i0 < end; i0 += 64) {
            uint32_t s, d;
            uint64_t peers;
            bool valid;
            rank(i0, s, d, peers, valid);
            const uint32_t cur = valid ? row[d] : 0u;  // read by all lanes of the digit first
            if (valid) L.idx[in ^ 1][cur + __popcll(peers & lt_mask)] = (uint16_t)s;
            if (valid && (peers & lt_mask) == 0) row[d] = (uint16_t)(cur + __popcll(peers));
        }
        __syncthreads();
        in ^= 1;
    }
    return in;
}

// H\eta(u) by a scan of the profile (rounds deeper than the signature).
C2_DEV uint32_t min_above(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                          const uint32_t *bj, uint32_t m, uint32_t b, uint32_t u, uint32_t eta) {
    uint64_t a, e;
    row_range(indptr, u, nnz, a, e);
    uint32_t best = b;
    for (uint64_t p = a; p < e; ++p) {
        const uint32_t it = indices[p];
        const uint32_t h = it < m ? bj[it] : b;
        if (h > eta && h < best) best = h;
    }
    return best;
}

// One workgroup per configuration j (n <= kWgMaxN).  Writes members[j*n ..),
// the first slot of each final cluster (cstart[j*n + c], c < ccount[j]) and
// ccount[j]; raises *status if max_rounds rounds left clusters unsplit; keeps
// the largest number of rounds used in *rctr.
__global__ __launch_bounds__(kWgThreads) void k_clu_wg(
    const int64_t *__restrict__ indptr, const uint32_t *__restrict__ indices, uint64_t nnz,
    uint32_t n, uint32_t m, const uint32_t *__restrict__ bucket, const uint32_t *__restrict__ sig,
    uint32_t b, uint32_t bb, uint32_t cap, uint32_t max_rounds, uint32_t *__restrict__ members,
    uint32_t *__restrict__ cstart, uint32_t *__restrict__ ccount, uint32_t *status,
    uint32_t *rctr) {
    __shared__ WgLds L;
    const uint32_t tid = threadIdx.x, j = blockIdx.x;
    const uint32_t *bj = bucket + (size_t)j * m;
    const uint32_t *sj = sig + (size_t)j * n * kSigD;
    const uint32_t vmask = (1u << bb) - 1u;
    for (uint32_t p = tid; p < n; p += kWgThreads) {
        L.uid[p] = (uint16_t)p;
        L.seg[p] = 0;
        L.key[p] = 0;
        L.st[p] = kFinal;
    }
    __syncthreads();
    if (tid == 0) L.st[0] = kRoot;
    __syncthreads();
    const uint32_t s0 = tid * kWgPer;  // this thread's slots / sorted entries
    uint32_t round = 0;
    for (;; ++round) {
        // (1) active slots in slot order, and the rank of each active segment
        uint32_t v[kWgPer];
#pragma unroll
        for (uint32_t i = 0; i < kWgPer; ++i) {
            const uint32_t p = s0 + i;
            uint32_t x = 0;
            if (p < n) {
                const uint32_t h = L.seg[p];
                const bool act = L.st[h] != kFinal;
                x = (act ? 1u : 0u) | ((act && h == p) ? 0x10000u : 0u);
            }
            v[i] = x;
        }
        const uint32_t tot = wg_scan(v, L.wsum);
        const uint32_t A = tot & 0xFFFFu, nseg = tot >> 16;
        if (A == 0) break;
        if (round >= max_rounds) {
            if (tid == 0 && status) atomicOr(status, 1u);
            break;
        }
#pragma unroll
        for (uint32_t i = 0; i < kWgPer; ++i) {
            const uint32_t p = s0 + i;
            if (p < n) {
                const uint32_t h = L.seg[p];
                if (L.st[h] != kFinal) {
                    L.idx[0][v[i] & 0xFFFFu] = (uint16_t)p;
                    if (h == p) L.idx[1][p] = (uint16_t)(v[i] >> 16);  // rank of the segment
                }
            }
        }
        __syncthreads();
        // (2) sort keys: rank of the segment, then the next hash value
        if (round < (uint32_t)kSigD) {
            uint32_t e[kWgPer];  // all lookups in flight first
#pragma unroll
            for (uint32_t i = 0; i < kWgPer; ++i) {
                const uint32_t q = tid + i * kWgThreads;
                e[i] = q < A ? sj[(size_t)L.uid[L.idx[0][q]] * kSigD + round] : 0u;
            }
#pragma unroll
            for (uint32_t i = 0; i < kWgPer; ++i) {
                const uint32_t q = tid + i * kWgThreads;
                if (q < A) {
                    const uint32_t p = L.idx[0][q];
                    const uint32_t ev = e[i] >= b ? b : e[i];  // b: no value above eta
                    L.key[p] = ((uint32_t)L.idx[1][L.seg[p]] << bb) | ev;
                }
            }
        } else {
            for (uint32_t q = tid; q < A; q += kWgThreads) {
                const uint32_t p = L.idx[0][q];
                uint32_t ev = min_above(indptr, indices, nnz, bj, m, b, L.uid[p], L.key[p]);
                if (ev >= b) ev = b;
                L.key[p] = ((uint32_t)L.idx[1][L.seg[p]] << bb) | ev;
            }
        }
        __syncthreads();
        // (3) stable sort of the active slots by key
        // at the top level every user has a value below b
        const uint32_t nbits = round == 0 ? bit_width_dev(b - 1) : bb + bit_width_dev(nseg - 1);
        const int res = wg_sort(L, A, nbits);
        uint16_t *sorted = L.idx[res];
        uint16_t *runs = L.idx[res ^ 1];
        // (4) groups: runs of equal keys in sorted order
        uint32_t hf[kWgPer];
#pragma unroll
        for (uint32_t i = 0; i < kWgPer; ++i) {
            const uint32_t q = s0 + i;
            hf[i] = (q < A && (q == 0 || L.key[sorted[q]] != L.key[sorted[q - 1]])) ? 1u : 0u;
        }
        const uint32_t nruns = wg_scan(hf, L.wsum);
#pragma unroll
        for (uint32_t i = 0; i < kWgPer; ++i) {
            const uint32_t q = s0 + i;
            if (q < A && (q == 0 || L.key[sorted[q]] != L.key[sorted[q - 1]])) runs[hf[i]] = (uint16_t)q;
        }
        __syncthreads();
        // per sorted entry: run start, run length, stays behind?
        uint32_t rs[kWgPer], rl[kWgPer], nr[kWgPer];
#pragma unroll
        for (uint32_t i = 0; i < kWgPer; ++i) {
            const uint32_t q = s0 + i;
            rs[i] = rl[i] = nr[i] = 0;
            if (q < A) {
                const uint32_t rid = hf[i] - ((q == 0 || L.key[sorted[q]] != L.key[sorted[q - 1]]) ? 0u : 1u);
                rs[i] = runs[rid];
                rl[i] = (rid + 1 < nruns ? runs[rid + 1] : A) - rs[i];
                const uint32_t p = sorted[q];
                const bool root = L.st[L.seg[p]] == kRoot;
                const bool resid = !root && ((L.key[p] & vmask) == b || rl[i] == 1);
                L.rflag[p] = resid ? 1u : 0u;
                nr[i] = resid ? 0u : 1u;
            }
        }
        __syncthreads();
        // (5) positions.  Groups: in sorted order from the parent's first slot.
        // Stay-behind users: after the parent's groups, in slot order.
        uint16_t *nrfirst = L.tab[0], *gcnt = L.tab[1], *rrhead = L.tab[2];
        wg_scan(nr, L.wsum);  // nr[i] = non-residual entries before sorted entry q
#pragma unroll
        for (uint32_t i = 0; i < kWgPer; ++i) {
            const uint32_t q = s0 + i;
            if (q < A) {
                const uint32_t rk = L.key[sorted[q]] >> bb;
                if (q == 0 || (L.key[sorted[q - 1]] >> bb) != rk) nrfirst[rk] = (uint16_t)nr[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t i = 0; i < kWgPer; ++i) {
            const uint32_t q = s0 + i;
            if (q < A) {
                const uint32_t rk = L.key[sorted[q]] >> bb;
                if (q + 1 == A || (L.key[sorted[q + 1]] >> bb) != rk)
                    gcnt[rk] = (uint16_t)(nr[i] + (L.rflag[sorted[q]] ? 0u : 1u) - nrfirst[rk]);
            }
        }
        uint32_t rr[kWgPer];
#pragma unroll
        for (uint32_t i = 0; i < kWgPer; ++i) {
            const uint32_t p = s0 + i;
            rr[i] = (p < n && L.st[L.seg[p]] != kFinal && L.rflag[p]) ? 1u : 0u;
        }
        wg_scan(rr, L.wsum);  // rr[i] = stay-behind slots before slot p
#pragma unroll
        for (uint32_t i = 0; i < kWgPer; ++i) {
            const uint32_t p = s0 + i;
            if (p < n && L.seg[p] == p && L.st[p] != kFinal) rrhead[L.key[p] >> bb] = (uint16_t)rr[i];
        }
        __syncthreads();
        // (6) gather, then move.  Packed per entry: new slot | new segment
        // start << 16; user | state << 16 (kNoState: not a segment start).
        constexpr uint32_t kNoState = 0xFFu;
        uint32_t gpos[kWgPer], gusr[kWgPer], gval[kWgPer];
#pragma unroll
        for (uint32_t i = 0; i < kWgPer; ++i) {
            gpos[i] = kNoValue;
            const uint32_t q = s0 + i;  // sorted entry: users that form groups
            if (q < A) {
                const uint32_t p = sorted[q];
                if (!L.rflag[p]) {
                    const uint32_t P = L.seg[p], rk = L.key[p] >> bb;
                    const uint32_t np = P + nr[i] - nrfirst[rk];
                    const uint32_t head = np - (q - rs[i]);
                    const uint32_t stt = q == rs[i] ? (rl[i] > cap ? kActive : kFinal) : kNoState;
                    gpos[i] = np | (head << 16);
                    gusr[i] = (uint32_t)L.uid[p] | (stt << 16);
                    gval[i] = L.key[p] & vmask;
                }
            }
        }
        uint32_t rpos[kWgPer], rusr[kWgPer], rval[kWgPer];
#pragma unroll
        for (uint32_t i = 0; i < kWgPer; ++i) {
            rpos[i] = kNoValue;
            const uint32_t p = s0 + i;  // slot: users that stay behind
            if (p < n && L.st[L.seg[p]] != kFinal && L.rflag[p]) {
                const uint32_t P = L.seg[p], rk = L.key[p] >> bb;
                const uint32_t head = P + gcnt[rk];
                rpos[i] = (head + rr[i] - rrhead[rk]) | (head << 16);
                rusr[i] = (uint32_t)L.uid[p] | ((rr[i] == rrhead[rk] ? kFinal : kNoState) << 16);
                rval[i] = L.key[p] & vmask;
            }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t i = 0; i < kWgPer; ++i) {
            if (gpos[i] != kNoValue) {
                const uint32_t np = gpos[i] & 0xFFFFu, stt = gusr[i] >> 16;
                L.uid[np] = (uint16_t)gusr[i];
                L.seg[np] = (uint16_t)(gpos[i] >> 16);
                L.key[np] = gval[i];
                if (stt != kNoState) L.st[np] = (uint8_t)stt;
            }
            if (rpos[i] != kNoValue) {
                const uint32_t np = rpos[i] & 0xFFFFu, stt = rusr[i] >> 16;
                L.uid[np] = (uint16_t)rusr[i];
                L.seg[np] = (uint16_t)(rpos[i] >> 16);
                L.key[np] = rval[i];
                if (stt != kNoState) L.st[np] = (uint8_t)stt;
            }
        }
#pragma unroll
        for (uint32_t i = 0; i < kWgPer; ++i) {
            const uint32_t p = s0 + i;
            if (p < n) L.rflag[p] = 0;
        }
        __syncthreads();
    }
    // output: the layout and the first slot of every final cluster
    uint32_t hf[kWgPer];
#pragma unroll
    for (uint32_t i = 0; i < kWgPer; ++i) {
        const uint32_t p = s0 + i;
        hf[i] = (p < n && L.seg[p] == p) ? 1u : 0u;
    }
    const uint32_t ncl = wg_scan(hf, L.wsum);
#pragma unroll
    for (uint32_t i = 0; i < kWgPer; ++i) {
        const uint32_t p = s0 + i;
        if (p < n) {
            members[(size_t)j * n + p] = L.uid[p];
            if (L.seg[p] == p) cstart[(size_t)j * n + hf[i]] = p;
        }
    }
    if (tid == 0) {
        ccount[j] = ncl;
        atomicMax(rctr, round);
    }
}

// cl_cfg_off, cl_off from the per-configuration cluster starts.
__global__ __launch_bounds__(256) void k_clu_wg_final(const uint32_t *cstart,
                                                      const uint32_t *ccount, uint32_t n,
                                                      uint32_t t, uint32_t *cl_off,
                                                      uint32_t *cl_cfg_off) {
    const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (uint64_t)t * n) return;
    const uint32_t j = (uint32_t)(x / n), c = (uint32_t)(x % n);
    if (c >= ccount[j]) return;
    uint32_t off = 0;
    for (uint32_t q = 0; q < j; ++q) off += ccount[q];
    cl_off[off + c] = j * n + cstart[x];
    if (c == 0) cl_cfg_off[j] = off;
    if (j == t - 1 && c == 0) {
        const uint32_t total = off + ccount[j];
        cl_cfg_off[t] = total;
        cl_off[total] = t * n;
    }
}

size_t cluster_wg_ws_bytes(uint32_t n, uint32_t t) {
    const size_t NE = (size_t)n * t;
    return 4 * (NE * kSigD + NE + 64 + 64);
}

bool cluster_wg_fits(uint32_t n, uint32_t b) {
    const uint32_t bb = bit_width(b);
    // keys hold (segment rank << bb) | value with ranks below kWgMaxN / 2
    return n >= 1 && n <= kWgMaxN && bb + bit_width(kRankTab - 1) <= 32;
}

hipError_t cluster_wg_run(const ClusterArgs &a, uint32_t *members, uint32_t *cl_off,
                          uint32_t *cl_cfg_off, char *scratch, uint32_t *status,
                          uint32_t max_rounds, uint32_t **rctr_out, hipStream_t s) {
    const size_t NE = (size_t)a.n * a.t;
    uint32_t *sig = reinterpret_cast<uint32_t *>(scratch);
    uint32_t *cstart = sig + NE * kSigD;
    uint32_t *ccount = cstart + NE;
    uint32_t *rctr = ccount + 64;
    if (rctr_out) *rctr_out = rctr;
    const dim3 sg((uint32_t)div_up(a.n, kSigUsers), a.t);
    if (a.m <= kSigTableMax)
        hipLaunchKernelGGL(k_signature<true>, sg, dim3(256), 4 * (size_t)a.m, s, a.indptr,
                           a.indices, a.nnz, a.n, a.m, a.bucket, sig, status, rctr);
    else
        hipLaunchKernelGGL(k_signature<false>, sg, dim3(256), 0, s, a.indptr, a.indices, a.nnz,
                           a.n, a.m, a.bucket, sig, status, rctr);
    hipLaunchKernelGGL(k_clu_wg, dim3(a.t), dim3(kWgThreads), 0, s, a.indptr, a.indices, a.nnz,
                       a.n, a.m, a.bucket, sig, a.b, a.bb, a.cap, max_rounds, members, cstart,
                       ccount, status, rctr);
    hipLaunchKernelGGL(k_clu_wg_final, dim3((uint32_t)div_up(NE, 256)), dim3(256), 0, s, cstart,
                       ccount, a.n, a.t, cl_off, cl_cfg_off);
    return hipGetLastError();
}

}  // namespace c2
