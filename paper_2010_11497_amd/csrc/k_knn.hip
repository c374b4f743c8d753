// Step 2 on the device: exact brute-force KNN inside every cluster
// (Section II-F, Algorithm 2, brute-force branch).
//
// Every user's profile is stored once as a bit row over the item universe
// (padded to a multiple of 64 items).  |P_u & P_v| is the dot product of two
// bit rows; |P_u | P_v| = |P_u| + |P_v| - |P_u & P_v|.  Two paths compute the
// dot products of a cluster's members, in tiles of (row block x column block):
//   - MFMA: 64-item chunks of the bit rows are expanded in LDS to 4-bit
//     e2m1 values (0 or 1.0) and multiplied with the gfx950 block-scaled
//     v_mfma_scale_f32_32x32x64_f8f6f4 at unit scale; the fp32 sums are
//     integer counts below 2^24, hence exact;
//   - bitmap: AND + population count of 32-bit words, for small clusters.
// Selection: every member of the row block owns a bounded heap of its k best
// candidates in LDS (worst at the root, exact Jaccard order) and offers each
// candidate that beats the root.
#include "c2_internal.h"
#include "c2_kernels.h"

namespace c2 {

constexpr int kStageThreads = 256;
constexpr int kStageWaves = kStageThreads / 64;
constexpr uint32_t kRowBlock = 64;   // rows (members) per bitmap work item
constexpr int kWordChunk = 16;       // bit-row words staged per step (bitmap path)
constexpr uint32_t kMR = 128;        // rows per MFMA work item (row owners)
constexpr uint32_t kMC = 128;        // columns per MFMA step
constexpr uint32_t kDefaultMfmaMin = 2;
constexpr uint32_t kPf = 4;          // chunks prefetched ahead (two pairs); rows pad to kPf chunks
constexpr uint32_t kGroupTiles = 4;  // column tiles per work item before a row block is split
constexpr uint32_t kMaxGroups = 4;   // column groups a row block is split into at most
constexpr uint32_t kUserBitsGrid = 2048;  // blocks of k_user_bits at most
constexpr uint32_t kBitmapPersistent = 256;  // persistent bitmap-path workgroups (batched form)
// batched planning counters: kCostClasses item counts, then scratch slots and
// bitmap items
constexpr uint32_t kCostClasses = 64;
constexpr uint32_t kSlotCtr = kCostClasses, kBitmapCtr = kCostClasses + 1;
constexpr uint32_t kPlanCtr = kCostClasses + 2;
// per-cluster dictionaries: automatic from rows of this many words, for
// clusters of at most kCompactMaxS members
constexpr uint32_t kCompactMinW = 512;
constexpr uint32_t kCompactMaxS = 8192;
constexpr uint32_t kCompactGrid = 1024;

// Words per bit row: the item universe padded to a multiple of 64 * kPf items,
// so the MFMA K loop runs whole unrolled groups.
uint32_t knn_wmax(uint32_t m) { return 2 * kPf * (uint32_t)div_up(m, 64 * kPf); }

size_t knn_stage_lds_bytes(uint32_t m, uint32_t wmax) {
    (void)m;
    return 4 * (size_t)kStageWaves * wmax;
}

C2_DEV void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ bit rows

// ubits[u][w]: bit (i & 31) of word i >> 5 is set iff item i is in P_u; rows
// are padded to a multiple of 64 items.  ulen[u] = |P_u|.  Row n is all zero:
// padding members of a tile point at it, so tile loads need no predicate.
// One wave per user, the row assembled in LDS and written out whole.
__global__ __launch_bounds__(kStageThreads) void k_user_bits(const int64_t *__restrict__ indptr,
                                                             const uint32_t *__restrict__ indices,
                                                             uint64_t nnz, uint32_t n, uint32_t m,
                                                             uint32_t Wg,
                                                             uint32_t *__restrict__ ubits,
                                                             uint32_t *__restrict__ ulen,
                                                             uint32_t *bmax_out,
                                                             uint32_t *plan_ctr) {
    extern __shared__ uint32_t lds[];
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t *rb = lds + wid * Wg;
    uint32_t longest = 0;
    // the next user's row range is loaded while this user's row is built
    const uint32_t step = gridDim.x * kStageWaves;
    uint32_t u = blockIdx.x * kStageWaves + wid;
    uint64_t na = 0, ne = 0;
    if (u < n) row_range(indptr, u, nnz, na, ne);
    for (; u <= n; u += step) {
        const uint64_t p0 = na, p1 = ne;
        na = ne = 0;
        if ((uint64_t)u + step < n) row_range(indptr, u + step, nnz, na, ne);
        for (uint32_t w = lane; w < Wg; w += 64) rb[w] = 0;
        wave_sync();
        for (uint64_t p = p0 + lane; p < p1; p += 64) {
            const uint32_t i = indices[p];
            if (i < m) atomicOr(&rb[i >> 5], 1u << (i & 31));
        }
        wave_sync();
        uint32_t *out = ubits + (size_t)u * Wg;
        for (uint32_t w = lane; w < Wg; w += 64) out[w] = rb[w];
        if (lane == 0) ulen[u] = (uint32_t)(p1 - p0);
        if (p1 - p0 > longest) longest = (uint32_t)(p1 - p0);
        wave_sync();
    }
    // the longest profile of this block (the grid is capped); the planning
    // kernels reduce the per-block values
    __shared__ uint32_t bmax;
    if (threadIdx.x == 0) bmax = 0;
    __syncthreads();
    if (lane == 0 && longest) atomicMax(&bmax, longest);
    __syncthreads();
    if (threadIdx.x == 0) bmax_out[blockIdx.x] = bmax;
    if (plan_ctr && blockIdx.x == 0 && threadIdx.x < kPlanCtr) plan_ctr[threadIdx.x] = 0;
}

// Longest profile, from the per-block values of k_user_bits (block-wide).
C2_DEV uint32_t block_max_len(const uint32_t *bmax, uint32_t nb) {
    __shared__ uint32_t red;
    if (threadIdx.x == 0) red = 0;
    __syncthreads();
    uint32_t v = 0;
    for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) v = bmax[i] > v ? bmax[i] : v;
    if (v) atomicMax(&red, v);
    __syncthreads();
    return red;
}

// --------------------------------------------------------------- selection

// Bounded heap of one row's best candidates, structure-of-arrays in LDS with
// the owner's index as the minor index (conflict-free).  Root = worst kept.
template <uint32_t STRIDE>
struct RowHeap {
    uint32_t *hI, *hU, *hV;  // [kMaxK][STRIDE]
    uint32_t me, k, cnt;
    uint32_t rI, rU, rV;     // root copy

    C2_DEV void get(uint32_t i, uint32_t &I, uint32_t &U, uint32_t &V) const {
        I = hI[i * STRIDE + me];
        U = hU[i * STRIDE + me];
        V = hV[i * STRIDE + me];
    }
    C2_DEV void put(uint32_t i, uint32_t I, uint32_t U, uint32_t V) {
        hI[i * STRIDE + me] = I;
        hU[i * STRIDE + me] = U;
        hV[i * STRIDE + me] = V;
    }
    // Sift (I, U, V) down from the root over `size` entries.
    C2_DEV void sift_down(uint32_t I, uint32_t U, uint32_t V, uint32_t size) {
        uint32_t pos = 0;
        for (;;) {
            uint32_t l = 2 * pos + 1;
            if (l >= size) break;
            uint32_t cI, cU, cV;
            get(l, cI, cU, cV);
            if (l + 1 < size) {
                uint32_t dI, dU, dV;
                get(l + 1, dI, dU, dV);
                if (jbetter(cI, cU, cV, dI, dU, dV)) { l = l + 1; cI = dI; cU = dU; cV = dV; }
            }
            if (!jbetter(I, U, V, cI, cU, cV)) break;
            put(pos, cI, cU, cV);
            pos = l;
        }
        put(pos, I, U, V);
    }
    C2_DEV void init(uint32_t *I, uint32_t *U, uint32_t *V, uint32_t owner, uint32_t kk) {
        hI = I; hU = U; hV = V; me = owner; k = kk; cnt = 0; rI = 0; rU = 1; rV = kPad;
    }
    C2_DEV void offer(uint32_t I, uint32_t U, uint32_t V) {
        if (cnt < k) {
            uint32_t pos = cnt++;
            while (pos > 0) {
                const uint32_t par = (pos - 1) >> 1;
                uint32_t pI, pU, pV;
                get(par, pI, pU, pV);
                if (!jbetter(pI, pU, pV, I, U, V)) break;
                put(pos, pI, pU, pV);
                pos = par;
            }
            put(pos, I, U, V);
            get(0, rI, rU, rV);
        } else if (jbetter(I, U, V, rI, rU, rV)) {
            sift_down(I, U, V, k);
            get(0, rI, rU, rV);
        }
    }
    // Write the kept entries best first, padded to k.
    C2_DEV void drain(uint32_t *out_id, uint32_t *out_I) {
        for (uint32_t r = cnt; r < k; ++r) {
            out_id[r] = kPad;
            out_I[r] = 0;
        }
        for (uint32_t size = cnt; size > 0; --size) {
            uint32_t I, U, V;
            get(0, I, U, V);
            out_id[size - 1] = V;
            out_I[size - 1] = I;
            if (size > 1) {
                uint32_t lI, lU, lV;
                get(size - 1, lI, lU, lV);
                sift_down(lI, lU, lV, size - 1);
            }
        }
    }
};

// Cluster c as seen by a work item.
struct ClusterView {
    uint32_t o, s, j;
};

C2_DEV ClusterView view(const KnnArgs &a, uint32_t c) {
    ClusterView v;
    v.o = a.cl_off[c];
    v.s = a.cl_off[c + 1] - v.o;
    v.j = v.o / a.n;
    return v;
}

C2_DEV uint32_t member(const KnnArgs &a, const ClusterView &v, uint32_t idx) {
    const uint32_t u = idx < v.s ? a.members[v.o + idx] : a.n;
    return u < a.n ? u : a.n;
}

// ------------------------------------------------------------ bitmap path
//
// One wave per work item (cluster, block of 64 rows); lane = row owner.  The
// lane keeps its row's 16-word chunk in registers and accumulates AND +
// popcount against each column row of a 64-column tile staged in LDS (read
// as a broadcast).

struct __attribute__((aligned(16))) BitmapLds {
    uint32_t colw[kRowBlock][kWordChunk];
    uint32_t clen[kRowBlock], cuid[kRowBlock];
    uint32_t hI[kMaxK * 64], hU[kMaxK * 64], hV[kMaxK * 64];
};

C2_DEV void bitmap_item(const KnnArgs &a, const uint32_t *ubits, const uint32_t *ulen,
                        uint32_t c, uint32_t rb, BitmapLds &L) {
    const uint32_t lane = threadIdx.x;
    const ClusterView cv = view(a, c);
    const uint32_t s = cv.s, W = a.wmax;
    const uint32_t ra = rb * kRowBlock + lane;
    const uint32_t ur = member(a, cv, ra);
    const bool active = ur < a.n;
    const uint32_t Lr = active ? ulen[ur] : 0;
    RowHeap<64> h;
    h.init(L.hI, L.hU, L.hV, lane, a.k);
    const uint32_t *myrow = ubits + (size_t)(active ? ur : 0) * W;
    for (uint32_t cb = 0; cb * kRowBlock < s; ++cb) {
        __syncthreads();
        const uint32_t uc = member(a, cv, cb * kRowBlock + lane);
        L.clen[lane] = uc < a.n ? ulen[uc] : 0;
        L.cuid[lane] = uc;
        __syncthreads();
        uint32_t acc[kRowBlock];
#pragma unroll
        for (int q = 0; q < (int)kRowBlock; ++q) acc[q] = 0;
        for (uint32_t w0 = 0; w0 < W; w0 += kWordChunk) {
            __syncthreads();
#pragma unroll
            for (int it = 0; it < kWordChunk; ++it) {
                const uint32_t idx = it * 64 + lane;
                const uint32_t cc = idx / kWordChunk, ww = idx % kWordChunk;
                const uint32_t ucc = L.cuid[cc];
                L.colw[cc][ww] = (ucc < a.n && w0 + ww < W) ? ubits[(size_t)ucc * W + w0 + ww] : 0u;
            }
            uint32_t r[kWordChunk];
#pragma unroll
            for (int ww = 0; ww < kWordChunk; ++ww)
                r[ww] = (active && w0 + ww < W) ? myrow[w0 + ww] : 0u;
            __syncthreads();
#pragma unroll
            for (int q = 0; q < (int)kRowBlock; ++q) {
                const uint4 *cw = reinterpret_cast<const uint4 *>(L.colw[q]);
                uint32_t x = acc[q];
#pragma unroll
                for (int v4 = 0; v4 < kWordChunk / 4; ++v4) {
                    const uint4 z = cw[v4];
                    x += __popc(r[4 * v4] & z.x) + __popc(r[4 * v4 + 1] & z.y) +
                         __popc(r[4 * v4 + 2] & z.z) + __popc(r[4 * v4 + 3] & z.w);
                }
                acc[q] = x;
            }
        }
        if (active) {
#pragma unroll
            for (int q = 0; q < (int)kRowBlock; ++q) {
                const uint32_t col = cb * kRowBlock + q;
                if (col < s && col != ra) {
                    const uint32_t I = acc[q];
                    h.offer(I, Lr + L.clen[q] - I, L.cuid[q]);
                }
            }
        }
    }
    if (active && cv.j < a.t) {
        const size_t base = ((size_t)ur * a.t + cv.j) * a.k;
        h.drain(a.part_id + base, a.part_I + base);
    }
}

// Plain form: block b handles items[b].  Batched form: persistent blocks take
// items from a device cursor until the list is exhausted.
__global__ __launch_bounds__(64) void k_knn_bitmap(KnnArgs a, const uint32_t *ubits,
                                                   const uint32_t *ulen, const uint64_t *items,
                                                   const uint32_t *n_items, uint32_t *cursor) {
    __shared__ BitmapLds L;
    __shared__ uint32_t next;
    const uint32_t total = *n_items;
    if (total == 0) return;  // the usual case: every cluster is on the MFMA path
    if (!cursor) {
        if (blockIdx.x >= total) return;
        const uint64_t it = items[blockIdx.x];
        bitmap_item(a, ubits, ulen, (uint32_t)(it >> 32), (uint32_t)it, L);
        return;
    }
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) next = atomicAdd(cursor, 1u);
        __syncthreads();
        const uint32_t i = next;
        if (i >= total) break;
        const uint64_t it = items[i];
        bitmap_item(a, ubits, ulen, (uint32_t)(it >> 32), (uint32_t)it, L);
    }
}

// -------------------------------------------------------------- MFMA path
//
// One block of 4 waves per work item (cluster, block of 128 rows).  For every
// 128-column tile of the cluster the block computes the 128 x 128 matrix of
// intersection counts: 256 threads stage their rows' raw bits in LDS two
// 64-item chunks at a time (double-buffered), and each wave expands the words
// of its 64 rows and 64 columns to fp4 nibbles in registers and multiplies
// its 64 x 64 sub-tile as 2 x 2 MFMAs of 32 x 32 x 64.  The counts are written
// to LDS transposed (16 bits each) so that the thread pair of row r reads it.
//
// Selection on this path uses an exact 32-bit similarity key,
//   key(I, U) = floor(I * (2^32 - 1) / U),
// which preserves the order of I/U exactly when U < 2^16 (two different
// fractions with denominators below 2^16 differ by more than 1/(2^32 - 1)),
// so the path is taken only when every profile has fewer than 2^15 items.
// A heap entry is the u64 (key << 32) | (0xFFFFFFFF - id): larger is better,
// and entries are distinct, so an entry beats the root iff it compares
// greater.  Each tile is first filtered against the heap root with a
// necessary fp32 test (and, when many pass, against the k best of the tile);
// the candidates that pass are inserted in a wave-uniform loop, where the
// exact comparison is made.

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// E8M0 block scales of 2^0 for all four operand blocks.
constexpr int kUnitScale = 0x7F7F7F7F;
// Operand format code of e2m1 (fp4) for the f8f6f4 MFMA family.
constexpr int kFmtFp4 = 4;

// C += A * B^T over 64 items for one 32 x 32 block: A and B hold, in lane l,
// 32 nibbles of row / column l % 32 for items [32 * (l / 32), +32).  Only the
// first four dwords of the 8-dword operands are read for fp4.
C2_DEV v16f mfma_fp4(v4i a, v4i b, v16f c) {
    const v8i A = {a[0], a[1], a[2], a[3], 0, 0, 0, 0};
    const v8i B = {b[0], b[1], b[2], b[3], 0, 0, 0, 0};
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, B, c, kFmtFp4, kFmtFp4, 0,
                                                           kUnitScale, 0, kUnitScale);
}

constexpr int kTile16Stride = 136;   // u16 per row of the transposed result tile
constexpr uint32_t kMfmaMaxLen = 1u << 15;
constexpr uint32_t kBisectSlack = 8;  // tile prefilter once more than k + this many pass
constexpr int kBisectSteps = 9;        // brackets the tile's k-th best code to 1/512 of the largest

struct __attribute__((aligned(16))) MfmaLds {
    union __attribute__((aligned(16))) {
        uint2 raw[2][2][kMR + kMC];  // [stage][word half][staged row]: bits of two chunks
        uint16_t itile[kMR][kTile16Stride];
    } u;
    uint32_t cuid[kMC], clen[kMC];
    uint64_t hk[kMaxK * kMR];
};

// 64 bits -> 32 bytes of e2m1 nibbles (0x2 = 1.0 for a set bit).  Dword s
// of a 32-bit word w holds, in byte q, bit 8q+2s of w in its low nibble and
// bit 8q+2s+1 in its high nibble: (w >> 2s) & 0x03030303 puts each byte's
// 2-bit pair in the low bits of that byte, and v_perm_b32 looks the pair up
// in a 4-byte table {0x00, 0x02, 0x20, 0x22} held in both sources (so either
// source order gives the same bytes).  Every row is expanded the same way,
// so item pairs stay aligned in the dot product whatever order the MFMA
// assigns to the nibbles.
constexpr uint32_t kPairLut = 0x22200200u;

C2_DEV uint4 nibbles32(uint32_t w) {
    return make_uint4(__builtin_amdgcn_perm(kPairLut, kPairLut, w & 0x03030303u),
                      __builtin_amdgcn_perm(kPairLut, kPairLut, (w >> 2) & 0x03030303u),
                      __builtin_amdgcn_perm(kPairLut, kPairLut, (w >> 4) & 0x03030303u),
                      __builtin_amdgcn_perm(kPairLut, kPairLut, (w >> 6) & 0x03030303u));
}

C2_DEV v4i as_v4i(uint4 x) { return v4i{(int)x.x, (int)x.y, (int)x.z, (int)x.w}; }

// Bits of chunks 2p and 2p+1 (row words 4p .. 4p+3).  The load is
// unconditional (p clamped into the row) so the compiler can count outstanding
// loads; pairs past the row are staged but never multiplied.
C2_DEV uint4 load_pair(const uint4 *row, uint32_t p, uint32_t npairs) {
    return row[p < npairs ? p : npairs - 1];
}

// I from key(I, U) and S = |P_u| + |P_v| (U = S - I): I/(S - I) is strictly
// increasing in I, and S*key/(2^32 - 1 + key) is within 2^-16 of I.
C2_DEV uint32_t key_to_I(uint32_t key, uint32_t S) {
    // the fp32 estimate is within 0.03 of I for S < 2^17 (checked for every
    // (I, U) with the reciprocal exact and 1-2 ulp off), so it rounds to I
    const float kt = (float)key;
    const float x = (float)S * kt * __builtin_amdgcn_rcpf(4294967295.0f + kt);
    return (uint32_t)(x + 0.5f);
}

struct KeyHeap {
    uint64_t *hk;  // [kMaxK][kMR], minor index = owner
    uint32_t me, k, cnt;
    uint64_t root;  // valid once full

    C2_DEV uint64_t get(uint32_t i) const { return hk[i * kMR + me]; }
    C2_DEV void put(uint32_t i, uint64_t v) { hk[i * kMR + me] = v; }
    // 4-ary min-heap: the children of p are 4p+1 .. 4p+4.  The four child
    // slots are read together (an index past the end reads the last entry
    // again, which never wins the strict comparisons), so each level costs one
    // LDS round trip.  A heap of at most 85 entries is at most three levels
    // below any node, so the descent is unrolled three times with no loop.
    // Returns the entry that ends up at pos.
    C2_DEV uint64_t sift_down(uint32_t pos, uint64_t v, uint32_t size) {
        uint64_t top = v;
        bool done = false;
        const uint32_t last = size - 1;
#pragma unroll
        for (int lvl = 0; lvl < 3; ++lvl) {
            const uint32_t c0 = 4 * pos + 1;
            done |= c0 >= size;
            const uint32_t i0 = c0 < last ? c0 : last;
            const uint64_t x0 = get(i0);
            const uint64_t x1 = get(c0 + 1 < last ? c0 + 1 : last);
            const uint64_t x2 = get(c0 + 2 < last ? c0 + 2 : last);
            const uint64_t x3 = get(c0 + 3 < last ? c0 + 3 : last);
            uint64_t best = x0;
            uint32_t bi = c0;
            if (x1 < best) { best = x1; bi = c0 + 1; }
            if (x2 < best) { best = x2; bi = c0 + 2; }
            if (x3 < best) { best = x3; bi = c0 + 3; }
            const bool mv = !done && v > best;
            if (mv) {
                put(pos, best);
                if (lvl == 0) top = best;
                pos = bi;
            }
            done |= !mv;
        }
        put(pos, v);
        return top;
    }
    C2_DEV void heapify(uint32_t size) {
        if (size < 2) return;
        for (int i = (int)(size - 2) / 4; i >= 0; --i) sift_down((uint32_t)i, get(i), size);
    }
    C2_DEV bool full() const { return cnt >= k; }
    // Until the heap holds k entries, entries are appended and then heapified
    // once; afterwards v replaces the root (the caller checked it beats it).
    C2_DEV void insert(uint64_t v) {
        if (cnt < k) {
            put(cnt++, v);
            if (cnt == k) {
                heapify(k);
                root = get(0);
            }
        } else {
            root = sift_down(0, v, k);
        }
    }
};

// Necessary condition for a candidate to beat the root, in fp32 with a margin
// that covers rounding: J > J_T implies I > sigma_T * (|P_u| + |P_v|).
C2_DEV bool may_beat(uint32_t I, uint32_t S, float sigma) {
    return (float)I >= sigma * (float)S * 0.999999f;
}

// floor(2^16 * I / S) for 0 <= I <= S/2, clamped to 15 bits (0 when S = 0).
// The fp32 estimate is within a relative 2^-22 of I/S.
C2_DEV uint32_t ratio_code(uint32_t I, uint32_t S) {
    const float f = (float)I * __builtin_amdgcn_rcpf((float)(S ? S : 1u)) * 65536.0f;
    const uint32_t c = (uint32_t)f;
    return c < 0x7FFFu ? c : 0x7FFFu;
}

// How many of the 64 codes packed two per word (15 bits each) are >= M, for
// M <= 0x7FFF: per half, bit 15 of (code | 0x8000) - M is set iff code >= M.
C2_DEV uint32_t codes_at_least(const uint32_t (&pk)[32], uint32_t M) {
    const uint32_t MM = M * 0x10001u;
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < 32; ++j) c += __popc(((pk[j] | 0x80008000u) - MM) & 0x80008000u);
    return c;
}

// Work item of the MFMA path: cluster c, row block rb, column group g of ng.
// A row block whose cluster spans more than kGroupTiles column tiles is split
// into ng <= kMaxGroups items over disjoint column ranges; each leaves its
// rows' k best (sorted keys) in scratch, and the item that finishes last
// merges them.  No item waits for another.
C2_DEV uint64_t mfma_item_code(uint32_t c, uint32_t rb, uint32_t g, uint32_t ng) {
    return ((uint64_t)c << 32) | ((uint64_t)rb << 8) | (g << 4) | (ng - 1);
}

struct MfmaScratch {
    uint64_t *keys;       // [slot][kMR][kMaxK]
    uint32_t *rb_done;    // per (cluster, row block) of a split row block
    const uint32_t *sbase;  // first slot of each cluster
    const uint32_t *cbits;  // compacted rows (nullptr: compaction off)
    const uint32_t *cw;     // words per compacted row of each cluster, 0 = full rows
    const uint64_t *coff;   // first word of each compacted cluster
};

C2_DEV void mfma_item(const KnnArgs &a, const uint32_t *ubits, const uint32_t *ulen,
                      const MfmaScratch &sc, uint64_t code, MfmaLds &L) {
    const uint32_t c = (uint32_t)(code >> 32), rb = (uint32_t)code >> 8;
    const uint32_t g = ((uint32_t)code >> 4) & 15u, ng = ((uint32_t)code & 15u) + 1;
    const uint32_t t = threadIdx.x, lane = t & 63, w = t >> 6;
    const uint32_t wr = w >> 1, wc = w & 1;
    const ClusterView cv = view(a, c);
    const uint32_t Wc = sc.cw ? sc.cw[c] : 0u;  // compacted row width, 0 = full rows
    const uint32_t s = cv.s, W = a.wmax, nchunks = (Wc ? Wc : W) / 2;
    const uint32_t *cbase = Wc ? sc.cbits + sc.coff[c] : nullptr;
    // selection: row r of the block belongs to the thread pair (2r, 2r + 1);
    // both filter half of each tile, the even thread keeps the heap
    const uint32_t r = t >> 1, half = t & 1;
    const uint32_t ra = rb * kMR + r;
    const uint32_t ur = member(a, cv, ra);
    const bool active = ur < a.n;
    const bool owner = active && half == 0;
    const uint32_t Lr = active ? ulen[ur] : 0;
    // staging: thread t < 128 expands row t of the block, t >= 128 column t - 128
    const uint32_t us_row = t < kMR ? member(a, cv, rb * kMR + t) : a.n;
    KeyHeap h;
    h.hk = L.hk;
    h.me = r;
    h.k = a.k;
    h.cnt = 0;
    h.root = 0;
    const uint32_t tiles = (s + kMC - 1) / kMC, per = (tiles + ng - 1) / ng;
    const uint32_t cb_end = (g + 1) * per < tiles ? (g + 1) * per : tiles;
    for (uint32_t cb = g * per; cb < cb_end; ++cb) {
        // staged row of this thread: owner row t, or column t - 128
        const uint32_t us = t < kMR ? us_row : member(a, cv, cb * kMC + (t - kMR));
        // the member's row over the cluster's dictionary, or its full row (the
        // all-zero row n for padding, which is at least as long as any row)
        const uint32_t pos = t < kMR ? rb * kMR + t : cb * kMC + (t - kMR);
        const uint64_t *src = reinterpret_cast<const uint64_t *>(
            cbase && pos < s ? cbase + (size_t)pos * Wc : ubits + (size_t)us * W);
        if (t >= kMR) {
            L.cuid[t - kMR] = us;
            L.clen[t - kMR] = us < a.n ? ulen[us] : 0;
        }
        v16f acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};
        // Staging: thread t stages its row's bits for two chunks at a time,
        // word half h of both chunks in raw[.][h][t], so that the 32 lanes of
        // a wave that read half h read 256 contiguous bytes.  Each wave reads
        // the words of its 64 A rows and 64 B rows and expands them to fp4
        // nibbles in registers right before the MFMAs: LDS carries 16 bytes
        // per row and pair of chunks instead of 64 bytes of nibbles per row
        // and chunk.  Pair p + 1 waits in pf[(p + 1) % 2], loaded two pairs
        // ahead; the loop is unrolled by 2 so the slot index is a constant.
        const uint4 *src4 = reinterpret_cast<const uint4 *>(src);
        const uint32_t npairs = nchunks / 2;  // even: rows are padded to 4 chunks
        uint4 pf[2];
        pf[1] = load_pair(src4, 1, npairs);
        {
            const uint4 x = load_pair(src4, 0, npairs);
            L.u.raw[0][0][t] = make_uint2(x.x, x.z);
            L.u.raw[0][1][t] = make_uint2(x.y, x.w);
        }
        pf[0] = load_pair(src4, 2, npairs);
        const uint32_t hh = lane >> 5, rr = lane & 31;
        for (uint32_t p0 = 0; p0 < npairs; p0 += 2) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const uint32_t pp = p0 + u;
                lds_barrier();
                const int st = u;
                const uint2 a0 = L.u.raw[st][hh][wr * 64 + rr];
                const uint2 a1 = L.u.raw[st][hh][wr * 64 + 32 + rr];
                const uint2 b0 = L.u.raw[st][hh][kMR + wc * 64 + rr];
                const uint2 b1 = L.u.raw[st][hh][kMR + wc * 64 + 32 + rr];
                {  // chunk 2pp
                    const v4i A0 = as_v4i(nibbles32(a0.x)), A1 = as_v4i(nibbles32(a1.x));
                    const v4i B0 = as_v4i(nibbles32(b0.x)), B1 = as_v4i(nibbles32(b1.x));
                    acc00 = mfma_fp4(A0, B0, acc00);
                    acc01 = mfma_fp4(A0, B1, acc01);
                    acc10 = mfma_fp4(A1, B0, acc10);
                    acc11 = mfma_fp4(A1, B1, acc11);
                }
                {  // chunk 2pp + 1
                    const v4i A0 = as_v4i(nibbles32(a0.y)), A1 = as_v4i(nibbles32(a1.y));
                    const v4i B0 = as_v4i(nibbles32(b0.y)), B1 = as_v4i(nibbles32(b1.y));
                    acc00 = mfma_fp4(A0, B0, acc00);
                    acc01 = mfma_fp4(A0, B1, acc01);
                    acc10 = mfma_fp4(A1, B0, acc10);
                    acc11 = mfma_fp4(A1, B1, acc11);
                }
                const int nx = (u + 1) & 1;
                L.u.raw[st ^ 1][0][t] = make_uint2(pf[nx].x, pf[nx].z);
                L.u.raw[st ^ 1][1][t] = make_uint2(pf[nx].y, pf[nx].w);
                pf[nx] = load_pair(src4, pp + 3, npairs);
            }
        }
        __syncthreads();
        // transpose through LDS: C[i][j] of a 32x32 block sits in lane j (+32),
        // register r at row 8*(r/4) + 4*(lane/32) + r%4
        {
            const uint32_t j0 = wc * 64 + (lane & 31), i0 = wr * 64 + 4 * (lane >> 5);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t i = i0 + 8 * (r >> 2) + (r & 3);
                L.u.itile[i][j0] = (uint16_t)(uint32_t)acc00[r];
                L.u.itile[i][j0 + 32] = (uint16_t)(uint32_t)acc01[r];
                L.u.itile[i + 32][j0] = (uint16_t)(uint32_t)acc10[r];
                L.u.itile[i + 32][j0 + 32] = (uint16_t)(uint32_t)acc11[r];
            }
        }
        __syncthreads();
        {
            const uint32_t ncol = s - cb * kMC < kMC ? s - cb * kMC : kMC;
            const uint32_t self = ra - cb * kMC;  // column index of the row's own member
            // the owner's heap state, shared with its helper lane (the root's
            // key word is all the filter needs)
            const uint32_t rhi = __shfl((uint32_t)(h.root >> 32), lane & ~1u);
            const bool full = __shfl((int)h.full(), lane & ~1u) != 0;
            // sigma = key_T / (2^32 - 1 + key_T): I >= sigma * (|P_u| + |P_v|) is necessary
            const float kt = (float)rhi;
            const float sigma = kt / (4294967295.0f + kt);
            // candidates half*64 .. half*64 + 63 that may beat the root (the
            // exact test is made again at insertion, against the root then)
            uint32_t m0 = 0u, m1 = 0u;
            const uint32_t q0 = half * 64;
#pragma unroll 1
            for (uint32_t q8 = 0; q8 < 64; q8 += 8) {
                const uint4 raw = *reinterpret_cast<const uint4 *>(&L.u.itile[r][q0 + q8]);
                const uint4 l0 = *reinterpret_cast<const uint4 *>(&L.clen[q0 + q8]);
                const uint4 l1 = *reinterpret_cast<const uint4 *>(&L.clen[q0 + q8 + 4]);
                const uint32_t pr[4] = {raw.x, raw.y, raw.z, raw.w};
                const uint32_t cl[8] = {l0.x, l0.y, l0.z, l0.w, l1.x, l1.y, l1.z, l1.w};
                uint32_t bits = 0;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint32_t q = q0 + q8 + e;
                    const uint32_t I = (pr[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
                    const bool ok = active & (q < ncol) & (q != self) &
                                    (!full | may_beat(I, Lr + cl[e], sigma));
                    bits |= (ok ? 1u : 0u) << e;
                }
                if (q8 < 32) m0 |= bits << q8;
                else m1 |= bits << (q8 - 32);
            }
            // When many candidates of a row pass (always in the first tile of
            // an item, where the heap is not yet full), drop those that are not
            // among the tile's own k best: a candidate with k better ones in
            // the same tile cannot be among the row's k best.  Each candidate
            // gets a 15-bit code of its I/S (floor(2^16 * I/S) in fp32, two
            // codes per word, 0 for columns that are not candidates), and
            // bisection finds a level L with at least k codes >= L.  A candidate
            // is dropped only when its code is below L - 1, a margin larger
            // than the rounding of the fp32 ratios, so those k candidates are
            // strictly better in exact arithmetic.
            const uint32_t npass = __popc(m0) + __popc(m1);
            const uint32_t npair = npass + __shfl_xor(npass, 1);
            if (__any(npair > a.k + kBisectSlack)) {
                uint32_t pk[32];
#pragma unroll
                for (int q2 = 0; q2 < 64; q2 += 2) {
                    const uint32_t q = q0 + q2;
                    const uint32_t I2 = *reinterpret_cast<const uint32_t *>(&L.u.itile[r][q]);
                    const uint2 l2 = *reinterpret_cast<const uint2 *>(&L.clen[q]);
                    const uint32_t c0 = active && q < ncol && q != self
                                            ? ratio_code(I2 & 0xFFFFu, Lr + l2.x) : 0u;
                    const uint32_t c1 = active && q + 1 < ncol && q + 1 != self
                                            ? ratio_code(I2 >> 16, Lr + l2.y) : 0u;
                    pk[q2 >> 1] = c0 | (c1 << 16);
                }
                uint32_t hi = 0;
#pragma unroll
                for (int j = 0; j < 32; ++j) hi = max(hi, max(pk[j] & 0xFFFFu, pk[j] >> 16));
                hi = max(hi, (uint32_t)__shfl_xor(hi, 1)) + 1;  // no code reaches hi
                uint32_t lo = 0;  // invariant: at least k codes >= lo
#pragma unroll 1
                for (int it = 0; it < kBisectSteps; ++it) {
                    const uint32_t mid = (lo + hi) >> 1;
                    const uint32_t c = codes_at_least(pk, mid);
                    if (c + __shfl_xor(c, 1) >= a.k) lo = mid;
                    else hi = mid;
                }
                if (npair > a.k + kBisectSlack && lo >= 2) {
                    const uint32_t M = (lo - 1) * 0x10001u;
                    uint32_t k0 = 0, k1 = 0;  // candidates whose code is >= lo - 1
#pragma unroll
                    for (int j = 0; j < 32; ++j) {
                        const uint32_t ge = ((pk[j] | 0x80008000u) - M) & 0x80008000u;
                        const uint32_t two = ((ge >> 15) & 1u) | ((ge >> 30) & 2u);
                        if (j < 16) k0 |= two << (2 * j);
                        else k1 |= two << (2 * (j - 16));
                    }
                    m0 &= k0;
                    m1 &= k1;
                }
            }
            // While a row's heap holds fewer than k entries, both threads of the
            // pair append passing candidates in parallel (the owner's first,
            // then its helper's, up to k in all); the owner heapifies once the
            // heap is full.  Candidates beyond k go through the insert loop.
            const uint32_t cnt0 = __shfl(h.cnt, lane & ~1u);
            if (__any(active && cnt0 < a.k)) {
                const uint32_t pmine = __popc(m0) + __popc(m1);
                const uint32_t pown = __shfl(pmine, lane & ~1u);
                const uint32_t room = active && cnt0 < a.k ? a.k - cnt0 : 0u;
                const uint32_t aown = pown < room ? pown : room;
                const uint32_t quota = half == 0 ? aown
                                                 : (pmine < room - aown ? pmine : room - aown);
                uint32_t slot = cnt0 + (half == 0 ? 0u : aown);
                for (uint32_t i = 0; i < quota; ++i) {
                    const bool lo = m0 != 0u;
                    const uint32_t bit = __ffs(lo ? m0 : m1) - 1;
                    if (lo) m0 &= m0 - 1;
                    else m1 &= m1 - 1;
                    const uint32_t q = q0 + (lo ? 0u : 32u) + bit;
                    const uint32_t I = L.u.itile[r][q];
                    const uint32_t U = Lr + L.clen[q] - I, uid = L.cuid[q];
                    h.put(slot++, ((uint64_t)jkey(I, U) << 32) | (0xFFFFFFFFu - uid));
                }
                const uint32_t ahelp = __shfl(quota, lane | 1u);
                if (owner && cnt0 < a.k) {
                    h.cnt = cnt0 + aown + ahelp;
                    if (h.cnt == a.k) {
                        h.heapify(a.k);
                        h.root = h.get(0);
                    }
                }
            }
            // the owner takes its helper's masks (adjacent lane)
            const uint32_t o0 = __shfl(m0, lane | 1u), o1 = __shfl(m1, lane | 1u);
            uint32_t msk[4] = {m0, m1, o0, o1};
            if (!owner) msk[0] = msk[1] = msk[2] = msk[3] = 0u;
            // wave-uniform loop: each owner inserts its next passing candidate
            while (__any((msk[0] | msk[1] | msk[2] | msk[3]) != 0u)) {
                const int wsel = msk[0] ? 0 : msk[1] ? 1 : msk[2] ? 2 : msk[3] ? 3 : -1;
                if (wsel >= 0) {
                    const uint32_t bit = __ffs(msk[wsel]) - 1;
                    msk[wsel] &= msk[wsel] - 1;
                    const uint32_t q = wsel * 32 + bit;
                    const uint32_t I = L.u.itile[r][q];
                    const uint32_t U = Lr + L.clen[q] - I, uid = L.cuid[q];
                    // keys are exact and distinct (the id is in the low word),
                    // so beating the root is one comparison
                    const uint64_t v = ((uint64_t)jkey(I, U) << 32) | (0xFFFFFFFFu - uid);
                    if (!h.full() || v > h.root) h.insert(v);
                }
            }
        }
        __syncthreads();
    }
    // The row's entries, best first, by rank: both threads of the pair take
    // every second slot of the heap (16 at most each) and count the entries
    // with a larger key (keys are distinct), which is each entry's position.
    const uint32_t cnt = __shfl(h.cnt, lane & ~1u);
    uint64_t mine[kMaxK / 2];
    uint32_t rk[kMaxK / 2];
#pragma unroll
    for (uint32_t i = 0; i < kMaxK / 2; ++i) {
        const uint32_t j = 2 * i + half;
        mine[i] = active && j < cnt ? h.get(j) : 0ull;
        rk[i] = 0;
    }
    for (uint32_t j = 0; j < kMaxK; ++j) {
        const uint64_t x = j < cnt ? h.get(j) : 0ull;
#pragma unroll
        for (uint32_t i = 0; i < kMaxK / 2; ++i) rk[i] += x > mine[i] ? 1u : 0u;
    }
    if (ng == 1) {
        if (active && cv.j < a.t) {
            const size_t base = ((size_t)ur * a.t + cv.j) * a.k;
            uint32_t *oid = a.part_id + base, *oI = a.part_I + base;
#pragma unroll
            for (uint32_t i = 0; i < kMaxK / 2; ++i)
                if (2 * i + half < cnt) {
                    const uint32_t uid = 0xFFFFFFFFu - (uint32_t)mine[i];
                    oid[rk[i]] = uid;
                    oI[rk[i]] = key_to_I((uint32_t)(mine[i] >> 32), Lr + ulen[uid]);
                }
            for (uint32_t q = cnt + half; q < a.k; q += 2) {
                oid[q] = kPad;
                oI[q] = 0;
            }
        }
        return;
    }
    // split row block: leave this group's sorted keys (0 = none) in scratch
    const uint32_t slot0 = sc.sbase[c] + rb * ng;
    if (active) {
        uint64_t *out = sc.keys + ((size_t)(slot0 + g) * kMR + r) * kMaxK;
#pragma unroll
        for (uint32_t i = 0; i < kMaxK / 2; ++i)
            if (2 * i + half < cnt) out[rk[i]] = mine[i];
        for (uint32_t q = cnt + half; q < a.k; q += 2) out[q] = 0;
    }
    __threadfence();
    __syncthreads();
    __shared__ uint32_t last;
    if (t == 0) last = atomicAdd(&sc.rb_done[slot0], 1u) == ng - 1;
    __syncthreads();
    if (!last || !owner || cv.j >= a.t) return;
    __threadfence();
    // the last group merges the ng sorted lists of each row (disjoint columns)
    const uint64_t *in = sc.keys + ((size_t)slot0 * kMR + r) * kMaxK;
    uint32_t ptr[kMaxGroups];
    uint64_t head[kMaxGroups];
#pragma unroll
    for (uint32_t q = 0; q < kMaxGroups; ++q) {
        ptr[q] = 0;
        head[q] = q < ng ? in[(size_t)q * kMR * kMaxK] : 0;
    }
    const size_t base = ((size_t)ur * a.t + cv.j) * a.k;
    for (uint32_t r = 0; r < a.k; ++r) {
        uint32_t best = 0;
#pragma unroll
        for (uint32_t q = 1; q < kMaxGroups; ++q)
            if (head[q] > head[best]) best = q;
        uint64_t v = 0;
#pragma unroll
        for (uint32_t q = 0; q < kMaxGroups; ++q)
            if (q == best) {
                v = head[q];
                ++ptr[q];
                head[q] = (v != 0 && ptr[q] < a.k) ? in[(size_t)q * kMR * kMaxK + ptr[q]] : 0;
            }
        if (v == 0) {
            a.part_id[base + r] = kPad;
            a.part_I[base + r] = 0;
        } else {
            const uint32_t uid = 0xFFFFFFFFu - (uint32_t)v;
            a.part_id[base + r] = uid;
            a.part_I[base + r] = key_to_I((uint32_t)(v >> 32), Lr + ulen[uid]);
        }
    }
}

__global__ __launch_bounds__(256, 2) void k_knn_mfma(KnnArgs a, const uint32_t *ubits,
                                                     const uint32_t *ulen, MfmaScratch sc,
                                                     const uint64_t *items,
                                                     const uint32_t *n_items, uint32_t *cursor) {
    __shared__ MfmaLds L;
    __shared__ uint32_t next;
    const uint32_t total = *n_items;
    if (!cursor) {
        if (blockIdx.x >= total) return;
        mfma_item(a, ubits, ulen, sc, items[blockIdx.x], L);
        return;
    }
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) next = atomicAdd(cursor, 1u);
        __syncthreads();
        const uint32_t i = next;
        if (i >= total) break;
        mfma_item(a, ubits, ulen, sc, items[i], L);
    }
}

// ------------------------------------------------------- cluster dictionaries
//
// Only items held by at least two members of a cluster can be in an
// intersection, so a cluster's pairwise counts need only those items (its
// local dictionary).  For each cluster of 2..kCompactMaxS members one block
// works from the members' CSR lists (a few hundred bytes per member, where
// the bit rows are W words):
//   1. every item sets its bit in `once` with a returning atomicOr, and in
//      `twice` when the bit was already set (LDS);
//   2. an exclusive prefix of popcounts of `twice` numbers the dictionary
//      items in item order (stored over `once`);
//   3. when the dictionary, padded to 256 items, is at most three quarters of
//      the row and fits the rest of the store, each wave sets the local bits
//      of one member at a time in an LDS row buffer and writes the row to
//      cbits; cw[c] then holds the compacted width, else 0.
// The dot products over the compacted rows equal those over the full rows.
// Clusters come from the MFMA work list, each at its first item (row block 0,
// group 0): in the batched form the list is costliest first, so the largest
// clusters start first and do not trail at the end of the pass.
template <int NT>
__global__ __launch_bounds__(NT) void k_compact(KnnArgs a, const uint64_t *__restrict__ items,
                                                const uint32_t *n_items,
                                                uint32_t *__restrict__ cbits,
                                                uint64_t cap, uint32_t *__restrict__ cw,
                                                uint64_t *__restrict__ coff,
                                                unsigned long long *ccur, uint32_t *cnext) {
    constexpr uint32_t NWV = NT / 64, G = 16, NG = NT / G;
    extern __shared__ uint32_t lds[];
    const uint32_t W = a.wmax, RB = 3 * W / 4;  // a compacted row has at most RB words
    uint32_t *once = lds, *twice = lds + W, *pre = lds;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    uint32_t *rowb = lds + 2 * W + wid * RB;
    __shared__ uint32_t wsum[NT / 64 + 1];
    __shared__ unsigned long long sh_off;
    __shared__ uint32_t sh_ok, sh_c;
    const uint32_t total_items = *n_items;
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            const uint32_t i = atomicAdd(cnext, 1u);
            // cluster of the item, or ~0 past the end; 0xFFFFFFFE: not a first item
            sh_c = i >= total_items ? 0xFFFFFFFFu
                   : ((uint32_t)items[i] >> 4) == 0 ? (uint32_t)(items[i] >> 32) : 0xFFFFFFFEu;
        }
        __syncthreads();
        const uint32_t c = sh_c;
        if (c == 0xFFFFFFFFu) break;
        if (c == 0xFFFFFFFEu) continue;
        const ClusterView cv = view(a, c);
        const uint32_t s = cv.s;
        if (s < 2 || s > kCompactMaxS) {
            if (tid == 0) cw[c] = 0;
            continue;
        }
        for (uint32_t w = tid; w < 2 * W; w += NT) lds[w] = 0;
        __syncthreads();
        // 1. dictionary: 16 lanes per member, 4 items per lane in flight; the
        //    next member's row range and the id after it are loaded while the
        //    current member's items are folded in
        {
            const uint32_t sub = tid & (G - 1), r0 = tid / G;
            uint64_t na = 0, ne = 0;
            uint32_t nu = r0 < s ? a.members[cv.o + r0] : a.n;
            if (nu < a.n) row_range(a.indptr, nu, a.nnz, na, ne);
            nu = r0 + NG < s ? a.members[cv.o + r0 + NG] : a.n;
            for (uint32_t r = r0; r < s; r += NG) {
                const uint64_t p0 = na, p1 = ne;
                na = ne = 0;
                if (nu < a.n) row_range(a.indptr, nu, a.nnz, na, ne);
                nu = r + 2 * NG < s ? a.members[cv.o + r + 2 * NG] : a.n;
                for (uint64_t p = p0 + sub; p < p1; p += 4 * G) {
                    uint32_t it[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        it[q] = p + q * G < p1 ? a.indices[p + q * G] : 0xFFFFFFFFu;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (it[q] >= a.m) continue;
                        const uint32_t bit = 1u << (it[q] & 31);
                        if (atomicOr(&once[it[q] >> 5], bit) & bit) atomicOr(&twice[it[q] >> 5], bit);
                    }
                }
            }
        }
        __syncthreads();
        // 2. local index of each word's first dictionary item
        const uint32_t per = (W + NT - 1) / NT, w0 = tid * per;
        uint32_t mine = 0;
        for (uint32_t w = w0; w < w0 + per && w < W; ++w) mine += __popc(twice[w]);
        uint32_t total;
        uint32_t run = block_excl_scan<uint32_t, NT>(mine, wsum, &total);
        for (uint32_t w = w0; w < w0 + per && w < W; ++w) {
            const uint32_t c2 = __popc(twice[w]);
            pre[w] = run;  // over `once`, which is no longer read
            run += c2;
        }
        const uint32_t wc = ((total ? total : 1u) + 255u) / 256u * 8u;  // words, a multiple of 8
        if (tid == 0) {
            sh_ok = 0;
            if (4 * wc <= 3 * W) {
                const unsigned long long need = (unsigned long long)s * wc;
                const unsigned long long off = atomicAdd(ccur, need);
                if (off + need <= cap) {
                    sh_ok = 1;
                    sh_off = off;
                }
            }
            cw[c] = sh_ok ? wc : 0u;
            if (sh_ok) coff[c] = sh_off;
        }
        __syncthreads();
        if (!sh_ok) continue;
        // 3. compacted rows, one member per wave at a time, with the next
        //    member's row range and the id after it in flight as in step 1
        uint64_t na = 0, ne = 0;
        uint32_t nu = wid < s ? a.members[cv.o + wid] : a.n;
        if (nu < a.n) row_range(a.indptr, nu, a.nnz, na, ne);
        nu = wid + NWV < s ? a.members[cv.o + wid + NWV] : a.n;
        for (uint32_t r = wid; r < s; r += NWV) {
            const uint64_t p0 = na, p1 = ne;
            na = ne = 0;
            if (nu < a.n) row_range(a.indptr, nu, a.nnz, na, ne);
            nu = r + 2 * NWV < s ? a.members[cv.o + r + 2 * NWV] : a.n;
            for (uint32_t o2 = lane; o2 < wc; o2 += 64) rowb[o2] = 0;
            wave_sync();
            for (uint64_t p = p0 + lane; p < p1; p += 2 * 64) {
                uint32_t it[2];
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    it[q] = p + q * 64 < p1 ? a.indices[p + q * 64] : 0xFFFFFFFFu;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    if (it[q] >= a.m) continue;
                    const uint32_t w = it[q] >> 5, b = it[q] & 31, d = twice[w];
                    if ((d >> b) & 1u) {
                        const uint32_t li = pre[w] + __popc(d & ((1u << b) - 1u));
                        atomicOr(&rowb[li >> 5], 1u << (li & 31));
                    }
                }
            }
            wave_sync();
            uint32_t *dst = cbits + sh_off + (size_t)r * wc;
            for (uint32_t o2 = lane; o2 < wc; o2 += 64) dst[o2] = rowb[o2];
            wave_sync();
        }
    }
}

// ---------------------------------------------------------------- planning

// Column groups of an MFMA cluster of s members.
C2_DEV uint32_t mfma_groups(uint32_t s, uint32_t group_tiles) {
    const uint32_t tiles = (s + kMC - 1) / kMC;
    if (tiles <= group_tiles) return 1;
    const uint32_t ng = (tiles + group_tiles - 1) / group_tiles;
    return ng < kMaxGroups ? ng : kMaxGroups;
}

// Per cluster (in `order`, or index order): number of MFMA items (low word)
// and bitmap items (high word), and the scratch slots of split row blocks;
// clusters of one member get padded lists here.
__global__ __launch_bounds__(256) void k_plan_count(KnnArgs a, const uint32_t *order,
                                                    uint32_t mfma_min, uint32_t group_tiles,
                                                    const uint32_t *bmax, uint32_t nbmax,
                                                    uint64_t *cnt, uint32_t *slots) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ncl = a.cl_cfg_off[a.t];
    if (block_max_len(bmax, nbmax) >= kMfmaMaxLen) mfma_min = 0xFFFFFFFFu;
    if (q >= a.NE) return;
    if (q >= ncl) { cnt[q] = 0; slots[q] = 0; return; }
    const uint32_t c = order ? order[q] : q;
    const ClusterView cv = view(a, c);
    uint64_t v = 0;
    uint32_t sl = 0;
    if (cv.s >= mfma_min && cv.s >= 2) {
        const uint32_t ng = mfma_groups(cv.s, group_tiles);
        v = (uint64_t)((cv.s + kMR - 1) / kMR) * ng;
        sl = ng > 1 ? (uint32_t)v : 0;
    } else if (cv.s >= 2) {
        v = (uint64_t)((cv.s + kRowBlock - 1) / kRowBlock) << 32;
    } else if (cv.s == 1) {
        const uint32_t u = member(a, cv, 0);
        if (u < a.n && cv.j < a.t) {
            const size_t base = ((size_t)u * a.t + cv.j) * a.k;
            for (uint32_t r = 0; r < a.k; ++r) {
                a.part_id[base + r] = kPad;
                a.part_I[base + r] = 0;
            }
        }
    }
    cnt[q] = v;
    slots[q] = sl;
}

__global__ __launch_bounds__(256) void k_plan_fill(KnnArgs a, const uint32_t *order,
                                                   uint32_t group_tiles, const uint64_t *off,
                                                   const uint32_t *slot_off,
                                                   uint64_t *items_m, uint64_t *items_b,
                                                   uint32_t *sbase, uint32_t *rb_done,
                                                   uint32_t *nitems, uint32_t *cursors) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) {
        const uint64_t tot = off[a.NE];
        nitems[0] = (uint32_t)tot;
        nitems[1] = (uint32_t)(tot >> 32);
        if (cursors) { cursors[0] = 0; cursors[1] = 0; }
    }
    if (q >= a.NE || q >= a.cl_cfg_off[a.t]) return;
    const uint32_t c = order ? order[q] : q;
    const uint64_t o0 = off[q], o1 = off[q + 1];
    const uint32_t bm = (uint32_t)o0, nm = (uint32_t)o1 - bm;
    const uint32_t bb = (uint32_t)(o0 >> 32), nbm = (uint32_t)(o1 >> 32) - bb;
    if (nm) {
        const uint32_t s = a.cl_off[c + 1] - a.cl_off[c];
        const uint32_t ng = mfma_groups(s, group_tiles), nrb = nm / ng;
        sbase[c] = slot_off[q];
        for (uint32_t r = 0; r < nrb; ++r) {
            for (uint32_t g = 0; g < ng; ++g) items_m[bm + r * ng + g] = mfma_item_code(c, r, g, ng);
            if (ng > 1) rb_done[slot_off[q] + r * ng] = 0;
        }
    }
    for (uint32_t r = 0; r < nbm; ++r) items_b[bb + r] = ((uint64_t)c << 32) | r;
}

// Batched planning without a sort.  The work items of the MFMA path fall into
// cost classes by the number of column tiles an item covers (more tiles =
// lower class index = taken first: the size-ordered queue of Section II-F).
// Each cluster takes a contiguous range inside its class by an atomic on the
// class counter, and scratch slots (split row blocks) and bitmap items by
// atomics on their counters; k_user_bits cleared the counters.  The order of
// clusters inside a class changes only the schedule, never a result.
// Positions inside each class come from per-block counts in LDS, then one
// global atomic per (block, counter): with one global atomic per cluster,
// thousands of clusters of one class serialise on one address.  The order
// of items inside a class is arbitrary either way.
__global__ __launch_bounds__(256) void k_plan_classes(KnnArgs a, uint32_t mfma_min,
                                                      uint32_t group_tiles,
                                                      const uint32_t *bmax, uint32_t nbmax,
                                                      uint32_t *pc, uint32_t *ccls,
                                                      uint32_t *cpos, uint32_t *sbase) {
    __shared__ uint32_t lcnt[kPlanCtr], lbase[kPlanCtr];
    for (uint32_t q = threadIdx.x; q < kPlanCtr; q += blockDim.x) lcnt[q] = 0;
    // (block_max_len begins with a barrier, which also orders the zeroing)
    if (block_max_len(bmax, nbmax) >= kMfmaMaxLen) mfma_min = 0xFFFFFFFFu;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = c < a.NE && c < a.cl_cfg_off[a.t];
    uint32_t cls = 0xFFFFFFFFu, ctr = 0, lpos = 0, lslot = 0;
    bool split = false;
    if (live) {
        const ClusterView cv = view(a, c);
        if (cv.s >= mfma_min && cv.s >= 2) {
            const uint32_t ng = mfma_groups(cv.s, group_tiles);
            const uint32_t tiles = (cv.s + kMC - 1) / kMC, per = (tiles + ng - 1) / ng;
            const uint32_t nit = ((cv.s + kMR - 1) / kMR) * ng;
            cls = kCostClasses - 1 - (per < kCostClasses - 1 ? per : kCostClasses - 1);
            ctr = cls;
            lpos = atomicAdd(&lcnt[cls], nit);
            split = ng > 1;
            if (split) lslot = atomicAdd(&lcnt[kSlotCtr], nit);
        } else if (cv.s >= 2) {
            cls = kCostClasses;
            ctr = kBitmapCtr;
            lpos = atomicAdd(&lcnt[kBitmapCtr], (cv.s + kRowBlock - 1) / kRowBlock);
        } else if (cv.s == 1) {
            const uint32_t u = member(a, cv, 0);
            if (u < a.n && cv.j < a.t) {
                const size_t base = ((size_t)u * a.t + cv.j) * a.k;
                for (uint32_t r = 0; r < a.k; ++r) {
                    a.part_id[base + r] = kPad;
                    a.part_I[base + r] = 0;
                }
            }
        }
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < kPlanCtr; q += blockDim.x)
        lbase[q] = lcnt[q] ? atomicAdd(&pc[q], lcnt[q]) : 0u;
    __syncthreads();
    if (!live) return;
    if (split) sbase[c] = lbase[kSlotCtr] + lslot;
    ccls[c] = cls;
    cpos[c] = cls == 0xFFFFFFFFu ? 0u : lbase[ctr] + lpos;
}

__global__ __launch_bounds__(256) void k_plan_items(KnnArgs a, uint32_t group_tiles,
                                                    const uint32_t *pc, const uint32_t *ccls,
                                                    const uint32_t *cpos, const uint32_t *sbase,
                                                    uint64_t *items_m, uint64_t *items_b,
                                                    uint32_t *rb_done, uint32_t *nitems,
                                                    uint32_t *cursors) {
    __shared__ uint32_t cbase[kCostClasses + 1];
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t q = 0; q < kCostClasses; ++q) {
            cbase[q] = run;
            run += pc[q];
        }
        cbase[kCostClasses] = run;
    }
    __syncthreads();
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c == 0) {
        nitems[0] = cbase[kCostClasses];
        nitems[1] = pc[kBitmapCtr];
        cursors[0] = 0;
        cursors[1] = 0;
    }
    if (c >= a.NE || c >= a.cl_cfg_off[a.t]) return;
    const uint32_t cls = ccls[c];
    if (cls < kCostClasses) {
        const uint32_t s = a.cl_off[c + 1] - a.cl_off[c];
        const uint32_t ng = mfma_groups(s, group_tiles), nrb = (s + kMR - 1) / kMR;
        const uint32_t b0 = cbase[cls] + cpos[c];
        for (uint32_t r = 0; r < nrb; ++r) {
            for (uint32_t g = 0; g < ng; ++g) items_m[b0 + r * ng + g] = mfma_item_code(c, r, g, ng);
            if (ng > 1) rb_done[sbase[c] + r * ng] = 0;
        }
    } else if (cls == kCostClasses) {
        const uint32_t s = a.cl_off[c + 1] - a.cl_off[c];
        const uint32_t nrb = (s + kRowBlock - 1) / kRowBlock;
        for (uint32_t r = 0; r < nrb; ++r) items_b[cpos[c] + r] = ((uint64_t)c << 32) | r;
    }
}

// --------------------------------------------------------------- host side

// Scratch slots of split row blocks: a cluster is split only when it spans
// more than one column tile (s > 128), and then takes
// ceil(s/128) * ng <= (s/128 + 1) * 4 < s/16 slots.
size_t knn_max_slots(uint32_t NE) { return (size_t)NE / 16 + 8; }

size_t knn_ws_bytes(uint32_t n, uint32_t NE, uint32_t wmax, KnnWs *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    KnnWs x;
    x.rows = take((size_t)4 * ((size_t)n + 1) * wmax);
    x.rlen = take(4 * ((size_t)n + 1));
    x.cnt = take(8 * ((size_t)NE + 1));
    x.items_m = take(8 * ((size_t)NE + NE / 16 + 64));
    x.slots = take(4 * ((size_t)NE + 1));
    x.sbase = take(4 * (size_t)NE);
    const size_t nslot = knn_max_slots(NE);
    x.rb_done = take(4 * nslot);
    x.skeys = take(8 * nslot * kMR * kMaxK);
    x.items_b = take(8 * (size_t)NE);
    x.csort_key = take(8 * (size_t)NE);
    x.csort_key_alt = take(8 * (size_t)NE);
    x.csort_val = take(4 * (size_t)NE);
    x.csort_val_alt = take(4 * (size_t)NE);
    const size_t hist = radix_hist_elems(NE);
    x.hist = take(4 * hist);
    x.htmp = take(4 * scan_tmp_elems((uint32_t)(hist > NE + 1 ? hist : NE + 1)));
    x.ctmp = take(8 * scan_tmp_elems(NE + 1));
    x.ctr = take(4 * 8);
    x.bmax = take(4 * kUserBitsGrid);
    x.pc = take(4 * kPlanCtr);
    x.ccls = take(4 * (size_t)NE);
    x.cpos = take(4 * (size_t)NE);
    // compacted rows: room for half of every member slot's full row, at most
    // 2^32 words, 16 GiB (2^24 when the automatic rule leaves compaction off)
    size_t cap = (size_t)NE * wmax / 2;
    const size_t cmax = wmax >= kCompactMinW ? ((size_t)1 << 32) : ((size_t)1 << 24);
    if (cap > cmax) cap = cmax;
    x.cbits_words = cap;
    x.cbits = take(4 * cap);
    x.cw = take(4 * (size_t)NE);
    x.coff = take(8 * (size_t)NE);
    x.ccur = take(16);
    x.total = off;
    if (w) *w = x;
    return off;
}

static uint32_t user_bits_grid(const KnnArgs &a) {
    const uint32_t grid = (uint32_t)div_up((uint64_t)a.n + 1, kStageWaves);
    return grid < kUserBitsGrid ? grid : kUserBitsGrid;
}

static hipError_t user_bits(const KnnArgs &a, const KnnPtrs &w, hipStream_t s) {
    const size_t lds = knn_stage_lds_bytes(a.m, a.wmax);
    hipError_t e = hipFuncSetAttribute((const void *)k_user_bits,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_user_bits, dim3(user_bits_grid(a)), dim3(kStageThreads), lds, s,
                       a.indptr, a.indices, a.nnz, a.n, a.m, a.wmax, w.rows, w.rlen, w.bmax, w.pc);
    return hipGetLastError();
}

static hipError_t plan(const KnnArgs &a, const KnnPtrs &w, const uint32_t *order,
                       const KnnOpts &o, bool batched, hipStream_t s) {
    const uint32_t mfma_min = o.mfma_min ? o.mfma_min : kDefaultMfmaMin;
    const uint32_t gt = o.group_tiles ? o.group_tiles : kGroupTiles;  // >= 1
    const dim3 g((uint32_t)div_up(a.NE, 256));
    hipLaunchKernelGGL(k_plan_count, g, dim3(256), 0, s, a, order, mfma_min, gt, w.bmax,
                       user_bits_grid(a), w.cnt, w.slots);
    hipError_t e = scan_u64(w.cnt, w.cnt, a.NE, w.ctmp, s);
    if (e != hipSuccess) return e;
    if ((e = scan_u32(w.slots, w.slots, a.NE, w.htmp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_fill, g, dim3(256), 0, s, a, order, gt, w.cnt, w.slots, w.items_m,
                       w.items_b, w.sbase, w.rb_done, w.ctr, batched ? w.ctr + 2 : nullptr);
    return hipGetLastError();
}

// k_compact's LDS: two W-word bitmaps and one 3W/4-word row buffer per wave;
// 8 waves up to 2048-word rows, else 4
static uint32_t compact_threads(uint32_t wmax) { return wmax <= 2048 ? 512u : 256u; }
static size_t compact_lds(uint32_t wmax) {
    return ((size_t)2 * wmax + (size_t)(compact_threads(wmax) / 64) * (3 * wmax / 4)) * 4;
}

static bool compact_on(const KnnArgs &a, const KnnOpts &o) {
    if (compact_lds(a.wmax) + 1024 > 160 * 1024) return false;
    return o.compact == 2 || (o.compact == 0 && a.wmax >= kCompactMinW);
}

static hipError_t launch_paths(const KnnArgs &a, const KnnPtrs &w, const KnnOpts &o,
                               uint32_t grid_m, uint32_t grid_b, bool batched, hipStream_t s) {
    // the events bracket the MFMA kernel, which carries the large clusters
    hipError_t e;
    if (o.ev_begin && (e = hipEventRecord(o.ev_begin, s)) != hipSuccess) return e;
    MfmaScratch sc;
    sc.keys = w.skeys;
    sc.rb_done = w.rb_done;
    sc.sbase = w.sbase;
    const bool cmp = compact_on(a, o);
    sc.cbits = cmp ? w.cbits : nullptr;
    sc.cw = cmp ? w.cw : nullptr;
    sc.coff = cmp ? w.coff : nullptr;
    if (grid_m)
        hipLaunchKernelGGL(k_knn_mfma, dim3(grid_m), dim3(256), 0, s, a, w.rows, w.rlen, sc,
                           w.items_m, w.ctr, batched ? w.ctr + 2 : nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (o.ev_end && (e = hipEventRecord(o.ev_end, s)) != hipSuccess) return e;
    if (grid_b)
        hipLaunchKernelGGL(k_knn_bitmap, dim3(grid_b), dim3(64), 0, s, a, w.rows, w.rlen,
                           w.items_b, w.ctr + 1, batched ? w.ctr + 3 : nullptr);
    return hipGetLastError();
}

static hipError_t compact(const KnnArgs &a, const KnnPtrs &w, const KnnOpts &o, hipStream_t s) {
    if (!compact_on(a, o)) return hipSuccess;
    const uint32_t nt = compact_threads(a.wmax);
    const size_t lds = compact_lds(a.wmax);
    const void *fn = nt == 512 ? (const void *)k_compact<512> : (const void *)k_compact<256>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    // allocation cursor (u64) and cluster cursor (u32)
    if ((e = launch_fill_u32(reinterpret_cast<uint32_t *>(w.ccur), 0, 4, s)) != hipSuccess) return e;
    uint32_t *cnext = reinterpret_cast<uint32_t *>(w.ccur) + 2;
    if (nt == 512)
        hipLaunchKernelGGL(k_compact<512>, dim3(kCompactGrid), dim3(512), lds, s, a, w.items_m,
                           w.ctr, w.cbits, (uint64_t)w.cbits_words, w.cw, w.coff, w.ccur, cnext);
    else
        hipLaunchKernelGGL(k_compact<256>, dim3(kCompactGrid), dim3(256), lds, s, a, w.items_m,
                           w.ctr, w.cbits, (uint64_t)w.cbits_words, w.cw, w.coff, w.ccur, cnext);
    return hipGetLastError();
}

hipError_t knn_plain(const KnnArgs &a, const KnnPtrs &w, const KnnOpts &o, hipStream_t s) {
    hipError_t e = user_bits(a, w, s);
    if (e != hipSuccess) return e;
    if ((e = plan(a, w, nullptr, o, false, s)) != hipSuccess) return e;
    // the dictionaries take their clusters from the work list the plan wrote
    if ((e = compact(a, w, o, s)) != hipSuccess) return e;
    uint32_t n[2] = {0, 0};
    e = hipMemcpyAsync(n, w.ctr, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    return launch_paths(a, w, o, n[0], n[1], false, s);
}

hipError_t knn_batched(const KnnArgs &a, const KnnPtrs &w, const KnnOpts &o, hipStream_t s) {
    hipError_t e = user_bits(a, w, s);
    if (e != hipSuccess) return e;
    // items by cost class, costliest first (the size-ordered queue of
    // Section II-F), without a sort
    const dim3 g((uint32_t)div_up(a.NE, 256));
    const uint32_t mfma_min = o.mfma_min ? o.mfma_min : kDefaultMfmaMin;
    const uint32_t gt = o.group_tiles ? o.group_tiles : kGroupTiles;
    hipLaunchKernelGGL(k_plan_classes, g, dim3(256), 0, s, a, mfma_min, gt, w.bmax,
                       user_bits_grid(a), w.pc, w.ccls, w.cpos, w.sbase);
    hipLaunchKernelGGL(k_plan_items, g, dim3(256), 0, s, a, gt, w.pc, w.ccls, w.cpos, w.sbase,
                       w.items_m, w.items_b, w.rb_done, w.ctr, w.ctr + 2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the dictionaries take their clusters from that list, largest first
    if ((e = compact(a, w, o, s)) != hipSuccess) return e;
    const uint32_t gm = o.persistent_wgs ? o.persistent_wgs : 512;
    return launch_paths(a, w, o, gm, kBitmapPersistent, true, s);
}

}  // namespace c2
