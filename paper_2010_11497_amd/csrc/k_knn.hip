// Step 2 on the device: exact brute-force KNN inside every cluster
// (Section II-F, Algorithm 2, brute-force branch).
//
// Staging.  Only items held by at least two members of a cluster can be in
// an intersection, so each cluster C is multiplied over its local dictionary
// D_C of such items.  One pass per cluster (k_dict) builds D_C from the
// members' CSR lists in LDS bitmaps over the item universe and numbers it in
// item order; every member's profile restricted to D_C becomes a bit row of
// Wc = 8 * ceil(|D_C| / 256) words in the cluster's region of the store.  The
// store is tiled for the MFMA operands: the rows of 32 consecutive members
// form a row block, and for each group of 256 dictionary positions a row
// block holds two 512-byte halves, half h holding words 4h .. 4h+3 of the
// group of each of its 32 rows (16 bytes per row).  A wave therefore loads a
// whole operand fragment (32 rows x 128 positions) with one coalesced 16-byte
// load per lane.  Clusters larger than kBigS members publish their
// dictionary maps and let every block write their rows (k_rows).
//
// Pairwise counts.  |P_u & P_v| is the dot product of two rows over D_C and
// |P_u | P_v| = |P_u| + |P_v| - |P_u & P_v|.  A work item is one row block of
// a cluster's members taken against its column tiles, by one wave, in one of
// three tile shapes chosen per cluster size (tunable): 32 x 32, 64 x 64, or
// 64 rows x 128 columns.  Per 64-position chunk the wave expands the bits of
// its column-member and row-member fragments to fp4 (e2m1) nibbles in
// registers (0x2 = 1.0 for a set bit) and issues one
// v_mfma_scale_f32_32x32x64_f8f6f4 per 32 x 32 block at unit block scale;
// the fp32 sums are integer counts below 2^24, hence exact.  The accumulators
// (up to 8 x 16 values per lane) stay in registers, two waves per SIMD so
// that one wave's selection runs beside the other's products: lane l holds
// row member 32 * bj + l % 32 of every block (bi, bj) against 16 column
// members, so selection reads its candidates straight from the accumulators.
//
// Selection.  Each row member keeps a bounded heap of its k best candidates
// in LDS, keyed by an exact 32-bit similarity key; each tile's candidates are
// filtered against the heap root and the survivors inserted, the two lanes
// that share a row taking turns.  A row block spanning more than group_tiles
// column tiles is split into up to 4 items over disjoint column ranges whose
// lists the last item to finish merges.
//
// Bitmap path: AND + population count over the same store, for clusters the
// tuning sends there and whenever some profile holds 2^15 items or more
// (where the 32-bit key is no longer exact).
#include "c2_internal.h"
#include "c2_kernels.h"

namespace c2 {

constexpr uint32_t kRowBlock = 64;   // rows (members) per bitmap work item
constexpr int kWordChunk = 16;       // row words staged per step (bitmap path)
constexpr uint32_t kRows = 64;       // rows of the largest MFMA tile (row members of a work item)
constexpr uint32_t kCols = 128;      // columns of the largest MFMA tile
constexpr uint32_t kDefaultMfmaMin = 2;
constexpr uint32_t kDefaultTile32 = 32;   // clusters up to this size: 32-row tiles
constexpr uint32_t kDefaultTile64 = 64;   // up to this size: 64 x 64 tiles, else 64 x 128
constexpr uint32_t kGroupTiles = 16; // column tiles per work item before a row block is split
constexpr uint32_t kMaxGroups = 4;   // column groups a row block is split into at most
constexpr uint32_t kLensGrid = 2048;  // blocks of k_lens at most
constexpr uint32_t kBitmapPersistent = 256;  // persistent bitmap-path workgroups (batched form)
constexpr uint32_t kDefaultWaves = 2048;     // persistent MFMA waves (8 per CU, 2 per SIMD)
// batched planning counters: kCostClasses item counts, then scratch slots and
// bitmap items
constexpr uint32_t kCostClasses = 64;
constexpr uint32_t kSlotCtr = kCostClasses, kBitmapCtr = kCostClasses + 1;
constexpr uint32_t kPlanCtr = kCostClasses + 2;
// staging
constexpr uint32_t kStageGrid = 1024;  // persistent staging blocks
constexpr uint32_t kStageThreads = 512;
constexpr uint32_t kBigS = 512;        // larger clusters: rows written by k_rows
constexpr uint32_t kWinW = 128;        // row words per staging window (16 groups)
constexpr uint32_t kWinStride = 132;   // LDS words per window row (bank spread, 16-B aligned)

C2_DEV void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

uint32_t dict_words(uint32_t m) { return (m + 31) / 32; }

// LDS word offset of the staging window after the two dictionary maps (16-byte aligned).
C2_DEV __host__ inline uint32_t win_offset(uint32_t Wm) { return (2 * Wm + 3) & ~3u; }

// ------------------------------------------------------------------ lengths

// ulen[u] = |P_u|; bmax[block] = the longest profile the block saw (the grid
// is capped); the first block also clears the planning counters.
__global__ __launch_bounds__(256) void k_lens(const int64_t *__restrict__ indptr, uint64_t nnz,
                                              uint32_t n, uint32_t *__restrict__ ulen,
                                              uint32_t *bmax_out, uint32_t *plan_ctr) {
    uint32_t longest = 0;
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        uint64_t a, e;
        row_range(indptr, u, nnz, a, e);
        const uint32_t l = (uint32_t)(e - a);
        ulen[u] = l;
        longest = l > longest ? l : longest;
    }
    __shared__ uint32_t bmax;
    if (threadIdx.x == 0) bmax = 0;
    __syncthreads();
    if (longest) atomicMax(&bmax, longest);
    __syncthreads();
    if (threadIdx.x == 0) bmax_out[blockIdx.x] = bmax;
    if (plan_ctr && blockIdx.x == 0 && threadIdx.x < kPlanCtr) plan_ctr[threadIdx.x] = 0;
}

// Longest profile, from the per-block values of k_lens (block-wide).
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

// ------------------------------------------------------------------ the store

// Rows per piece of a cluster of s members: 32, or s when the cluster has
// fewer (its one row block is not padded; a fragment load then reads past the
// piece, into the next piece or past the block, which reads as 0, and the rows
// it reads there are never used).
C2_DEV uint32_t piece_rows(uint32_t s) { return s < 32 ? s : 32u; }

// Word w of the row at position p of a cluster whose rows have Wc = 8 * G
// words (the tiled layout described at the top), P rows per piece.
C2_DEV size_t store_word(uint32_t p, uint32_t w, uint32_t G, uint32_t P) {
    return ((((size_t)(p >> 5) * G + (w >> 3)) * 2 + ((w >> 2) & 1)) * P * 4) + (p & 31) * 4 + (w & 3);
}

struct StoreView {
    const uint32_t *bits;
    const uint32_t *cw;    // words per row of each cluster, 0 = not staged
    const uint64_t *coff;  // first word of each cluster's rows
};

// Work item of the MFMA path: cluster c, row block rb of 32 * NB rows (nbc =
// log2 NB), column group g of ng.
C2_DEV uint64_t mfma_item_code(uint32_t c, uint32_t rb, uint32_t nbc, uint32_t g, uint32_t ng) {
    return ((uint64_t)c << 32) | ((uint64_t)rb << 8) | (nbc << 6) | (g << 4) | (ng - 1);
}
// Tile shapes: 0 = 32 rows x 32 columns, 1 = 64 x 64, 2 = 64 x 128.
C2_DEV uint32_t shape_rows(uint32_t tc) { return tc == 0 ? 32u : 64u; }
C2_DEV uint32_t shape_cols(uint32_t tc) { return 32u << tc; }

// The first item of a cluster: row block 0, column group 0.
C2_DEV bool first_item(uint64_t code) {
    return ((uint32_t)code >> 8) == 0 && (((uint32_t)code >> 4) & 3u) == 0;
}

// ------------------------------------------------------------------ staging

// Dictionary rank of item i: its position among the dictionary items (in item
// order) if it is one; for any item, the number of dictionary items below it
// (non-decreasing in i).
C2_DEV uint32_t dict_rank(const uint32_t *twice, const uint32_t *pre, uint32_t i, bool &in) {
    const uint32_t w = i >> 5, b = i & 31, d = twice[w];
    in = (d >> b) & 1u;
    return pre[w] + __popc(d & ((1u << b) - 1u));
}

// Writes the tiled rows of the 32-row blocks [u0, u1) of cluster cv (G groups
// per row) from the dictionary maps in LDS.  NT threads, NT/32 lanes per member;
// win: 32 x kWinStride words of LDS.
template <int NT>
C2_DEV void write_rows(const KnnArgs &a, const ClusterView &cv, uint32_t u0, uint32_t u1,
                       uint32_t G, uint32_t *__restrict__ dst, const uint32_t *twice,
                       const uint32_t *pre, uint32_t *win) {
    const uint32_t P = piece_rows(cv.s);
    constexpr uint32_t NL = NT / 32;
    const uint32_t tid = threadIdx.x, r = tid / NL, sub = tid % NL, lane = tid & 63;
    const uint32_t gshift = lane & ~(NL - 1);
    const uint32_t Wc = 8 * G;
    for (uint32_t unit = u0; unit < u1; ++unit) {
        const uint32_t p = unit * 32 + r;
        uint64_t cur = 0, end = 0;
        if (p < cv.s) {
            const uint32_t u = a.members[cv.o + p];
            if (u < a.n) row_range(a.indptr, u, a.nnz, cur, end);
        }
        for (uint32_t wb = 0; wb < Wc; wb += kWinW) {
            const uint32_t ww = Wc - wb < kWinW ? Wc - wb : kWinW;
            for (uint32_t x = tid; x < 32 * kWinStride; x += NT) win[x] = 0;
            __syncthreads();
            const uint32_t dhi = (wb + ww) * 32, dlo = wb * 32;
            for (;;) {
                const uint64_t idx = cur + sub;
                const bool valid = idx < end;
                bool in = false;
                uint32_t d = 0;
                if (valid) {  // an item >= m (invalid input) is passed over
                    const uint32_t it = a.indices[idx];
                    if (it < a.m) d = dict_rank(twice, pre, it, in);
                }
                const bool used = valid && d < dhi;
                if (used && in) atomicOr(&win[r * kWinStride + ((d - dlo) >> 5)], 1u << (d & 31));
                const uint64_t bal = __ballot(used);
                const uint32_t nused = __popcll((bal >> gshift) & ((NL == 64 ? ~0ull : (1ull << NL) - 1)));
                cur += nused;
                if (nused < NL) break;
            }
            __syncthreads();
            // pieces of this window: (group x, half h) of P rows, 16 bytes per row
            const uint32_t npiece = (ww / 8) * 2;
            for (uint32_t e = tid; e < 32 * npiece; e += NT) {
                const uint32_t rr = e & 31, fh = e >> 5, x = fh >> 1, h = fh & 1;
                if (rr >= P) continue;
                const uint4 v = *reinterpret_cast<const uint4 *>(&win[rr * kWinStride + x * 8 + h * 4]);
                const size_t o = ((((size_t)unit * G + wb / 8 + x) * 2 + h) * P * 4) + rr * 4;
                *reinterpret_cast<uint4 *>(dst + o) = v;
            }
            __syncthreads();
        }
    }
}

struct StageArgs {
    uint32_t *bits;
    uint64_t cap;              // words
    uint32_t *cw;
    uint64_t *coff;
    unsigned long long *ccur;  // allocation cursor (words)
    uint32_t *cnext;           // cluster cursor of k_dict
    uint32_t *rnext;           // entry cursor of k_rows
    uint32_t *dslot;           // map slot of each big cluster
    uint32_t *dmap;            // [slot][2 * Wm]: twice, then pre
    uint32_t *dcur;            // map slot cursor
    uint64_t *rlist;           // row work of the big clusters: c << 32 | first unit << 8 | units
    uint32_t *rcount;          // entries of rlist
    uint32_t row_units;        // 32-row units per entry (2..8)
    uint32_t claim;            // work-list items a k_dict block claims at a time (1..64)
    uint32_t *status;          // bit 0 set when the store overflows
};

// One block per cluster of >= 2 members (taken at the cluster's first MFMA or
// bitmap item, in work-list order, costliest first in the batched form; a
// block claims st.claim consecutive items at a time and takes the clusters
// whose first items they hold, one after the other):
// dictionary bitmaps `once` and `twice` over the items (LDS), numbering, a
// region of the store, then the rows (clusters of at most kBigS members) or
// the published maps and the cluster's entries in the row list (larger ones).
__global__ __launch_bounds__(kStageThreads) void k_dict(KnnArgs a, const uint64_t *__restrict__ items,
                                                        const uint32_t *n_items, StageArgs st) {
    constexpr uint32_t NT = kStageThreads, G16 = 16, NG = NT / G16;
    extern __shared__ uint32_t lds[];
    const uint32_t Wm = a.Wm;
    uint32_t *once = lds, *twice = lds + Wm, *pre = lds, *win = lds + win_offset(Wm);
    const uint32_t tid = threadIdx.x;
    __shared__ uint32_t wsum[NT / 64 + 1];
    __shared__ unsigned long long sh_off;
    __shared__ uint32_t sh_ok, sh_slot, sh_rbase, sh_n, sh_end;
    __shared__ uint32_t sh_list[64];
    const uint32_t total_items = *n_items;
    for (;;) {
        __syncthreads();
        if (tid < 64) {  // wave 0 claims the items and lists their clusters
            uint32_t base = 0;
            if (tid == 0) base = atomicAdd(st.cnext, st.claim);
            base = __shfl(base, 0);
            const uint32_t i = base + tid;
            const bool in = tid < st.claim && i < total_items;
            const uint64_t code = in ? items[i] : 0ull;
            const bool f = in && first_item(code);
            const uint64_t bal = __ballot(f);
            if (f) sh_list[__popcll(bal & ((1ull << tid) - 1))] = (uint32_t)(code >> 32);
            if (tid == 0) {
                sh_n = (uint32_t)__popcll(bal);
                sh_end = base >= total_items;
            }
        }
        __syncthreads();
        if (sh_end) break;
        const uint32_t nlist = sh_n;
        for (uint32_t ci = 0; ci < nlist; ++ci) {
            if (ci) __syncthreads();  // the previous cluster is done with the LDS
            const uint32_t c = sh_list[ci];
            const ClusterView cv = view(a, c);
            const uint32_t s = cv.s;
            for (uint32_t w = tid; w < 2 * Wm; w += NT) lds[w] = 0;
            __syncthreads();
            // 1. dictionary: 16 lanes per member, 4 items per lane in flight; the
            //    next member's row range and the id after it are loaded while the
            //    current member's items are folded in
            {
                const uint32_t sub = tid & (G16 - 1), r0 = tid / G16;
                uint64_t na = 0, ne = 0;
                uint32_t nu = r0 < s ? a.members[cv.o + r0] : a.n;
                if (nu < a.n) row_range(a.indptr, nu, a.nnz, na, ne);
                nu = r0 + NG < s ? a.members[cv.o + r0 + NG] : a.n;
                for (uint32_t r = r0; r < s; r += NG) {
                    const uint64_t p0 = na, p1 = ne;
                    na = ne = 0;
                    if (nu < a.n) row_range(a.indptr, nu, a.nnz, na, ne);
                    nu = r + 2 * NG < s ? a.members[cv.o + r + 2 * NG] : a.n;
                    for (uint64_t p = p0 + sub; p < p1; p += 4 * G16) {
                        uint32_t it[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            it[q] = p + q * G16 < p1 ? a.indices[p + q * G16] : 0xFFFFFFFFu;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            if (it[q] >= a.m) continue;
                            const uint32_t bit = 1u << (it[q] & 31);
                            if (atomicOr(&once[it[q] >> 5], bit) & bit)
                                atomicOr(&twice[it[q] >> 5], bit);
                        }
                    }
                }
            }
            __syncthreads();
            // 2. rank of each word's first dictionary item (over `once`)
            const uint32_t per = (Wm + NT - 1) / NT, w0 = tid * per;
            uint32_t mine = 0;
            for (uint32_t w = w0; w < w0 + per && w < Wm; ++w) mine += __popc(twice[w]);
            uint32_t total;
            uint32_t run = block_excl_scan<uint32_t, NT>(mine, wsum, &total);
            for (uint32_t w = w0; w < w0 + per && w < Wm; ++w) {
                const uint32_t c2 = __popc(twice[w]);
                pre[w] = run;
                run += c2;
            }
            const uint32_t G = total ? (total + 255u) / 256u : 1u;
            if (tid == 0) {
                const unsigned long long rows = s < 32 ? s : (unsigned long long)((s + 31) / 32) * 32;
                const unsigned long long need = rows * 8 * G;
                const unsigned long long off = atomicAdd(st.ccur, need);
                sh_ok = off + need <= st.cap;
                sh_off = off;
                st.cw[c] = sh_ok ? 8 * G : 0u;
                st.coff[c] = off;
                if (!sh_ok) atomicOr(st.status, 1u);
                sh_slot = sh_ok && s > kBigS ? atomicAdd(st.dcur, 1u) : 0xFFFFFFFFu;
                if (sh_slot != 0xFFFFFFFFu) st.dslot[c] = sh_slot;
            }
            __syncthreads();
            if (!sh_ok) continue;
            if (sh_slot != 0xFFFFFFFFu) {
                uint32_t *dm = st.dmap + (size_t)sh_slot * 2 * Wm;
                for (uint32_t w = tid; w < Wm; w += NT) {
                    dm[w] = twice[w];
                    dm[Wm + w] = pre[w];
                }
                const uint32_t nblk = (s + 31) / 32, ne = (nblk + st.row_units - 1) / st.row_units;
                if (tid == 0) sh_rbase = atomicAdd(st.rcount, ne);
                __syncthreads();
                for (uint32_t e = tid; e < ne; e += NT) {
                    const uint32_t u0 = e * st.row_units;
                    const uint32_t nu = nblk - u0 < st.row_units ? nblk - u0 : st.row_units;
                    st.rlist[sh_rbase + e] = ((uint64_t)c << 32) | ((uint64_t)u0 << 8) | nu;
                }
                continue;
            }
            write_rows<NT>(a, cv, 0, (s + 31) / 32, G, st.bits + sh_off, twice, pre, win);
        }
    }
}

// Rows of the clusters larger than kBigS members: every block takes entries
// of the row list (runs of 32-row units of one cluster, which k_dict appended
// when it published the cluster's maps), loads the cluster's maps into LDS
// (kept while consecutive entries share the cluster) and writes the rows.
__global__ __launch_bounds__(kStageThreads) void k_rows(KnnArgs a, StageArgs st) {
    constexpr uint32_t NT = kStageThreads;
    extern __shared__ uint32_t lds[];
    const uint32_t Wm = a.Wm;
    uint32_t *twice = lds, *pre = lds + Wm, *win = lds + win_offset(Wm);
    const uint32_t tid = threadIdx.x;
    __shared__ uint64_t sh_code;
    uint32_t loaded = 0xFFFFFFFFu;
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            const uint32_t i = atomicAdd(st.rnext, 1u);
            sh_code = i < *st.rcount ? st.rlist[i] : ~0ull;
        }
        __syncthreads();
        const uint64_t code = sh_code;
        if (code == ~0ull) break;
        const uint32_t c = (uint32_t)(code >> 32);
        const ClusterView cv = view(a, c);
        if (c != loaded) {
            const uint32_t *dm = st.dmap + (size_t)st.dslot[c] * 2 * Wm;
            for (uint32_t w = tid; w < 2 * Wm; w += NT) lds[w] = dm[w];
            loaded = c;
            __syncthreads();
        }
        const uint32_t u0 = (uint32_t)code >> 8, u1 = u0 + ((uint32_t)code & 0xFFu);
        write_rows<NT>(a, cv, u0, u1, st.cw[c] / 8, st.bits + st.coff[c], twice, pre, win);
    }
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

// ------------------------------------------------------------ bitmap path
//
// One wave per work item (cluster, block of 64 rows); lane = row owner.  The
// lane keeps its row's 16-word chunk in registers and accumulates AND +
// popcount against each column row of a 64-column tile staged in LDS (read
// as a broadcast).  Rows come from the store.

struct __attribute__((aligned(16))) BitmapLds {
    uint32_t colw[kRowBlock][kWordChunk];
    uint32_t clen[kRowBlock], cuid[kRowBlock];
    uint32_t hI[kMaxK * 64], hU[kMaxK * 64], hV[kMaxK * 64];
    uint32_t cnt[kRowBlock][64];  // the tile's counts, [column][row owner]
};

C2_DEV void bitmap_item(const KnnArgs &a, const StoreView &sv, const uint32_t *ulen, uint32_t c,
                        uint32_t rb, BitmapLds &L) {
    const uint32_t lane = threadIdx.x;
    const ClusterView cv = view(a, c);
    const uint32_t s = cv.s, W = sv.cw[c], G = W / 8, P = piece_rows(s);
    if (W == 0) return;  // not staged (store overflow, flagged in the status word)
    const uint32_t *base = sv.bits + sv.coff[c];
    const uint32_t ra = rb * kRowBlock + lane;
    const bool active = ra < s;
    const uint32_t ur = active ? a.members[cv.o + ra] : kPad;
    const uint32_t Lr = active ? ulen[ur] : 0;
    RowHeap<64> h;
    h.init(L.hI, L.hU, L.hV, lane, a.k);
    for (uint32_t cb = 0; cb * kRowBlock < s; ++cb) {
        __syncthreads();
        const uint32_t pc = cb * kRowBlock + lane;
        const uint32_t uc = pc < s ? a.members[cv.o + pc] : kPad;
        L.clen[lane] = pc < s ? ulen[uc] : 0;
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
                const uint32_t p = cb * kRowBlock + cc;
                L.colw[cc][ww] = (p < s && w0 + ww < W) ? base[store_word(p, w0 + ww, G, P)] : 0u;
            }
            uint32_t r[kWordChunk];
#pragma unroll
            for (int ww = 0; ww < kWordChunk; ++ww)
                r[ww] = (active && w0 + ww < W) ? base[store_word(ra, w0 + ww, G, P)] : 0u;
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
        // the counts go through LDS so that the offer loop need not be unrolled
#pragma unroll
        for (int q = 0; q < (int)kRowBlock; ++q) L.cnt[q][lane] = acc[q];
        if (active) {
#pragma unroll 1
            for (uint32_t q = 0; q < kRowBlock; ++q) {
                const uint32_t col = cb * kRowBlock + q;
                if (col < s && col != ra) {
                    const uint32_t I = L.cnt[q][lane];
                    h.offer(I, Lr + L.clen[q] - I, L.cuid[q]);
                }
            }
        }
    }
    if (active && cv.j < a.t) {
        const size_t base_o = ((size_t)ur * a.t + cv.j) * a.k;
        h.drain(a.part_id + base_o, a.part_I + base_o);
    }
}

// Plain form: block b handles items[b].  Batched form: persistent blocks take
// items from a device cursor until the list is exhausted.
__global__ __launch_bounds__(64) void k_knn_bitmap(KnnArgs a, StoreView sv, const uint32_t *ulen,
                                                   const uint64_t *items, const uint32_t *n_items,
                                                   uint32_t *cursor) {
    __shared__ BitmapLds L;
    __shared__ uint32_t next;
    const uint32_t total = *n_items;
    if (total == 0) return;  // the usual case: every cluster is on the MFMA path
    if (!cursor) {
        if (blockIdx.x >= total) return;
        const uint64_t it = items[blockIdx.x];
        bitmap_item(a, sv, ulen, (uint32_t)(it >> 32), (uint32_t)it >> 8, L);
        return;
    }
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) next = atomicAdd(cursor, 1u);
        __syncthreads();
        const uint32_t i = next;
        if (i >= total) break;
        const uint64_t it = items[i];
        bitmap_item(a, sv, ulen, (uint32_t)(it >> 32), (uint32_t)it >> 8, L);
    }
}

// -------------------------------------------------------------- MFMA path
//
// Selection on this path uses an exact 32-bit similarity key,
//   key(I, U) = floor(I * (2^32 - 1) / U),
// which preserves the order of I/U exactly when U < 2^16 (two different
// fractions with denominators below 2^16 differ by more than 1/(2^32 - 1)),
// so the path is taken only when every profile has fewer than 2^15 items.
// A heap entry is the u64 (key << 32) | (0xFFFFFFFF - id): larger is better,
// and entries are distinct, so an entry beats the root iff it compares
// greater.  Each tile's candidates are first filtered against the heap root
// with a necessary fp32 test; those that pass are inserted in a wave-uniform
// loop, where the exact comparison is made.

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// E8M0 block scales of 2^0 for all four operand blocks.
constexpr int kUnitScale = 0x7F7F7F7F;
// Operand format code of e2m1 (fp4) for the f8f6f4 MFMA family.
constexpr int kFmtFp4 = 4;

// C += A * B^T over 64 positions for one 32 x 32 block: A and B hold, in lane
// l, 32 nibbles of row / column l % 32 for positions [32 * (l / 32), +32).
// Only the first four dwords of the 8-dword operands are read for fp4.
C2_DEV v16f mfma_fp4(v4i a, v4i b, v16f c) {
    const v8i A = {a[0], a[1], a[2], a[3], 0, 0, 0, 0};
    const v8i B = {b[0], b[1], b[2], b[3], 0, 0, 0, 0};
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, B, c, kFmtFp4, kFmtFp4, 0,
                                                           kUnitScale, 0, kUnitScale);
}

constexpr uint32_t kMfmaMaxLen = 1u << 15;
// Word 3 of a raw buffer resource on gfx9 parts: 32-bit data format, no
// swizzle; loads past num_records return 0.
constexpr int kBufferFlags = 0x00020000;

// 32 bits -> 16 bytes of e2m1 nibbles (0x2 = 1.0 for a set bit).  Dword s of
// the result holds, in byte q, bit 8q+2s of w in its low nibble and bit
// 8q+2s+1 in its high nibble: (w >> 2s) & 0x03030303 puts each byte's 2-bit
// pair in the low bits of that byte, and v_perm_b32 looks the pair up in a
// 4-byte table {0x00, 0x02, 0x20, 0x22} held in both sources (so either
// source order gives the same bytes).  Every row is expanded the same way,
// so positions stay aligned in the dot product whatever order the MFMA gives
// the nibbles.
constexpr uint32_t kPairLut = 0x22200200u;

C2_DEV v4i nibbles32(uint32_t w) {
    return v4i{(int)__builtin_amdgcn_perm(kPairLut, kPairLut, w & 0x03030303u),
               (int)__builtin_amdgcn_perm(kPairLut, kPairLut, (w >> 2) & 0x03030303u),
               (int)__builtin_amdgcn_perm(kPairLut, kPairLut, (w >> 4) & 0x03030303u),
               (int)__builtin_amdgcn_perm(kPairLut, kPairLut, (w >> 6) & 0x03030303u)};
}

C2_DEV uint32_t u4get(const uint4 &x, int q) { return q == 0 ? x.x : q == 1 ? x.y : q == 2 ? x.z : x.w; }

// I from key(I, U) and S = |P_u| + |P_v| (U = S - I): I/(S - I) is strictly
// increasing in I, and S*key/(2^32 - 1 + key) is within 2^-16 of I.
C2_DEV uint32_t key_to_I(uint32_t key, uint32_t S) {
    // the fp32 estimate is within 0.03 of I for S < 2^17 (checked for every
    // (I, U) with the reciprocal exact and 1-2 ulp off), so it rounds to I
    const float kt = (float)key;
    const float x = (float)S * kt * __builtin_amdgcn_rcpf(4294967295.0f + kt);
    return (uint32_t)(x + 0.5f);
}

// Bounded heap of one row's k best keys in LDS, hk[slot * kRows + row].
struct KeyHeap {
    uint64_t *hk;
    uint32_t me, k, cnt;
    uint64_t root;  // valid once full

    C2_DEV uint64_t get(uint32_t i) const { return hk[i * kRows + me]; }
    C2_DEV void put(uint32_t i, uint64_t v) { hk[i * kRows + me] = v; }
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
    // Until the heap holds k entries, entries are appended and then heapified
    // once; afterwards v replaces the root if it beats it.
    C2_DEV void insert(uint64_t v) {
        if (cnt < k) {
            put(cnt++, v);
            if (cnt == k) {
                heapify(k);
                root = get(0);
            }
        } else if (v > root) {
            root = sift_down(0, v, k);
        }
    }
};

// Necessary condition for a candidate to beat the root: J > J_T implies
// I > sigma_T * (|P_u| + |P_v|), sigma_T = J_T / (1 + J_T).  It is taken in
// fp32 on the accumulator as I >= fma(s, |P_v|, s * |P_u|) with
// s = sigma_T * (1 - 1e-6) fixed per row and round: the roundings of the
// products and of sigma_T (a reciprocal within 1 ulp) stay far below the
// 1e-6 margin, so no candidate that can beat the root is turned away.  An
// empty or filling heap has s = 0, and every real column passes.  The same
// comparison drops what is not a candidate: a padded column has length +inf
// (fma gives +inf, or NaN when s = 0) and a row past the cluster's end has
// s = NaN; a comparison with NaN is false.
struct BeatTest {
    float s, sL;
    C2_DEV BeatTest(float sigma, uint32_t Lr, bool act)
        : s(act ? sigma * 0.999999f : __builtin_nanf("")), sL(s * (float)Lr) {}
    C2_DEV bool operator()(float I, float Lv) const { return I >= __builtin_fmaf(s, Lv, sL); }
};

// sigma of the root's key kt: kt / (2^32 - 1 + kt), at most sigma_T since kt
// is J_T * (2^32 - 1) rounded down.
C2_DEV float sigma_of(uint32_t key) {
    const float kt = (float)key;
    return kt * __builtin_amdgcn_rcpf(4294967295.0f + kt);
}
// The key half of heap R's root (the high word of the u64 entry).
C2_DEV uint32_t root_key(const uint64_t *hk, uint32_t R) {
    return reinterpret_cast<const uint32_t *>(hk)[2 * R + 1];
}
// The bit of the accumulator position that holds column `self` in a lane
// whose first column is c0 (columns c0 + 8 * (r / 4) + r % 4), or 0.
C2_DEV uint32_t self_bit(uint32_t self, uint32_t c0) {
    const uint32_t d = self - c0;
    return d < 32 && !(d & 4) ? 1u << (4 * (d >> 3) + (d & 3)) : 0u;
}

struct MfmaScratch {
    uint64_t *keys;         // [slot][kRows][k], at the start of the store
    uint32_t *rb_done;      // per (cluster, row block) of a split row block
    const uint32_t *sbase;  // first slot of each cluster
};

struct __attribute__((aligned(16))) WaveLds {
    uint64_t hk[kMaxK * kRows];  // heaps, [slot][row]
    uint32_t hcnt[kRows];        // entries per heap
    uint32_t cuid[kCols];
    float clen[kCols];           // profile lengths, +inf past the last column
    uint32_t scr[64 * 8];        // 16 counts (u16) per lane
};

// Column member of the accumulator value r of block bi in lane half hh.
C2_DEV uint32_t acc_col(uint32_t bi, uint32_t r, uint32_t hh) {
    return 32 * bi + 8 * (r >> 2) + 4 * hh + (r & 3);
}

// Buffer resource over 32-row block x of a cluster (its `bytes` bytes from
// uint4 x * xstride of `frag`), or an empty one for x >= nblk.
C2_DEV __amdgpu_buffer_rsrc_t block_rsrc(const uint4 *frag, uint32_t x, uint32_t nblk,
                                         uint32_t xstride, uint32_t bytes) {
    const bool ok = x < nblk;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint4 *>(frag + (size_t)(ok ? x : 0) * xstride),
                                             (short)0, ok ? (int)bytes : 0, kBufferFlags);
}

C2_DEV uint4 buf_load16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
    return make_uint4(v[0], v[1], v[2], v[3]);
}

// The NC column-member and NR row-member fragments of one group.
template <int NR, int NC>
C2_DEV void load_group(const __amdgpu_buffer_rsrc_t (&rA)[NC], const __amdgpu_buffer_rsrc_t (&rB)[NR],
                       uint32_t off, uint4 (&xa)[NC], uint4 (&xb)[NR]) {
#pragma unroll
    for (int i = 0; i < NC; ++i) xa[i] = buf_load16(rA[i], off);
#pragma unroll
    for (int i = 0; i < NR; ++i) xb[i] = buf_load16(rB[i], off);
}

// acc[bi][bj] += the counts of one group (four 64-position chunks): the
// row-member operands of a chunk are expanded first, the column-member ones
// one at a time, each feeding NR MFMAs.
template <int NR, int NC>
C2_DEV void mult_group(const uint4 (&xa)[NC], const uint4 (&xb)[NR], v16f (&acc)[NC][NR]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v4i B[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) B[i] = nibbles32(u4get(xb[i], q));
#pragma unroll
        for (int bi = 0; bi < NC; ++bi) {
            const v4i A = nibbles32(u4get(xa[bi], q));
#pragma unroll
            for (int bj = 0; bj < NR; ++bj) acc[bi][bj] = mfma_fp4(A, B[bj], acc[bi][bj]);
        }
    }
}

// Per-tile selection state shared by the rounds of one lane.
struct SelCtx {
    uint32_t k, lane, lr, hh, rowpos;
};

// One selection round: the 16 candidates of accumulator block (BI, BJ) for the
// lane's row member 32 * BJ + lr.  The fp32 filter runs on all lanes; the
// candidates that pass are staged in LDS and offered to the heap with the
// exact key, which decides (a candidate that ties the root passes the filter
// and is turned away there), the two lanes of the row taking turns (lower
// half first).  The exact key is computed only in the insert loop, whose
// iterations follow each lane's own candidates: a check of the 16 positions
// in turn would run every position that any lane holds.
template <int BJ, int BI>
C2_DEV void select_round(const v16f &acc, uint32_t Lr, bool act, const SelCtx &cx, WaveLds &L) {
    const uint32_t R = 32 * BJ + cx.lr;
    const uint32_t self = cx.rowpos + 32 * BJ;
    const uint32_t cnt0 = L.hcnt[R];
    const bool full = cnt0 >= cx.k;
    const BeatTest beats(full ? sigma_of(root_key(L.hk, R)) : 0.0f, Lr, act);
    const uint32_t sbit = self_bit(self, 32 * BI + 4 * cx.hh);
    uint32_t mask = 0;
    uint32_t pk[8];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const uint32_t col = acc_col(BI, r, cx.hh);
        const uint32_t I = (uint32_t)acc[r];
        const bool ok = beats(acc[r], L.clen[col]);
        mask |= (ok ? 1u : 0u) << r;
        if (r & 1) pk[r >> 1] |= I << 16;
        else pk[r >> 1] = I;
    }
    mask &= ~sbit;
    if (!__any(mask != 0u)) return;
#pragma unroll
    for (int q = 0; q < 8; ++q) L.scr[cx.lane * 8 + q] = pk[q];
    wave_sync();
    KeyHeap h;
    h.hk = L.hk;
    h.me = R;
    h.k = cx.k;
#pragma unroll 1
    for (uint32_t pass = 0; pass < 2; ++pass) {
        uint32_t m = cx.hh == pass ? mask : 0u;
        if (m) {
            h.cnt = L.hcnt[R];
            h.root = h.cnt >= cx.k ? L.hk[R] : 0ull;
        }
        while (__any(m != 0u)) {
            if (m) {
                const uint32_t r = __ffs(m) - 1;
                m &= m - 1;
                const uint32_t I = (L.scr[cx.lane * 8 + (r >> 1)] >> (16 * (r & 1))) & 0xFFFFu;
                const uint32_t col = acc_col(BI, r, cx.hh);
                const uint32_t U = Lr + (uint32_t)L.clen[col] - I, uid = L.cuid[col];
                const uint64_t v = ((uint64_t)jkey(I, U) << 32) | (0xFFFFFFFFu - uid);
                h.insert(v);
            }
        }
        if (cx.hh == pass && mask) L.hcnt[R] = h.cnt;
        wave_sync();
    }
}

// Row ownership for two row blocks: after the swap, lane (lr, hh) holds in
// acc[bi][h] the counts of its own row member 32 * hh + lr against the
// columns of lane half h (v_permlane32_swap exchanges the upper 32 lanes of
// its first operand with the lower 32 lanes of its second), so that each row
// is selected by one lane and no two lanes touch one heap.
// (Whole vectors in and out: writing single elements of the accumulator
// vectors in place compiled to wrong code.)
typedef uint32_t v16u __attribute__((ext_vector_type(16)));
template <int NC>
C2_DEV void own_rows(v16f (&acc)[NC][2]) {
#pragma unroll
    for (int bi = 0; bi < NC; ++bi) {
        const v16u x = __builtin_bit_cast(v16u, acc[bi][0]), y = __builtin_bit_cast(v16u, acc[bi][1]);
        v16u nx, ny;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const auto p = __builtin_amdgcn_permlane32_swap(x[r], y[r], false, false);
            nx[r] = p[0];
            ny[r] = p[1];
        }
        acc[bi][0] = __builtin_bit_cast(v16f, nx);
        acc[bi][1] = __builtin_bit_cast(v16f, ny);
    }
}

// One selection round on owned rows: the 16 candidates of column block BI,
// lane half H, for the lane's own row member 32 * hh + lr (filter and
// exact-key insert as in select_round).
template <int H, int BI>
C2_DEV void select_own(const v16f &acc, uint32_t Lr, bool act, const SelCtx &cx, WaveLds &L) {
    const uint32_t R = 32 * cx.hh + cx.lr;
    const uint32_t self = cx.rowpos + 32 * cx.hh;
    const uint32_t cnt0 = L.hcnt[R];
    const bool full = cnt0 >= cx.k;
    const uint64_t root = full ? L.hk[R] : 0ull;
    const BeatTest beats(full ? sigma_of(root_key(L.hk, R)) : 0.0f, Lr, act);
    const uint32_t sbit = self_bit(self, 32 * BI + 4 * H);
    uint32_t mask = 0;
    uint32_t pk[8];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const uint32_t col = acc_col(BI, r, H);
        const uint32_t I = (uint32_t)acc[r];
        const bool ok = beats(acc[r], L.clen[col]);
        mask |= (ok ? 1u : 0u) << r;
        if (r & 1) pk[r >> 1] |= I << 16;
        else pk[r >> 1] = I;
    }
    mask &= ~sbit;
    if (!__any(mask != 0u)) return;
#pragma unroll
    for (int q = 0; q < 8; ++q) L.scr[cx.lane * 8 + q] = pk[q];
    wave_sync();
    KeyHeap h;
    h.hk = L.hk;
    h.me = R;
    h.k = cx.k;
    h.cnt = cnt0;
    h.root = root;
    uint32_t m = mask;
    while (__any(m != 0u)) {
        if (m) {
            const uint32_t r = __ffs(m) - 1;
            m &= m - 1;
            const uint32_t I = (L.scr[cx.lane * 8 + (r >> 1)] >> (16 * (r & 1))) & 0xFFFFu;
            const uint32_t col = acc_col(BI, r, H);
            const uint32_t U = Lr + (uint32_t)L.clen[col] - I, uid = L.cuid[col];
            h.insert(((uint64_t)jkey(I, U) << 32) | (0xFFFFFFFFu - uid));
        }
    }
    if (mask) L.hcnt[R] = h.cnt;
    wave_sync();
}

template <int NC, int IDX>
struct OwnRounds {
    static C2_DEV void run(v16f (&acc)[NC][2], uint32_t Lr, bool act, const SelCtx &cx, WaveLds &L) {
        constexpr int H = IDX / NC, BI = IDX % NC;
        select_own<H, BI>(acc[BI][H], Lr, act, cx, L);
        OwnRounds<NC, IDX + 1>::run(acc, Lr, act, cx, L);
    }
};
template <int NC>
struct OwnRounds<NC, 2 * NC> {
    static C2_DEV void run(v16f (&)[NC][2], uint32_t, bool, const SelCtx &, WaveLds &) {}
};

// The NR x NC rounds with compile-time block indices (the accumulators stay
// in registers only if every index into them is a constant).
template <int NR, int NC, int IDX>
struct Rounds {
    static C2_DEV void run(v16f (&acc)[NC][NR], const uint32_t (&Lr)[NR], const bool (&act)[NR],
                           const SelCtx &cx, WaveLds &L) {
        constexpr int BJ = IDX / NC, BI = IDX % NC;
        select_round<BJ, BI>(acc[BI][BJ], Lr[BJ], act[BJ], cx, L);
        Rounds<NR, NC, IDX + 1>::run(acc, Lr, act, cx, L);
    }
};
template <int NR, int NC>
struct Rounds<NR, NC, NR * NC> {
    static C2_DEV void run(v16f (&)[NC][NR], const uint32_t (&)[NR], const bool (&)[NR],
                           const SelCtx &, WaveLds &) {}
};

// Work item of one wave: the TRR = 32 * NR row members of row block rb against
// the cluster's column tiles of TRC = 32 * NC members in column group g.
template <int NR, int NC>
C2_DEV void mfma_item(const KnnArgs &a, const StoreView &sv, const uint32_t *ulen,
                      const MfmaScratch &sc, uint64_t code, WaveLds &L) {
    constexpr uint32_t TRR = 32 * NR, TRC = 32 * NC;
    const uint32_t lane = threadIdx.x & 63, lr = lane & 31, hh = lane >> 5;
    const uint32_t c = (uint32_t)(code >> 32), rb = (uint32_t)code >> 8;
    const uint32_t g = ((uint32_t)code >> 4) & 3u, ng = ((uint32_t)code & 15u) + 1;
    const ClusterView cv = view(a, c);
    const uint32_t s = cv.s, Wc = sv.cw[c];
    if (Wc == 0) return;  // not staged (store overflow, flagged in the status word)
    const uint32_t G = Wc / 8, nblk = (s + 31) / 32, P = piece_rows(s);
    // Fragment (32-row block x, group gg, half hh) of this lane: 16 bytes at
    // byte (gg * 2P + hh * P + lr) * 16 of row block x, whose G * 2P * 16
    // bytes start at uint4 x * G * 2P of the cluster's rows.  Each row block
    // is read through a buffer resource of exactly its size: past it (groups
    // >= G, lanes beyond a short piece, blocks >= nblk) the loads return 0.
    const uint4 *frag = reinterpret_cast<const uint4 *>(sv.bits + sv.coff[c]);
    const uint32_t voff = (hh * P + lr) * 16, gbytes = 2 * P * 16, xbytes = G * gbytes;
    // row members of this lane: position rb * TRR + 32 * bj + lr
    uint32_t Lr[NR];
    bool act[NR];
#pragma unroll
    for (int bj = 0; bj < NR; ++bj) {
        const uint32_t p = rb * TRR + 32 * bj + lr;
        act[bj] = p < s;
        Lr[bj] = act[bj] ? ulen[a.members[cv.o + p]] : 0u;
    }
    for (uint32_t q = lane; q < TRR; q += 64) L.hcnt[q] = 0;
    __amdgpu_buffer_rsrc_t rB[NR];
#pragma unroll
    for (int bj = 0; bj < NR; ++bj) rB[bj] = block_rsrc(frag, rb * NR + bj, nblk, G * 2 * P, xbytes);
    const uint32_t tiles = (s + TRC - 1) / TRC, per = (tiles + ng - 1) / ng;
    const uint32_t cb_end = (g + 1) * per < tiles ? (g + 1) * per : tiles;
    for (uint32_t cb = g * per; cb < cb_end; ++cb) {
        wave_sync();
        for (uint32_t q = lane; q < TRC; q += 64) {
            const uint32_t p = cb * TRC + q;
            const uint32_t u = p < s ? a.members[cv.o + p] : kPad;
            L.cuid[q] = u;
            L.clen[q] = p < s ? (float)ulen[u] : __builtin_inff();
        }
        __amdgpu_buffer_rsrc_t rA[NC];
#pragma unroll
        for (int bi = 0; bi < NC; ++bi) rA[bi] = block_rsrc(frag, cb * NC + bi, nblk, G * 2 * P, xbytes);
        v16f acc[NC][NR];
#pragma unroll
        for (int bi = 0; bi < NC; ++bi)
#pragma unroll
            for (int bj = 0; bj < NR; ++bj) acc[bi][bj] = v16f{};
        // K loop, two groups per step: group gg + 1 is in flight while group
        // gg is multiplied, and the loads of gg + 2 and gg + 3 follow
        uint4 xa0[NC], xb0[NR], xa1[NC], xb1[NR];
        load_group<NR, NC>(rA, rB, voff, xa0, xb0);
        load_group<NR, NC>(rA, rB, voff + gbytes, xa1, xb1);
        // (G >= 1: written as a do-while so that no zero-trip path keeps a
        // second copy of the zero accumulators alive across the loop)
        uint32_t gg = 0;
        do {
            mult_group<NR, NC>(xa0, xb0, acc);
            load_group<NR, NC>(rA, rB, voff + (gg + 2) * gbytes, xa0, xb0);
            if (gg + 1 < G) mult_group<NR, NC>(xa1, xb1, acc);
            load_group<NR, NC>(rA, rB, voff + (gg + 3) * gbytes, xa1, xb1);
            gg += 2;
        } while (gg < G);
        wave_sync();
        // selection: NR x NC rounds of 16 candidates, one per accumulator block
        SelCtx cx;
        cx.k = a.k;
        cx.lane = lane;
        cx.lr = lr;
        cx.hh = hh;
        cx.rowpos = rb * TRR + lr - cb * TRC;  // column of the lane's row member in block bj = 0
        if constexpr (NR == 2) {
            own_rows<NC>(acc);
            OwnRounds<NC, 0>::run(acc, hh ? Lr[NR - 1] : Lr[0], hh ? act[NR - 1] : act[0], cx, L);
        } else {
            Rounds<NR, NC, 0>::run(acc, Lr, act, cx, L);
        }
    }
    // The rows' entries, best first, by rank: the lane of half bj % 2 drains
    // row 32 * bj + lr (for NR = 1 the lower lanes drain the one row).
    const uint32_t slot0 = ng > 1 ? sc.sbase[c] + rb * ng : 0u;
    const uint32_t bj0 = NR > 1 ? hh : 0u, bstep = NR > 1 ? 2u : 1u;
    const uint32_t bjn = NR > 1 || hh == 0 ? NR : 0u;
#pragma unroll 1
    for (uint32_t bj = bj0; bj < bjn; bj += bstep) {
        const uint32_t R = 32 * bj + lr, p = rb * TRR + R;
        if (p >= s) continue;
        const uint32_t u = a.members[cv.o + p], Lu = ulen[u];
        const uint32_t cnt = L.hcnt[R];
        uint64_t ent[kMaxK];
        uint32_t rk[kMaxK];
#pragma unroll
        for (uint32_t i = 0; i < kMaxK; ++i) {
            ent[i] = i < cnt ? L.hk[i * kRows + R] : 0ull;
            rk[i] = 0;
        }
#pragma unroll
        for (uint32_t i = 0; i < kMaxK; ++i)
#pragma unroll
            for (uint32_t j2 = 0; j2 < kMaxK; ++j2) rk[i] += ent[j2] > ent[i] ? 1u : 0u;
        if (ng == 1) {
            if (cv.j >= a.t) continue;
            const size_t base = ((size_t)u * a.t + cv.j) * a.k;
#pragma unroll
            for (uint32_t i = 0; i < kMaxK; ++i)
                if (i < cnt) {
                    const uint32_t uid = 0xFFFFFFFFu - (uint32_t)ent[i];
                    a.part_id[base + rk[i]] = uid;
                    a.part_I[base + rk[i]] = key_to_I((uint32_t)(ent[i] >> 32), Lu + ulen[uid]);
                }
            for (uint32_t q = cnt; q < a.k; ++q) {
                a.part_id[base + q] = kPad;
                a.part_I[base + q] = 0;
            }
        } else {
            uint64_t *out = sc.keys + ((size_t)(slot0 + g) * kRows + R) * a.k;
#pragma unroll
            for (uint32_t i = 0; i < kMaxK; ++i)
                if (i < cnt) out[rk[i]] = ent[i];
            for (uint32_t q = cnt; q < a.k; ++q) out[q] = 0;
        }
    }
    if (ng == 1) return;
    // split row block: the item that finishes last merges the ng sorted lists
    __threadfence();
    wave_sync();
    uint32_t last = 0;
    if (lane == 0) last = atomicAdd(&sc.rb_done[slot0], 1u) == ng - 1;
    last = __shfl(last, 0);
    if (!last || cv.j >= a.t) return;
    __threadfence();
#pragma unroll 1
    for (uint32_t bj = bj0; bj < bjn; bj += bstep) {
        const uint32_t R = 32 * bj + lr, p = rb * TRR + R;
        if (p >= s) continue;
        const uint32_t u = a.members[cv.o + p], Lu = ulen[u];
        const uint64_t *in = sc.keys + ((size_t)slot0 * kRows + R) * a.k;
        uint32_t ptr[kMaxGroups];
        uint64_t head[kMaxGroups];
#pragma unroll
        for (uint32_t q = 0; q < kMaxGroups; ++q) {
            ptr[q] = 0;
            head[q] = q < ng ? in[(size_t)q * kRows * a.k] : 0;
        }
        const size_t base = ((size_t)u * a.t + cv.j) * a.k;
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
                    head[q] = (v != 0 && ptr[q] < a.k) ? in[(size_t)q * kRows * a.k + ptr[q]] : 0;
                }
            if (v == 0) {
                a.part_id[base + r] = kPad;
                a.part_I[base + r] = 0;
            } else {
                const uint32_t uid = 0xFFFFFFFFu - (uint32_t)v;
                a.part_id[base + r] = uid;
                a.part_I[base + r] = key_to_I((uint32_t)(v >> 32), Lu + ulen[uid]);
            }
        }
    }
}

C2_DEV void mfma_dispatch(const KnnArgs &a, const StoreView &sv, const uint32_t *ulen,
                          const MfmaScratch &sc, uint64_t code, WaveLds &L) {
    switch ((uint32_t)code >> 6 & 3u) {
    case 0: mfma_item<1, 1>(a, sv, ulen, sc, code, L); break;
    case 1: mfma_item<2, 2>(a, sv, ulen, sc, code, L); break;
    default: mfma_item<2, 4>(a, sv, ulen, sc, code, L); break;
    }
}

// Four waves per block, each with its own work item and LDS; two waves per
// SIMD (each up to 8 x 16 accumulator values per lane in 256 registers), so
// that one wave's selection runs beside the other's matrix products.  The
// waves of a block take consecutive items, which the plan orders so that
// they share their column tiles (the same column group of consecutive row
// blocks), read at about the same time through the CU's caches.  Plain form:
// wave w of block b takes items[4b + w]; batched form: persistent waves take
// items from a device cursor.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_knn_mfma(KnnArgs a, StoreView sv, const uint32_t *ulen, MfmaScratch sc,
                const uint64_t *items, const uint32_t *n_items, uint32_t *cursor) {
    __shared__ WaveLds Ls[4];
    WaveLds &L = Ls[threadIdx.x >> 6];
    const uint32_t total = *n_items;
    // the next item: the wave's own (plain form) or the cursor's (batched);
    // wave-uniform, so the item and everything derived from it live in SGPRs
    auto next = [&]() -> uint32_t {
        uint32_t i = 0;
        if ((threadIdx.x & 63) == 0) i = atomicAdd(cursor, 1u);
        return __builtin_amdgcn_readfirstlane(__shfl(i, 0));
    };
    uint32_t i = cursor ? next() : __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    while (i < total) {
        mfma_dispatch(a, sv, ulen, sc, items[i], L);
        if (!cursor) break;
        i = next();
        wave_sync();
    }
}

// ---------------------------------------------------------------- planning

// Tile shape code of a cluster of s members: 0 (32 x 32 tiles), 1 (64 x 64) or
// 2 (64 rows x 128 columns).
C2_DEV uint32_t tile_code(uint32_t s, uint32_t t32, uint32_t t64) {
    return s <= t32 ? 0u : s <= t64 ? 1u : 2u;
}

// Column groups of an MFMA cluster of s members in tile shape tc.  Only the
// largest shape's row blocks are split (their scratch slots then number at
// most (s/64 + 1) * 4 < s / 8).
C2_DEV uint32_t mfma_groups(uint32_t s, uint32_t tc, uint32_t group_tiles) {
    if (tc < 2) return 1;
    const uint32_t tiles = (s + kCols - 1) / kCols;
    if (tiles <= group_tiles) return 1;
    const uint32_t ng = (tiles + group_tiles - 1) / group_tiles;
    return ng < kMaxGroups ? ng : kMaxGroups;
}

struct PlanOpts {
    uint32_t mfma_min, group_tiles, t32, t64;
};

// Per cluster (index order): number of MFMA items (low word) and bitmap
// items (high word), and the scratch slots of split row blocks; clusters of
// one member get padded lists here.
__global__ __launch_bounds__(256) void k_plan_count(KnnArgs a, PlanOpts po, const uint32_t *bmax,
                                                    uint32_t nbmax, uint64_t *cnt, uint32_t *slots) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ncl = a.cl_cfg_off[a.t];
    uint32_t mfma_min = po.mfma_min;
    if (block_max_len(bmax, nbmax) >= kMfmaMaxLen) mfma_min = 0xFFFFFFFFu;
    if (q >= a.NE) return;
    if (q >= ncl) { cnt[q] = 0; slots[q] = 0; return; }
    const ClusterView cv = view(a, q);
    uint64_t v = 0;
    uint32_t sl = 0;
    if (cv.s >= mfma_min && cv.s >= 2) {
        const uint32_t tc = tile_code(cv.s, po.t32, po.t64), TRR = shape_rows(tc);
        const uint32_t ng = mfma_groups(cv.s, tc, po.group_tiles);
        v = (uint64_t)((cv.s + TRR - 1) / TRR) * ng;
        sl = ng > 1 ? (uint32_t)v : 0;
    } else if (cv.s >= 2) {
        v = (uint64_t)((cv.s + kRowBlock - 1) / kRowBlock) << 32;
    } else if (cv.s == 1) {
        const uint32_t u = a.members[cv.o];
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

// Bitmap items (64 rows) carry the 64-row shape code, so that the staging
// kernels can take clusters and row blocks from either list.
__global__ __launch_bounds__(256) void k_plan_fill(KnnArgs a, PlanOpts po, const uint64_t *off,
                                                   const uint32_t *slot_off, uint64_t *items_m,
                                                   uint64_t *items_b, uint32_t *sbase,
                                                   uint32_t *rb_done, uint32_t *nitems,
                                                   uint32_t *cursors) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) {
        const uint64_t tot = off[a.NE];
        nitems[0] = (uint32_t)tot;
        nitems[1] = (uint32_t)(tot >> 32);
        if (cursors) { cursors[0] = 0; cursors[1] = 0; }
    }
    if (q >= a.NE || q >= a.cl_cfg_off[a.t]) return;
    const uint64_t o0 = off[q], o1 = off[q + 1];
    const uint32_t bm = (uint32_t)o0, nm = (uint32_t)o1 - bm;
    const uint32_t bb = (uint32_t)(o0 >> 32), nbm = (uint32_t)(o1 >> 32) - bb;
    if (nm) {
        const uint32_t s = a.cl_off[q + 1] - a.cl_off[q];
        const uint32_t tc = tile_code(s, po.t32, po.t64);
        const uint32_t ng = mfma_groups(s, tc, po.group_tiles), nrb = nm / ng;
        sbase[q] = slot_off[q];
        for (uint32_t r = 0; r < nrb; ++r) {
            for (uint32_t g = 0; g < ng; ++g) items_m[bm + g * nrb + r] = mfma_item_code(q, r, tc, g, ng);
            if (ng > 1) rb_done[slot_off[q] + r * ng] = 0;
        }
    }
    for (uint32_t r = 0; r < nbm; ++r) items_b[bb + r] = mfma_item_code(q, r, 1, 0, 1);
}

// Batched planning without a sort.  The work items of the MFMA path fall into
// cost classes by the work an item covers (column tiles times tile area, on a
// log scale: more work = lower class index = taken first, the size-ordered
// queue of Section II-F).  Each cluster takes a contiguous range inside its
// class by an atomic on the class counter, and scratch slots (split row
// blocks) and bitmap items by atomics on their counters; k_lens cleared the
// counters.  Positions come from per-block counts in LDS, then one global
// atomic per (block, counter).  The order of clusters inside a class changes
// only the schedule, never a result.
__global__ __launch_bounds__(256) void k_plan_classes(KnnArgs a, PlanOpts po, const uint32_t *bmax,
                                                      uint32_t nbmax, uint32_t *pc, uint32_t *ccls,
                                                      uint32_t *cpos, uint32_t *sbase) {
    __shared__ uint32_t lcnt[kPlanCtr], lbase[kPlanCtr];
    for (uint32_t q = threadIdx.x; q < kPlanCtr; q += blockDim.x) lcnt[q] = 0;
    // (block_max_len begins with a barrier, which also orders the zeroing)
    uint32_t mfma_min = po.mfma_min;
    if (block_max_len(bmax, nbmax) >= kMfmaMaxLen) mfma_min = 0xFFFFFFFFu;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = c < a.NE && c < a.cl_cfg_off[a.t];
    uint32_t cls = 0xFFFFFFFFu, ctr = 0, lpos = 0, lslot = 0;
    bool split = false;
    if (live) {
        const ClusterView cv = view(a, c);
        if (cv.s >= mfma_min && cv.s >= 2) {
            const uint32_t tc = tile_code(cv.s, po.t32, po.t64);
            const uint32_t TRR = shape_rows(tc), TRC = shape_cols(tc);
            const uint32_t ng = mfma_groups(cv.s, tc, po.group_tiles);
            const uint32_t tiles = (cv.s + TRC - 1) / TRC, per = (tiles + ng - 1) / ng;
            const uint32_t nit = ((cv.s + TRR - 1) / TRR) * ng;
            // work of one item in 32 x 32 blocks: per * (TRR / 32) * (TRC / 32), log scale
            const uint32_t work = per * (TRR / 32) * (TRC / 32);
            const uint32_t lv = 4 * bit_width_dev(work);
            cls = kCostClasses - 1 - (lv < kCostClasses - 1 ? lv : kCostClasses - 1);
            ctr = cls;
            lpos = atomicAdd(&lcnt[cls], nit);
            split = ng > 1;
            if (split) lslot = atomicAdd(&lcnt[kSlotCtr], nit);
        } else if (cv.s >= 2) {
            cls = kCostClasses;
            ctr = kBitmapCtr;
            lpos = atomicAdd(&lcnt[kBitmapCtr], (cv.s + kRowBlock - 1) / kRowBlock);
        } else if (cv.s == 1) {
            const uint32_t u = a.members[cv.o];
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

__global__ __launch_bounds__(256) void k_plan_items(KnnArgs a, PlanOpts po, const uint32_t *pc,
                                                    const uint32_t *ccls, const uint32_t *cpos,
                                                    const uint32_t *sbase, uint64_t *items_m,
                                                    uint64_t *items_b, uint32_t *rb_done,
                                                    uint32_t *nitems, uint32_t *cursors) {
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
        const uint32_t tc = tile_code(s, po.t32, po.t64), TRR = shape_rows(tc);
        const uint32_t ng = mfma_groups(s, tc, po.group_tiles), nrb = (s + TRR - 1) / TRR;
        const uint32_t b0 = cbase[cls] + cpos[c];
        for (uint32_t r = 0; r < nrb; ++r) {
            for (uint32_t g = 0; g < ng; ++g) items_m[b0 + g * nrb + r] = mfma_item_code(c, r, tc, g, ng);
            if (ng > 1) rb_done[sbase[c] + r * ng] = 0;
        }
    } else if (cls == kCostClasses) {
        const uint32_t s = a.cl_off[c + 1] - a.cl_off[c];
        const uint32_t nrb = (s + kRowBlock - 1) / kRowBlock;
        for (uint32_t r = 0; r < nrb; ++r) items_b[cpos[c] + r] = mfma_item_code(c, r, 1, 0, 1);
    }
}

// ------------------------------------------------------- full rows (Hyrec)

// rows[u][w]: bit (i & 31) of word i >> 5 is set iff item i is in P_u, rows
// padded to W words; one wave per user, the row assembled in LDS and written
// out whole.  Used by the Hyrec branch of Algorithm 2.
__global__ __launch_bounds__(256) void k_user_bits(const int64_t *__restrict__ indptr,
                                                   const uint32_t *__restrict__ indices,
                                                   uint64_t nnz, uint32_t n, uint32_t m,
                                                   uint32_t W, uint32_t *__restrict__ rows) {
    extern __shared__ uint32_t lds[];
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t *rb = lds + wid * W;
    for (uint32_t u = blockIdx.x * nw + wid; u < n; u += gridDim.x * nw) {
        uint64_t p0, p1;
        row_range(indptr, u, nnz, p0, p1);
        for (uint32_t w = lane; w < W; w += 64) rb[w] = 0;
        wave_sync();
        for (uint64_t p = p0 + lane; p < p1; p += 64) {
            const uint32_t i = indices[p];
            if (i < m) atomicOr(&rb[i >> 5], 1u << (i & 31));
        }
        wave_sync();
        uint32_t *out = rows + (size_t)u * W;
        for (uint32_t w = lane; w < W; w += 64) out[w] = rb[w];
        wave_sync();
    }
}

uint32_t full_row_words(uint32_t m) { return 8 * (uint32_t)div_up(m, 256); }

hipError_t launch_user_bits(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                            uint32_t n, uint32_t m, uint32_t *rows, hipStream_t s) {
    const uint32_t W = full_row_words(m);
    uint32_t nw = (uint32_t)((160 * 1024) / ((size_t)4 * W));
    nw = nw > 4 ? 4 : nw;
    if (nw == 0) return hipErrorInvalidValue;
    const size_t lds = (size_t)4 * nw * W;
    hipError_t e = hipFuncSetAttribute((const void *)k_user_bits,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const uint64_t want = div_up(n, nw);
    const uint32_t grid = (uint32_t)(want < kLensGrid ? want : kLensGrid);
    hipLaunchKernelGGL(k_user_bits, dim3(grid), dim3(64 * nw), lds, s, indptr, indices, nnz, n, m,
                       W, rows);
    return hipGetLastError();
}

// --------------------------------------------------------------- host side

// Scratch slots of split row blocks: a cluster is split only when it spans
// more than one column tile of 128 (s > 128, 64-row blocks), and then takes
// ceil(s/64) * ng <= (s/64 + 1) * 4 < s/8 slots.
size_t knn_max_slots(uint32_t NE) { return (size_t)NE / 8 + 8; }

// Map slots: clusters of more than kBigS members.
static size_t knn_max_maps(uint32_t NE) { return (size_t)NE / (kBigS + 1) + 1; }
// Entries of the row list: at least two 32-row units each, so at most
// ceil(units / 2) <= s / 64 + 2 per cluster.
static size_t knn_max_row_entries(uint32_t NE) { return (size_t)NE / 64 + 2 * knn_max_maps(NE) + 16; }

size_t knn_ws_fixed(uint32_t n, uint32_t NE, uint32_t m, KnnWs *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    KnnWs x;
    x.rlen = take(4 * ((size_t)n + 1));
    x.cnt = take(8 * ((size_t)NE + 1));
    x.items_m = take(8 * ((size_t)NE + NE / 16 + 64));
    x.slots = take(4 * ((size_t)NE + 1));
    x.sbase = take(4 * (size_t)NE);
    const size_t nslot = knn_max_slots(NE);
    x.rb_done = take(4 * nslot);
    x.items_b = take(8 * (size_t)NE);
    x.ctmp = take(8 * scan_tmp_elems(NE + 1));
    x.htmp = take(4 * scan_tmp_elems(NE + 1));
    x.ctr = take(4 * 16);
    x.bmax = take(4 * kLensGrid);
    x.pc = take(4 * kPlanCtr);
    x.ccls = take(4 * (size_t)NE);
    x.cpos = take(4 * (size_t)NE);
    x.cw = take(4 * (size_t)NE);
    x.coff = take(8 * (size_t)NE);
    x.ccur = take(16);
    x.dslot = take(4 * (size_t)NE);
    x.dmap = take((size_t)4 * 2 * dict_words(m) * knn_max_maps(NE));
    x.rlist = take(8 * knn_max_row_entries(NE));
    x.store = off;
    x.total = off;
    if (w) *w = x;
    return off;
}

// Default room for the store: the scratch of split row blocks, taken as one
// slot of 64 rows x 32 keys (u64) per 64 slots of the partition (the slots a
// partition needs when its clusters above 2048 members hold half the slots),
// and the dictionary rows of every cluster, where a member's row over its
// cluster's dictionary takes about 4 words per profile item on the workloads
// measured, plus the row padding (8 words at least per row, 32-row blocks),
// capped by the rows over the whole item universe.  A partition that needs
// more is reported (c2_local_knn, header bytes 8..15).
size_t knn_store_default_bytes(uint32_t n, uint32_t NE, uint32_t m, uint64_t nnz, uint32_t t) {
    const double tnnz = (double)nnz * t;
    double words = 4.0 * tnnz + 16.0 * NE + 8192.0;
    const double full = ((double)NE + 31.0 * NE / 2.0) * full_row_words(m);
    if (words > full) words = full;
    words += (double)NE / 64.0 * kRows * kMaxK * 2.0;
    (void)n;
    return ((size_t)words > 1024 ? (size_t)words : 1024) * 4;  // 4 KiB at least
}

static uint32_t lens_grid(uint32_t n) {
    const uint32_t grid = (uint32_t)div_up((uint64_t)n, 256);
    return grid < kLensGrid ? (grid ? grid : 1) : kLensGrid;
}

static PlanOpts plan_opts(const KnnOpts &o) {
    PlanOpts po;
    po.mfma_min = o.mfma_min ? o.mfma_min : kDefaultMfmaMin;
    po.group_tiles = o.group_tiles ? o.group_tiles : kGroupTiles;
    po.t32 = o.tile32_max ? o.tile32_max : kDefaultTile32;
    po.t64 = o.tile64_max ? o.tile64_max : kDefaultTile64;
    if (po.t64 < po.t32) po.t64 = po.t32;
    return po;
}

static hipError_t lens(const KnnArgs &a, const KnnPtrs &w, hipStream_t s) {
    hipLaunchKernelGGL(k_lens, dim3(lens_grid(a.n)), dim3(256), 0, s, a.indptr, a.nnz, a.n,
                       w.rlen, w.bmax, w.pc);
    return hipGetLastError();
}

static size_t stage_lds(uint32_t Wm) { return ((size_t)win_offset(Wm) + 32 * kWinStride) * 4; }

static StageArgs stage_args(const KnnArgs &a, const KnnPtrs &w) {
    StageArgs st;
    st.bits = w.store;
    st.cap = w.store_words;
    st.cw = w.cw;
    st.coff = w.coff;
    st.ccur = w.ccur;
    st.cnext = w.ctr + 4;
    st.rnext = w.ctr + 5;
    st.dslot = w.dslot;
    st.dmap = w.dmap;
    st.dcur = w.ctr + 6;
    st.rlist = w.rlist;
    st.rcount = w.ctr + 9;
    // entries of 8 units (256 rows) when the partition gives every staging
    // block many of them, down to one 64-row block on small inputs
    const uint32_t per_block = (uint32_t)((uint64_t)a.NE / 32 / kStageGrid / 8);
    st.row_units = per_block >= 8 ? 8u : per_block >= 4 ? 4u : 2u;
    // the same for k_dict's claims: one item at a time on small inputs, where
    // one block per cluster keeps the largest clusters apart, up to 64
    const uint32_t claim = (uint32_t)((uint64_t)a.NE / kStageGrid / 256);
    st.claim = claim >= 64 ? 64u : claim >= 16 ? 16u : claim >= 4 ? 4u : 1u;
    st.status = w.status;
    return st;
}

// The store begins with the scratch of the split row blocks (nslots slots of
// kRows x k keys, u64): the cursor of the dictionary rows starts past it, so
// that a scratch larger than the store fails every cluster's allocation.
__global__ void k_store_init(unsigned long long *ccur, const uint32_t *nslots, uint32_t slot_words) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const unsigned long long w = (unsigned long long)(*nslots) * slot_words;
        ccur[0] = (w + 63ull) & ~63ull;
    }
}

// Staging of every cluster with >= 2 members, from the work lists the plan
// wrote (the MFMA list, then the bitmap list; both start with each cluster's
// first item).  nslots: the plan's count of scratch slots.
static hipError_t stage(const KnnArgs &a, const KnnPtrs &w, const uint32_t *nslots, hipStream_t s) {
    const size_t lds = stage_lds(a.Wm);
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)k_dict, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void *)k_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds)) != hipSuccess)
        return e;
    // allocation cursor (u64, past the scratch); the cursors of k_dict (both
    // lists), of k_rows, of the map slots and the row list's count (ctr 4..9)
    hipLaunchKernelGGL(k_store_init, dim3(1), dim3(64), 0, s, w.ccur, nslots, kRows * a.k * 2);
    if ((e = launch_fill_u32(w.ctr + 4, 0, 6, s)) != hipSuccess) return e;
    const StageArgs st = stage_args(a, w);
    hipLaunchKernelGGL(k_dict, dim3(kStageGrid), dim3(kStageThreads), lds, s, a, w.items_m, w.ctr, st);
    // clusters on the bitmap path
    StageArgs sb = st;
    sb.cnext = w.ctr + 7;
    hipLaunchKernelGGL(k_dict, dim3(kStageGrid / 4), dim3(kStageThreads), lds, s, a, w.items_b,
                       w.ctr + 1, sb);
    // the rows of the big clusters of both lists
    hipLaunchKernelGGL(k_rows, dim3(kStageGrid), dim3(kStageThreads), lds, s, a, st);
    return hipGetLastError();
}

static hipError_t launch_paths(const KnnArgs &a, const KnnPtrs &w, const KnnOpts &o,
                               uint32_t grid_m, uint32_t grid_b, bool batched, hipStream_t s) {
    hipError_t e;
    StoreView sv;
    sv.bits = w.store;
    sv.cw = w.cw;
    sv.coff = w.coff;
    MfmaScratch sc;
    sc.keys = reinterpret_cast<uint64_t *>(w.store);
    sc.rb_done = w.rb_done;
    sc.sbase = w.sbase;
    // the events bracket the MFMA kernel, which carries the large clusters
    if (o.ev_begin && (e = hipEventRecord(o.ev_begin, s)) != hipSuccess) return e;
    if (grid_m)
        hipLaunchKernelGGL(k_knn_mfma, dim3((uint32_t)div_up(grid_m, 4)), dim3(256), 0, s, a, sv,
                           w.rlen, sc, w.items_m, w.ctr, batched ? w.ctr + 2 : nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (o.ev_end && (e = hipEventRecord(o.ev_end, s)) != hipSuccess) return e;
    if (grid_b)
        hipLaunchKernelGGL(k_knn_bitmap, dim3(grid_b), dim3(64), 0, s, a, sv, w.rlen, w.items_b,
                           w.ctr + 1, batched ? w.ctr + 3 : nullptr);
    return hipGetLastError();
}

hipError_t knn_plain(const KnnArgs &a, const KnnPtrs &w, const KnnOpts &o, hipStream_t s) {
    hipError_t e = lens(a, w, s);
    if (e != hipSuccess) return e;
    const PlanOpts po = plan_opts(o);
    const dim3 g((uint32_t)div_up(a.NE, 256));
    hipLaunchKernelGGL(k_plan_count, g, dim3(256), 0, s, a, po, w.bmax, lens_grid(a.n), w.cnt,
                       w.slots);
    if ((e = scan_u64(w.cnt, w.cnt, a.NE, w.ctmp, s)) != hipSuccess) return e;
    if ((e = scan_u32(w.slots, w.slots, a.NE, w.htmp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_fill, g, dim3(256), 0, s, a, po, w.cnt, w.slots, w.items_m,
                       w.items_b, w.sbase, w.rb_done, w.ctr, nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_fill_u32(w.status, 0, 1, s)) != hipSuccess) return e;
    if ((e = stage(a, w, w.slots + a.NE, s)) != hipSuccess) return e;
    uint32_t n[3] = {0, 0, 0};
    e = hipMemcpyAsync(n, w.ctr, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(n + 2, w.status, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (n[2]) return hipErrorOutOfMemory;  // the store is too small (*ccur: the words needed)
    return launch_paths(a, w, o, n[0], n[1], false, s);
}

hipError_t knn_batched(const KnnArgs &a, const KnnPtrs &w, const KnnOpts &o, hipStream_t s) {
    hipError_t e = lens(a, w, s);
    if (e != hipSuccess) return e;
    // items by cost class, costliest first (the size-ordered queue of
    // Section II-F), without a sort
    const PlanOpts po = plan_opts(o);
    const dim3 g((uint32_t)div_up(a.NE, 256));
    hipLaunchKernelGGL(k_plan_classes, g, dim3(256), 0, s, a, po, w.bmax, lens_grid(a.n), w.pc,
                       w.ccls, w.cpos, w.sbase);
    hipLaunchKernelGGL(k_plan_items, g, dim3(256), 0, s, a, po, w.pc, w.ccls, w.cpos, w.sbase,
                       w.items_m, w.items_b, w.rb_done, w.ctr, w.ctr + 2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_fill_u32(w.status, 0, 1, s)) != hipSuccess) return e;
    // the dictionaries take their clusters from that list, largest first
    if ((e = stage(a, w, w.pc + kSlotCtr, s)) != hipSuccess) return e;
    const uint32_t gm = o.persistent_wgs ? o.persistent_wgs : kDefaultWaves;
    return launch_paths(a, w, o, gm, kBitmapPersistent, true, s);
}

}  // namespace c2
