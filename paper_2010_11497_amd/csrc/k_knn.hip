// Step 2 on the device: exact brute-force KNN inside every cluster
// (Section II-F, Algorithm 2, brute-force branch).
//
// Staging: per cluster, the local dictionary is the set of items held by at
// least two members (an item held once can never be in an intersection);
// each member becomes a bit row over that dictionary, padded to a multiple of
// 64 items.  Intersection sizes |P_u & P_v| are then dot products of bit rows;
// |P_u | P_v| = |P_u| + |P_v| - |P_u & P_v| uses the full profile lengths.
//
// Per-user selection: every member of the row block owns a bounded heap of
// its k best candidates in LDS (worst at the root, exact Jaccard order), and
// offers each candidate that beats the root.
#include "c2_internal.h"
#include "c2_kernels.h"

namespace c2 {

constexpr int kStageThreads = 256;
constexpr int kStageWaves = kStageThreads / 64;
constexpr uint32_t kRowBlock = 64;   // rows (members) per work item
constexpr int kWordChunk = 16;       // bit-row words staged per step

uint32_t knn_wmax(uint32_t m) { return 2 * (uint32_t)div_up(m, 64); }

size_t knn_stage_lds_bytes(uint32_t m, uint32_t wmax) {
    const size_t mw = div_up(m, 32);
    return 4 * (3 * mw + (size_t)kStageWaves * wmax);
}

C2_DEV void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ staging

__global__ __launch_bounds__(kStageThreads) void k_knn_stage(
    const int64_t *__restrict__ indptr, const uint32_t *__restrict__ indices, uint64_t nnz,
    uint32_t n, uint32_t m, uint32_t t, uint32_t k, const uint32_t *__restrict__ members,
    const uint32_t *__restrict__ cl_off, const uint32_t *__restrict__ cl_cfg_off, uint32_t wmax,
    uint32_t *__restrict__ rows, uint32_t *__restrict__ rlen, uint32_t *__restrict__ cl_W,
    uint32_t *__restrict__ part_id, uint32_t *__restrict__ part_I) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t wsum[kStageWaves + 1];
    const uint32_t mw = (m + 31) / 32;
    uint32_t *seen1 = lds, *seen2 = lds + mw, *pref = lds + 2 * mw;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    uint32_t *rb = lds + 3 * mw + wid * wmax;
    const uint32_t ncl = cl_cfg_off[t];
    const uint32_t per = (mw + kStageThreads - 1) / kStageThreads;
    for (uint32_t c = blockIdx.x; c < ncl; c += gridDim.x) {
        const uint32_t o = cl_off[c], s = cl_off[c + 1] - o;
        if (s <= 1) {
            const uint32_t u = s == 1 ? members[o] : n, j = o / n;
            if (u < n && j < t && tid < k) {
                part_id[((size_t)u * t + j) * k + tid] = kPad;
                part_I[((size_t)u * t + j) * k + tid] = 0;
            }
            if (tid == 0) cl_W[c] = 0;
            continue;
        }
        for (uint32_t w = tid; w < mw; w += kStageThreads) seen1[w] = seen2[w] = 0;
        __syncthreads();
        for (uint32_t a = wid; a < s; a += kStageWaves) {
            uint64_t p0, p1;
            row_range(indptr, members[o + a], nnz, p0, p1);
            for (uint64_t p = p0 + lane; p < p1; p += 64) {
                const uint32_t i = indices[p];
                if (i < m) {
                    const uint32_t bit = 1u << (i & 31);
                    if (atomicOr(&seen1[i >> 5], bit) & bit) atomicOr(&seen2[i >> 5], bit);
                }
            }
        }
        __syncthreads();
        // dictionary rank of every twice-seen item: prefix popcount over words
        uint32_t loc = 0;
        for (uint32_t w = tid * per; w < mw && w < (tid + 1) * per; ++w) loc += __popc(seen2[w]);
        uint32_t D;
        uint32_t pre = block_excl_scan<uint32_t, kStageThreads>(loc, wsum, &D);
        for (uint32_t w = tid * per; w < mw && w < (tid + 1) * per; ++w) {
            pref[w] = pre;
            pre += __popc(seen2[w]);
        }
        const uint32_t W = 2 * ((D + 63) / 64);
        if (tid == 0) cl_W[c] = W;
        __syncthreads();
        for (uint32_t a = wid; a < s; a += kStageWaves) {
            const uint32_t u = members[o + a];
            for (uint32_t w = lane; w < W; w += 64) rb[w] = 0;
            wave_sync();
            uint64_t p0, p1;
            row_range(indptr, u, nnz, p0, p1);
            for (uint64_t p = p0 + lane; p < p1; p += 64) {
                const uint32_t i = indices[p];
                if (i < m) {
                    const uint32_t bit = 1u << (i & 31), sw = seen2[i >> 5];
                    if (sw & bit) {
                        const uint32_t li = pref[i >> 5] + __popc(sw & (bit - 1));
                        atomicOr(&rb[li >> 5], 1u << (li & 31));
                    }
                }
            }
            wave_sync();
            uint32_t *out = rows + (size_t)(o + a) * wmax;
            for (uint32_t w = lane; w < W; w += 64) out[w] = rb[w];
            if (lane == 0) rlen[o + a] = (uint32_t)(p1 - p0);
            wave_sync();
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------- selection

// Bounded heap of one row's best candidates, structure-of-arrays in LDS with
// the row's lane as the minor index (conflict-free).  Root = worst kept.
struct RowHeap {
    uint32_t *hI, *hU, *hV;  // [kMaxK][64]
    uint32_t lane, k, cnt;
    uint32_t rI, rU, rV;     // root copy

    C2_DEV void get(uint32_t i, uint32_t &I, uint32_t &U, uint32_t &V) const {
        I = hI[i * 64 + lane];
        U = hU[i * 64 + lane];
        V = hV[i * 64 + lane];
    }
    C2_DEV void put(uint32_t i, uint32_t I, uint32_t U, uint32_t V) {
        hI[i * 64 + lane] = I;
        hU[i * 64 + lane] = U;
        hV[i * 64 + lane] = V;
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
// as a broadcast).

struct BitmapLds {
    uint32_t colw[kRowBlock][kWordChunk];
    uint32_t clen[kRowBlock], cuid[kRowBlock];
    uint32_t hI[kMaxK * 64], hU[kMaxK * 64], hV[kMaxK * 64];
};

C2_DEV void bitmap_item(const KnnArgs &a, const uint32_t *rows, const uint32_t *rlen,
                        const uint32_t *cl_W, uint32_t c, uint32_t rb, BitmapLds &L) {
    const uint32_t lane = threadIdx.x;
    const uint32_t o = a.cl_off[c], s = a.cl_off[c + 1] - o, j = o / a.n;
    const uint32_t W = cl_W[c], wmax = a.wmax;
    const uint32_t ra = rb * kRowBlock + lane;
    const bool active = ra < s;
    const uint32_t Lr = active ? rlen[o + ra] : 0;
    RowHeap h;
    h.hI = L.hI; h.hU = L.hU; h.hV = L.hV;
    h.lane = lane; h.k = a.k; h.cnt = 0; h.rI = 0; h.rU = 1; h.rV = kPad;
    const uint32_t *myrow = rows + (size_t)(o + (active ? ra : 0)) * wmax;
    for (uint32_t cb = 0; cb * kRowBlock < s; ++cb) {
        const uint32_t ci = cb * kRowBlock + lane;
        __syncthreads();
        L.clen[lane] = ci < s ? rlen[o + ci] : 0;
        L.cuid[lane] = ci < s ? a.members[o + ci] : kPad;
        uint32_t acc[kRowBlock];
#pragma unroll
        for (int q = 0; q < (int)kRowBlock; ++q) acc[q] = 0;
        for (uint32_t w0 = 0; w0 < W; w0 += kWordChunk) {
            __syncthreads();
#pragma unroll
            for (int it = 0; it < kWordChunk; ++it) {
                const uint32_t idx = it * 64 + lane;
                const uint32_t cc = idx / kWordChunk, ww = idx % kWordChunk;
                const uint32_t col = cb * kRowBlock + cc;
                L.colw[cc][ww] = (col < s && w0 + ww < W) ? rows[(size_t)(o + col) * wmax + w0 + ww]
                                                          : 0u;
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
        __syncthreads();
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
    const uint32_t u = active ? a.members[o + ra] : a.n;
    if (u < a.n && j < a.t) {
        const size_t base = ((size_t)u * a.t + j) * a.k;
        h.drain(a.part_id + base, a.part_I + base);
    }
}

// Plain form: block b handles items[b].  Batched form: persistent blocks take
// items from a device cursor until the list is exhausted.
__global__ __launch_bounds__(64) void k_knn_bitmap(KnnArgs a, const uint32_t *rows,
                                                   const uint32_t *rlen, const uint32_t *cl_W,
                                                   const uint64_t *items,
                                                   const uint32_t *n_items, uint32_t *cursor) {
    __shared__ BitmapLds L;
    __shared__ uint32_t next;
    const uint32_t total = *n_items;
    if (!cursor) {
        if (blockIdx.x >= total) return;
        const uint64_t it = items[blockIdx.x];
        bitmap_item(a, rows, rlen, cl_W, (uint32_t)(it >> 32), (uint32_t)it, L);
        return;
    }
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) next = atomicAdd(cursor, 1u);
        __syncthreads();
        const uint32_t i = next;
        if (i >= total) break;
        const uint64_t it = items[i];
        bitmap_item(a, rows, rlen, cl_W, (uint32_t)(it >> 32), (uint32_t)it, L);
    }
}

// ---------------------------------------------------------------- planning

// nrb[c] = row blocks of cluster c (0 for clusters with fewer than 2 members).
__global__ __launch_bounds__(256) void k_plan_count(const uint32_t *cl_off,
                                                    const uint32_t *cl_cfg_off, uint32_t t,
                                                    const uint32_t *order, uint32_t NE,
                                                    uint32_t *nrb) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ncl = cl_cfg_off[t];
    if (q >= NE) return;
    if (q >= ncl) { nrb[q] = 0; return; }
    const uint32_t c = order ? order[q] : q;
    const uint32_t s = cl_off[c + 1] - cl_off[c];
    nrb[q] = s >= 2 ? (s + kRowBlock - 1) / kRowBlock : 0;
}

__global__ __launch_bounds__(256) void k_plan_fill(const uint32_t *cl_cfg_off, uint32_t t,
                                                   const uint32_t *order, uint32_t NE,
                                                   const uint32_t *item_off, uint64_t *items,
                                                   uint32_t *cursor) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0 && cursor) *cursor = 0;
    if (q >= NE || q >= cl_cfg_off[t]) return;
    const uint32_t c = order ? order[q] : q;
    const uint32_t b0 = item_off[q], nb = item_off[q + 1] - b0;
    for (uint32_t r = 0; r < nb; ++r) items[b0 + r] = ((uint64_t)c << 32) | r;
}

// Sort keys for the largest-first order: (n - size) so that ascending order
// is descending size, ties by cluster index (stable sort).
__global__ __launch_bounds__(256) void k_plan_keys(const uint32_t *cl_off,
                                                   const uint32_t *cl_cfg_off, uint32_t t,
                                                   uint32_t NE, uint64_t *key, uint32_t *val) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= NE || c >= cl_cfg_off[t]) return;
    const uint32_t s = cl_off[c + 1] - cl_off[c];
    key[c] = (uint64_t)(NE - s);
    val[c] = c;
}

// --------------------------------------------------------------- host side

size_t knn_ws_bytes(uint32_t NE, uint32_t wmax, KnnWs *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    KnnWs x;
    x.rows = take((size_t)4 * NE * wmax);
    x.rlen = take(4 * (size_t)NE);
    x.cl_W = take(4 * (size_t)NE);
    x.nrb = take(4 * ((size_t)NE + 1));
    x.item_off = take(4 * ((size_t)NE + 1));
    x.items = take(8 * (size_t)NE);
    x.csort_key = take(8 * (size_t)NE);
    x.csort_key_alt = take(8 * (size_t)NE);
    x.csort_val = take(4 * (size_t)NE);
    x.csort_val_alt = take(4 * (size_t)NE);
    const size_t hist = radix_hist_elems(NE);
    x.hist = take(4 * hist);
    x.htmp = take(4 * scan_tmp_elems((uint32_t)(hist > NE + 1 ? hist : NE + 1)));
    x.ctr = take(4 * 8);
    x.total = off;
    if (w) *w = x;
    return off;
}

static hipError_t stage(const KnnArgs &a, const KnnPtrs &w, uint32_t grid, hipStream_t s) {
    const size_t lds = knn_stage_lds_bytes(a.m, a.wmax);
    hipError_t e = hipFuncSetAttribute((const void *)k_knn_stage,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_knn_stage, dim3(grid), dim3(kStageThreads), lds, s, a.indptr, a.indices,
                       a.nnz, a.n, a.m, a.t, a.k, a.members, a.cl_off, a.cl_cfg_off, a.wmax,
                       w.rows, w.rlen, w.cl_W, a.part_id, a.part_I);
    return hipGetLastError();
}

hipError_t knn_plain(const KnnArgs &a, const KnnPtrs &w, hipStream_t s) {
    uint32_t ncl = 0;
    hipError_t e = hipMemcpyAsync(&ncl, a.cl_cfg_off + a.t, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (ncl == 0) return hipSuccess;
    if ((e = stage(a, w, ncl < 65535 ? ncl : 65535, s)) != hipSuccess) return e;
    const dim3 g((uint32_t)div_up(a.NE, 256));
    hipLaunchKernelGGL(k_plan_count, g, dim3(256), 0, s, a.cl_off, a.cl_cfg_off, a.t, nullptr,
                       a.NE, w.nrb);
    if ((e = scan_u32(w.nrb, w.item_off, a.NE, w.htmp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_fill, g, dim3(256), 0, s, a.cl_cfg_off, a.t, nullptr, a.NE,
                       w.item_off, w.items, nullptr);
    uint32_t nitems = 0;
    e = hipMemcpyAsync(&nitems, w.item_off + a.NE, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess || nitems == 0) return e;
    hipLaunchKernelGGL(k_knn_bitmap, dim3(nitems), dim3(64), 0, s, a, w.rows, w.rlen, w.cl_W,
                       w.items, w.item_off + a.NE, nullptr);
    return hipGetLastError();
}

hipError_t knn_batched(const KnnArgs &a, const KnnPtrs &w, uint32_t persistent_wgs,
                       hipStream_t s) {
    hipError_t e = stage(a, w, 2048, s);
    if (e != hipSuccess) return e;
    const dim3 g((uint32_t)div_up(a.NE, 256));
    // largest clusters first (the size-ordered queue of Section II-F)
    hipLaunchKernelGGL(k_plan_keys, g, dim3(256), 0, s, a.cl_off, a.cl_cfg_off, a.t, a.NE,
                       w.csort_key, w.csort_val);
    bool in_alt = false;
    e = radix_sort(w.csort_key, w.csort_val, w.csort_key_alt, w.csort_val_alt, a.cl_cfg_off + a.t,
                   a.NE, bit_width(a.NE), w.hist, w.htmp, &in_alt, s);
    if (e != hipSuccess) return e;
    const uint32_t *order = in_alt ? w.csort_val_alt : w.csort_val;
    hipLaunchKernelGGL(k_plan_count, g, dim3(256), 0, s, a.cl_off, a.cl_cfg_off, a.t, order, a.NE,
                       w.nrb);
    if ((e = scan_u32(w.nrb, w.item_off, a.NE, w.htmp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_fill, g, dim3(256), 0, s, a.cl_cfg_off, a.t, order, a.NE,
                       w.item_off, w.items, w.ctr);
    const uint32_t grid = persistent_wgs ? persistent_wgs : 2048;
    hipLaunchKernelGGL(k_knn_bitmap, dim3(grid), dim3(64), 0, s, a, w.rows, w.rlen, w.cl_W,
                       w.items, w.item_off + a.NE, w.ctr);
    return hipGetLastError();
}

}  // namespace c2
