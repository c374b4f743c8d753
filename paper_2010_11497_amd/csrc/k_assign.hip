// Learned cluster assigner: an embedding bag over the user's items and a
// two-layer MLP whose output is one bucket per hash configuration.  It takes
// the place of FastRandomHash's top-level grouping; FastRandomHash stays the
// fallback (low-confidence users, and the split of oversized groups).
//
//   e_u   = mean_{i in P_u} E[i]             E bf16 [m][64], fp32 sum, -> bf16
//   h_u   = ReLU(W1 e_u + b1)                W1 bf16 [256][64], b1 fp32, -> bf16
//   z_u   = W2 h_u + b2                      W2 bf16 [t*b][256], b2 fp32, fp32
//   key_j = argmax_{c < b} z_u[j*b + c]      lowest index on ties
//   gap_j = top-1 minus top-2 logit of head j
//
// k_assign_hidden: one wave per user (8 item rows per gather), W1 staged
//                  (transposed, fp32) in LDS.
// k_assign_keys:   the logits as a bf16 MFMA product (32x32x16), buckets as
//                  the M dimension and users as N, the per-head argmax fused
//                  into the epilogue, so the n x t*b logits never reach HBM.
// k_embag_fwd/bwd: the embedding bag alone in fp32, for training.
#include "c2_internal.h"
#include "c2_kernels.h"

namespace c2 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

C2_DEV float bf16_to_f32(uint16_t x) { return __uint_as_float((uint32_t)x << 16); }

// round to nearest even (finite inputs)
C2_DEV uint16_t f32_to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Sum of E rows over the items of row u with wide gathers: lane = 8 * g + d8
// loads dimensions [8*d8, 8*d8+8) of every 8th item (g = 0..7), so one load
// instruction brings in 8 item rows; the 8 partial sums per dimension are
// then added across g.
// Returns the count; lane l receives the sum of dimension l in `sum`.
C2_DEV uint32_t bag_sum_wide(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                             uint32_t m, const uint16_t *E, uint32_t u, int lane, float &sum) {
    uint64_t a, e;
    row_range(indptr, u, nnz, a, e);
    const int g = lane >> 3, d8 = lane & 7;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (uint64_t c = a; c < e; c += 64) {
        const uint32_t cnt = (uint32_t)(e - c < 64 ? e - c : 64);
        const uint32_t mine = (uint32_t)lane < cnt ? indices[c + lane] : 0xFFFFFFFFu;
        for (uint32_t q = 0; q < cnt; q += 8) {
            const uint32_t i = __shfl(mine, (int)(q + g));
            if (q + g < cnt && i < m) {
                const uint4 v = *reinterpret_cast<const uint4 *>(E + (size_t)i * kAsgDim + 8 * d8);
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    acc[2 * x] += __uint_as_float(w[x] << 16);
                    acc[2 * x + 1] += __uint_as_float(w[x] & 0xFFFF0000u);
                }
            }
        }
    }
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        acc[x] += __shfl_xor(acc[x], 8);
        acc[x] += __shfl_xor(acc[x], 16);
        acc[x] += __shfl_xor(acc[x], 32);
    }
    // lane l wants dimension l = 8 * d8' + x': held (after the reduction) by
    // every lane with d8 == l / 8, in acc[l % 8]
    float r = 0.f;
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        const float y = __shfl(acc[x], lane >> 3);
        r = (lane & 7) == x ? y : r;
    }
    sum = r;
    return (uint32_t)(e - a);
}

constexpr int kHidWaves = 8;

__global__ __launch_bounds__(64 * kHidWaves) void k_assign_hidden(
    const int64_t *__restrict__ indptr, const uint32_t *__restrict__ indices, uint64_t nnz,
    uint32_t n, uint32_t m, const uint16_t *__restrict__ E, const uint16_t *__restrict__ W1,
    const float *__restrict__ b1, uint16_t *__restrict__ h) {
    __shared__ float w1t[kAsgDim][kAsgHidden];
    for (uint32_t x = threadIdx.x; x < kAsgDim * kAsgHidden; x += 64 * kHidWaves) {
        const uint32_t o = x / kAsgDim, k = x % kAsgDim;
        w1t[k][o] = bf16_to_f32(W1[x]);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    float bias[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) bias[q] = b1[lane + 64 * q];
    for (uint32_t u = blockIdx.x * kHidWaves + wid; u < n; u += gridDim.x * kHidWaves) {
        float s;
        const uint32_t len = bag_sum_wide(indptr, indices, nnz, m, E, u, lane, s);
        const float eu = bf16_to_f32(f32_to_bf16(len ? s / (float)len : 0.f));
        float acc[4] = {bias[0], bias[1], bias[2], bias[3]};
#pragma unroll 16
        for (int k = 0; k < kAsgDim; ++k) {
            const float ek = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(eu), k));
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = fmaf(w1t[k][lane + 64 * q], ek, acc[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            h[(size_t)u * kAsgHidden + lane + 64 * q] = f32_to_bf16(acc[q] > 0.f ? acc[q] : 0.f);
    }
}

// ---------------------------------------------------------------- logits

constexpr int kKeyWaves = 8;
constexpr int kKeyUsers = 64 * kKeyWaves;  // 64 users (two 32-column blocks) per wave
constexpr int kTileB = 64;                 // buckets per tile (two MFMA row blocks)
constexpr int kRowPad = kAsgHidden + 8;    // bf16 per LDS row (breaks bank aliasing)
constexpr int kSteps = kAsgHidden / 16;    // MFMA k-steps per tile
constexpr int kTileChunks = kTileB * kAsgHidden / 8;             // 16-byte chunks per tile
constexpr int kChunksPerThread = kTileChunks / (64 * kKeyWaves);  // 4

struct Best {
    float v1, v2;
    uint32_t idx;
};

C2_DEV void best_reset(Best &b) {
    b.v1 = -__builtin_huge_valf();
    b.v2 = -__builtin_huge_valf();
    b.idx = 0xFFFFFFFFu;
}

// buckets arrive in ascending order per lane: strict '>' keeps the lowest
template <bool kSecond>
C2_DEV void best_push(Best &b, float v, uint32_t c) {
    if constexpr (kSecond) {
        if (v > b.v1) {
            b.v2 = b.v1;
            b.v1 = v;
            b.idx = c;
        } else if (v > b.v2) {
            b.v2 = v;
        }
    } else {
        const bool gt = v > b.v1;
        b.v1 = gt ? v : b.v1;
        b.idx = gt ? c : b.idx;
    }
}

// lanes l and l^32 hold the same user over disjoint bucket sets
C2_DEV void best_combine(Best &b) {
    const float o1 = __shfl_xor(b.v1, 32), o2 = __shfl_xor(b.v2, 32);
    const uint32_t oi = __shfl_xor(b.idx, 32);
    if (o1 > b.v1) {
        b.v2 = fmaxf(o2, b.v1);
        b.v1 = o1;
        b.idx = oi;
    } else if (o1 == b.v1) {
        b.v2 = b.v1;
        b.idx = oi < b.idx ? oi : b.idx;
    } else {
        b.v2 = fmaxf(b.v2, o1);
    }
}

// kSecond: also track the runner-up (for the gap output or the fallback)
template <bool kSecond>
__global__ __launch_bounds__(64 * kKeyWaves) void k_assign_keys(
    const uint16_t *__restrict__ h, uint32_t n, const uint16_t *__restrict__ W2,
    const float *__restrict__ b2, uint32_t t, uint32_t b, const uint32_t *__restrict__ frh,
    float min_gap, uint32_t *__restrict__ keys, float *__restrict__ gap) {
    __shared__ __attribute__((aligned(16))) uint16_t wt[2][kTileB * kRowPad];
    __shared__ float bt[2][kTileB];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t ubase = blockIdx.x * kKeyUsers + wid * 64;
    const int half = lane >> 5, col = lane & 31;

    // this wave's users as MFMA B fragments: B[k][j] = h[user j][k]
    bf16x8 bf[2][kSteps];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const uint32_t u = ubase + c * 32 + col;
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
            uint4 v = make_uint4(0, 0, 0, 0);
            if (u < n)
                v = *reinterpret_cast<const uint4 *>(h + (size_t)u * kAsgHidden + 16 * s + 8 * half);
            bf[c][s] = __builtin_bit_cast(bf16x8, v);
        }
    }

    const uint32_t tiles_per_head = b / kTileB;
    const uint32_t ntiles = t * tiles_per_head;
    // cooperative tile load: 64 rows x 512 B in 16-byte chunks, four per
    // thread, held in named registers between the load and the LDS store
    static_assert(kChunksPerThread == 4, "four chunks per thread");
    const uint32_t q0 = threadIdx.x, qs = 64 * kKeyWaves;
    const uint32_t g0 = (q0 / 32) * kAsgHidden + (q0 % 32) * 8;  // element offset in the tile
    const uint32_t gs = (qs / 32) * kAsgHidden;                    // step between a thread's chunks
    const uint32_t l0 = (q0 / 32) * kRowPad + (q0 % 32) * 8;
    const uint32_t ls = (qs / 32) * kRowPad;
    uint4 p0, p1, p2, p3;
    float pbias = 0.f;
#define C2_LOAD_TILE(T)                                                                        \
    do {                                                                                       \
        const uint16_t *src_ = W2 + (size_t)(T) * kTileB * kAsgHidden + g0;                    \
        p0 = *reinterpret_cast<const uint4 *>(src_);                                           \
        p1 = *reinterpret_cast<const uint4 *>(src_ + gs);                                      \
        p2 = *reinterpret_cast<const uint4 *>(src_ + 2 * gs);                                  \
        p3 = *reinterpret_cast<const uint4 *>(src_ + 3 * gs);                                  \
        pbias = threadIdx.x < kTileB ? b2[(size_t)(T) * kTileB + threadIdx.x] : 0.f;           \
    } while (0)
#define C2_STORE_TILE(BUF)                                                                     \
    do {                                                                                       \
        uint16_t *dst_ = &wt[BUF][l0];                                                         \
        *reinterpret_cast<uint4 *>(dst_) = p0;                                                 \
        *reinterpret_cast<uint4 *>(dst_ + ls) = p1;                                            \
        *reinterpret_cast<uint4 *>(dst_ + 2 * ls) = p2;                                        \
        *reinterpret_cast<uint4 *>(dst_ + 3 * ls) = p3;                                        \
        if (threadIdx.x < kTileB) bt[BUF][threadIdx.x] = pbias;                                \
    } while (0)

    C2_LOAD_TILE(0);
    C2_STORE_TILE(0);
    __syncthreads();

    Best best[2];
    best_reset(best[0]);
    best_reset(best[1]);
    for (uint32_t T = 0; T < ntiles; ++T) {
        const int buf = T & 1;
        if (T + 1 < ntiles) C2_LOAD_TILE(T + 1);
        // accumulators start at the bias of their bucket row
        f32x16 acc[2][2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float bias = bt[buf][32 * rb + 8 * (r / 4) + 4 * half + (r % 4)];
                acc[rb][0][r] = bias;
                acc[rb][1][r] = bias;
            }
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const bf16x8 a = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const uint4 *>(
                                &wt[buf][(32 * rb + col) * kRowPad + 8 * half + 16 * s]));
                acc[rb][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bf[0][s], acc[rb][0], 0, 0, 0);
                acc[rb][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bf[1][s], acc[rb][1], 0, 0, 0);
            }
        }
        const uint32_t tin = T % tiles_per_head;
        if constexpr (kSecond) {
            // a group whose maximum does not beat the runner-up changes nothing
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    const f32x16 &v = acc[rb][cb];
                    float mx = fmaxf(fmaxf(v[0], v[1]), v[2]);
#pragma unroll
                    for (int r = 3; r < 15; r += 2) mx = fmaxf(fmaxf(mx, v[r]), v[r + 1]);
                    mx = fmaxf(mx, v[15]);
                    if (mx > best[cb].v2) {
#pragma unroll
                        for (int r = 0; r < 16; ++r)
                            best_push<true>(best[cb], v[r],
                                            tin * kTileB + 32 * rb + 8 * (r / 4) + 4 * half + (r % 4));
                    }
                }
        } else {
            // the lane's 16 values of a row block rarely hold a new maximum once
            // a few tiles have passed: take their maximum first, and search for
            // the first (lowest) bucket holding it only when it beats the best
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    const f32x16 &v = acc[rb][cb];
                    float mx = fmaxf(fmaxf(v[0], v[1]), v[2]);
#pragma unroll
                    for (int r = 3; r < 15; r += 2) mx = fmaxf(fmaxf(mx, v[r]), v[r + 1]);
                    mx = fmaxf(mx, v[15]);
                    if (mx > best[cb].v1) {
                        int first = 15;
#pragma unroll
                        for (int r = 14; r >= 0; --r) first = v[r] == mx ? r : first;
                        best[cb].v1 = mx;
                        best[cb].idx = tin * kTileB + 32 * rb + 8 * (first / 4) + 4 * half + (first % 4);
                    }
                }
        }
        if (tin == tiles_per_head - 1) {
            const uint32_t j = T / tiles_per_head;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                best_combine(best[c]);
                const uint32_t u = ubase + c * 32 + col;
                if (half == 0 && u < n) {
                    uint32_t key = best[c].idx;
                    if constexpr (kSecond) {
                        const float g = best[c].v1 - best[c].v2;
                        if (frh && g < min_gap) key = b + frh[(size_t)j * n + u];
                        if (gap) gap[(size_t)j * n + u] = g;
                    }
                    keys[(size_t)j * n + u] = key;
                }
                best_reset(best[c]);
            }
        }
        // buf ^ 1 was last read before the previous barrier: store the next
        // tile there, then one barrier publishes it and retires buf
        if (T + 1 < ntiles) C2_STORE_TILE(buf ^ 1);
        __syncthreads();
    }
#undef C2_LOAD_TILE
#undef C2_STORE_TILE
}

// -------------------------------------------------------------- training

__global__ __launch_bounds__(256) void k_embag_fwd(const int64_t *__restrict__ indptr,
                                                   const uint32_t *__restrict__ indices,
                                                   uint64_t nnz, uint32_t n, uint32_t m,
                                                   const uint32_t *__restrict__ rows,
                                                   uint32_t nrows, const uint16_t *__restrict__ E,
                                                   float *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const uint32_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nrows) return;
    const uint32_t u = rows ? rows[r] : r;
    float s = 0.f;
    uint32_t len = 0;
    if (u < n) len = bag_sum_wide(indptr, indices, nnz, m, E, u, lane, s);
    out[(size_t)r * kAsgDim + lane] = len ? s / (float)len : 0.f;
}

__global__ __launch_bounds__(256) void k_embag_bwd(const int64_t *__restrict__ indptr,
                                                   const uint32_t *__restrict__ indices,
                                                   uint64_t nnz, uint32_t n, uint32_t m,
                                                   const uint32_t *__restrict__ rows,
                                                   uint32_t nrows, const float *__restrict__ grad,
                                                   float *__restrict__ dE) {
    const int lane = threadIdx.x & 63;
    const uint32_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nrows) return;
    const uint32_t u = rows ? rows[r] : r;
    if (u >= n) return;
    uint64_t a, e;
    row_range(indptr, u, nnz, a, e);
    if (e == a) return;
    const float g = grad[(size_t)r * kAsgDim + lane] / (float)(e - a);
    for (uint64_t p = a; p < e; ++p) {
        const uint32_t i = indices[p];
        if (i < m) atomicAdd(&dE[(size_t)i * kAsgDim + lane], g);
    }
}

// ------------------------------------------------------------------ host

hipError_t launch_assign_hidden(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                                uint32_t n, uint32_t m, const uint16_t *E, const uint16_t *W1,
                                const float *b1, uint16_t *h, hipStream_t s) {
    uint32_t blocks = (uint32_t)div_up(n, kHidWaves);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_assign_hidden, dim3(blocks), dim3(64 * kHidWaves), 0, s, indptr, indices,
                       nnz, n, m, E, W1, b1, h);
    return hipGetLastError();
}

hipError_t launch_assign_keys(const uint16_t *h, uint32_t n, const uint16_t *W2, const float *b2,
                              uint32_t t, uint32_t b, const uint32_t *frh, float min_gap,
                              uint32_t *keys, float *gap, hipStream_t s) {
    const dim3 grid((uint32_t)div_up(n, kKeyUsers)), block(64 * kKeyWaves);
    if (frh || gap)
        hipLaunchKernelGGL(k_assign_keys<true>, grid, block, 0, s, h, n, W2, b2, t, b, frh,
                           min_gap, keys, gap);
    else
        hipLaunchKernelGGL(k_assign_keys<false>, grid, block, 0, s, h, n, W2, b2, t, b, frh,
                           min_gap, keys, gap);
    return hipGetLastError();
}

hipError_t launch_embag(const int64_t *indptr, const uint32_t *indices, uint64_t nnz, uint32_t n,
                        uint32_t m, const uint32_t *rows, uint32_t nrows, const uint16_t *E,
                        float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_embag_fwd, dim3((uint32_t)div_up(nrows, 4)), dim3(256), 0, s, indptr,
                       indices, nnz, n, m, rows, nrows, E, out);
    return hipGetLastError();
}

hipError_t launch_embag_backward(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                                 uint32_t n, uint32_t m, const uint32_t *rows, uint32_t nrows,
                                 const float *grad, float *dE, hipStream_t s) {
    hipLaunchKernelGGL(k_embag_bwd, dim3((uint32_t)div_up(nrows, 4)), dim3(256), 0, s, indptr,
                       indices, nnz, n, m, rows, nrows, grad, dE);
    return hipGetLastError();
}

}  // namespace c2
