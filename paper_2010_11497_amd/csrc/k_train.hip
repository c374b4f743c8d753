// Training step of the learned cluster assigner: forward, loss and gradients
// of one batch, and the Adam update.
//
// A batch is R = 2B profile rows: rows 0..B-1 are users u_i, rows B..2B-1
// their exact neighbours v_i, and w_i = v_{i-1 mod B} is u_i's
// non-neighbour.  Forward (the inference model with its bf16 roundings):
//   e = bf16(mean_{i in P_r} E[i])                          [R][64]
//   h = bf16(ReLU(e W1^T + b1))                             [R][256]
//   z = h W2^T + b2                                         [R][t*b], fp32
//   p_{r,j} = softmax of z_r over head j's b buckets
// Loss, with s_ij = <p_{u_i,j}, p_{v_i,j}>, n_ij = <p_{u_i,j}, p_{w_i,j}>,
// q_j = mean_r p_{r,j} and H the entropy:
//   L = -mean log max(s, 1e-12) - w_neg mean log(1 - clip(n, 0, 1 - 1e-6))
//       + w_bal mean_j sum_c q_jc log(q_jc b + 1e-12) + w_ent mean H
// Backward: dL/dp is the sum of the pair terms and the balance term dq/R;
// through the softmax dz = p (g - <p, g>) - w_ent/(R t) p (log p + H).  The
// bf16 roundings pass gradients unchanged.
//
// Kernels.  The four dense products (z, dW2 = dz^T h, dh = dz W2 and the
// small W1 ones) run on one bf16 MFMA GEMM (v_mfma_f32_32x32x16_bf16, 128 x
// 128 tiles, four waves of 64 x 64, K staged through LDS in steps of 32 with
// the next step's global loads in flight); operands stored with K outermost
// are transposed on their way into LDS, and long-K products are split over K
// into fp32 partial sums reduced by a second kernel.  The softmax statistics
// are row kernels (one block per row and head), the column means and sums
// column kernels over row slices, and dz one block per pair and head that
// writes both rows' gradients as bf16, the operand of the two products that
// follow.  No step depends on atomics except the embedding bag's backward
// (shared with the library's embedding-bag kernels).
#include "c2_internal.h"
#include "c2_kernels.h"

namespace c2 {
namespace {

typedef __bf16 trbf16x8 __attribute__((ext_vector_type(8)));
typedef float trf32x16 __attribute__((ext_vector_type(16)));

C2_DEV float tr_f32(uint16_t x) { return __uint_as_float((uint32_t)x << 16); }

// round to nearest even (finite inputs)
C2_DEV uint16_t tr_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

constexpr int kTrThreads = 256;

C2_DEV float block_sum(float v, float *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();                       // red may still be read by a previous call
    if (lane == 0) red[wid] = v;
    __syncthreads();
    float s = 0.f;
#pragma unroll
    for (int w = 0; w < kTrThreads / 64; ++w) s += red[w];
    return s;
}

C2_DEV float block_max(float v, float *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    float s = red[0];
#pragma unroll
    for (int w = 1; w < kTrThreads / 64; ++w) s = fmaxf(s, red[w]);
    return s;
}

// ------------------------------------------------------------------- GEMM

constexpr int kGM = 128, kGN = 128, kGK = 32;
constexpr int kGRow = kGK + 8;     // bf16 per LDS row: 80 bytes, 16-byte aligned rows

enum : int { kEpiF32 = 0, kEpiBiasF32 = 1, kEpiBiasReluBf16 = 2 };

struct GemmArgs {
    const uint16_t *A, *B;   // C[m][n] = sum_k A(m,k) B(n,k)
    uint32_t lda, ldb;
    uint32_t M, N, K;
    uint32_t kslice;          // K range of blockIdx.z (a multiple of kGK)
    float *C;                 // fp32 output, slice z at C + z * cstride
    uint16_t *C16;            // bf16 output (kEpiBiasReluBf16)
    uint32_t ldc;
    size_t cstride;
    const float *bias;        // per column n
};

// One operand tile (128 rows of the M or N side x 32 of K) as two 16-byte
// chunks per thread.  Not transposed: X(r, k) = X[r * ld + k], a chunk is 8
// consecutive k of one row; transposed: X(r, k) = X[k * ld + r], a chunk is
// 8 consecutive rows of one k.  Out-of-range chunks read as zeros (the
// contiguous extent is a multiple of 8).
template <bool T>
C2_DEV void gemm_load(const uint16_t *X, uint32_t ld, uint32_t r0, uint32_t rdim, uint32_t k0,
                      uint32_t kend, uint4 (&v)[2]) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const uint32_t c = threadIdx.x + kTrThreads * q;
        v[q] = make_uint4(0, 0, 0, 0);
        if constexpr (!T) {
            const uint32_t row = c >> 2, kc = (c & 3) * 8;
            if (r0 + row < rdim && k0 + kc < kend)
                v[q] = *reinterpret_cast<const uint4 *>(X + (size_t)(r0 + row) * ld + k0 + kc);
        } else {
            const uint32_t kr = c >> 4, rc = (c & 15) * 8;
            if (k0 + kr < kend && r0 + rc < rdim)
                v[q] = *reinterpret_cast<const uint4 *>(X + (size_t)(k0 + kr) * ld + r0 + rc);
        }
    }
}

// ... into LDS as [row][k] (k contiguous), the layout the MFMA fragments read
template <bool T>
C2_DEV void gemm_store(uint16_t *L, const uint4 (&v)[2]) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const uint32_t c = threadIdx.x + kTrThreads * q;
        if constexpr (!T) {
            const uint32_t row = c >> 2, kc = (c & 3) * 8;
            *reinterpret_cast<uint4 *>(L + row * kGRow + kc) = v[q];
        } else {
            const uint32_t kr = c >> 4, rc = (c & 15) * 8;
            const uint32_t w[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                L[(rc + 2 * i) * kGRow + kr] = (uint16_t)(w[i] & 0xFFFFu);
                L[(rc + 2 * i + 1) * kGRow + kr] = (uint16_t)(w[i] >> 16);
            }
        }
    }
}

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(kTrThreads) void k_gemm_bf16(GemmArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t As[2][kGM * kGRow];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][kGN * kGRow];
    const uint32_t m0 = blockIdx.x * kGM, n0 = blockIdx.y * kGN;
    const uint32_t kb = blockIdx.z * a.kslice;
    const uint32_t ke = a.K < kb + a.kslice ? a.K : kb + a.kslice;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wm = wid & 1, wn = wid >> 1, half = lane >> 5, col = lane & 31;
    trf32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    uint4 ra[2], rb[2];
    if (kb < ke) {
        gemm_load<TA>(a.A, a.lda, m0, a.M, kb, ke, ra);
        gemm_load<TB>(a.B, a.ldb, n0, a.N, kb, ke, rb);
        gemm_store<TA>(As[0], ra);
        gemm_store<TB>(Bs[0], rb);
    }
    __syncthreads();
    int buf = 0;
    for (uint32_t k0 = kb; k0 < ke; k0 += kGK) {
        const bool more = k0 + kGK < ke;
        if (more) {
            gemm_load<TA>(a.A, a.lda, m0, a.M, k0 + kGK, ke, ra);
            gemm_load<TB>(a.B, a.ldb, n0, a.N, k0 + kGK, ke, rb);
        }
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            trbf16x8 av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                av[i] = __builtin_bit_cast(trbf16x8, *reinterpret_cast<const uint4 *>(
                    &As[buf][(wm * 64 + i * 32 + col) * kGRow + ks * 16 + half * 8]));
                bv[i] = __builtin_bit_cast(trbf16x8, *reinterpret_cast<const uint4 *>(
                    &Bs[buf][(wn * 64 + i * 32 + col) * kGRow + ks * 16 + half * 8]));
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i], bv[j], acc[i][j],
                                                                        0, 0, 0);
        }
        if (more) {
            gemm_store<TA>(As[buf ^ 1], ra);
            gemm_store<TB>(Bs[buf ^ 1], rb);
        }
        __syncthreads();
        buf ^= 1;
    }
    // lane (half, col) of block (i, j) holds rows 8(r/4) + 4 half + r%4, column col
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const uint32_t n = n0 + wn * 64 + j * 32 + col;
            if (n >= a.N) continue;
            const float bias = (EPI != kEpiF32) ? a.bias[n] : 0.f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t m = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                if (m >= a.M) continue;
                const float v = acc[i][j][r] + bias;
                const size_t at = (size_t)m * a.ldc + n;
                if constexpr (EPI == kEpiBiasReluBf16)
                    a.C16[at] = tr_bf16(v > 0.f ? v : 0.f);
                else
                    a.C[blockIdx.z * a.cstride + at] = v;
            }
        }
}

// sum of S fp32 slices; optionally masked by h > 0 and also written as bf16
__global__ __launch_bounds__(kTrThreads) void k_slices_sum(const float *__restrict__ part,
                                                           uint32_t S, size_t count,
                                                           const uint16_t *__restrict__ mask,
                                                           float *__restrict__ out,
                                                           uint16_t *__restrict__ out16) {
    for (size_t i = blockIdx.x * (size_t)kTrThreads + threadIdx.x; i < count;
         i += (size_t)gridDim.x * kTrThreads) {
        float v = 0.f;
        for (uint32_t s = 0; s < S; ++s) v += part[s * count + i];
        if (mask && mask[i] == 0) v = 0.f;     // h = bf16(ReLU(pre)) is 0 exactly where pre <= 0
        out[i] = v;
        if (out16) out16[i] = tr_bf16(v);
    }
}

__global__ __launch_bounds__(kTrThreads) void k_to_bf16(const float *__restrict__ in, size_t count,
                                                        uint16_t *__restrict__ out) {
    for (size_t i = blockIdx.x * (size_t)kTrThreads + threadIdx.x; i < count;
         i += (size_t)gridDim.x * kTrThreads)
        out[i] = tr_bf16(in[i]);
}

// ------------------------------------------------------- softmax and loss

struct LossArgs {
    uint32_t R, B, t, b, T;   // rows, pairs, heads, buckets per head, T = t * b
    float w_neg, w_bal, w_ent;
    const float *z;           // [R][T]
    float *lse, *H, *D;       // [R][t]
    float *s, *sn;            // [B][t]
    float *q, *dq;            // [T]
};

// one block per (row, head): log-sum-exp and entropy of p = softmax(z)
__global__ __launch_bounds__(kTrThreads) void k_row_stats(LossArgs a) {
    __shared__ float red[kTrThreads / 64];
    const uint32_t r = blockIdx.x / a.t, j = blockIdx.x % a.t;
    const float *z = a.z + (size_t)r * a.T + (size_t)j * a.b;
    float mx = -__builtin_huge_valf();
    for (uint32_t c = threadIdx.x; c < a.b; c += kTrThreads) mx = fmaxf(mx, z[c]);
    mx = block_max(mx, red);
    float se = 0.f, sze = 0.f;
    for (uint32_t c = threadIdx.x; c < a.b; c += kTrThreads) {
        const float d = z[c] - mx, ex = __expf(d);
        se += ex;
        sze += d * ex;
    }
    se = block_sum(se, red);
    sze = block_sum(sze, red);
    if (threadIdx.x == 0) {
        const float ls = __logf(se);
        a.lse[blockIdx.x] = mx + ls;
        a.H[blockIdx.x] = ls - sze / se;      // -sum p log p = log S - sum p (z - max)
    }
}

// one block per (pair i, head j): s = <p_u, p_v>, n = <p_u, p_w>
__global__ __launch_bounds__(kTrThreads) void k_pair_stats(LossArgs a) {
    __shared__ float red[kTrThreads / 64];
    const uint32_t i = blockIdx.x / a.t, j = blockIdx.x % a.t;
    const uint32_t u = i, v = a.B + i, w = a.B + (i + a.B - 1) % a.B;
    const float lu = a.lse[u * a.t + j], lv = a.lse[v * a.t + j], lw = a.lse[w * a.t + j];
    const size_t off = (size_t)j * a.b;
    const float *zu = a.z + (size_t)u * a.T + off, *zv = a.z + (size_t)v * a.T + off,
                *zw = a.z + (size_t)w * a.T + off;
    float s = 0.f, sn = 0.f;
    for (uint32_t c = threadIdx.x; c < a.b; c += kTrThreads) {
        const float pu = __expf(zu[c] - lu);
        s += pu * __expf(zv[c] - lv);
        sn += pu * __expf(zw[c] - lw);
    }
    s = block_sum(s, red);
    sn = block_sum(sn, red);
    if (threadIdx.x == 0) {
        a.s[blockIdx.x] = s;
        a.sn[blockIdx.x] = sn;
    }
}

// column sums over a slice of rows: block (x = 256 columns, y = row slice);
// kind 0 sums p (from z and lse), kind 1 bf16 values, kind 2 fp32 values
template <int KIND>
__global__ __launch_bounds__(kTrThreads) void k_col_part(const void *__restrict__ X, uint32_t rows,
                                                         uint32_t cols, uint32_t rows_per,
                                                         const float *__restrict__ lse,
                                                         uint32_t t, uint32_t b,
                                                         float *__restrict__ part) {
    const uint32_t c = blockIdx.x * kTrThreads + threadIdx.x;
    if (c >= cols) return;
    const uint32_t r0 = blockIdx.y * rows_per;
    const uint32_t r1 = rows < r0 + rows_per ? rows : r0 + rows_per;
    float acc = 0.f;
    for (uint32_t r = r0; r < r1; ++r) {
        const size_t at = (size_t)r * cols + c;
        if constexpr (KIND == 0)
            acc += __expf(static_cast<const float *>(X)[at] - lse[(size_t)r * t + c / b]);
        else if constexpr (KIND == 1)
            acc += tr_f32(static_cast<const uint16_t *>(X)[at]);
        else
            acc += static_cast<const float *>(X)[at];
    }
    part[(size_t)blockIdx.y * cols + c] = acc;
}

// q = column means of p, and the balance term's derivative dq
__global__ __launch_bounds__(kTrThreads) void k_q_finish(const float *__restrict__ part, uint32_t S,
                                                         LossArgs a) {
    const uint32_t c = blockIdx.x * kTrThreads + threadIdx.x;
    if (c >= a.T) return;
    float v = 0.f;
    for (uint32_t s = 0; s < S; ++s) v += part[(size_t)s * a.T + c];
    const float q = v / (float)a.R, qb = q * (float)a.b;
    a.q[c] = q;
    a.dq[c] = a.w_bal / (float)a.t * (__logf(qb + 1e-12f) + qb / (qb + 1e-12f));
}

__global__ __launch_bounds__(kTrThreads) void k_cols_finish(const float *__restrict__ part,
                                                            uint32_t S, uint32_t cols,
                                                            float *__restrict__ out) {
    const uint32_t c = blockIdx.x * kTrThreads + threadIdx.x;
    if (c >= cols) return;
    float v = 0.f;
    for (uint32_t s = 0; s < S; ++s) v += part[(size_t)s * cols + c];
    out[c] = v;
}

// one block per (row, head): D = <p, dq>
__global__ __launch_bounds__(kTrThreads) void k_row_dot(LossArgs a) {
    __shared__ float red[kTrThreads / 64];
    const uint32_t r = blockIdx.x / a.t, j = blockIdx.x % a.t;
    const float l = a.lse[blockIdx.x];
    const float *z = a.z + (size_t)r * a.T + (size_t)j * a.b;
    const float *dq = a.dq + (size_t)j * a.b;
    float d = 0.f;
    for (uint32_t c = threadIdx.x; c < a.b; c += kTrThreads) d += __expf(z[c] - l) * dq[c];
    d = block_sum(d, red);
    if (threadIdx.x == 0) a.D[blockIdx.x] = d;
}

C2_DEV float pos_grad(float s, float Bt) { return s >= 1e-12f ? -1.f / (s * Bt) : 0.f; }

C2_DEV float neg_grad(float sn, float w_neg, float Bt) {
    return (sn >= 0.f && sn <= 1.f - 1e-6f) ? w_neg / ((1.f - sn) * Bt) : 0.f;
}

// one block per (pair i, head j): dz of rows u_i and v_i (bf16).  u_i's
// gradient of p takes v_i (pair term) and w_i (non-neighbour term); v_i's
// takes u_i and u_{i+1}, whose non-neighbour it is.
__global__ __launch_bounds__(kTrThreads) void k_dz(LossArgs a, uint16_t *__restrict__ dz) {
    const uint32_t i = blockIdx.x / a.t, j = blockIdx.x % a.t;
    const uint32_t i1 = (i + 1) % a.B;
    const uint32_t u = i, v = a.B + i, w = a.B + (i + a.B - 1) % a.B, u1 = i1;
    const float Bt = (float)a.B * (float)a.t, invR = 1.f / (float)a.R;
    const float went = a.w_ent / ((float)a.R * (float)a.t);
    const float s = a.s[i * a.t + j], sn = a.sn[i * a.t + j], sn1 = a.sn[i1 * a.t + j];
    const float ds = pos_grad(s, Bt), dn = neg_grad(sn, a.w_neg, Bt),
                dn1 = neg_grad(sn1, a.w_neg, Bt);
    const float lu = a.lse[u * a.t + j], lv = a.lse[v * a.t + j], lw = a.lse[w * a.t + j],
                lu1 = a.lse[u1 * a.t + j];
    const float Hu = a.H[u * a.t + j], Hv = a.H[v * a.t + j];
    // <p, g> of each row: the pair terms are s and n by definition
    const float Gu = ds * s + dn * sn + a.D[u * a.t + j] * invR;
    const float Gv = ds * s + dn1 * sn1 + a.D[v * a.t + j] * invR;
    const size_t off = (size_t)j * a.b;
    const float *zu = a.z + (size_t)u * a.T + off, *zv = a.z + (size_t)v * a.T + off,
                *zw = a.z + (size_t)w * a.T + off, *zu1 = a.z + (size_t)u1 * a.T + off;
    const float *dq = a.dq + off;
    uint16_t *du = dz + (size_t)u * a.T + off, *dv = dz + (size_t)v * a.T + off;
    for (uint32_t c = threadIdx.x; c < a.b; c += kTrThreads) {
        const float lpu = zu[c] - lu, lpv = zv[c] - lv;
        const float pu = __expf(lpu), pv = __expf(lpv);
        const float pw = __expf(zw[c] - lw), pu1 = __expf(zu1[c] - lu1);
        const float b = dq[c] * invR;
        const float gu = ds * pv + dn * pw + b, gv = ds * pu + dn1 * pu1 + b;
        du[c] = tr_bf16(pu * (gu - Gu) - went * pu * (lpu + Hu));
        dv[c] = tr_bf16(pv * (gv - Gv) - went * pv * (lpv + Hv));
    }
}

// loss parts: total, pos, neg, bal, ent
__global__ __launch_bounds__(kTrThreads) void k_loss(LossArgs a, float *__restrict__ loss) {
    __shared__ float red[kTrThreads / 64];
    float pos = 0.f, neg = 0.f, bal = 0.f, ent = 0.f;
    const uint32_t Bt = a.B * a.t, Rt = a.R * a.t;
    for (uint32_t x = threadIdx.x; x < Bt; x += kTrThreads) {
        pos += __logf(fmaxf(a.s[x], 1e-12f));
        neg += log1pf(-fminf(fmaxf(a.sn[x], 0.f), 1.f - 1e-6f));
    }
    for (uint32_t c = threadIdx.x; c < a.T; c += kTrThreads) {
        const float q = a.q[c];
        bal += q * __logf(q * (float)a.b + 1e-12f);
    }
    for (uint32_t x = threadIdx.x; x < Rt; x += kTrThreads) ent += a.H[x];
    pos = -block_sum(pos, red) / (float)Bt;
    neg = -a.w_neg * block_sum(neg, red) / (float)Bt;
    bal = a.w_bal * block_sum(bal, red) / (float)a.t;
    ent = a.w_ent * block_sum(ent, red) / (float)Rt;
    if (threadIdx.x == 0) {
        loss[0] = pos + neg + bal + ent;
        loss[1] = pos;
        loss[2] = neg;
        loss[3] = bal;
        loss[4] = ent;
    }
}

// --------------------------------------------------------------------- Adam

__global__ __launch_bounds__(kTrThreads) void k_adam(float *__restrict__ p,
                                                     const float *__restrict__ g,
                                                     float *__restrict__ m1,
                                                     float *__restrict__ m2, size_t n, float lr,
                                                     float beta1, float beta2, float eps,
                                                     float bc1, float bc2,
                                                     uint16_t *__restrict__ p16) {
    for (size_t i = blockIdx.x * (size_t)kTrThreads + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kTrThreads) {
        const float gi = g[i];
        const float a = beta1 * m1[i] + (1.f - beta1) * gi;
        const float b = beta2 * m2[i] + (1.f - beta2) * gi * gi;
        m1[i] = a;
        m2[i] = b;
        const float x = p[i] - lr * (a / bc1) / (sqrtf(b / bc2) + eps);
        p[i] = x;
        if (p16) p16[i] = tr_bf16(x);
    }
}

// -------------------------------------------------------------------- host

uint32_t grid_for(size_t count) {
    const size_t g = (count + kTrThreads - 1) / kTrThreads;
    return (uint32_t)(g < 8192 ? (g ? g : 1) : 8192);
}

template <bool TA, bool TB, int EPI>
hipError_t gemm(const GemmArgs &a, uint32_t splits, hipStream_t s) {
    const dim3 grid((uint32_t)div_up(a.M, kGM), (uint32_t)div_up(a.N, kGN), splits);
    hipLaunchKernelGGL((k_gemm_bf16<TA, TB, EPI>), grid, dim3(kTrThreads), 0, s, a);
    return hipGetLastError();
}

// K split into `splits` slices of a multiple of kGK
uint32_t kslice_for(uint32_t K, uint32_t splits) {
    const uint32_t per = (uint32_t)div_up(K, splits);
    return (uint32_t)div_up(per, kGK) * kGK;
}

constexpr uint32_t kColSlices = 16;   // row slices of the column sums
constexpr uint32_t kSplitDh = 16;     // K slices of dh = dz W2 (K = t*b)
constexpr uint32_t kSplitW1 = 8;      // K slices of dW1 = dpre^T e (K = R)

struct TrainLayout {
    size_t e32, e16, h16, z, dz16, lse, H, D, s, sn, q, dq, colpart, dhpart, dpre32, dpre16, de,
        w1part, total;
};

TrainLayout train_layout(uint32_t R, uint32_t t, uint32_t b) {
    const size_t T = (size_t)t * b, B = R / 2;
    TrainLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    L.e32 = take((size_t)R * kAsgDim * 4);
    L.e16 = take((size_t)R * kAsgDim * 2);
    L.h16 = take((size_t)R * kAsgHidden * 2);
    L.z = take((size_t)R * T * 4);
    L.dz16 = take((size_t)R * T * 2);
    L.lse = take((size_t)R * t * 4);
    L.H = take((size_t)R * t * 4);
    L.D = take((size_t)R * t * 4);
    L.s = take(B * t * 4);
    L.sn = take(B * t * 4);
    L.q = take(T * 4);
    L.dq = take(T * 4);
    L.colpart = take((size_t)kColSlices * (T > kAsgHidden ? T : kAsgHidden) * 4);
    L.dhpart = take((size_t)kSplitDh * R * kAsgHidden * 4);
    L.dpre32 = take((size_t)R * kAsgHidden * 4);
    L.dpre16 = take((size_t)R * kAsgHidden * 2);
    L.de = take((size_t)R * kAsgDim * 4);
    L.w1part = take((size_t)kSplitW1 * kAsgHidden * kAsgDim * 4);
    L.total = off;
    return L;
}

}  // namespace

size_t train_ws_bytes(uint32_t nrows, uint32_t t, uint32_t b) {
    return train_layout(nrows, t, b).total;
}

hipError_t launch_train_grad(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                             uint32_t n, uint32_t m, const uint32_t *rows, uint32_t R,
                             const uint16_t *E, const uint16_t *W1, const float *b1,
                             const uint16_t *W2, const float *b2, uint32_t t, uint32_t b,
                             float w_neg, float w_bal, float w_ent, float *loss, float *dE,
                             float *dW1, float *db1, float *dW2, float *db2, void *ws,
                             hipStream_t s) {
    const TrainLayout L = train_layout(R, t, b);
    char *base = static_cast<char *>(ws);
    auto F = [&](size_t off) { return reinterpret_cast<float *>(base + off); };
    auto H16 = [&](size_t off) { return reinterpret_cast<uint16_t *>(base + off); };
    const uint32_t T = t * b, B = R / 2;
    hipError_t e;
    // forward: e (fp32, then bf16), h = bf16(ReLU(e W1^T + b1)), z = h W2^T + b2
    if ((e = launch_embag(indptr, indices, nnz, n, m, rows, R, E, F(L.e32), s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_for((size_t)R * kAsgDim)), dim3(kTrThreads), 0, s,
                       F(L.e32), (size_t)R * kAsgDim, H16(L.e16));
    GemmArgs g{};
    g.A = H16(L.e16); g.lda = kAsgDim; g.B = W1; g.ldb = kAsgDim;
    g.M = R; g.N = kAsgHidden; g.K = kAsgDim; g.kslice = kslice_for(g.K, 1);
    g.C16 = H16(L.h16); g.ldc = kAsgHidden; g.bias = b1;
    if ((e = gemm<false, false, kEpiBiasReluBf16>(g, 1, s)) != hipSuccess) return e;
    g = GemmArgs{};
    g.A = H16(L.h16); g.lda = kAsgHidden; g.B = W2; g.ldb = kAsgHidden;
    g.M = R; g.N = T; g.K = kAsgHidden; g.kslice = kslice_for(g.K, 1);
    g.C = F(L.z); g.ldc = T; g.bias = b2;
    if ((e = gemm<false, false, kEpiBiasF32>(g, 1, s)) != hipSuccess) return e;

    // softmax statistics, pair products, column means, <p, dq>, dz, loss
    LossArgs la{R, B, t, b, T, w_neg, w_bal, w_ent, F(L.z), F(L.lse), F(L.H), F(L.D), F(L.s),
                F(L.sn), F(L.q), F(L.dq)};
    hipLaunchKernelGGL(k_row_stats, dim3(R * t), dim3(kTrThreads), 0, s, la);
    hipLaunchKernelGGL(k_pair_stats, dim3(B * t), dim3(kTrThreads), 0, s, la);
    const uint32_t rows_per = (uint32_t)div_up(R, kColSlices);
    hipLaunchKernelGGL(k_col_part<0>, dim3((uint32_t)div_up(T, kTrThreads), kColSlices),
                       dim3(kTrThreads), 0, s, (const void *)F(L.z), R, T, rows_per, F(L.lse), t,
                       b, F(L.colpart));
    hipLaunchKernelGGL(k_q_finish, dim3((uint32_t)div_up(T, kTrThreads)), dim3(kTrThreads), 0, s,
                       F(L.colpart), kColSlices, la);
    hipLaunchKernelGGL(k_row_dot, dim3(R * t), dim3(kTrThreads), 0, s, la);
    hipLaunchKernelGGL(k_dz, dim3(B * t), dim3(kTrThreads), 0, s, la, H16(L.dz16));
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(kTrThreads), 0, s, la, loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    // db2 = column sums of dz; dW2 = dz^T h
    hipLaunchKernelGGL(k_col_part<1>, dim3((uint32_t)div_up(T, kTrThreads), kColSlices),
                       dim3(kTrThreads), 0, s, (const void *)H16(L.dz16), R, T, rows_per,
                       (const float *)nullptr, t, b, F(L.colpart));
    hipLaunchKernelGGL(k_cols_finish, dim3((uint32_t)div_up(T, kTrThreads)), dim3(kTrThreads), 0,
                       s, F(L.colpart), kColSlices, T, db2);
    g = GemmArgs{};
    g.A = H16(L.dz16); g.lda = T; g.B = H16(L.h16); g.ldb = kAsgHidden;
    g.M = T; g.N = kAsgHidden; g.K = R; g.kslice = kslice_for(g.K, 1);
    g.C = dW2; g.ldc = kAsgHidden;
    if ((e = gemm<true, true, kEpiF32>(g, 1, s)) != hipSuccess) return e;

    // dh = dz W2 over K slices, reduced with the ReLU mask: dpre (fp32, bf16)
    g = GemmArgs{};
    g.A = H16(L.dz16); g.lda = T; g.B = W2; g.ldb = kAsgHidden;
    g.M = R; g.N = kAsgHidden; g.K = T; g.kslice = kslice_for(T, kSplitDh);
    g.C = F(L.dhpart); g.ldc = kAsgHidden; g.cstride = (size_t)R * kAsgHidden;
    const uint32_t sdh = (uint32_t)div_up(T, g.kslice);
    if ((e = gemm<false, true, kEpiF32>(g, sdh, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_slices_sum, dim3(grid_for((size_t)R * kAsgHidden)), dim3(kTrThreads), 0,
                       s, F(L.dhpart), sdh, (size_t)R * kAsgHidden, H16(L.h16), F(L.dpre32),
                       H16(L.dpre16));
    // db1 = column sums of dpre; dW1 = dpre^T e; de = dpre W1
    hipLaunchKernelGGL(k_col_part<2>, dim3(1, kColSlices), dim3(kTrThreads), 0, s,
                       (const void *)F(L.dpre32), R, (uint32_t)kAsgHidden, rows_per,
                       (const float *)nullptr, t, b, F(L.colpart));
    hipLaunchKernelGGL(k_cols_finish, dim3(1), dim3(kTrThreads), 0, s, F(L.colpart), kColSlices,
                       (uint32_t)kAsgHidden, db1);
    g = GemmArgs{};
    g.A = H16(L.dpre16); g.lda = kAsgHidden; g.B = H16(L.e16); g.ldb = kAsgDim;
    g.M = kAsgHidden; g.N = kAsgDim; g.K = R; g.kslice = kslice_for(R, kSplitW1);
    g.C = F(L.w1part); g.ldc = kAsgDim; g.cstride = (size_t)kAsgHidden * kAsgDim;
    const uint32_t sw1 = (uint32_t)div_up(R, g.kslice);
    if ((e = gemm<true, true, kEpiF32>(g, sw1, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_slices_sum, dim3(grid_for((size_t)kAsgHidden * kAsgDim)),
                       dim3(kTrThreads), 0, s, F(L.w1part), sw1, (size_t)kAsgHidden * kAsgDim,
                       (const uint16_t *)nullptr, dW1, (uint16_t *)nullptr);
    g = GemmArgs{};
    g.A = H16(L.dpre16); g.lda = kAsgHidden; g.B = W1; g.ldb = kAsgDim;
    g.M = R; g.N = kAsgDim; g.K = kAsgHidden; g.kslice = kslice_for(g.K, 1);
    g.C = F(L.de); g.ldc = kAsgDim;
    if ((e = gemm<false, true, kEpiF32>(g, 1, s)) != hipSuccess) return e;
    // dE: the embedding bag's backward into a cleared gradient
    if ((e = launch_fill_u32(reinterpret_cast<uint32_t *>(dE), 0, m * kAsgDim, s)) != hipSuccess)
        return e;
    return launch_embag_backward(indptr, indices, nnz, n, m, rows, R, F(L.de), dE, s);
}

hipError_t launch_adam(float *p, const float *g, float *m1, float *m2, size_t n, float lr,
                       float beta1, float beta2, float eps, float bc1, float bc2, uint16_t *p16,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(kTrThreads), 0, s, p, g, m1, m2, n, lr,
                       beta1, beta2, eps, bc1, bc2, p16);
    return hipGetLastError();
}

}  // namespace c2
