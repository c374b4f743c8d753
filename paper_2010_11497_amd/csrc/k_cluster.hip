// Step 1 on the device: grouping by FastRandomHash and recursive splitting
// (Algorithm 1 and Section II-D, Fig. 3), level-synchronously.
//
// State: the t*n slots of `members` (configuration j owns slots [j*n, j*n+n))
// are partitioned into contiguous segments, one per cluster.  seg[p] is the
// first slot of p's segment; at that first slot s, state[s] says whether the
// segment is final, still to be split (active) or a configuration root, eta1[s]
// is its index + 1 (the smallest hash value its split may use) and len[s] its
// size.  A round regroups every active segment in place:
//   mark   : number the active slots and active segments (one u64 scan);
//   fill   : per active slot, the next hash value e' = min{h(i) >= eta1}
//            (the precomputed FastRandomHash key at a root), as the sort key
//            (segment rank, e');
//   sort   : stable radix sort of the keys, which keeps users in slot order
//            inside each new group;
//   classify: group sizes; a user stays behind (residual) if it has no e', or
//            is alone with its e', unless its segment is a root;
//   scatter: inside each parent segment, the groups in ascending e' first,
//            then the users that stayed, in their previous order; new segments
//            larger than cap become active, the others final.
// With externally given top-level keys (a learned assignment) the root's
// groups start their split from eta1 = 0, i.e. from H_j(u) itself.
// Every step is a grid over all t*n slots whose work depends only on device
// data, so the rounds can be enqueued without synchronising.
#include "c2_internal.h"
#include "c2_kernels.h"

namespace c2 {

constexpr int kFillLanes = 8;

__global__ __launch_bounds__(256) void k_clu_init(uint32_t *E_uid, uint32_t *E_seg,
                                                  uint32_t *S_state, uint32_t *S_eta1,
                                                  uint32_t *S_len, uint32_t n, uint32_t NE,
                                                  uint32_t *ctr, uint32_t nctr) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nctr) ctr[p] = 0;
    if (p >= NE) return;
    const uint32_t u = p % n;
    E_uid[p] = u;
    E_seg[p] = p - u;
    if (u == 0) {
        S_state[p] = kRoot;
        S_eta1[p] = 0;
        S_len[p] = n;
    }
}

// mark[p] = active(p) | (active head(p) << 32), scanned afterwards.
__global__ __launch_bounds__(256) void k_clu_mark(const uint32_t *E_seg, const uint32_t *S_state,
                                                  uint64_t *mark, uint32_t NE) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NE) return;
    const uint32_t s = E_seg[p];
    const bool act = S_state[s] != kFinal;
    mark[p] = (uint64_t)act | ((uint64_t)(act && s == p) << 32);
}

// LANES lanes per slot: kFillLanes for the split rounds, which scan the
// profile; one at the top level (round 0), which only reads the given keys.
template <int LANES>
__global__ __launch_bounds__(256) void k_clu_fill(
    const int64_t *__restrict__ indptr, const uint32_t *__restrict__ indices, uint64_t nnz,
    uint32_t n, uint32_t m, const uint32_t *__restrict__ bucket, const uint32_t *__restrict__ keys0,
    uint32_t b, uint32_t bb, const uint32_t *E_uid, const uint32_t *E_seg, const uint32_t *S_state,
    const uint32_t *S_eta1, const uint32_t *S_len, const uint64_t *mark, uint32_t NE,
    uint32_t *A_uid, uint32_t *A_rank, uint32_t *P_start, uint32_t *P_len, uint32_t *P_state,
    uint32_t *P_q0, uint64_t *key, uint32_t *val) {
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid / LANES >= NE) return;
    const uint32_t p = (uint32_t)(gid / LANES);
    const uint32_t gl = threadIdx.x % LANES;
    const uint32_t s = E_seg[p];
    const uint32_t st = S_state[s];
    if (st == kFinal) return;
    const uint32_t q = (uint32_t)mark[p];
    const uint32_t rank = (uint32_t)(mark[s] >> 32);
    const uint32_t u = E_uid[p], j = p / n;
    uint32_t e;
    if (st == kRoot) {
        e = keys0[(size_t)j * n + u];
    } else {
        e = group_min_above<LANES>(indptr, indices, nnz, bucket + (size_t)j * m, m, b, u,
                                   S_eta1[s], gl);
    }
    if (gl == 0) {
        A_uid[q] = u;
        A_rank[q] = rank;
        key[q] = ((uint64_t)rank << bb) | (e > b ? b : e);
        val[q] = q;
        if (p == s) {
            P_start[rank] = s;
            P_len[rank] = S_len[s];
            P_state[rank] = st;
            P_q0[rank] = q;
        }
    }
}

// First index in [lo, hi) whose key is >= k (strict = false) or > k (true).
C2_DEV uint32_t bound(const uint64_t *keys, uint32_t lo, uint32_t hi, uint64_t k, bool strict) {
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        const uint64_t x = keys[mid];
        if (x < k || (strict && x == k)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Group bounds of each sorted entry and residual flags.  flg[q] low word:
// sorted entry q keeps a group; flg[v] high word: original entry v stays.
__global__ __launch_bounds__(256) void k_clu_classify(const uint64_t *skey, const uint32_t *sval,
                                                      const uint32_t *n_act, uint32_t NE,
                                                      uint32_t b, uint32_t bb,
                                                      const uint32_t *P_len,
                                                      const uint32_t *P_state,
                                                      const uint32_t *P_q0, uint32_t *glb,
                                                      uint32_t *glen, uint64_t *flg) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nA = *n_act;
    if (q >= NE) return;
    if (q >= nA) {
        flg[q] = 0;
        return;
    }
    const uint64_t k = skey[q];
    const uint32_t r = (uint32_t)(k >> bb);
    const uint32_t e = (uint32_t)(k & ((1ull << bb) - 1));
    const uint32_t lo = P_q0[r], hi = lo + P_len[r];
    const uint32_t lb = bound(skey, lo, hi, k, false);
    const uint32_t ub = bound(skey, lb, hi, k, true);
    const uint32_t len = ub - lb;
    const bool resid = P_state[r] == kActive && (e >= b || len == 1);
    glb[q] = lb;
    glen[q] = len;
    uint32_t *f32 = reinterpret_cast<uint32_t *>(flg);
    f32[2 * (size_t)q] = resid ? 0u : 1u;
    f32[2 * (size_t)sval[q] + 1] = resid ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_clu_scatter(
    const uint64_t *skey, const uint32_t *sval, const uint32_t *n_act, uint32_t bb, uint32_t cap,
    const uint32_t *A_uid, const uint32_t *A_rank, const uint32_t *P_start, const uint32_t *P_len,
    const uint32_t *P_q0, const uint32_t *glb, const uint32_t *glen, const uint64_t *fs,
    const uint32_t *P_state, uint32_t given_keys, uint32_t *E_uid, uint32_t *E_seg,
    uint32_t *S_state, uint32_t *S_eta1, uint32_t *S_len, uint32_t *new_active) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= *n_act) return;
    // (a) q as a sorted entry: place it inside its group
    {
        const uint64_t fq = fs[q], fq1 = fs[q + 1];
        if ((uint32_t)fq1 != (uint32_t)fq) {
            const uint64_t k = skey[q];
            const uint32_t r = (uint32_t)(k >> bb);
            const uint32_t e = (uint32_t)(k & ((1ull << bb) - 1));
            const uint32_t s = P_start[r];
            const uint32_t X0 = (uint32_t)fs[P_q0[r]];
            const uint32_t lb = glb[q], len = glen[q];
            const uint32_t gs = s + (uint32_t)fs[lb] - X0;
            const uint32_t np = s + (uint32_t)fq - X0;
            E_uid[np] = A_uid[sval[q]];
            E_seg[np] = gs;
            if (q == lb) {
                const bool big = len > cap;
                S_state[gs] = big ? kActive : kFinal;
                S_eta1[gs] = (given_keys && P_state[r] == kRoot) ? 0u : e + 1;
                S_len[gs] = len;
                if (big) atomicAdd(new_active, 1u);
            }
        }
    }
    // (b) q as an original entry: users that stay go after the groups, in order
    {
        const uint32_t R = (uint32_t)(fs[q] >> 32), R1 = (uint32_t)(fs[q + 1] >> 32);
        if (R1 != R) {
            const uint32_t r = A_rank[q];
            const uint32_t s = P_start[r], q0 = P_q0[r], L = P_len[r];
            const uint32_t R0 = (uint32_t)(fs[q0] >> 32);
            const uint32_t rc = (uint32_t)(fs[q0 + L] >> 32) - R0;
            const uint32_t start = s + (L - rc);
            const uint32_t np = start + (R - R0);
            E_uid[np] = A_uid[q];
            E_seg[np] = start;
            if (R == R0) {
                S_state[start] = kFinal;
                S_eta1[start] = 0;
                S_len[start] = rc;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_clu_heads(const uint32_t *E_seg, uint32_t *flag,
                                                   uint32_t NE) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NE) flag[p] = E_seg[p] == p ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_clu_final(const uint32_t *E_seg, const uint32_t *hs,
                                                   uint32_t n, uint32_t t, uint32_t NE,
                                                   uint32_t *cl_off, uint32_t *cl_cfg_off,
                                                   const uint32_t *ctr_last, uint32_t *status) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NE) return;
    if (E_seg[p] == p) {
        const uint32_t idx = hs[p];
        cl_off[idx] = p;
        if (p % n == 0) cl_cfg_off[p / n] = idx;
    }
    if (p == 0) {
        const uint32_t total = hs[NE];
        cl_off[total] = NE;
        cl_cfg_off[t] = total;
        if (status) *status = (ctr_last && *ctr_last) ? 1u : 0u;
    }
}

// --------------------------------------------------------------- host side

size_t cluster_ws_elems(const ClusterDims &d, ClusterWs *w) {
    // carve a ClusterWs out of a u32-aligned region (w == nullptr: size only)
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t NE = d.NE;
    ClusterWs x;
    x.E_seg = take(4 * NE);
    x.S_state = take(4 * NE);
    x.S_eta1 = take(4 * NE);
    x.S_len = take(4 * NE);
    x.mark = take(8 * (NE + 1));
    x.mtmp = take(8 * scan_tmp_elems((uint32_t)NE));
    x.A_uid = take(4 * NE);
    x.A_rank = take(4 * NE);
    x.P_start = take(4 * d.NP);
    x.P_len = take(4 * d.NP);
    x.P_state = take(4 * d.NP);
    x.P_q0 = take(4 * d.NP);
    x.key = take(8 * NE);
    x.key_alt = take(8 * NE);
    x.val = take(4 * (NE + 1));
    x.val_alt = take(4 * (NE + 1));
    x.hist = take(4 * radix_hist_elems((uint32_t)NE));
    const size_t hmax = radix_hist_elems((uint32_t)NE) > NE + 1 ? radix_hist_elems((uint32_t)NE)
                                                                  : NE + 1;
    x.htmp = take(4 * scan_tmp_elems((uint32_t)hmax));
    x.glb = take(4 * NE);
    x.glen = take(4 * NE);
    x.flg = take(8 * (NE + 1));
    x.ftmp = take(8 * scan_tmp_elems((uint32_t)NE));
    x.keys0 = take(4 * NE);
    x.bt = take(4 * d.TM);
    x.ctr = take(4 * (kMaxRounds + 2));
    x.status = take(4 * 4);
    x.total = off;
    if (w) *w = x;
    return off;
}

static inline dim3 grid_for(uint64_t threads, uint32_t bs = 256) {
    return dim3((uint32_t)div_up(threads, bs));
}

hipError_t cluster_round(const ClusterArgs &a, const ClusterPtrs &c, uint32_t round,
                         hipStream_t s) {
    const uint32_t NE = a.NE;
    hipLaunchKernelGGL(k_clu_mark, grid_for(NE), dim3(256), 0, s, c.E_seg, c.S_state, c.mark, NE);
    hipError_t e = scan_u64(c.mark, c.mark, NE, c.mtmp, s);
    if (e != hipSuccess) return e;
    // (round 0: every slot is at the top level)
    if (round == 0)
        hipLaunchKernelGGL(k_clu_fill<1>, grid_for((uint64_t)NE), dim3(256), 0, s,
                           a.indptr, a.indices, a.nnz, a.n, a.m, a.bucket,
                           a.keys_in ? a.keys_in : c.keys0, a.b, a.bb,
                           c.E_uid, c.E_seg, c.S_state, c.S_eta1, c.S_len, c.mark, NE, c.A_uid,
                           c.A_rank, c.P_start, c.P_len, c.P_state, c.P_q0, c.key, c.val);
    else
        hipLaunchKernelGGL(k_clu_fill<kFillLanes>, grid_for((uint64_t)NE * kFillLanes), dim3(256),
                           0, s, a.indptr, a.indices, a.nnz, a.n, a.m, a.bucket,
                           a.keys_in ? a.keys_in : c.keys0, a.b, a.bb,
                           c.E_uid, c.E_seg, c.S_state, c.S_eta1, c.S_len, c.mark, NE, c.A_uid,
                           c.A_rank, c.P_start, c.P_len, c.P_state, c.P_q0, c.key, c.val);
    const uint32_t *n_act = reinterpret_cast<const uint32_t *>(c.mark + NE);
    const uint32_t rank_bits = round == 0 ? bit_width(a.t - 1) : bit_width(a.NP - 1);
    bool in_alt = false;
    e = radix_sort(c.key, c.val, c.key_alt, c.val_alt, n_act, NE, rank_bits + a.bb, c.hist,
                   c.htmp, &in_alt, s);
    if (e != hipSuccess) return e;
    const uint64_t *skey = in_alt ? c.key_alt : c.key;
    const uint32_t *sval = in_alt ? c.val_alt : c.val;
    hipLaunchKernelGGL(k_clu_classify, grid_for(NE), dim3(256), 0, s, skey, sval, n_act, NE, a.b,
                       a.bb, c.P_len, c.P_state, c.P_q0, c.glb, c.glen, c.flg);
    e = scan_u64(c.flg, c.flg, NE, c.ftmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_clu_scatter, grid_for(NE), dim3(256), 0, s, skey, sval, n_act, a.bb,
                       a.cap, c.A_uid, c.A_rank, c.P_start, c.P_len, c.P_q0, c.glb, c.glen, c.flg,
                       c.P_state, a.keys_in ? 1u : 0u, c.E_uid, c.E_seg, c.S_state, c.S_eta1,
                       c.S_len, c.ctr + 1 + round);
    return hipGetLastError();
}

hipError_t cluster_init(const ClusterArgs &a, const ClusterPtrs &c, hipStream_t s) {
    hipLaunchKernelGGL(k_clu_init, grid_for(a.NE > kMaxRounds + 2 ? a.NE : kMaxRounds + 2),
                       dim3(256), 0, s, c.E_uid, c.E_seg, c.S_state, c.S_eta1, c.S_len, a.n, a.NE,
                       c.ctr, (uint32_t)(kMaxRounds + 2));
    if (a.keys_in) return hipGetLastError();
    return launch_frh_keys_rows(a.indptr, a.indices, a.nnz, a.n, a.m, a.bucket, a.t, a.b, c.bt,
                                c.keys0, s);
}

hipError_t cluster_finish(const ClusterArgs &a, const ClusterPtrs &c, uint32_t rounds,
                          uint32_t *cl_off, uint32_t *cl_cfg_off, hipStream_t s) {
    const uint32_t NE = a.NE;
    hipLaunchKernelGGL(k_clu_heads, grid_for(NE), dim3(256), 0, s, c.E_seg, c.val, NE);
    hipError_t e = scan_u32(c.val, c.val, NE, c.htmp, s);
    if (e != hipSuccess) return e;
    const uint32_t *last = rounds ? c.ctr + rounds : nullptr;
    hipLaunchKernelGGL(k_clu_final, grid_for(NE), dim3(256), 0, s, c.E_seg, c.val, a.n, a.t, NE,
                       cl_off, cl_cfg_off, last, c.status);
    return hipGetLastError();
}

}  // namespace c2
