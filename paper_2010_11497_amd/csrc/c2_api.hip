// C ABI of libc2.so: argument checks, workspace carving and the host-side
// orchestration of the kernels.  Declarations and contracts: include/c2.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "../../include/c2.h"
#include "c2_internal.h"
#include "c2_kernels.h"

using namespace c2;

namespace {

thread_local char g_err[512] = "";

c2_status fail(c2_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

c2_status hip_fail(hipError_t e, const char *where) {
    return fail(C2_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define C2_TRY(expr, where)                                    \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return hip_fail(e_, where);      \
    } while (0)

constexpr size_t kHeader = 256;  // status word(s) at the start of every workspace

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

c2_status check_sizes(uint32_t n, uint32_t m, uint64_t nnz, const c2_params *p, bool need_p) {
    if (n == 0 || n > 0x7FFFFFFFu) return fail(C2_E_ARG, "n = %u out of range [1, 2^31)", n);
    if (m == 0) return fail(C2_E_ARG, "m must be >= 1");
    if (m > kMaxItems) return fail(C2_E_UNSUPPORTED, "m = %u > %u items", m, kMaxItems);
    if (nnz >= (1ull << 40)) return fail(C2_E_UNSUPPORTED, "nnz too large");
    if (!need_p) return C2_OK;
    if (!p) return fail(C2_E_ARG, "params is NULL");
    if (p->t < 1 || p->t > 64) return fail(C2_E_ARG, "t = %u out of range [1, 64]", p->t);
    if (p->b < 1 || p->b > (1u << 31)) return fail(C2_E_ARG, "b = %u out of range [1, 2^31]", p->b);
    if (p->cap < 1) return fail(C2_E_ARG, "cap must be >= 1");
    if (p->k < 1 || p->k > kMaxK) return fail(C2_E_ARG, "k = %u out of range [1, %u]", p->k, kMaxK);
    if ((uint64_t)p->t * n >= 0xFFFFFFFFull) return fail(C2_E_UNSUPPORTED, "t*n >= 2^32");
    return C2_OK;
}

c2_status check_profiles(const c2_profiles *P) {
    if (!P) return fail(C2_E_ARG, "profiles is NULL");
    if (!P->indptr || (!P->indices && P->nnz)) return fail(C2_E_ARG, "profile pointers are NULL");
    return C2_OK;
}

// Brute force: members, cl_off, cl_cfg and the partial lists ahead of the
// local-KNN region.
size_t brute_head(uint32_t n, uint32_t k) {
    return kHeader + al(4 * (size_t)n) + al(4 * ((size_t)n + 1)) + al(8) + 2 * al(4 * (size_t)n * k);
}

// Smallest workspace a call accepts: the fixed part and a minimal store (the
// store takes whatever the caller gives beyond the fixed part).
size_t knn_min_bytes(uint32_t n, uint32_t NE, uint32_t m) {
    return knn_ws_fixed(n, NE, m, nullptr) + 4096;
}

ClusterDims cdims(uint32_t n, uint32_t m, const c2_params *p) {
    ClusterDims d;
    d.NE = (size_t)p->t * n;
    d.TM = (size_t)p->t * m;
    size_t np = d.NE / ((size_t)p->cap + 1);
    d.NP = (np > p->t ? np : p->t) + 1;
    return d;
}

// Scratch of the clustering step: the grid rounds' state, or the workgroup
// path's signatures and cluster starts, whichever is larger.
size_t cluster_scratch_bytes(uint32_t n, uint32_t m, const c2_params *p) {
    const size_t g = cluster_ws_elems(cdims(n, m, p), nullptr);
    const size_t w = cluster_wg_ws_bytes(n, p->t);
    return g > w ? g : w;
}

struct BuildLayout {
    size_t bucket, members, cl_off, cl_cfg, part_id, part_I, scratch, knn_fixed, total;
};

BuildLayout build_layout(uint32_t n, uint32_t m, uint64_t nnz, const c2_params *p) {
    BuildLayout L;
    size_t off = kHeader;
    auto take = [&](size_t b) { size_t o = off; off += al(b); return o; };
    const size_t NE = (size_t)p->t * n;
    L.bucket = take(4 * (size_t)p->t * m);
    L.members = take(4 * NE);
    L.cl_off = take(4 * (NE + 1));
    L.cl_cfg = take(4 * ((size_t)p->t + 1));
    L.part_id = take(4 * NE * p->k);
    L.part_I = take(4 * NE * p->k);
    L.scratch = off;
    const size_t cw = cluster_scratch_bytes(n, m, p);
    L.knn_fixed = knn_ws_fixed(n, (uint32_t)NE, m, nullptr);
    const size_t kw = L.knn_fixed + knn_store_default_bytes(n, (uint32_t)NE, m, nnz, p->t);
    L.total = off + (cw > kw ? cw : kw);
    return L;
}

// Smallest workspace c2_build accepts: the outputs of the stages, then the
// clustering scratch or the local KNN's fixed part and a minimal store.
size_t build_min_bytes(uint32_t n, uint32_t m, uint64_t nnz, const c2_params *p) {
    const BuildLayout L = build_layout(n, m, nnz, p);
    const size_t cw = cluster_scratch_bytes(n, m, p), kw = L.knn_fixed + 4096;
    return L.scratch + (cw > kw ? cw : kw);
}

ClusterPtrs cluster_ptrs(char *base, const ClusterWs &w, uint32_t *members, uint32_t *status) {
    ClusterPtrs c;
    auto u32 = [&](size_t o) { return reinterpret_cast<uint32_t *>(base + o); };
    auto u64 = [&](size_t o) { return reinterpret_cast<uint64_t *>(base + o); };
    c.E_uid = members;
    c.E_seg = u32(w.E_seg);
    c.S_state = u32(w.S_state);
    c.S_eta1 = u32(w.S_eta1);
    c.S_len = u32(w.S_len);
    c.mark = u64(w.mark);
    c.mtmp = u64(w.mtmp);
    c.A_uid = u32(w.A_uid);
    c.A_rank = u32(w.A_rank);
    c.P_start = u32(w.P_start);
    c.P_len = u32(w.P_len);
    c.P_state = u32(w.P_state);
    c.P_q0 = u32(w.P_q0);
    c.key = u64(w.key);
    c.key_alt = u64(w.key_alt);
    c.val = u32(w.val);
    c.val_alt = u32(w.val_alt);
    c.hist = u32(w.hist);
    c.htmp = u32(w.htmp);
    c.glb = u32(w.glb);
    c.glen = u32(w.glen);
    c.flg = u64(w.flg);
    c.ftmp = u64(w.ftmp);
    c.keys0 = u32(w.keys0);
    c.bt = u32(w.bt);
    c.ctr = u32(w.ctr);
    c.status = status;
    return c;
}

// Pointers into a local-KNN region of `bytes` bytes at base (the store takes
// what the fixed part leaves); status: the caller's header word for overflow.
KnnPtrs knn_ptrs(char *base, size_t bytes, const KnnWs &w, uint32_t *status) {
    KnnPtrs k;
    auto u32 = [&](size_t o) { return reinterpret_cast<uint32_t *>(base + o); };
    auto u64 = [&](size_t o) { return reinterpret_cast<uint64_t *>(base + o); };
    k.rlen = u32(w.rlen);
    k.cnt = u64(w.cnt);
    k.items_m = u64(w.items_m);
    k.items_b = u64(w.items_b);
    k.slots = u32(w.slots);
    k.sbase = u32(w.sbase);
    k.rb_done = u32(w.rb_done);
    k.htmp = u32(w.htmp);
    k.ctmp = u64(w.ctmp);
    k.ctr = u32(w.ctr);
    k.bmax = u32(w.bmax);
    k.pc = u32(w.pc);
    k.ccls = u32(w.ccls);
    k.cpos = u32(w.cpos);
    k.cw = u32(w.cw);
    k.coff = u64(w.coff);
    // the allocation cursor of the store sits in the caller's header (bytes
    // 8..15, after the two status words) when there is one: every cluster adds
    // its need to it whether or not it fits, so afterwards it holds the store
    // words the whole partition needs
    k.ccur = status ? reinterpret_cast<unsigned long long *>(status + 1)
                    : reinterpret_cast<unsigned long long *>(base + w.ccur);
    k.dslot = u32(w.dslot);
    k.dmap = u32(w.dmap);
    k.rlist = u64(w.rlist);
    k.store = u32(w.store);
    k.store_words = bytes > w.store ? (bytes - w.store) / 4 : 0;
    k.status = status;
    return k;
}

// Workspace of c2_local_knn_alg2: the local-KNN scratch (whose bit rows the
// Hyrec kernels read), the rewritten partition, and Hyrec's double-buffered
// lists over the largest possible cluster.
struct Alg2Layout {
    size_t rows, cl_off, cfg, keyA, keyB, IA, IB, upd, knn, total;
};

Alg2Layout alg2_layout(uint32_t n, uint32_t m, uint64_t nnz, const c2_params *p) {
    Alg2Layout L;
    size_t off = kHeader;
    auto take = [&](size_t b) { size_t o = off; off += al(b); return o; };
    const size_t NE = (size_t)p->t * n;
    L.rows = take((size_t)4 * n * full_row_words(m));
    L.cl_off = take(4 * (NE + 1));
    L.cfg = take(4 * ((size_t)p->t + 1));
    L.keyA = take(8 * (size_t)n * p->k);
    L.keyB = take(8 * (size_t)n * p->k);
    L.IA = take(4 * (size_t)n * p->k);
    L.IB = take(4 * (size_t)n * p->k);
    L.upd = take(256);
    L.knn = off;
    L.total = off + knn_ws_fixed(n, (uint32_t)NE, m, nullptr) +
              knn_store_default_bytes(n, (uint32_t)NE, m, nnz, p->t);
    return L;
}

uint32_t rounds_from(const c2_tuning *tune) {
    uint32_t r = tune && tune->split_rounds ? tune->split_rounds : 8;
    return r > kMaxRounds ? kMaxRounds : r;
}

// Clustering on an explicit scratch region (clusters of `ws` header status).
// Header of a workspace: word 0 = split rounds left clusters unsplit
// (batched clustering), word 1 = the local KNN's store overflowed, bytes
// 8..15 = the store words the last local KNN needed (u64).  Each stage writes
// its own words; c2_check_complete reads the two status words.
c2_status run_cluster(const c2_profiles *P, const uint32_t *bucket, const c2_params *p, int form,
                      const c2_tuning *tune, uint32_t rounds_batched, uint32_t *members, uint32_t *cl_off,
                      uint32_t *cl_cfg_off, char *scratch, uint32_t *status, hipStream_t s,
                      uint32_t *rounds_used, const uint32_t *keys_in = nullptr) {
    ClusterWs w;
    const ClusterDims d = cdims(P->n, P->m, p);
    cluster_ws_elems(d, &w);
    const ClusterPtrs c = cluster_ptrs(scratch, w, members, status);
    ClusterArgs a;
    a.indptr = P->indptr;
    a.indices = P->indices;
    a.nnz = P->nnz;
    a.n = P->n;
    a.m = P->m;
    a.t = p->t;
    a.b = p->b;
    a.bb = bit_width(p->b);
    a.cap = p->cap;
    a.bucket = bucket;
    a.NE = (uint32_t)d.NE;
    a.NP = (uint32_t)d.NP;
    a.keys_in = keys_in;
    const uint32_t path = tune ? tune->cluster_path : 0;
    if (!keys_in && path != 1 && cluster_wg_fits(a.n, a.b)) {
        uint32_t *rctr = nullptr;
        const uint32_t maxr = form == C2_FORM_PLAIN ? kMaxRounds : rounds_batched;
        C2_TRY(cluster_wg_run(a, members, cl_off, cl_cfg_off, scratch, status, maxr, &rctr, s),
               "cluster (workgroup)");
        if (form == C2_FORM_PLAIN) {
            uint32_t h[2] = {0, 0};
            C2_TRY(hipMemcpyAsync(&h[0], rctr, 4, hipMemcpyDeviceToHost, s), "copy");
            C2_TRY(hipMemcpyAsync(&h[1], status, 4, hipMemcpyDeviceToHost, s), "copy");
            C2_TRY(hipStreamSynchronize(s), "sync");
            if (h[1]) return fail(C2_E_UNSUPPORTED, "more than %u split rounds", kMaxRounds);
            if (rounds_used) *rounds_used = h[0];
        }
        return C2_OK;
    }
    C2_TRY(cluster_init(a, c, s), "cluster init");
    uint32_t r = 0;
    if (form == C2_FORM_PLAIN) {
        for (;; ++r) {
            if (r >= kMaxRounds) return fail(C2_E_UNSUPPORTED, "more than %u split rounds", kMaxRounds);
            C2_TRY(cluster_round(a, c, r, s), "cluster round");
            uint32_t more = 0;
            C2_TRY(hipMemcpyAsync(&more, c.ctr + 1 + r, 4, hipMemcpyDeviceToHost, s), "copy");
            C2_TRY(hipStreamSynchronize(s), "sync");
            if (!more) { ++r; break; }
        }
        C2_TRY(cluster_finish(a, c, 0, cl_off, cl_cfg_off, s), "cluster finish");
    } else {
        for (r = 0; r < rounds_batched; ++r) C2_TRY(cluster_round(a, c, r, s), "cluster round");
        C2_TRY(cluster_finish(a, c, rounds_batched, cl_off, cl_cfg_off, s), "cluster finish");
    }
    if (rounds_used) *rounds_used = r;
    return C2_OK;
}

// The local KNN on a region of `bytes` bytes at `scratch`; *status (a header
// word of the caller's workspace) is set when the store overflows (batched).
c2_status run_knn(const c2_profiles *P, const uint32_t *members, const uint32_t *cl_off,
                  const uint32_t *cl_cfg_off, uint32_t t, uint32_t k, int form,
                  const c2_tuning *tune, uint32_t *part_id, uint32_t *part_I, char *scratch,
                  size_t bytes, uint32_t *status, hipStream_t s) {
    KnnWs w;
    const uint32_t NE = t * P->n;
    knn_ws_fixed(P->n, NE, P->m, &w);
    if (bytes < w.total) return fail(C2_E_WORKSPACE, "local knn: workspace too small");
    KnnArgs a;
    a.indptr = P->indptr;
    a.indices = P->indices;
    a.nnz = P->nnz;
    a.n = P->n;
    a.m = P->m;
    a.t = t;
    a.k = k;
    a.members = members;
    a.cl_off = cl_off;
    a.cl_cfg_off = cl_cfg_off;
    a.NE = NE;
    a.Wm = dict_words(P->m);
    a.part_id = part_id;
    a.part_I = part_I;
    const KnnPtrs kp = knn_ptrs(scratch, bytes, w, status);
    KnnOpts o;
    if (tune) {
        o.persistent_wgs = tune->persistent_wgs;
        o.mfma_min = tune->mfma_min_rows;
        o.group_tiles = tune->group_tiles;
        o.tile32_max = tune->tile32_max;
        o.tile64_max = tune->tile64_max;
        o.ev_begin = (hipEvent_t)tune->ev_knn_begin;
        o.ev_end = (hipEvent_t)tune->ev_knn_end;
    }
    hipError_t e = form == C2_FORM_PLAIN ? knn_plain(a, kp, o, s) : knn_batched(a, kp, o, s);
    if (e == hipErrorOutOfMemory)
        return fail(C2_E_WORKSPACE,
                    "local knn: the dictionary rows of this partition need more than the %llu "
                    "bytes of store the workspace leaves (pass a larger workspace)",
                    (unsigned long long)kp.store_words * 4);
    if (e != hipSuccess) return hip_fail(e, "local knn");
    return C2_OK;
}

c2_status check_ws(void *ws, size_t have, size_t need) {
    if (!ws) return fail(C2_E_ARG, "workspace is NULL");
    if (have < need) return fail(C2_E_WORKSPACE, "workspace %zu bytes < %zu needed", have, need);
    return C2_OK;
}

c2_status check_form(int form) {
    if (form != C2_FORM_PLAIN && form != C2_FORM_BATCHED) return fail(C2_E_ARG, "bad form %d", form);
    return C2_OK;
}

// ------------------------------------------------------------ no allocation
//
// Workspace of c2_build_noalloc: a fixed array in device memory, one copy per
// GPU, held from the module's load until the process ends.  Host code never
// passes the array's name to a kernel or copy (on the host it is a stand-in,
// not a device address): the device address comes from hipGetSymbolAddress,
// taken once per device with that device current, and is kept here.
constexpr size_t kNoAllocBytes = (size_t)256 << 20;
constexpr int kNoAllocDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Bit 0: split rounds left clusters unsplit; bit 1: the store overflowed.
__global__ void k_copy_status(const uint32_t *src, uint32_t *dst) {
    *dst = (src[0] ? 1u : 0u) | (src[1] ? 2u : 0u);
}

std::mutex g_noalloc_mu;
char *g_noalloc_base[kNoAllocDevices] = {};

// Device address of this GPU's copy of the array (the current device).
c2_status noalloc_base(char **out) {
    int dev = 0;
    C2_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kNoAllocDevices)
        return fail(C2_E_UNSUPPORTED, "device %d: at most %d devices", dev, kNoAllocDevices);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_base[dev]) {
        void *ptr = nullptr;
        C2_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(C2_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_noalloc_base[dev] = reinterpret_cast<char *>(ptr);
    }
    *out = g_noalloc_base[dev];
    return C2_OK;
}

}  // namespace

extern "C" {

const char *c2_last_error(void) { return g_err; }

size_t c2_workspace_bytes(uint32_t n, uint32_t m, uint64_t nnz, const c2_params *p, int op) {
    c2_params one = {1, 1, 1, 1};
    switch (op) {
    case C2_OP_VALIDATE:
        if (check_sizes(n, m, nnz, nullptr, false) != C2_OK) return 0;
        return kHeader;
    case C2_OP_CLUSTER:
        if (check_sizes(n, m, nnz, p, true) != C2_OK) return 0;
        return kHeader + cluster_scratch_bytes(n, m, p);
    case C2_OP_LOCAL_KNN:
        if (check_sizes(n, m, nnz, p, true) != C2_OK) return 0;
        return kHeader + knn_ws_fixed(n, p->t * n, m, nullptr) +
               knn_store_default_bytes(n, p->t * n, m, nnz, p->t);
    case C2_OP_BUILD:
        if (check_sizes(n, m, nnz, p, true) != C2_OK) return 0;
        return build_layout(n, m, nnz, p).total;
    case C2_OP_BRUTE_FORCE: {
        one.k = p ? p->k : 1;
        if (check_sizes(n, m, nnz, &one, true) != C2_OK) return 0;
        // one cluster: its rows over the whole item universe at most, after
        // the scratch of its row blocks (up to 4 column groups each)
        return brute_head(n, one.k) + knn_ws_fixed(n, n, m, nullptr) +
               (size_t)4 * (((size_t)n + 31) / 32 * 32) * full_row_words(m) +
               (((size_t)n + 63) / 64) * 4 * 64 * one.k * 8 + 4096;
    }
    case C2_OP_LOCAL_KNN_ALG2:
        if (check_sizes(n, m, nnz, p, true) != C2_OK) return 0;
        return alg2_layout(n, m, nnz, p).total;
    case C2_OP_LOCAL_KNN_MIN:
        if (check_sizes(n, m, nnz, p, true) != C2_OK) return 0;
        return kHeader + knn_min_bytes(n, p->t * n, m);
    case C2_OP_FINGERPRINT:
        if (check_sizes(n, m, nnz, nullptr, false) != C2_OK) return 0;
        if (!p || p->b < 1 || p->b > kFpMaxBits) {
            fail(C2_E_ARG, "fingerprint bits (p->b) out of range [1, %u]", kFpMaxBits);
            return 0;
        }
        return kHeader + fingerprint_ws_bytes(n, p->b);
    default:
        fail(C2_E_ARG, "unknown op %d", op);
        return 0;
    }
}

c2_status c2_validate(const c2_profiles *P, void *ws, size_t ws_bytes, void *stream) {
    c2_status st;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, nullptr, false)) != C2_OK) return st;
    if ((st = check_ws(ws, ws_bytes, kHeader)) != C2_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    uint32_t *err = reinterpret_cast<uint32_t *>(ws);
    C2_TRY(launch_fill_u32(err, 0, 1, s), "validate");
    C2_TRY(launch_validate(P->indptr, P->indices, P->nnz, P->n, P->m, err, s), "validate");
    uint32_t h = 0;
    C2_TRY(hipMemcpyAsync(&h, err, 4, hipMemcpyDeviceToHost, s), "validate copy");
    C2_TRY(hipStreamSynchronize(s), "validate sync");
    if (h) {
        return fail(C2_E_PROFILE, "invalid profiles:%s%s%s%s", (h & 1) ? " indptr ends" : "",
                    (h & 2) ? " empty row" : "", (h & 4) ? " item >= m" : "",
                    (h & 8) ? " items not strictly increasing" : "");
    }
    return C2_OK;
}

c2_status c2_fingerprint(const c2_profiles *P, const uint32_t *g, uint32_t B, int64_t *fp_indptr,
                         uint32_t *fp_indices, uint64_t *fp_nnz, void *ws, size_t ws_bytes,
                         void *stream) {
    c2_status st;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, nullptr, false)) != C2_OK) return st;
    if (!g || !fp_indptr || (!fp_indices && P->nnz) || !fp_nnz) return fail(C2_E_ARG, "NULL pointer");
    if (B < 1 || B > kFpMaxBits) return fail(C2_E_ARG, "B = %u out of range [1, %u]", B, kFpMaxBits);
    const c2_params q = {1, B, 1, 1};
    if ((st = check_ws(ws, ws_bytes, c2_workspace_bytes(P->n, P->m, P->nnz, &q, C2_OP_FINGERPRINT))) != C2_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    uint32_t *err = reinterpret_cast<uint32_t *>(ws);
    C2_TRY(launch_fill_u32(err, 0, 1, s), "fingerprint");
    C2_TRY(launch_fingerprint(P->indptr, P->indices, P->nnz, P->n, P->m, g, B, fp_indptr,
                              fp_indices, reinterpret_cast<char *>(ws) + kHeader, err, s),
           "fingerprint");
    uint32_t h = 0;
    int64_t total = 0;
    C2_TRY(hipMemcpyAsync(&h, err, 4, hipMemcpyDeviceToHost, s), "fingerprint copy");
    C2_TRY(hipMemcpyAsync(&total, fp_indptr + P->n, 8, hipMemcpyDeviceToHost, s), "fingerprint copy");
    C2_TRY(hipStreamSynchronize(s), "fingerprint sync");
    if (h & 1) return fail(C2_E_PROFILE, "a profile holds an item >= m");
    if (h & 2) return fail(C2_E_ARG, "g holds a position >= B = %u", B);
    *fp_nnz = (uint64_t)total;
    return C2_OK;
}

c2_status c2_assign_hidden(const c2_profiles *P, const uint16_t *E, const uint16_t *W1,
                           const float *b1, uint16_t *h, void *stream) {
    c2_status st;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, nullptr, false)) != C2_OK) return st;
    if (!E || !W1 || !b1 || !h) return fail(C2_E_ARG, "NULL pointer");
    C2_TRY(launch_assign_hidden(P->indptr, P->indices, P->nnz, P->n, P->m, E, W1, b1, h,
                                (hipStream_t)stream),
           "assign hidden");
    return C2_OK;
}

c2_status c2_assign_keys(const uint16_t *h, uint32_t n, const uint16_t *W2, const float *b2,
                         uint32_t t, uint32_t b, const uint32_t *frh_keys, float min_gap,
                         uint32_t *keys, float *gap, void *stream) {
    if (!h || !W2 || !b2 || !keys) return fail(C2_E_ARG, "NULL pointer");
    if (n == 0 || n > 0x7FFFFFFFu) return fail(C2_E_ARG, "n = %u out of range [1, 2^31)", n);
    if (t < 1 || t > 64) return fail(C2_E_ARG, "t = %u out of range [1, 64]", t);
    if (b < 64 || b % 64 || b > (1u << 23)) return fail(C2_E_ARG, "b = %u: a multiple of 64 in [64, 2^23]", b);
    if ((uint64_t)t * n >= 0xFFFFFFFFull) return fail(C2_E_UNSUPPORTED, "t*n >= 2^32");
    C2_TRY(launch_assign_keys(h, n, W2, b2, t, b, frh_keys, min_gap, keys, gap,
                              (hipStream_t)stream),
           "assign keys");
    return C2_OK;
}

c2_status c2_embag(const c2_profiles *P, const uint32_t *rows, uint32_t nrows, const uint16_t *E,
                   float *out, void *stream) {
    c2_status st;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, nullptr, false)) != C2_OK) return st;
    if (!E || !out) return fail(C2_E_ARG, "NULL pointer");
    if (nrows == 0) return C2_OK;
    C2_TRY(launch_embag(P->indptr, P->indices, P->nnz, P->n, P->m, rows, nrows, E, out,
                        (hipStream_t)stream),
           "embedding bag");
    return C2_OK;
}

c2_status c2_embag_backward(const c2_profiles *P, const uint32_t *rows, uint32_t nrows,
                            const float *grad, float *dE, void *stream) {
    c2_status st;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, nullptr, false)) != C2_OK) return st;
    if (!grad || !dE) return fail(C2_E_ARG, "NULL pointer");
    if (nrows == 0) return C2_OK;
    C2_TRY(launch_embag_backward(P->indptr, P->indices, P->nnz, P->n, P->m, rows, nrows, grad, dE,
                                 (hipStream_t)stream),
           "embedding bag backward");
    return C2_OK;
}

size_t c2_assign_train_workspace_bytes(uint32_t nrows, uint32_t t, uint32_t b) {
    if (nrows < 2 || nrows % 2 || t < 1 || t > 64 || b < 64 || b % 64 || b > (1u << 23)) {
        fail(C2_E_ARG, "training batch: nrows = %u (even, >= 2), t = %u, b = %u", nrows, t, b);
        return 0;
    }
    return train_ws_bytes(nrows, t, b);
}

c2_status c2_assign_train_grad(const c2_profiles *P, const uint32_t *rows, uint32_t nrows,
                               const uint16_t *E, const uint16_t *W1, const float *b1,
                               const uint16_t *W2, const float *b2, uint32_t t, uint32_t b,
                               const c2_train_opts *opts, float *loss, float *dE, float *dW1,
                               float *db1, float *dW2, float *db2, void *ws, size_t ws_bytes,
                               void *stream) {
    c2_status st;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, nullptr, false)) != C2_OK) return st;
    if (!rows || !E || !W1 || !b1 || !W2 || !b2 || !opts || !loss || !dE || !dW1 || !db1 ||
        !dW2 || !db2)
        return fail(C2_E_ARG, "NULL pointer");
    const size_t need = c2_assign_train_workspace_bytes(nrows, t, b);
    if (need == 0) return C2_E_ARG;
    if ((uint64_t)nrows * t * b >= (1ull << 40)) return fail(C2_E_UNSUPPORTED, "batch too large");
    if ((st = check_ws(ws, ws_bytes, need)) != C2_OK) return st;
    C2_TRY(launch_train_grad(P->indptr, P->indices, P->nnz, P->n, P->m, rows, nrows, E, W1, b1,
                             W2, b2, t, b, opts->w_neg, opts->w_bal, opts->w_ent, loss, dE, dW1,
                             db1, dW2, db2, ws, (hipStream_t)stream),
           "assign training step");
    return C2_OK;
}

c2_status c2_adam_step(float *param, const float *grad, float *m1, float *m2, uint64_t count,
                       float lr, float beta1, float beta2, float eps, uint32_t step,
                       uint16_t *param_bf16, void *stream) {
    if (!param || !grad || !m1 || !m2) return fail(C2_E_ARG, "NULL pointer");
    if (step < 1) return fail(C2_E_ARG, "step counts from 1");
    if (count == 0) return C2_OK;
    const float bc1 = (float)(1.0 - pow((double)beta1, (double)step));
    const float bc2 = (float)(1.0 - pow((double)beta2, (double)step));
    C2_TRY(launch_adam(param, grad, m1, m2, count, lr, beta1, beta2, eps, bc1, bc2, param_bf16,
                       (hipStream_t)stream),
           "adam");
    return C2_OK;
}

c2_status c2_hash_items(const uint64_t *tab, uint32_t t, uint32_t b, uint32_t m, uint32_t *bucket,
                        void *stream) {
    if (!tab || !bucket) return fail(C2_E_ARG, "NULL pointer");
    if (t < 1 || t > 64 || b < 1 || m < 1) return fail(C2_E_ARG, "bad t/b/m");
    C2_TRY(launch_hash_items(tab, t, b, m, bucket, (hipStream_t)stream), "hash items");
    return C2_OK;
}

c2_status c2_frh_keys(const c2_profiles *P, const uint32_t *bucket, uint32_t t, uint32_t *keys,
                      void *stream) {
    c2_status st;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, nullptr, false)) != C2_OK) return st;
    if (!bucket || !keys) return fail(C2_E_ARG, "NULL pointer");
    if (t < 1 || t > 64) return fail(C2_E_ARG, "bad t");
    C2_TRY(launch_frh_keys(P->indptr, P->indices, P->nnz, P->n, P->m, bucket, t, 0xFFFFFFFFu, keys,
                           (hipStream_t)stream),
           "frh keys");
    return C2_OK;
}

c2_status c2_cluster(const c2_profiles *P, const uint32_t *bucket, const c2_params *p, int form,
                     const c2_tuning *tune, uint32_t *members, uint32_t *cl_off,
                     uint32_t *cl_cfg_off, void *ws, size_t ws_bytes, void *stream) {
    c2_status st;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, p, true)) != C2_OK) return st;
    if ((st = check_form(form)) != C2_OK) return st;
    if (!bucket || !members || !cl_off || !cl_cfg_off) return fail(C2_E_ARG, "NULL pointer");
    if ((st = check_ws(ws, ws_bytes, c2_workspace_bytes(P->n, P->m, P->nnz, p, C2_OP_CLUSTER))) != C2_OK)
        return st;
    char *base = reinterpret_cast<char *>(ws);
    C2_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(base) + 1, 0, 1, (hipStream_t)stream),
           "status");
    return run_cluster(P, bucket, p, form, tune, rounds_from(tune), members, cl_off, cl_cfg_off,
                       base + kHeader, reinterpret_cast<uint32_t *>(base), (hipStream_t)stream,
                       nullptr);
}

c2_status c2_cluster_keys(const c2_profiles *P, const uint32_t *keys, const uint32_t *bucket,
                          const c2_params *p, int form, const c2_tuning *tune, uint32_t *members,
                          uint32_t *cl_off, uint32_t *cl_cfg_off, void *ws, size_t ws_bytes,
                          void *stream) {
    c2_status st;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, p, true)) != C2_OK) return st;
    if ((st = check_form(form)) != C2_OK) return st;
    if (!keys || !bucket || !members || !cl_off || !cl_cfg_off) return fail(C2_E_ARG, "NULL pointer");
    if ((st = check_ws(ws, ws_bytes, c2_workspace_bytes(P->n, P->m, P->nnz, p, C2_OP_CLUSTER))) != C2_OK)
        return st;
    char *base = reinterpret_cast<char *>(ws);
    C2_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(base) + 1, 0, 1, (hipStream_t)stream),
           "status");
    return run_cluster(P, bucket, p, form, tune, rounds_from(tune), members, cl_off, cl_cfg_off,
                       base + kHeader, reinterpret_cast<uint32_t *>(base), (hipStream_t)stream,
                       nullptr, keys);
}

c2_status c2_check_complete(const void *ws, void *stream) {
    if (!ws) return fail(C2_E_ARG, "workspace is NULL");
    uint32_t h[2] = {0, 0};
    hipStream_t s = (hipStream_t)stream;
    C2_TRY(hipMemcpyAsync(h, ws, 8, hipMemcpyDeviceToHost, s), "status copy");
    C2_TRY(hipStreamSynchronize(s), "status sync");
    if (h[0]) return fail(C2_E_INCOMPLETE, "batched clustering needs more split rounds");
    if (h[1])
        return fail(C2_E_WORKSPACE, "the workspace's store could not hold every cluster's "
                                    "dictionary rows (pass a larger workspace)");
    return C2_OK;
}

c2_status c2_local_knn(const c2_profiles *P, const uint32_t *members, const uint32_t *cl_off,
                       const uint32_t *cl_cfg_off, const c2_params *p, int form,
                       const c2_tuning *tune, uint32_t *part_id, uint32_t *part_I, void *ws,
                       size_t ws_bytes, void *stream) {
    c2_status st;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, p, true)) != C2_OK) return st;
    if ((st = check_form(form)) != C2_OK) return st;
    if (!members || !cl_off || !cl_cfg_off || !part_id || !part_I) return fail(C2_E_ARG, "NULL pointer");
    if ((st = check_ws(ws, ws_bytes, kHeader + knn_min_bytes(P->n, p->t * P->n, P->m))) != C2_OK)
        return st;
    char *base = reinterpret_cast<char *>(ws);
    C2_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(base), 0, 1, (hipStream_t)stream), "status");
    return run_knn(P, members, cl_off, cl_cfg_off, p->t, p->k, form, tune, part_id, part_I,
                   base + kHeader, ws_bytes - kHeader, reinterpret_cast<uint32_t *>(base) + 1,
                   (hipStream_t)stream);
}

c2_status c2_local_knn_alg2(const c2_profiles *P, const uint32_t *members, const uint32_t *cl_off,
                            const uint32_t *cl_cfg_off, const c2_params *p, const c2_hyrec *hy,
                            const c2_tuning *tune, uint32_t *part_id, uint32_t *part_I, void *ws,
                            size_t ws_bytes, void *stream) {
    c2_status st;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, p, true)) != C2_OK) return st;
    if (!members || !cl_off || !cl_cfg_off || !part_id || !part_I || !hy)
        return fail(C2_E_ARG, "NULL pointer");
    if (hy->rho < 1) return fail(C2_E_ARG, "rho must be >= 1");
    const Alg2Layout L = alg2_layout(P->n, P->m, P->nnz, p);
    if ((st = check_ws(ws, ws_bytes, L.knn + knn_min_bytes(P->n, p->t * P->n, P->m))) != C2_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    char *base = reinterpret_cast<char *>(ws);
    uint32_t *status = reinterpret_cast<uint32_t *>(base) + 1;
    const uint32_t t = p->t, k = p->k, n = P->n;
    const uint64_t NE = (uint64_t)t * n;
    // the partition on the host: which clusters take Hyrec
    std::vector<uint32_t> cfg(t + 1);
    C2_TRY(hipMemcpyAsync(cfg.data(), cl_cfg_off, 4 * (t + 1), hipMemcpyDeviceToHost, s), "copy");
    C2_TRY(hipStreamSynchronize(s), "sync");
    const uint32_t ncl = cfg[t];
    if (ncl < 1 || ncl > NE) return fail(C2_E_ARG, "cl_cfg_off[t] = %u out of range", ncl);
    std::vector<uint32_t> off(ncl + 1);
    C2_TRY(hipMemcpyAsync(off.data(), cl_off, 4 * ((size_t)ncl + 1), hipMemcpyDeviceToHost, s), "copy");
    C2_TRY(hipStreamSynchronize(s), "sync");
    const uint64_t thr = (uint64_t)hy->rho * k * k;
    std::vector<uint32_t> big;
    for (uint32_t c = 0; c < ncl; ++c) {
        if (off[c + 1] < off[c] || off[c + 1] > NE) return fail(C2_E_ARG, "cl_off not monotone");
        const uint32_t sz = off[c + 1] - off[c];
        if (sz >= 2 && sz >= thr) big.push_back(c);
    }
    if (big.empty())
        return run_knn(P, members, cl_off, cl_cfg_off, t, k, C2_FORM_PLAIN, tune, part_id, part_I,
                       base + L.knn, ws_bytes - L.knn, status, s);
    if (ncl >= (1u << 24) || n >= (1u << 28))
        return fail(C2_E_UNSUPPORTED, "Hyrec needs fewer than 2^24 clusters and 2^28 users");
    {   // exact keys need |P_u| + |P_v| < 2^16
        std::vector<int64_t> ip((size_t)n + 1);
        C2_TRY(hipMemcpyAsync(ip.data(), P->indptr, 8 * ((size_t)n + 1), hipMemcpyDeviceToHost, s), "copy");
        C2_TRY(hipStreamSynchronize(s), "sync");
        for (uint32_t u = 0; u < n; ++u)
            if (ip[u + 1] - ip[u] >= (1 << 15))
                return fail(C2_E_UNSUPPORTED, "Hyrec clusters need profiles shorter than 2^15 items");
    }
    // brute force on the rest: every Hyrec cluster becomes singletons (pad lists),
    // overwritten below
    std::vector<uint32_t> off2, cfg2(t + 1);
    off2.reserve(ncl + 1);
    size_t bi = 0;
    for (uint32_t j = 0; j < t; ++j) {
        cfg2[j] = (uint32_t)off2.size();
        for (uint32_t c = cfg[j]; c < cfg[j + 1]; ++c) {
            if (bi < big.size() && big[bi] == c) {
                for (uint32_t x = off[c]; x < off[c + 1]; ++x) off2.push_back(x);
                ++bi;
            } else {
                off2.push_back(off[c]);
            }
        }
    }
    cfg2[t] = (uint32_t)off2.size();
    off2.push_back((uint32_t)NE);
    uint32_t *d_off2 = reinterpret_cast<uint32_t *>(base + L.cl_off);
    uint32_t *d_cfg2 = reinterpret_cast<uint32_t *>(base + L.cfg);
    C2_TRY(hipMemcpyAsync(d_off2, off2.data(), 4 * off2.size(), hipMemcpyHostToDevice, s), "copy");
    C2_TRY(hipMemcpyAsync(d_cfg2, cfg2.data(), 4 * ((size_t)t + 1), hipMemcpyHostToDevice, s), "copy");
    st = run_knn(P, members, d_off2, d_cfg2, t, k, C2_FORM_PLAIN, tune, part_id, part_I,
                 base + L.knn, ws_bytes - L.knn, status, s);
    C2_TRY(hipStreamSynchronize(s), "sync");  // off2 / cfg2 copied before they go
    if (st != C2_OK) return st;
    // Hyrec on the big clusters, over full bit rows and the profile lengths the
    // local KNN left
    const uint32_t wmax = full_row_words(P->m);
    uint32_t *rows = reinterpret_cast<uint32_t *>(base + L.rows);
    C2_TRY(launch_user_bits(P->indptr, P->indices, P->nnz, n, P->m, rows, s), "hyrec rows");
    KnnWs kw;
    knn_ws_fixed(n, (uint32_t)NE, P->m, &kw);
    const KnnPtrs kp = knn_ptrs(base + L.knn, ws_bytes - L.knn, kw, nullptr);
    uint64_t *kA = reinterpret_cast<uint64_t *>(base + L.keyA);
    uint64_t *kB = reinterpret_cast<uint64_t *>(base + L.keyB);
    uint32_t *iA = reinterpret_cast<uint32_t *>(base + L.IA);
    uint32_t *iB = reinterpret_cast<uint32_t *>(base + L.IB);
    uint32_t *upd = reinterpret_cast<uint32_t *>(base + L.upd);
    for (uint32_t c : big) {
        uint32_t j = 0;
        while (cfg[j + 1] <= c) ++j;
        const uint32_t *S = members + off[c];
        const uint32_t sz = off[c + 1] - off[c];
        C2_TRY(launch_hyrec_step(rows, kp.rlen, wmax, S, sz, k, c, hy->seed, true, nullptr, kA,
                                 iA, upd, s),
               "hyrec init");
        for (uint32_t it = 0; it < hy->max_iter; ++it) {
            C2_TRY(launch_fill_u32(upd, 0, 1, s), "hyrec");
            C2_TRY(launch_hyrec_step(rows, kp.rlen, wmax, S, sz, k, c, hy->seed, false, kA, kB,
                                     iB, upd, s),
                   "hyrec step");
            uint32_t h = 0;
            C2_TRY(hipMemcpyAsync(&h, upd, 4, hipMemcpyDeviceToHost, s), "copy");
            C2_TRY(hipStreamSynchronize(s), "sync");
            uint64_t *tk = kA; kA = kB; kB = tk;
            uint32_t *ti = iA; iA = iB; iB = ti;
            if ((double)h < hy->delta * (double)k * (double)sz) break;
        }
        C2_TRY(launch_hyrec_out(S, sz, k, j, t, kA, iA, part_id, part_I, s), "hyrec out");
    }
    return C2_OK;
}

c2_status c2_merge(const c2_profiles *P, const uint32_t *part_id, const uint32_t *part_I,
                   const c2_params *p, uint32_t *knn_id, uint32_t *knn_I, uint32_t *knn_U,
                   void *stream) {
    c2_status st;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, p, true)) != C2_OK) return st;
    if (!part_id || !part_I || !knn_id || !knn_I || !knn_U) return fail(C2_E_ARG, "NULL pointer");
    C2_TRY(launch_merge(P->indptr, nullptr, P->nnz, P->n, p->t, p->k, part_id, part_I, knn_id,
                        knn_I, knn_U, (hipStream_t)stream),
           "merge");
    return C2_OK;
}

static c2_status build_impl(const c2_profiles *P, const uint64_t *tab, const c2_params *p,
                            int form, const c2_tuning *tune, uint32_t rounds_batched,
                            uint32_t *knn_id, uint32_t *knn_I, uint32_t *knn_U, char *base,
                            size_t ws_bytes, hipStream_t s, uint32_t *rounds_used) {
    const BuildLayout L = build_layout(P->n, P->m, P->nnz, p);
    uint32_t *bucket = reinterpret_cast<uint32_t *>(base + L.bucket);
    uint32_t *members = reinterpret_cast<uint32_t *>(base + L.members);
    uint32_t *cl_off = reinterpret_cast<uint32_t *>(base + L.cl_off);
    uint32_t *cl_cfg = reinterpret_cast<uint32_t *>(base + L.cl_cfg);
    uint32_t *pid = reinterpret_cast<uint32_t *>(base + L.part_id);
    uint32_t *pI = reinterpret_cast<uint32_t *>(base + L.part_I);
    C2_TRY(launch_hash_items(tab, p->t, p->b, P->m, bucket, s), "hash items");
    c2_status st = run_cluster(P, bucket, p, form, tune, rounds_batched, members, cl_off, cl_cfg,
                               base + L.scratch, reinterpret_cast<uint32_t *>(base), s,
                               rounds_used);
    if (st != C2_OK) return st;
    st = run_knn(P, members, cl_off, cl_cfg, p->t, p->k, form, tune, pid, pI, base + L.scratch,
                 ws_bytes - L.scratch, reinterpret_cast<uint32_t *>(base) + 1, s);
    if (st != C2_OK) return st;
    // the local KNN left the profile lengths at the start of its workspace
    KnnWs kw;
    knn_ws_fixed(P->n, p->t * P->n, P->m, &kw);
    const uint32_t *rlen = reinterpret_cast<const uint32_t *>(base + L.scratch + kw.rlen);
    C2_TRY(launch_merge(P->indptr, rlen, P->nnz, P->n, p->t, p->k, pid, pI, knn_id, knn_I, knn_U,
                        s),
           "merge");
    return C2_OK;
}

c2_status c2_build(const c2_profiles *P, const uint64_t *tab, const c2_params *p, int form,
                   const c2_tuning *tune, uint32_t *knn_id, uint32_t *knn_I, uint32_t *knn_U,
                   void *ws, size_t ws_bytes, void *stream) {
    c2_status st;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, p, true)) != C2_OK) return st;
    if ((st = check_form(form)) != C2_OK) return st;
    if (!tab || !knn_id || !knn_I || !knn_U) return fail(C2_E_ARG, "NULL pointer");
    if ((st = check_ws(ws, ws_bytes, build_min_bytes(P->n, P->m, P->nnz, p))) != C2_OK) return st;
    return build_impl(P, tab, p, form, tune, rounds_from(tune), knn_id, knn_I, knn_U,
                      reinterpret_cast<char *>(ws), ws_bytes, (hipStream_t)stream, nullptr);
}

c2_status c2_build_noalloc(const c2_profiles *P, const uint64_t *tab, const c2_params *p,
                           int form, const c2_tuning *tune, uint32_t *knn_id, uint32_t *knn_I,
                           uint32_t *knn_U, uint32_t *status_out, void *stream) {
    c2_status st;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, p, true)) != C2_OK) return st;
    if ((st = check_form(form)) != C2_OK) return st;
    if (!tab || !knn_id || !knn_I || !knn_U) return fail(C2_E_ARG, "NULL pointer");
    const size_t need = c2_workspace_bytes(P->n, P->m, P->nnz, p, C2_OP_BUILD);
    if (need == 0) return C2_E_ARG;
    if (need > kNoAllocBytes)
        return fail(C2_E_WORKSPACE,
                    "c2_build_noalloc: these sizes need %zu bytes of workspace, more than its "
                    "fixed %zu (use c2_build with a caller workspace)", need, kNoAllocBytes);
    char *base = nullptr;
    if ((st = noalloc_base(&base)) != C2_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    st = build_impl(P, tab, p, form, tune, rounds_from(tune), knn_id, knn_I, knn_U, base,
                    kNoAllocBytes, s, nullptr);
    if (st != C2_OK) return st;
    if (status_out) {
        hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(1), 0, s,
                           reinterpret_cast<const uint32_t *>(base), status_out);
        C2_TRY(hipGetLastError(), "status copy");
    }
    return C2_OK;
}

c2_status c2_brute_force(const c2_profiles *P, uint32_t k, uint32_t *knn_id, uint32_t *knn_I,
                         uint32_t *knn_U, void *ws, size_t ws_bytes, void *stream) {
    c2_status st;
    c2_params one = {1, 1, 1, k};
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, &one, true)) != C2_OK) return st;
    if (!knn_id || !knn_I || !knn_U) return fail(C2_E_ARG, "NULL pointer");
    if ((st = check_ws(ws, ws_bytes, brute_head(P->n, k) + knn_min_bytes(P->n, P->n, P->m))) != C2_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    char *base = reinterpret_cast<char *>(ws);
    size_t off = kHeader;
    uint32_t *members = reinterpret_cast<uint32_t *>(base + off);
    off += al(4 * (size_t)P->n);
    uint32_t *cl_off = reinterpret_cast<uint32_t *>(base + off);
    off += al(4 * ((size_t)P->n + 1));
    uint32_t *cl_cfg = reinterpret_cast<uint32_t *>(base + off);
    off += al(8);
    uint32_t *pid = reinterpret_cast<uint32_t *>(base + off);
    off += al(4 * (size_t)P->n * k);
    uint32_t *pI = reinterpret_cast<uint32_t *>(base + off);
    off += al(4 * (size_t)P->n * k);
    C2_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(base), 0, 1, s), "status");
    // one cluster holding every user: members = 0..n-1, cl_off = {0, n}, cl_cfg = {0, 1}
    C2_TRY(launch_iota(members, P->n, s), "brute force setup");
    C2_TRY(launch_fill_u32(cl_off, 0, 1, s), "brute force setup");
    C2_TRY(launch_fill_u32(cl_off + 1, P->n, 1, s), "brute force setup");
    C2_TRY(launch_fill_u32(cl_cfg, 0, 1, s), "brute force setup");
    C2_TRY(launch_fill_u32(cl_cfg + 1, 1, 1, s), "brute force setup");
    st = run_knn(P, members, cl_off, cl_cfg, 1, k, C2_FORM_BATCHED, nullptr, pid, pI, base + off,
                 ws_bytes - off, reinterpret_cast<uint32_t *>(base) + 1, s);
    if (st != C2_OK) return st;
    C2_TRY(launch_merge(P->indptr, nullptr, P->nnz, P->n, 1, k, pid, pI, knn_id, knn_I, knn_U, s),
           "merge");
    return C2_OK;
}

struct c2_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint32_t rounds;
};

c2_status c2_graph_create(const c2_profiles *P, const uint64_t *tab, const c2_params *p,
                          const c2_tuning *tune, uint32_t *knn_id, uint32_t *knn_I,
                          uint32_t *knn_U, void *ws, size_t ws_bytes, void *stream,
                          c2_graph **out) {
    c2_status st;
    if (!out) return fail(C2_E_ARG, "out is NULL");
    *out = nullptr;
    if ((st = check_profiles(P)) != C2_OK) return st;
    if ((st = check_sizes(P->n, P->m, P->nnz, p, true)) != C2_OK) return st;
    if (!tab || !knn_id || !knn_I || !knn_U) return fail(C2_E_ARG, "NULL pointer");
    if ((st = check_ws(ws, ws_bytes, build_min_bytes(P->n, P->m, P->nnz, p))) != C2_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    char *base = reinterpret_cast<char *>(ws);
    // plain build once: learns the number of split rounds and loads the kernels
    uint32_t rounds = 0;
    st = build_impl(P, tab, p, C2_FORM_PLAIN, tune, 0, knn_id, knn_I, knn_U, base, ws_bytes, s,
                    &rounds);
    if (st != C2_OK) return st;
    C2_TRY(hipStreamSynchronize(s), "graph warm-up");
    hipStream_t cap;
    C2_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "capture stream");
    c2_graph *g = new (std::nothrow) c2_graph;
    if (!g) { (void)hipStreamDestroy(cap); return fail(C2_E_ARG, "out of host memory"); }
    g->rounds = rounds + 1;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = build_impl(P, tab, p, C2_FORM_BATCHED, tune, g->rounds, knn_id, knn_I, knn_U, base,
                        ws_bytes, cap, nullptr);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(cap, &graph);
        if (st == C2_OK && e2 != hipSuccess) st = hip_fail(e2, "end capture");
        if (st == C2_OK) {
            g->graph = graph;
            e2 = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
            if (e2 != hipSuccess) st = hip_fail(e2, "graph instantiate");
        } else if (graph) {
            (void)hipGraphDestroy(graph);
            graph = nullptr;
        }
        if (st != C2_OK && graph) (void)hipGraphDestroy(graph);
    } else {
        st = hip_fail(e, "begin capture");
    }
    const hipError_t ed = hipStreamDestroy(cap);
    if (st == C2_OK && ed != hipSuccess) st = hip_fail(ed, "capture stream destroy");
    if (st != C2_OK) {
        delete g;
        return st;
    }
    *out = g;
    return C2_OK;
}

c2_status c2_graph_launch(c2_graph *g, void *stream) {
    if (!g) return fail(C2_E_ARG, "graph is NULL");
    C2_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream), "graph launch");
    return C2_OK;
}

c2_status c2_graph_destroy(c2_graph *g) {
    if (!g) return C2_OK;
    const hipError_t e1 = hipGraphExecDestroy(g->exec);
    const hipError_t e2 = hipGraphDestroy(g->graph);
    delete g;
    if (e1 != hipSuccess) return hip_fail(e1, "graph exec destroy");
    if (e2 != hipSuccess) return hip_fail(e2, "graph destroy");
    return C2_OK;
}

}  // extern "C"
