// Launchers and workspace descriptors shared by the host-side API.
#pragma once

#include "c2_internal.h"

namespace c2 {

constexpr uint32_t kMaxRounds = 4096;

// ---- hashing / validation
hipError_t launch_hash_items(const uint64_t *tab, uint32_t t, uint32_t b, uint32_t m,
                             uint32_t *bucket, hipStream_t s);
// The same keys through an item-major copy of the table (bt: t * m u32 of scratch).
hipError_t launch_frh_keys_rows(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                                uint32_t n, uint32_t m, const uint32_t *bucket, uint32_t t,
                                uint32_t b, uint32_t *bt, uint32_t *keys, hipStream_t s);
hipError_t launch_frh_keys(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                           uint32_t n, uint32_t m, const uint32_t *bucket, uint32_t t, uint32_t b,
                           uint32_t *keys, hipStream_t s);
hipError_t launch_validate(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                           uint32_t n, uint32_t m, uint32_t *err, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint32_t n, hipStream_t s);
hipError_t launch_iota(uint32_t *p, uint32_t n, hipStream_t s);

// ---- GoldFinger fingerprints
constexpr uint32_t kFpMaxBits = 8192;
size_t fingerprint_ws_bytes(uint32_t n, uint32_t B);
hipError_t launch_fingerprint(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                              uint32_t n, uint32_t m, const uint32_t *g, uint32_t B,
                              int64_t *fp_indptr, uint32_t *fp_indices, void *ws, uint32_t *err,
                              hipStream_t s);

// ---- learned assigner (embedding bag dim 64, hidden 256)
constexpr int kAsgDim = 64;
constexpr int kAsgHidden = 256;
hipError_t launch_assign_hidden(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                                uint32_t n, uint32_t m, const uint16_t *E, const uint16_t *W1,
                                const float *b1, uint16_t *h, hipStream_t s);
hipError_t launch_assign_keys(const uint16_t *h, uint32_t n, const uint16_t *W2, const float *b2,
                              uint32_t t, uint32_t b, const uint32_t *frh, float min_gap,
                              uint32_t *keys, float *gap, hipStream_t s);
hipError_t launch_embag(const int64_t *indptr, const uint32_t *indices, uint64_t nnz, uint32_t n,
                        uint32_t m, const uint32_t *rows, uint32_t nrows, const uint16_t *E,
                        float *out, hipStream_t s);
hipError_t launch_embag_backward(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                                 uint32_t n, uint32_t m, const uint32_t *rows, uint32_t nrows,
                                 const float *grad, float *dE, hipStream_t s);

// ---- training of the assigner
size_t train_ws_bytes(uint32_t nrows, uint32_t t, uint32_t b);
hipError_t launch_train_grad(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                             uint32_t n, uint32_t m, const uint32_t *rows, uint32_t R,
                             const uint16_t *E, const uint16_t *W1, const float *b1,
                             const uint16_t *W2, const float *b2, uint32_t t, uint32_t b,
                             float w_neg, float w_bal, float w_ent, float *loss, float *dE,
                             float *dW1, float *db1, float *dW2, float *db2, void *ws,
                             hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m1, float *m2, size_t n, float lr,
                       float beta1, float beta2, float eps, float bc1, float bc2, uint16_t *p16,
                       hipStream_t s);

// ---- clustering
struct ClusterDims {
    size_t NE;  // t*n slots
    size_t NP;  // most segments that can be split in one round
    size_t TM;  // t*m: the item-major bucket table of the top-level keys
};
struct ClusterWs {  // byte offsets inside the clustering workspace
    size_t E_seg, S_state, S_eta1, S_len, mark, mtmp, A_uid, A_rank, P_start, P_len, P_state,
        P_q0, key, key_alt, val, val_alt, hist, htmp, glb, glen, flg, ftmp, keys0, bt, ctr, status,
        total;
};
struct ClusterPtrs {
    uint32_t *E_uid, *E_seg, *S_state, *S_eta1, *S_len;
    uint64_t *mark, *mtmp;
    uint32_t *A_uid, *A_rank, *P_start, *P_len, *P_state, *P_q0;
    uint64_t *key, *key_alt;
    uint32_t *val, *val_alt, *hist, *htmp, *glb, *glen;
    uint64_t *flg, *ftmp;
    uint32_t *keys0, *bt, *ctr, *status;
};
struct ClusterArgs {
    const int64_t *indptr;
    const uint32_t *indices;
    uint64_t nnz;
    uint32_t n, m, t, b, bb, cap;
    const uint32_t *bucket;
    uint32_t NE, NP;
    // top-level keys given per user ([t][n], < b) instead of H_j(u); the
    // oversized top-level groups are then split by FastRandomHash from H_j(u)
    const uint32_t *keys_in = nullptr;
};
size_t cluster_ws_elems(const ClusterDims &d, ClusterWs *w);
// one workgroup per configuration (n <= kWgMaxN), all split rounds in LDS
constexpr uint32_t kWgMaxN = 8192;
constexpr int kSigD = 4;  // smallest distinct hash values kept per (configuration, user)
size_t cluster_wg_ws_bytes(uint32_t n, uint32_t t);
bool cluster_wg_fits(uint32_t n, uint32_t b);
hipError_t cluster_wg_run(const ClusterArgs &a, uint32_t *members, uint32_t *cl_off,
                          uint32_t *cl_cfg_off, char *scratch, uint32_t *status,
                          uint32_t max_rounds, uint32_t **rctr_out, hipStream_t s);
hipError_t cluster_init(const ClusterArgs &a, const ClusterPtrs &c, hipStream_t s);
hipError_t cluster_round(const ClusterArgs &a, const ClusterPtrs &c, uint32_t round,
                         hipStream_t s);
hipError_t cluster_finish(const ClusterArgs &a, const ClusterPtrs &c, uint32_t rounds,
                          uint32_t *cl_off, uint32_t *cl_cfg_off, hipStream_t s);

// ---- local KNN
struct KnnArgs {
    const int64_t *indptr;
    const uint32_t *indices;
    uint64_t nnz;
    uint32_t n, m, t, k;
    const uint32_t *members, *cl_off, *cl_cfg_off;
    uint32_t NE;  // t*n member slots
    uint32_t Wm;  // words of an item bitmap (m bits): the dictionary maps
    uint32_t *part_id, *part_I;
};
struct KnnWs {  // byte offsets; the store takes the rest of the region
    size_t rlen, cnt, items_m, items_b, slots, sbase, rb_done, htmp, ctmp, ctr, bmax, pc,
        ccls, cpos, cw, coff, ccur, dslot, dmap, rlist, store, total;
};
struct KnnPtrs {
    uint32_t *rlen;
    uint64_t *cnt, *items_m, *items_b;
    uint32_t *slots, *sbase, *rb_done;
    uint32_t *htmp;
    uint64_t *ctmp;
    uint32_t *ctr, *bmax, *pc, *ccls, *cpos;
    uint32_t *cw;                  // words per dictionary row of each cluster, 0 = not staged
    uint64_t *coff;                // first word of each cluster's rows in the store
    unsigned long long *ccur;      // allocation cursor of the store
    uint32_t *dslot, *dmap;        // dictionary maps of the clusters larger than kBigS
    uint64_t *rlist;               // row work of those clusters (cluster, first 32-row unit, units)
    uint32_t *store;               // the rows of every cluster over its dictionary
    uint64_t store_words;          // capacity of the store
    uint32_t *status;              // set to 1 when the store is too small (caller's header word)
};
// Workspace of the local KNN without the store, and the store's default size.
size_t knn_ws_fixed(uint32_t n, uint32_t NE, uint32_t m, KnnWs *w);
size_t knn_store_default_bytes(uint32_t n, uint32_t NE, uint32_t m, uint64_t nnz, uint32_t t);
uint32_t dict_words(uint32_t m);
// Full bit rows over all items (words per row), for the Hyrec branch.
uint32_t full_row_words(uint32_t m);
hipError_t launch_user_bits(const int64_t *indptr, const uint32_t *indices, uint64_t nnz,
                            uint32_t n, uint32_t m, uint32_t *rows, hipStream_t s);
struct KnnOpts {
    uint32_t persistent_wgs = 0;
    uint32_t mfma_min = 0;
    uint32_t group_tiles = 0;
    uint32_t tile32_max = 0, tile64_max = 0;  // cluster sizes up to which 32- / 64-row tiles are used
    hipEvent_t ev_begin = nullptr, ev_end = nullptr;
};
// Both return hipErrorOutOfMemory (plain form) when the store cannot hold the
// partition's dictionary rows; the batched form sets *status instead.
hipError_t knn_plain(const KnnArgs &a, const KnnPtrs &w, const KnnOpts &o, hipStream_t s);
hipError_t knn_batched(const KnnArgs &a, const KnnPtrs &w, const KnnOpts &o, hipStream_t s);

// ---- Hyrec branch of Algorithm 2
hipError_t launch_hyrec_step(const uint32_t *rows, const uint32_t *rlen, uint32_t W,
                             const uint32_t *S, uint32_t s, uint32_t k, uint32_t cl,
                             uint64_t seed, bool init, const uint64_t *okey, uint64_t *nkey,
                             uint32_t *nI, uint32_t *updates, hipStream_t st);
hipError_t launch_hyrec_out(const uint32_t *S, uint32_t s, uint32_t k, uint32_t j, uint32_t t,
                            const uint64_t *key, const uint32_t *I, uint32_t *part_id,
                            uint32_t *part_I, hipStream_t st);

// ---- merge
// ulen: the profile lengths when the caller has them, else nullptr (read from indptr)
hipError_t launch_merge(const int64_t *indptr, const uint32_t *ulen, uint64_t nnz, uint32_t n,
                        uint32_t t, uint32_t k, const uint32_t *part_id, const uint32_t *part_I,
                        uint32_t *knn_id, uint32_t *knn_I, uint32_t *knn_U, hipStream_t s);

}  // namespace c2
