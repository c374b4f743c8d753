/*
 * c2.h -- C ABI of libc2.so, Cluster-and-Conquer (C^2) KNN-graph construction
 * on AMD MI355X (gfx950).
 *
 * The method (Giakkoupis, Kermarrec, Ruas, Taiani, "Cluster-and-Conquer: When
 * Randomness Meets Graph Locality", arXiv 2010.11497) builds an approximate
 * k-nearest-neighbour graph over users whose profiles are item sets, under
 * Jaccard similarity, in three steps (Section II-C):
 *   1. FastRandomHash clustering with t hash functions into b buckets, with
 *      recursive splitting of clusters larger than N  -> c2_hash_items,
 *      c2_frh_keys, c2_cluster;
 *   2. an exact (brute-force) KNN graph inside every cluster -> c2_local_knn;
 *   3. a merge of each user's t partial lists            -> c2_merge.
 * c2_build runs the three steps; c2_graph_* capture the batched form of
 * c2_build in a HIP graph; c2_brute_force computes the exact graph.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named in c2_profiles and every array argument are DEVICE
 *    pointers unless the comment says "host".  They are owned by the caller;
 *    the library never frees or retains them.  The library keeps no state
 *    between calls except a per-thread error string (c2_last_error) and the
 *    graph objects the caller creates.
 *  - `stream` is a hipStream_t (passed as void*; NULL = the default stream).
 *    Work is enqueued on it and the call returns without waiting, except where
 *    a comment says "synchronous".
 *  - Argument errors are detected on the host before anything is enqueued and
 *    returned as a status; nothing is enqueued then.  Profile contents are only
 *    checked by c2_validate: the other calls assume validated input (on
 *    invalid input they return unspecified results but read and write only
 *    inside the buffers the arguments describe).
 *  - No C++ exception crosses this interface.
 *
 * Similarity order (exact; readings of the paper where it is silent)
 * -------------------------------------------------------------------
 *  For a user u and candidates v, w with I = |P_u & P_x| and U = |P_u | P_x|:
 *  v ranks before w iff I_v * U_w > I_w * U_v, or the products are equal and
 *  v < w.  u is never its own neighbour.  Zero-similarity neighbours are
 *  kept.  A list with fewer than k candidates is padded with id C2_PAD and
 *  I = U = 0.  A neighbour that appears in several partial lists is kept once.
 */
#ifndef C2_H
#define C2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t c2_status;

#define C2_OK 0
#define C2_E_ARG (-1)          /* bad argument (null pointer, size out of range) */
#define C2_E_PROFILE (-2)      /* profile data invalid (c2_validate only) */
#define C2_E_WORKSPACE (-3)    /* workspace smaller than c2_workspace_bytes */
#define C2_E_HIP (-4)          /* a HIP runtime call failed */
#define C2_E_UNSUPPORTED (-5)  /* sizes outside what the library supports */
#define C2_E_INCOMPLETE (-6)   /* batched clustering needed more split rounds */

#define C2_PAD 0xFFFFFFFFu     /* padding id in neighbour lists */

/* Limits of the library: n <= 2^31 - 1 users and t*n < 2^32, m <= 2^19 items
 * (two m-bit dictionary bitmaps per cluster live in the 160 KiB of LDS),
 * nnz < 2^40, every profile shorter than 2^20 items, 1 <= t <= 64,
 * 1 <= b <= 2^31, cap >= 1, 1 <= k <= 32. */

/* Users and their profiles in CSR form (Section II-A: U, I and P_u).
 * Row u is indices[indptr[u] .. indptr[u+1]): strictly increasing item ids
 * < m, at least one item per user. */
typedef struct c2_profiles {
    uint32_t n;               /* users */
    uint32_t m;               /* items */
    uint64_t nnz;             /* indptr[n] */
    const int64_t *indptr;    /* device, [n+1], indptr[0] = 0 */
    const uint32_t *indices;  /* device, [nnz] */
} c2_profiles;

/* Parameters of the method (Section II-D, II-F, IV-C): t hash functions,
 * b buckets per function, cap = N (clusters larger than N are split), k
 * neighbours per user. */
typedef struct c2_params {
    uint32_t t, b, cap, k;
} c2_params;

/* Execution forms of the same arithmetic. */
#define C2_FORM_PLAIN 0    /* host-driven: cluster tables read back, one launch per stage */
#define C2_FORM_BATCHED 1  /* device-driven: no host sync, persistent local-KNN launch over
                              all clusters of all configurations, largest first; capturable */

/* Tile and schedule choices of c2_local_knn (written by the autotuner).  A
 * NULL pointer or a zero field means the built-in default.  None of them
 * changes a result. */
typedef struct c2_tuning {
    uint32_t mfma_min_rows;   /* clusters with at least this many members use the
                                 MFMA path, smaller ones the bitmap path (default 2) */
    uint32_t persistent_wgs;  /* MFMA path, batched form: persistent waves (four per
                                 256-thread block; default 2048, two per SIMD) */
    uint32_t split_rounds;    /* split rounds enqueued by the batched form */
    uint32_t group_tiles;     /* MFMA path: a row block whose cluster spans more than this many
                                 column tiles is split into up to 4 work items over disjoint
                                 column ranges (default 16) */
    uint32_t cluster_path;    /* 0: automatic; 1: grid rounds (any size); 2: one workgroup per
                                 configuration with every split round in LDS (n <= 8192 and
                                 bit_width(b) <= 20; otherwise the grid rounds are used) */
    void *ev_knn_begin;       /* optional hipEvent_t (host handles, caller-owned): recorded on */
    void *ev_knn_end;         /* the stream right before / after the pairwise local-KNN kernel */
    uint32_t tile32_max;      /* MFMA path tile shape per cluster: clusters of at most this many */
    uint32_t tile64_max;      /* members take 32 x 32 tiles (default 32), of at most tile64_max
                                 64 x 64 tiles (default 64), larger ones 64-row x 128-column
                                 tiles */
} c2_tuning;

/* Workspace queries: which call the size is for. */
#define C2_OP_VALIDATE 0
#define C2_OP_CLUSTER 1
#define C2_OP_LOCAL_KNN 2
#define C2_OP_BUILD 3
#define C2_OP_BRUTE_FORCE 4
#define C2_OP_FINGERPRINT 5
#define C2_OP_LOCAL_KNN_ALG2 6
#define C2_OP_LOCAL_KNN_MIN 7  /* the smallest workspace c2_local_knn accepts: its fixed part
                                  plus a 4096-byte store (the store takes every byte beyond
                                  the fixed part) */

/* Message for the last non-OK status returned on this thread (host string,
 * valid until the next call on this thread). */
const char *c2_last_error(void);

/* Bytes of device workspace the call `op` needs for these sizes (host-only,
 * no device work).  Returns 0 and sets the error string if the sizes are
 * unsupported. */
size_t c2_workspace_bytes(uint32_t n, uint32_t m, uint64_t nnz, const c2_params *p, int op);

/* Checks the profiles: indptr[0] = 0, indptr non-decreasing with every row
 * non-empty, indptr[n] = nnz, items < m and strictly increasing in each row.
 * Synchronous: returns C2_OK or C2_E_PROFILE.  ws: C2_OP_VALIDATE bytes. */
c2_status c2_validate(const c2_profiles *P, void *ws, size_t ws_bytes, void *stream);

/* Item hashes (Section II-D; Eq. 3's generative function h_j, one per
 * configuration): bucket[j*m + i] = h_j(i) in [0, b) for j < t, i < m.
 * h_j is simple tabulation hashing of the item id's 4 bytes with the random
 * 64-bit tables tab[j][0..3][0..255] (device, uint64[t][4][256], drawn by the
 * caller), x = T0[i & 255] ^ T1[(i >> 8) & 255] ^ T2[(i >> 16) & 255] ^
 * T3[i >> 24], reduced to [0, b) as the high word of the 128-bit product x * b.
 * (The paper names Jenkins' hash without variant or seeding; this function is
 * this library's reading.) */
c2_status c2_hash_items(const uint64_t *tab, uint32_t t, uint32_t b, uint32_t m,
                        uint32_t *bucket, void *stream);

/* FastRandomHash (Eq. 3): keys[j*n + u] = min_{i in P_u} bucket[j*m + i]. */
c2_status c2_frh_keys(const c2_profiles *P, const uint32_t *bucket, uint32_t t,
                      uint32_t *keys, void *stream);

/* Step 1 (Algorithm 1 and the recursive splitting of Section II-D, Fig. 3).
 * Input: bucket[t][m] from c2_hash_items (or any table of values < b).
 * Users of configuration j are grouped by H_j(u); a cluster with index eta
 * holding more than cap users is split by H\eta(u) = min{h_j(i) : i in P_u,
 * h_j(i) > eta}: users sharing a new value form a new cluster (split again
 * if it is still larger than cap); users with no value above eta, or alone
 * with theirs, stay behind and form a final cluster that is never split.
 * Outputs (device):
 *   members[t*n]   configuration j's users occupy members[j*n .. j*n+n),
 *                  grouped by final cluster, ascending inside each cluster;
 *   cl_off[t*n+1]  cluster c holds members[cl_off[c] .. cl_off[c+1]); only
 *                  the first (total clusters + 1) entries are written;
 *   cl_cfg_off[t+1] clusters of configuration j are [cl_cfg_off[j], cl_cfg_off[j+1]).
 * Cluster order: ascending top-level hash value; a split cluster is replaced
 * by its sub-clusters in ascending new value (each recursively), followed by
 * the users that stayed behind.
 * form: C2_FORM_PLAIN reads the number of clusters still to split after every
 * round (synchronises the stream once per round); C2_FORM_BATCHED enqueues
 * tune->split_rounds rounds (default 8) without synchronising and records on
 * the device whether that was enough (see c2_check_complete).
 * ws: C2_OP_CLUSTER bytes; also holds the status read by c2_check_complete. */
c2_status c2_cluster(const c2_profiles *P, const uint32_t *bucket, const c2_params *p,
                     int form, const c2_tuning *tune, uint32_t *members, uint32_t *cl_off,
                     uint32_t *cl_cfg_off, void *ws, size_t ws_bytes, void *stream);

/* Step 1 with the top-level buckets given per user instead of computed by
 * FastRandomHash: keys[j*n + u] < p->b is user u's bucket in configuration j
 * (e.g. from a learned assigner, c2_assign_keys).  Users with equal keys form
 * a cluster; a cluster larger than p->cap is split by FastRandomHash on
 * `bucket` (as c2_hash_items writes it, values < p->b), starting from H_j(u)
 * and then recursively as in c2_cluster.  Cluster order: ascending key, a
 * split cluster replaced as in c2_cluster.  Always runs the grid rounds
 * (tune->cluster_path is not used).  Outputs, forms and ws as c2_cluster. */
c2_status c2_cluster_keys(const c2_profiles *P, const uint32_t *keys, const uint32_t *bucket,
                          const c2_params *p, int form, const c2_tuning *tune, uint32_t *members,
                          uint32_t *cl_off, uint32_t *cl_cfg_off, void *ws, size_t ws_bytes,
                          void *stream);

/* Synchronous: C2_OK if the last batched c2_cluster / c2_build that used this
 * workspace split every oversized cluster and the last local KNN found room
 * for every cluster's dictionary rows; C2_E_INCOMPLETE if split rounds were
 * missing, C2_E_WORKSPACE if the store was too small (the results are then
 * invalid). */
c2_status c2_check_complete(const void *ws, void *stream);

/* Step 2 (Section II-F, Algorithm 2, brute-force branch): for every cluster
 * of any partition given as (members, cl_off, cl_cfg_off) in c2_cluster's
 * layout (members need not be sorted), and every member u of a
 * configuration-j cluster C, the k best users of C \ {u}:
 *   part_id[(u*t + j)*k + r], part_I[(u*t + j)*k + r]  (device, [n][t][k]),
 * best first, padded with (C2_PAD, 0).  Every (u, j) slot is written exactly
 * once, so every user must appear once per configuration.
 * Pairwise intersections are exact integer counts over bit rows built per
 * cluster from the CSR lists, over the cluster's dictionary (the items held
 * by at least two of its members; no other item can be in an intersection):
 * the MFMA path expands 64-position chunks of the rows to fp4 (e2m1) values 0
 * and 1 and multiplies them with the gfx950 block-scaled MFMA at unit scale,
 * whose fp32 sums of 0/1 products are exact integer counts (used when every
 * profile has fewer than 2^15 items, where an exact 32-bit similarity key
 * exists); the bitmap path uses AND and population count.
 * form: C2_FORM_PLAIN reads the cluster table back (synchronises once) and
 * launches one grid over (cluster, row block) pairs in cluster order;
 * C2_FORM_BATCHED plans on the device and runs one persistent launch that
 * takes (cluster, row block) pairs largest cluster first.
 * tune: NULL or c2_tuning.
 * ws: C2_OP_LOCAL_KNN bytes by default.  The rows live in a store that takes
 * all of the workspace beyond a fixed part, so a caller may pass more (or
 * less, down to the fixed part and 4 KiB); the default holds about four
 * words per (configuration, profile item), which covered every workload
 * measured.  When a partition's rows do not fit, the plain form returns
 * C2_E_WORKSPACE and the batched form leaves its results invalid and makes
 * c2_check_complete(ws) return C2_E_WORKSPACE.  Either way, after the call
 * bytes 8..15 of ws hold (u64, device, in stream order) the store bytes / 4
 * that the partition needs, so a caller can retry with C2_OP_LOCAL_KNN_MIN
 * bytes + 4 times that. */
c2_status c2_local_knn(const c2_profiles *P, const uint32_t *members, const uint32_t *cl_off,
                       const uint32_t *cl_cfg_off, const c2_params *p, int form,
                       const c2_tuning *tune, uint32_t *part_id, uint32_t *part_I,
                       void *ws, size_t ws_bytes, void *stream);

/* Parameters of Algorithm 2's Hyrec branch (Section II-F; Hyrec, delta and the
 * iteration cap in Section IV-B and IV-C; rho = 5 in Section II-F). */
typedef struct c2_hyrec {
    uint32_t rho;       /* clusters of at least rho*k^2 members take Hyrec */
    uint32_t max_iter;  /* iterations at most (30 in the paper) */
    double delta;       /* stop when fewer than delta*k*|C| entries changed (0.001) */
    uint64_t seed;      /* seed of the initial random graph */
} c2_hyrec;

/* Step 2 as Algorithm 2: c2_local_knn (brute force) in clusters of fewer than
 * rho*k^2 members, Hyrec in the others.  The paper does not fix Hyrec's
 * random choices; this form is deterministic: member a's initial list is the
 * k best distinct of k uniform draws among the cluster's other members, draw
 * q being SplitMix64 output number c + 1 from state `seed`, c = (cluster <<
 * 40) | (a << 12) | q (cluster = index in cl_off, a = position in the
 * cluster), reduced mod (|C| - 1) and shifted past a.  Each iteration then
 * replaces, for all members at once, a's list by the k best distinct of its
 * list and its neighbours' lists (a excluded), in the exact order.  It stops
 * after an iteration that changed fewer than delta*k*|C| list entries, or
 * after max_iter iterations.  Plain form only (synchronous: it reads the
 * partition and the update counts on the host).  C2_E_UNSUPPORTED if a Hyrec
 * cluster is needed and some profile holds 2^15 items or more.  Outputs as
 * c2_local_knn.  ws: C2_OP_LOCAL_KNN_ALG2 bytes. */
c2_status c2_local_knn_alg2(const c2_profiles *P, const uint32_t *members, const uint32_t *cl_off,
                            const uint32_t *cl_cfg_off, const c2_params *p, const c2_hyrec *hy,
                            const c2_tuning *tune, uint32_t *part_id, uint32_t *part_I, void *ws,
                            size_t ws_bytes, void *stream);

/* Step 3 (Section II-G, Algorithm 3): knn(u) = the k best entries of the union
 * of u's t partial lists (part_* as written by c2_local_knn), each neighbour
 * once, best first, padded with (C2_PAD, 0, 0).  Outputs (device, [n][k]):
 * knn_id, knn_I = |P_u & P_v|, knn_U = |P_u | P_v|. */
c2_status c2_merge(const c2_profiles *P, const uint32_t *part_id, const uint32_t *part_I,
                   const c2_params *p, uint32_t *knn_id, uint32_t *knn_I, uint32_t *knn_U,
                   void *stream);

/* The whole method: c2_hash_items, c2_frh_keys, c2_cluster, c2_local_knn,
 * c2_merge on the workspace.  tab as in c2_hash_items.  Outputs as c2_merge.
 * ws: C2_OP_BUILD bytes by default; the store of the local KNN takes what is
 * left after the other stages' buffers (see c2_local_knn). */
c2_status c2_build(const c2_profiles *P, const uint64_t *tab, const c2_params *p, int form,
                   const c2_tuning *tune, uint32_t *knn_id, uint32_t *knn_I, uint32_t *knn_U,
                   void *ws, size_t ws_bytes, void *stream);

/* c2_build for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, forms, arithmetic and outputs as c2_build, but the workspace is
 * a fixed array of 256 MiB in device memory that the library holds on each
 * GPU it runs on until the process ends; the call itself allocates nothing.
 * C2_E_WORKSPACE (nothing enqueued) when c2_workspace_bytes(..., C2_OP_BUILD)
 * exceeds 256 MiB.  Every call on one GPU uses that GPU's one array, so calls
 * that overlap on one GPU (other streams, other host threads) race and give
 * undefined results; calls on one stream are ordered and safe.
 * status_out: NULL, or a device u32 that receives, in stream order, 0 if the
 * build split every oversized cluster and 1 if the batched form needed more
 * split rounds (the c2_check_complete condition; the plain form writes 0). */
c2_status c2_build_noalloc(const c2_profiles *P, const uint64_t *tab, const c2_params *p,
                           int form, const c2_tuning *tune, uint32_t *knn_id, uint32_t *knn_I,
                           uint32_t *knn_U, uint32_t *status_out, void *stream);

/* The exact KNN graph (Section IV-B, brute force): c2_local_knn on one cluster
 * holding all users.  Outputs as c2_merge.  ws: C2_OP_BRUTE_FORCE bytes. */
c2_status c2_brute_force(const c2_profiles *P, uint32_t k, uint32_t *knn_id, uint32_t *knn_I,
                         uint32_t *knn_U, void *ws, size_t ws_bytes, void *stream);

/* GoldFinger fingerprints (Section II-F; 1024 bits in Section IV-C; their
 * effect in Section V-D, Table 5): the local similarities may be computed on
 * a compact B-bit vector per user instead of the profile.  The fingerprint of
 * user u is the set F_u = { g(i) : i in P_u } of bit positions, g an item hash
 * into [0, B) (c2_hash_items with t = 1, b = B and tables of its own), and
 * the Jaccard index of F_u and F_v is the estimate of the users' similarity.
 * The fingerprints are written as CSR profiles over B items, so that
 * c2_local_knn, c2_merge and c2_brute_force run on them unchanged (then
 * knn_I = |F_u & F_v| and knn_U = |F_u | F_v|).
 *   g           device, [m], every value < B
 *   B           bits, 1..8192
 *   fp_indptr   device int64 [n+1]; fp_indices device u32 with room for
 *               P->nnz entries (|F_u| <= |P_u|); each row strictly increasing
 *   fp_nnz      host; receives fp_indptr[n]
 * Synchronous.  C2_E_PROFILE if a row holds an item >= m, C2_E_ARG if g
 * holds a value >= B (outputs then undefined).  ws: C2_OP_FINGERPRINT bytes,
 * queried with p->b = B (the other fields of p are not used). */
c2_status c2_fingerprint(const c2_profiles *P, const uint32_t *g, uint32_t B, int64_t *fp_indptr,
                         uint32_t *fp_indices, uint64_t *fp_nnz, void *ws, size_t ws_bytes,
                         void *stream);

/* Learned cluster assigner: a per-user bucket in each of the t configurations
 * from a small network over the user's items, in place of FastRandomHash's
 * top-level grouping (then c2_cluster_keys, c2_local_knn and c2_merge, whose
 * exact arithmetic is unchanged).  FastRandomHash remains the fallback: for
 * users whose best logit does not clear the second by min_gap, and for the
 * split of groups larger than the cap.  The paper has no such component;
 * model and fallback rules are this library's own.
 *   e_u = mean over i in P_u of E[i]      (fp32 sum, rounded to bf16)
 *   h_u = ReLU(W1 e_u + b1)               (fp32, rounded to bf16)
 *   z_u = W2 h_u + b2                     (bf16 products, fp32 sums)
 *   key_j(u) = argmax over c < b of z_u[j*b + c], lowest c on ties.
 * Weights (device, row-major, caller-owned): E bf16 [m][C2_ASSIGN_DIM],
 * W1 bf16 [C2_ASSIGN_HIDDEN][C2_ASSIGN_DIM], b1 fp32 [C2_ASSIGN_HIDDEN],
 * W2 bf16 [t*b][C2_ASSIGN_HIDDEN], b2 fp32 [t*b].  bf16 is passed as its
 * 16-bit pattern (uint16_t). */
#define C2_ASSIGN_DIM 64
#define C2_ASSIGN_HIDDEN 256

/* h [n][C2_ASSIGN_HIDDEN] bf16 (device) = h_u for every user. */
c2_status c2_assign_hidden(const c2_profiles *P, const uint16_t *E, const uint16_t *W1,
                           const float *b1, uint16_t *h, void *stream);

/* keys [t][n] (device u32): key_j(u), or b + frh_keys[j*n + u] when frh_keys
 * (device [t][n], values < b, e.g. c2_frh_keys) is not NULL and the gap
 * z(top 1) - z(top 2) of head j is below min_gap.  gap [t][n] (device fp32,
 * may be NULL) receives that gap.  Cluster the keys with p->b >= 2b when the
 * fallback is on (b otherwise).  b: a multiple of 64.  The n x t*b logits are
 * never written: the argmax runs in the product's epilogue. */
c2_status c2_assign_keys(const uint16_t *h, uint32_t n, const uint16_t *W2, const float *b2,
                         uint32_t t, uint32_t b, const uint32_t *frh_keys, float min_gap,
                         uint32_t *keys, float *gap, void *stream);

/* Training support.  out [nrows][C2_ASSIGN_DIM] fp32 (device) = e_u in fp32
 * (not rounded) for u = rows[r] (device u32 [nrows]; NULL = rows 0..nrows-1). */
c2_status c2_embag(const c2_profiles *P, const uint32_t *rows, uint32_t nrows, const uint16_t *E,
                   float *out, void *stream);

/* dE [m][C2_ASSIGN_DIM] fp32 (device) += the gradient of the mean bag
 * through out, given grad [nrows][C2_ASSIGN_DIM] fp32: each item of row r gets
 * grad[r] / |P_u|.  Atomic fp32 adds: the summation order is not fixed. */
c2_status c2_embag_backward(const c2_profiles *P, const uint32_t *rows, uint32_t nrows,
                            const float *grad, float *dE, void *stream);

/* One training step of the assigner: loss and gradients of a batch of
 * nrows = 2B profile rows (rows, device u32 [nrows]): rows 0..B-1 are users
 * u_i, rows B..2B-1 exact neighbours v_i of theirs, and v_{i-1 mod B} is u_i's
 * non-neighbour.  With p the per-head softmax of the logits z (the forward
 * above: e and h rounded to bf16, z = h W2^T + b2 in fp32), s_i = <p(u_i),
 * p(v_i)>, n_i = <p(u_i), p(v_{i-1})>, q = the batch mean of p and H the
 * entropy, averaged over heads and pairs or rows:
 *   L = -mean log max(s, 1e-12) - w_neg mean log(1 - clip(n, 0, 1 - 1e-6))
 *       + w_bal mean_j sum_c q log(q b + 1e-12) + w_ent mean H
 * (the library's own objective; the paper has no learned assigner).
 * Outputs (device, caller-owned): loss fp32 [5] = total, pair, non-neighbour,
 * balance and entropy terms; dE fp32 [m][C2_ASSIGN_DIM] (overwritten),
 * dW1 fp32 [C2_ASSIGN_HIDDEN][C2_ASSIGN_DIM], db1 fp32 [C2_ASSIGN_HIDDEN],
 * dW2 fp32 [t*b][C2_ASSIGN_HIDDEN], db2 fp32 [t*b]: the gradients of L with
 * respect to the weights the forward read (the bf16 copies), the roundings
 * passing gradients unchanged.  The products run on bf16 MFMA with fp32
 * sums; the logits' gradient is rounded to bf16 as their operand.  b: a
 * multiple of 64; nrows even and >= 2.  ws: at least
 * c2_assign_train_workspace_bytes(nrows, t, b) bytes (device).  Asynchronous,
 * capturable (no host synchronisation, no memset). */
typedef struct c2_train_opts {
    float w_neg, w_bal, w_ent;
} c2_train_opts;

size_t c2_assign_train_workspace_bytes(uint32_t nrows, uint32_t t, uint32_t b);

c2_status c2_assign_train_grad(const c2_profiles *P, const uint32_t *rows, uint32_t nrows,
                               const uint16_t *E, const uint16_t *W1, const float *b1,
                               const uint16_t *W2, const float *b2, uint32_t t, uint32_t b,
                               const c2_train_opts *opts, float *loss, float *dE, float *dW1,
                               float *db1, float *dW2, float *db2, void *ws, size_t ws_bytes,
                               void *stream);

/* Adam (Kingma and Ba, Algorithm 1) on count fp32 parameters in place:
 * m1 = beta1 m1 + (1 - beta1) g, m2 = beta2 m2 + (1 - beta2) g^2,
 * param -= lr (m1 / (1 - beta1^step)) / (sqrt(m2 / (1 - beta2^step)) + eps),
 * step counted from 1.  param_bf16 (may be NULL) receives the updated values
 * rounded to bf16, the copy the next forward reads.  All device. */
c2_status c2_adam_step(float *param, const float *grad, float *m1, float *m2, uint64_t count,
                       float lr, float beta1, float beta2, float eps, uint32_t step,
                       uint16_t *param_bf16, void *stream);

/* HIP-graph form of c2_build (C2_FORM_BATCHED) on fixed buffers.  Create
 * runs one plain clustering synchronously to learn how many split rounds the
 * data needs, then captures the batched build with that many rounds (plus
 * one) on `stream`.  Launch replays it (asynchronous); after it, the result is
 * valid if c2_check_complete(ws) is C2_OK (data changed in place may need
 * more rounds).  Destroy releases the graph (host handle) and frees it even
 * when the runtime reports an error, which it returns as C2_E_HIP. */
typedef struct c2_graph c2_graph;
c2_status c2_graph_create(const c2_profiles *P, const uint64_t *tab, const c2_params *p,
                          const c2_tuning *tune, uint32_t *knn_id, uint32_t *knn_I,
                          uint32_t *knn_U, void *ws, size_t ws_bytes, void *stream,
                          c2_graph **out);
c2_status c2_graph_launch(c2_graph *g, void *stream);
c2_status c2_graph_destroy(c2_graph *g);

#ifdef __cplusplus
}
#endif

#endif /* C2_H */
