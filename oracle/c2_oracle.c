/*
 * c2_oracle.c -- plain CPU oracle for the Cluster-and-Conquer (C^2) hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The GPU library never links,
 * includes or calls it, and this file shares no code with it.
 *
 * It computes, slowly and plainly, what the paper defines:
 *   - Jaccard similarity |Pu & Pv| / |Pu | Pv| over item-set profiles
 *     (Section II-A), compared exactly as integer cross products, ties broken
 *     by the smaller neighbour id;
 *   - the exact KNN graph by brute force (Section IV-B, "Brute force");
 *   - FastRandomHash H(u) = min over the profile of h(i)  (Eq. 3), with t
 *     hash functions giving t clustering configurations (Algorithm 1);
 *   - recursive splitting of clusters larger than N with
 *     H\eta(u) = min{ h(i) : i in Pu, h(i) > eta }  (Section II-D, Fig. 3);
 *   - brute-force local KNN inside every cluster, clusters taken largest first
 *     from a size-ordered queue by a pool of threads (Section II-F,
 *     Algorithm 2, brute-force branch);
 *   - the merge of each user's t partial lists into one bounded list
 *     (Section II-G, Algorithm 3).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - a user is not its own neighbour;
 *   - the order on candidates is J descending, then neighbour id ascending;
 *   - zero-similarity neighbours are kept; rows with fewer than k candidates
 *     are padded with id 0xFFFFFFFF and I = 0;
 *   - a neighbour found in several partial lists is kept once;
 *   - buckets are numbered [0, b) instead of [1, b];
 *   - a cluster is split iff its size is strictly larger than N; the users
 *     that stay behind (no item hashing above eta, or alone in their new
 *     cluster) form a final cluster that is never split again;
 *   - a sub-cluster is a different cluster from a top-level cluster with the
 *     same hash value;
 *   - the item hash is simple tabulation hashing over the 4 bytes of the item
 *     id with 64-bit random tables, reduced to [0, b) by the high word of the
 *     128-bit product x*b (the paper names Jenkins' hash without a variant or
 *     seeding).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORC_PAD 0xFFFFFFFFu
#define ORC_NONE 0xFFFFFFFFFFFFFFFFull

/* ---------------------------------------------------------------- order -- */

/* Does candidate a = (Ia, Ua, va) rank before candidate b for the same user?
 * J_a > J_b  <=>  Ia * Ub > Ib * Ua  (all U >= 1), ties go to the smaller id. */
static int better(uint32_t Ia, uint32_t Ua, uint32_t va,
                  uint32_t Ib, uint32_t Ub, uint32_t vb)
{
    uint64_t l = (uint64_t)Ia * Ub, r = (uint64_t)Ib * Ua;
    if (l != r) return l > r;
    return va < vb;
}

typedef struct { uint32_t v, I, U; } cand_t;

static int cand_cmp(const void *pa, const void *pb)
{
    const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
    if (better(a->I, a->U, a->v, b->I, b->U, b->v)) return -1;
    if (better(b->I, b->U, b->v, a->I, a->U, a->v)) return 1;
    return 0;
}

/* ----------------------------------------------------------- validation -- */

/* 0 = ok, -1 = bad sizes, -2 = bad profile (empty, unsorted, duplicate or
 * out-of-range item). */
int orc_validate(uint32_t n, uint32_t m, const int64_t *indptr,
                 const uint32_t *indices)
{
    if (n == 0 || m == 0) return -1;
    if (indptr[0] != 0) return -2;
    for (uint32_t u = 0; u < n; ++u) {
        int64_t a = indptr[u], e = indptr[u + 1];
        if (e <= a) return -2;
        for (int64_t p = a; p < e; ++p) {
            if (indices[p] >= m) return -2;
            if (p > a && indices[p] <= indices[p - 1]) return -2;
        }
    }
    return 0;
}

/* ------------------------------------------------------------- hashing -- */

/* h_j(i) for j < t, i < m into bucket[j*m + i].  tab is uint64[t][4][256]. */
void orc_hash_items(const uint64_t *tab, uint32_t t, uint64_t b, uint32_t m,
                    uint32_t *bucket)
{
    for (uint32_t j = 0; j < t; ++j) {
        const uint64_t *T = tab + (size_t)j * 4 * 256;
        for (uint32_t i = 0; i < m; ++i) {
            uint64_t x = T[0 * 256 + (i & 255u)] ^ T[1 * 256 + ((i >> 8) & 255u)]
                       ^ T[2 * 256 + ((i >> 16) & 255u)] ^ T[3 * 256 + (i >> 24)];
            unsigned __int128 p = (unsigned __int128)x * b;
            bucket[(size_t)j * m + i] = (uint32_t)(p >> 64);
        }
    }
}

/* FastRandomHash keys, Eq. 3: keys[j*n + u] = min_{i in P_u} h_j(i). */
void orc_frh_keys(uint32_t n, uint32_t m, const int64_t *indptr,
                  const uint32_t *indices, const uint32_t *bucket, uint32_t t,
                  uint32_t *keys)
{
    for (uint32_t j = 0; j < t; ++j)
        for (uint32_t u = 0; u < n; ++u) {
            uint32_t best = 0xFFFFFFFFu;
            for (int64_t p = indptr[u]; p < indptr[u + 1]; ++p) {
                uint32_t h = bucket[(size_t)j * m + indices[p]];
                if (h < best) best = h;
            }
            keys[(size_t)j * n + u] = best;
        }
}

/* ---------------------------------------------------------- clustering -- */

typedef struct { uint64_t key; uint32_t uid; } kv_t;

static int kv_cmp(const void *pa, const void *pb)
{
    const kv_t *a = (const kv_t *)pa, *b = (const kv_t *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->uid != b->uid) return a->uid < b->uid ? -1 : 1;
    return 0;
}

static int u32_cmp(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    return a < b ? -1 : a > b;
}

typedef struct {
    const int64_t *indptr;
    const uint32_t *indices;
    const uint32_t *h;      /* bucket row of the current configuration */
    uint32_t cap;
    uint32_t *members;      /* output slots of the current configuration */
    uint32_t *cl_off;       /* global cluster offsets */
    uint32_t base;          /* j*n */
    uint32_t pos;           /* next free slot, relative to base */
    uint32_t ncl;           /* clusters emitted so far, all configurations */
    uint32_t *depth_hist;   /* optional: clusters per split depth */
    uint32_t max_depth;
} split_ctx;

static void emit(split_ctx *c, const uint32_t *users, uint32_t cnt,
                 uint32_t depth)
{
    c->cl_off[c->ncl++] = c->base + c->pos;
    memcpy(c->members + c->pos, users, cnt * sizeof(uint32_t));
    qsort(c->members + c->pos, cnt, sizeof(uint32_t), u32_cmp);
    c->pos += cnt;
    if (depth > c->max_depth) c->max_depth = depth;
}

/* H\eta(u) = min{ h(i) : i in P_u, h(i) > eta }, or ORC_NONE.  eta = ORC_ALL
 * stands for "below every hash value": then the result is H(u) itself. */
#define ORC_ALL (ORC_NONE - 1)
static uint64_t next_hash(const split_ctx *c, uint32_t u, uint64_t eta)
{
    uint64_t best = ORC_NONE;
    for (int64_t p = c->indptr[u]; p < c->indptr[u + 1]; ++p) {
        uint64_t h = c->h[c->indices[p]];
        if ((eta == ORC_ALL || h > eta) && h < best) best = h;
    }
    return best;
}

/* A cluster C with index eta (the hash value that produced it).  If it is no
 * larger than N it is final.  Otherwise each member gets H\eta; members with
 * the same new value form a new cluster that is split again in turn; members
 * with no new value or alone with theirs remain in C, which is then final. */
static void split(split_ctx *c, const uint32_t *users, uint32_t cnt,
                  uint64_t eta, uint32_t depth)
{
    if (cnt <= c->cap) { emit(c, users, cnt, depth); return; }
    kv_t *kv = (kv_t *)malloc((size_t)cnt * sizeof(kv_t));
    uint32_t *stay = (uint32_t *)malloc((size_t)cnt * sizeof(uint32_t));
    uint32_t nkv = 0, nstay = 0;
    for (uint32_t q = 0; q < cnt; ++q) {
        uint64_t e = next_hash(c, users[q], eta);
        if (e == ORC_NONE) stay[nstay++] = users[q];
        else { kv[nkv].key = e; kv[nkv].uid = users[q]; ++nkv; }
    }
    qsort(kv, nkv, sizeof(kv_t), kv_cmp);
    uint32_t *grp = (uint32_t *)malloc((size_t)cnt * sizeof(uint32_t));
    for (uint32_t a = 0; a < nkv;) {
        uint32_t e = a;
        while (e < nkv && kv[e].key == kv[a].key) ++e;
        if (e - a == 1) {
            stay[nstay++] = kv[a].uid;
        } else {
            for (uint32_t q = a; q < e; ++q) grp[q - a] = kv[q].uid;
            split(c, grp, e - a, kv[a].key, depth + 1);
        }
        a = e;
    }
    if (nstay) emit(c, stay, nstay, depth);
    free(grp);
    free(stay);
    free(kv);
}

/* Top-level grouping of configuration j followed by the recursive split.
 * keys0 == NULL: the group key is H_j(u) (Eq. 3) and an oversized group is
 * split from its own hash value.  Otherwise keys0[j*n + u] is an externally
 * assigned bucket (a learned assignment); an oversized group of such users is
 * split by FastRandomHash from the start, i.e. by H_j(u), then recursively. */
static int cluster_impl(uint32_t n, uint32_t m, const int64_t *indptr,
                        const uint32_t *indices, const uint32_t *keys0,
                        const uint32_t *bucket, uint32_t t, uint32_t cap,
                        uint32_t *members, uint32_t *cl_off, uint32_t *cl_cfg_off)
{
    split_ctx c;
    memset(&c, 0, sizeof(c));
    c.indptr = indptr;
    c.indices = indices;
    c.cap = cap;
    c.cl_off = cl_off;
    kv_t *kv = (kv_t *)malloc((size_t)n * sizeof(kv_t));
    uint32_t *grp = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    for (uint32_t j = 0; j < t; ++j) {
        c.h = bucket + (size_t)j * m;
        c.members = members + (size_t)j * n;
        c.base = j * n;
        c.pos = 0;
        cl_cfg_off[j] = c.ncl;
        /* B_j[H_j(u)] <- B_j[H_j(u)] + {u} */
        for (uint32_t u = 0; u < n; ++u) {
            uint64_t best = ORC_NONE;
            if (keys0) {
                best = keys0[(size_t)j * n + u];
            } else {
                for (int64_t p = indptr[u]; p < indptr[u + 1]; ++p) {
                    uint64_t h = c.h[indices[p]];
                    if (h < best) best = h;
                }
            }
            kv[u].key = best;
            kv[u].uid = u;
        }
        qsort(kv, n, sizeof(kv_t), kv_cmp);
        for (uint32_t a = 0; a < n;) {
            uint32_t e = a;
            while (e < n && kv[e].key == kv[a].key) ++e;
            for (uint32_t q = a; q < e; ++q) grp[q - a] = kv[q].uid;
            split(&c, grp, e - a, keys0 ? ORC_ALL : kv[a].key, 0);
            a = e;
        }
    }
    cl_cfg_off[t] = c.ncl;
    cl_off[c.ncl] = t * n;
    free(grp);
    free(kv);
    return (int)c.max_depth;
}

/* Step 1 (Algorithm 1 + recursive splitting) for all t configurations.
 * members[j*n .. j*n+n) receives configuration j's users grouped by final
 * cluster, each cluster's members ascending.  cl_off[c] is the start slot of
 * cluster c (global over configurations, cl_off[total] = t*n), and clusters of
 * configuration j are [cl_cfg_off[j], cl_cfg_off[j+1]).  Cluster order: top-level
 * clusters by ascending hash value; a split cluster is replaced by its
 * sub-clusters (ascending new hash value, each recursively) followed by the
 * users that stayed behind.  Returns the deepest split level reached. */
int orc_cluster(uint32_t n, uint32_t m, const int64_t *indptr,
                const uint32_t *indices, const uint32_t *bucket, uint32_t t,
                uint32_t cap, uint32_t *members, uint32_t *cl_off,
                uint32_t *cl_cfg_off)
{
    return cluster_impl(n, m, indptr, indices, NULL, bucket, t, cap, members,
                        cl_off, cl_cfg_off);
}

/* The same with top-level groups given by keys0[t][n] (ascending key order),
 * FastRandomHash on `bucket` splitting the oversized ones. */
int orc_cluster_keys(uint32_t n, uint32_t m, const int64_t *indptr,
                     const uint32_t *indices, const uint32_t *keys0,
                     const uint32_t *bucket, uint32_t t, uint32_t cap,
                     uint32_t *members, uint32_t *cl_off, uint32_t *cl_cfg_off)
{
    return cluster_impl(n, m, indptr, indices, keys0, bucket, t, cap, members,
                        cl_off, cl_cfg_off);
}

/* ----------------------------------------------------- local KNN (Alg.2) -- */

typedef struct {
    uint32_t n, t, k;
    const int64_t *indptr;
    const uint32_t *indices;
    const uint32_t *members;
    const uint32_t *cl_off;
    const uint32_t *cl_cfg_off;
    uint32_t ncl;
    const uint32_t *order;  /* clusters, largest first */
    uint32_t next;          /* queue head, guarded by mu */
    pthread_mutex_t mu;
    uint32_t *part_id, *part_I;
    uint32_t m;
    /* Algorithm 2: clusters of at least rho*k^2 members take Hyrec */
    int alg2;
    uint32_t rho, max_iter;
    double delta;
    uint64_t seed;
} lknn_ctx;

static uint32_t cfg_of_cluster(const lknn_ctx *c, uint32_t cl)
{
    uint32_t j = 0;
    while (c->cl_cfg_off[j + 1] <= cl) ++j;
    return j;
}

static uint32_t plen(const int64_t *indptr, uint32_t u)
{
    return (uint32_t)(indptr[u + 1] - indptr[u]);
}

/* |P_u & P_v| with P_u marked in mark[]. */
static uint32_t inter_marked(const lknn_ctx *c, const uint8_t *mark, uint32_t v)
{
    uint32_t I = 0;
    for (int64_t p = c->indptr[v]; p < c->indptr[v + 1]; ++p)
        I += mark[c->indices[p]];
    return I;
}

/* Brute force inside one cluster: every member's k best co-members. */
static void local_cluster(lknn_ctx *c, uint32_t cl, uint8_t *mark,
                          cand_t *cand)
{
    uint32_t j = cfg_of_cluster(c, cl);
    const uint32_t *S = c->members + c->cl_off[cl];
    uint32_t s = c->cl_off[cl + 1] - c->cl_off[cl];
    for (uint32_t a = 0; a < s; ++a) {
        uint32_t u = S[a];
        for (int64_t p = c->indptr[u]; p < c->indptr[u + 1]; ++p)
            mark[c->indices[p]] = 1;
        uint32_t nc = 0, Lu = plen(c->indptr, u);
        for (uint32_t q = 0; q < s; ++q) {
            uint32_t v = S[q];
            if (v == u) continue;
            uint32_t I = inter_marked(c, mark, v);
            cand[nc].v = v;
            cand[nc].I = I;
            cand[nc].U = Lu + plen(c->indptr, v) - I;
            ++nc;
        }
        for (int64_t p = c->indptr[u]; p < c->indptr[u + 1]; ++p)
            mark[c->indices[p]] = 0;
        qsort(cand, nc, sizeof(cand_t), cand_cmp);
        uint32_t *oid = c->part_id + ((size_t)u * c->t + j) * c->k;
        uint32_t *oI = c->part_I + ((size_t)u * c->t + j) * c->k;
        for (uint32_t r = 0; r < c->k; ++r) {
            oid[r] = r < nc ? cand[r].v : ORC_PAD;
            oI[r] = r < nc ? cand[r].I : 0;
        }
    }
}

/* ------------------------------------------- Hyrec branch (Algorithm 2) -- */

/* SplitMix64 (Steele, Lea and Flood, 2014): the (c+1)-th output of the
 * generator whose state starts at `seed`; the state advances by the golden
 * gamma and each output is the state passed through the published mixer. */
static uint64_t splitmix_at(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + 0x9e3779b97f4a7c15ull * (c + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix_at(uint64_t seed, uint64_t c) { return splitmix_at(seed, c); }

/* Sort candidates (v = member position; positions follow ids), keep each
 * position once, return the k best in out (count through *nout). */
static void topk_distinct(cand_t *cand, uint32_t nc, uint32_t k, cand_t *out,
                          uint32_t *nout)
{
    qsort(cand, nc, sizeof(cand_t), cand_cmp);
    uint32_t o = 0;
    for (uint32_t q = 0; q < nc && o < k; ++q) {
        if (o > 0 && cand[q].v == out[o - 1].v) continue;
        out[o++] = cand[q];
    }
    *nout = o;
}

/* Hyrec on one cluster, deterministic form: the initial graph gives member a
 * the k best of k uniform draws among the other members (SplitMix64 counter
 * (cluster << 40) | (a << 12) | q); then, synchronously, every member's new
 * list is the k best of its list and its neighbours' lists (Section IV-B:
 * neighbours' neighbours), until fewer than delta*k*s list entries changed in
 * an iteration or max_iter iterations ran. */
static void hyrec_cluster(lknn_ctx *c, uint32_t cl, uint8_t *mark)
{
    const uint32_t j = cfg_of_cluster(c, cl), k = c->k;
    const uint32_t *S = c->members + c->cl_off[cl];
    const uint32_t s = c->cl_off[cl + 1] - c->cl_off[cl];
    cand_t *cur = (cand_t *)malloc((size_t)s * k * sizeof(cand_t));
    cand_t *nxt = (cand_t *)malloc((size_t)s * k * sizeof(cand_t));
    uint32_t *ncur = (uint32_t *)calloc(s, sizeof(uint32_t));
    uint32_t *nnxt = (uint32_t *)calloc(s, sizeof(uint32_t));
    cand_t *cand = (cand_t *)malloc((size_t)(k + k * k) * sizeof(cand_t));
    for (uint32_t a = 0; a < s; ++a) {
        const uint32_t u = S[a], Lu = plen(c->indptr, u);
        for (int64_t p = c->indptr[u]; p < c->indptr[u + 1]; ++p) mark[c->indices[p]] = 1;
        uint32_t nc = 0;
        for (uint32_t q = 0; q < k; ++q) {
            uint64_t r = splitmix_at(c->seed, ((uint64_t)cl << 40) | ((uint64_t)a << 12) | q);
            uint32_t b = (uint32_t)(r % (s - 1));
            if (b >= a) ++b;
            uint32_t I = inter_marked(c, mark, S[b]);
            cand[nc].v = b; cand[nc].I = I; cand[nc].U = Lu + plen(c->indptr, S[b]) - I;
            ++nc;
        }
        for (int64_t p = c->indptr[u]; p < c->indptr[u + 1]; ++p) mark[c->indices[p]] = 0;
        topk_distinct(cand, nc, k, cur + (size_t)a * k, &ncur[a]);
    }
    for (uint32_t it = 0; it < c->max_iter; ++it) {
        uint64_t updates = 0;
        for (uint32_t a = 0; a < s; ++a) {
            const uint32_t u = S[a], Lu = plen(c->indptr, u);
            for (int64_t p = c->indptr[u]; p < c->indptr[u + 1]; ++p) mark[c->indices[p]] = 1;
            uint32_t nc = 0;
            const cand_t *la = cur + (size_t)a * k;
            for (uint32_t q = 0; q < ncur[a]; ++q) {
                cand[nc++] = la[q];
                const cand_t *lb = cur + (size_t)la[q].v * k;
                for (uint32_t r = 0; r < ncur[la[q].v]; ++r) {
                    const uint32_t b = lb[r].v;
                    if (b == a) continue;
                    uint32_t I = inter_marked(c, mark, S[b]);
                    cand[nc].v = b; cand[nc].I = I; cand[nc].U = Lu + plen(c->indptr, S[b]) - I;
                    ++nc;
                }
            }
            for (int64_t p = c->indptr[u]; p < c->indptr[u + 1]; ++p) mark[c->indices[p]] = 0;
            cand_t *na = nxt + (size_t)a * k;
            topk_distinct(cand, nc, k, na, &nnxt[a]);
            for (uint32_t q = 0; q < nnxt[a]; ++q) {
                int found = 0;
                for (uint32_t r = 0; r < ncur[a] && !found; ++r) found = la[r].v == na[q].v;
                updates += !found;
            }
        }
        cand_t *tc = cur; cur = nxt; nxt = tc;
        uint32_t *tn = ncur; ncur = nnxt; nnxt = tn;
        if ((double)updates < c->delta * (double)k * (double)s) break;
    }
    for (uint32_t a = 0; a < s; ++a) {
        const uint32_t u = S[a];
        uint32_t *oid = c->part_id + ((size_t)u * c->t + j) * k;
        uint32_t *oI = c->part_I + ((size_t)u * c->t + j) * k;
        for (uint32_t q = 0; q < k; ++q) {
            oid[q] = q < ncur[a] ? S[cur[(size_t)a * k + q].v] : ORC_PAD;
            oI[q] = q < ncur[a] ? cur[(size_t)a * k + q].I : 0;
        }
    }
    free(cand); free(nnxt); free(ncur); free(nxt); free(cur);
}

static void *lknn_worker(void *arg)
{
    lknn_ctx *c = (lknn_ctx *)arg;
    uint8_t *mark = (uint8_t *)calloc(c->m, 1);
    uint32_t smax = 0;
    for (uint32_t cl = 0; cl < c->ncl; ++cl) {
        uint32_t s = c->cl_off[cl + 1] - c->cl_off[cl];
        if (s > smax) smax = s;
    }
    cand_t *cand = (cand_t *)malloc((size_t)(smax + 1) * sizeof(cand_t));
    for (;;) {
        pthread_mutex_lock(&c->mu);
        uint32_t q = c->next++;
        pthread_mutex_unlock(&c->mu);
        if (q >= c->ncl) break;
        const uint32_t cl = c->order[q];
        const uint32_t s = c->cl_off[cl + 1] - c->cl_off[cl];
        if (c->alg2 && s >= 2 && (uint64_t)s >= (uint64_t)c->rho * c->k * c->k)
            hyrec_cluster(c, cl, mark);
        else
            local_cluster(c, cl, mark, cand);
    }
    free(cand);
    free(mark);
    return NULL;
}

static const uint32_t *g_sort_off; /* qsort context for cluster order */
static int by_size_desc(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    uint32_t sa = g_sort_off[a + 1] - g_sort_off[a];
    uint32_t sb = g_sort_off[b + 1] - g_sort_off[b];
    if (sa != sb) return sa > sb ? -1 : 1;
    return a < b ? -1 : a > b;
}

/* Step 2: partial KNN of every cluster.  part_id/part_I are [n][t][k]; slot
 * (u, j) holds u's k best co-members in its configuration-j cluster, best
 * first, padded with (0xFFFFFFFF, 0). */
static void local_knn_impl(uint32_t n, uint32_t m, const int64_t *indptr,
                           const uint32_t *indices, uint32_t t, uint32_t k,
                           const uint32_t *members, const uint32_t *cl_off,
                           const uint32_t *cl_cfg_off, uint32_t *part_id,
                           uint32_t *part_I, int nthreads, int alg2, uint32_t rho,
                           double delta, uint32_t max_iter, uint64_t seed)
{
    lknn_ctx c;
    memset(&c, 0, sizeof(c));
    c.alg2 = alg2; c.rho = rho; c.delta = delta; c.max_iter = max_iter; c.seed = seed;
    c.n = n; c.t = t; c.k = k; c.m = m;
    c.indptr = indptr; c.indices = indices;
    c.members = members; c.cl_off = cl_off; c.cl_cfg_off = cl_cfg_off;
    c.ncl = cl_cfg_off[t];
    c.part_id = part_id; c.part_I = part_I;
    uint32_t *order = (uint32_t *)malloc((size_t)c.ncl * sizeof(uint32_t) + 4);
    for (uint32_t q = 0; q < c.ncl; ++q) order[q] = q;
    g_sort_off = cl_off;
    qsort(order, c.ncl, sizeof(uint32_t), by_size_desc);
    c.order = order;
    pthread_mutex_init(&c.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = (pthread_t *)malloc((size_t)nthreads * sizeof(pthread_t));
    for (int w = 0; w < nthreads; ++w) pthread_create(&th[w], NULL, lknn_worker, &c);
    for (int w = 0; w < nthreads; ++w) pthread_join(th[w], NULL);
    pthread_mutex_destroy(&c.mu);
    free(th);
    free(order);
}

void orc_local_knn(uint32_t n, uint32_t m, const int64_t *indptr,
                   const uint32_t *indices, uint32_t t, uint32_t k,
                   const uint32_t *members, const uint32_t *cl_off,
                   const uint32_t *cl_cfg_off, uint32_t *part_id,
                   uint32_t *part_I, int nthreads)
{
    local_knn_impl(n, m, indptr, indices, t, k, members, cl_off, cl_cfg_off,
                   part_id, part_I, nthreads, 0, 0, 0.0, 0, 0);
}

/* Algorithm 2: brute force in clusters of fewer than rho*k^2 members, Hyrec
 * (hyrec_cluster) in the others. */
void orc_local_knn_alg2(uint32_t n, uint32_t m, const int64_t *indptr,
                        const uint32_t *indices, uint32_t t, uint32_t k,
                        const uint32_t *members, const uint32_t *cl_off,
                        const uint32_t *cl_cfg_off, uint32_t rho, double delta,
                        uint32_t max_iter, uint64_t seed, uint32_t *part_id,
                        uint32_t *part_I, int nthreads)
{
    local_knn_impl(n, m, indptr, indices, t, k, members, cl_off, cl_cfg_off,
                   part_id, part_I, nthreads, 1, rho, delta, max_iter, seed);
}

/* ---------------------------------------------------------- merge (Alg.3) -- */

/* Step 3: knn(u) = the k best of the union of u's t partial lists, each
 * neighbour once.  knn_U is |P_u | P_v| = |P_u| + |P_v| - I. */
void orc_merge(uint32_t n, const int64_t *indptr, uint32_t t, uint32_t k,
               const uint32_t *part_id, const uint32_t *part_I,
               uint32_t *knn_id, uint32_t *knn_I, uint32_t *knn_U)
{
    cand_t *cand = (cand_t *)malloc((size_t)t * k * sizeof(cand_t) + 16);
    for (uint32_t u = 0; u < n; ++u) {
        uint32_t nc = 0, Lu = plen(indptr, u);
        for (uint32_t j = 0; j < t; ++j)
            for (uint32_t r = 0; r < k; ++r) {
                size_t at = ((size_t)u * t + j) * k + r;
                uint32_t v = part_id[at];
                if (v == ORC_PAD) continue;
                cand[nc].v = v;
                cand[nc].I = part_I[at];
                cand[nc].U = Lu + plen(indptr, v) - part_I[at];
                ++nc;
            }
        qsort(cand, nc, sizeof(cand_t), cand_cmp);
        uint32_t out = 0;
        for (uint32_t q = 0; q < nc && out < k; ++q) {
            if (out > 0 && cand[q].v == knn_id[(size_t)u * k + out - 1]) continue;
            knn_id[(size_t)u * k + out] = cand[q].v;
            knn_I[(size_t)u * k + out] = cand[q].I;
            knn_U[(size_t)u * k + out] = cand[q].U;
            ++out;
        }
        for (; out < k; ++out) {
            knn_id[(size_t)u * k + out] = ORC_PAD;
            knn_I[(size_t)u * k + out] = 0;
            knn_U[(size_t)u * k + out] = 0;
        }
    }
    free(cand);
}

/* ------------------------------------------------- exact KNN (definition) -- */

typedef struct {
    uint32_t n, m, k;
    const int64_t *indptr;
    const uint32_t *indices;
    const uint32_t *rows;   /* users whose list is wanted */
    uint32_t nrows;
    uint32_t next;
    pthread_mutex_t mu;
    uint32_t *knn_id, *knn_I, *knn_U;  /* [nrows][k] */
    /* candidate restriction (definition form of C^2), or NULL for all users */
    const uint32_t *members, *cl_off, *pos_cl; /* pos_cl[j*n+u] = cluster of u */
    uint32_t t;
} bf_ctx;

static void topk_row(bf_ctx *c, uint32_t r, uint8_t *mark, cand_t *cand,
                     uint32_t *stamp)
{
    uint32_t u = c->rows[r];
    uint32_t Lu = plen(c->indptr, u), nc = 0;
    for (int64_t p = c->indptr[u]; p < c->indptr[u + 1]; ++p)
        mark[c->indices[p]] = 1;
    lknn_ctx lc;
    lc.indptr = c->indptr;
    lc.indices = c->indices;
    if (!c->members) {
        for (uint32_t v = 0; v < c->n; ++v) {
            if (v == u) continue;
            uint32_t I = inter_marked(&lc, mark, v);
            cand[nc].v = v; cand[nc].I = I; cand[nc].U = Lu + plen(c->indptr, v) - I;
            ++nc;
        }
    } else {
        /* Cand(u) = users sharing at least one final cluster with u */
        stamp[u] = r + 1;
        for (uint32_t j = 0; j < c->t; ++j) {
            uint32_t cl = c->pos_cl[(size_t)j * c->n + u];
            for (uint32_t q = c->cl_off[cl]; q < c->cl_off[cl + 1]; ++q) {
                uint32_t v = c->members[q];
                if (stamp[v] == r + 1) continue;
                stamp[v] = r + 1;
                uint32_t I = inter_marked(&lc, mark, v);
                cand[nc].v = v; cand[nc].I = I; cand[nc].U = Lu + plen(c->indptr, v) - I;
                ++nc;
            }
        }
    }
    for (int64_t p = c->indptr[u]; p < c->indptr[u + 1]; ++p)
        mark[c->indices[p]] = 0;
    qsort(cand, nc, sizeof(cand_t), cand_cmp);
    for (uint32_t q = 0; q < c->k; ++q) {
        size_t at = (size_t)r * c->k + q;
        c->knn_id[at] = q < nc ? cand[q].v : ORC_PAD;
        c->knn_I[at] = q < nc ? cand[q].I : 0;
        c->knn_U[at] = q < nc ? cand[q].U : 0;
    }
}

static void *bf_worker(void *arg)
{
    bf_ctx *c = (bf_ctx *)arg;
    uint8_t *mark = (uint8_t *)calloc(c->m, 1);
    cand_t *cand = (cand_t *)malloc((size_t)c->n * sizeof(cand_t));
    uint32_t *stamp = (uint32_t *)calloc(c->n, sizeof(uint32_t));
    for (;;) {
        pthread_mutex_lock(&c->mu);
        uint32_t r = c->next++;
        pthread_mutex_unlock(&c->mu);
        if (r >= c->nrows) break;
        topk_row(c, r, mark, cand, stamp);
    }
    free(stamp);
    free(cand);
    free(mark);
    return NULL;
}

static void run_rows(bf_ctx *c, int nthreads)
{
    pthread_mutex_init(&c->mu, NULL);
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = (pthread_t *)malloc((size_t)nthreads * sizeof(pthread_t));
    for (int w = 0; w < nthreads; ++w) pthread_create(&th[w], NULL, bf_worker, c);
    for (int w = 0; w < nthreads; ++w) pthread_join(th[w], NULL);
    pthread_mutex_destroy(&c->mu);
    free(th);
}

/* Exact KNN of the listed users over all n users (brute force). Outputs are
 * [nrows][k]. */
void orc_brute_force(uint32_t n, uint32_t m, const int64_t *indptr,
                     const uint32_t *indices, uint32_t k, const uint32_t *rows,
                     uint32_t nrows, uint32_t *knn_id, uint32_t *knn_I,
                     uint32_t *knn_U, int nthreads)
{
    bf_ctx c;
    memset(&c, 0, sizeof(c));
    c.n = n; c.m = m; c.k = k; c.indptr = indptr; c.indices = indices;
    c.rows = rows; c.nrows = nrows;
    c.knn_id = knn_id; c.knn_I = knn_I; c.knn_U = knn_U;
    run_rows(&c, nthreads);
}

/* The C^2 graph by its definition: knn(u) = the k best users among those that
 * share at least one final cluster with u, in any configuration.  Same layout
 * as orc_brute_force. */
void orc_candidate_topk(uint32_t n, uint32_t m, const int64_t *indptr,
                        const uint32_t *indices, uint32_t t, uint32_t k,
                        const uint32_t *members, const uint32_t *cl_off,
                        const uint32_t *cl_cfg_off, const uint32_t *rows,
                        uint32_t nrows, uint32_t *knn_id, uint32_t *knn_I,
                        uint32_t *knn_U, int nthreads)
{
    uint32_t ncl = cl_cfg_off[t];
    uint32_t *pos_cl = (uint32_t *)malloc((size_t)t * n * sizeof(uint32_t));
    for (uint32_t cl = 0; cl < ncl; ++cl) {
        uint32_t j = 0;
        while (cl_cfg_off[j + 1] <= cl) ++j;
        for (uint32_t q = cl_off[cl]; q < cl_off[cl + 1]; ++q)
            pos_cl[(size_t)j * n + members[q]] = cl;
    }
    bf_ctx c;
    memset(&c, 0, sizeof(c));
    c.n = n; c.m = m; c.k = k; c.indptr = indptr; c.indices = indices;
    c.rows = rows; c.nrows = nrows;
    c.knn_id = knn_id; c.knn_I = knn_I; c.knn_U = knn_U;
    c.members = members; c.cl_off = cl_off; c.pos_cl = pos_cl; c.t = t;
    run_rows(&c, nthreads);
    free(pos_cl);
}
