/*
 * rkmips.h -- C ABI of the exact Reverse k-Maximum Inner Product Search library for
 * AMD Instinct MI355X (gfx950).
 *
 * Problem (Definition 1 of "SAH: Shifting-aware Asymmetric Hashing for Reverse
 * k-Maximum Inner Product Search", Huang, Wang, Tung, AAAI 2023): given items P
 * (n x d), users U (m x d), a query item q and k >= 1, return every user u for
 * which q is among the k largest inner products of u over P united with {q}.
 *
 * Exactness contract.  Inner products are decided in a canonical IEEE double form:
 *   FP32 / BF16 storage: s(u,x) = (((0 + u_0 x_0) + u_1 x_1) + ...) + u_{d-1} x_{d-1}
 *     in FP64, index order (each FP32 product is exact in FP64);
 *   FP8 e4m3 storage with per-vector FP32 scales: s(u,x) = (su * sx) * S, S the
 *     exact sum of the decoded code products (one rounding).
 * lambda_u^(j) is the j-th largest s(u,p) over P (-inf for j > n), and
 *   u is in the answer  <=>  s(u,q) >= lambda_u^(k)
 * (the query wins ties, as the paper's query algorithms prune only on a strict
 * "<": Alg. 5 and Alg. 2).  The returned sets are exactly these sets.  Bulk work
 * runs in FP32/BF16/FP8 on the matrix cores; every decision closer than a derived
 * error bound is taken again in the canonical FP64 form on the GPU.
 *
 * Conventions.
 *  - Vector inputs are DEVICE pointers to row-major contiguous matrices, rows of
 *    d elements: float (RKMIPS_F32), uint16 BF16 bit patterns (RKMIPS_BF16) or
 *    uint8 OCP e4m3fn codes (RKMIPS_FP8_E4M3, with one FP32 scale per row in a
 *    device array; scale pointers are NULL for the other types).
 *  - Inputs are borrowed for the duration of a call; the index copies what it keeps.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls are ordered on it.
 *  - Every entry point validates its arguments before any device work.  On error it
 *    returns a negative status, writes no output, leaks nothing, and
 *    rkmips_last_error() describes the failure (thread-local text).
 *  - No C++ exception crosses this interface.
 *  - An index is read-only after it is built: concurrent rkmips_query_batch calls on
 *    different streams are safe.  Freeing an index while calls use it is not.
 */
#ifndef RKMIPS_H
#define RKMIPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rkmips_index rkmips_index;    /* opaque; owns all device memory of an index   */
typedef struct rkmips_result rkmips_result;  /* opaque; owns the outputs of one query batch  */

typedef enum { RKMIPS_F32 = 0, RKMIPS_BF16 = 1, RKMIPS_FP8_E4M3 = 2 } rkmips_dtype;

typedef enum {
    RKMIPS_OK = 0,
    RKMIPS_EINVAL = -1,   /* invalid argument (null pointer, size, non-finite value, ...) */
    RKMIPS_ENOMEM = -2,   /* device or host allocation failed, or a memory budget is too small */
    RKMIPS_EDEVICE = -3,  /* a HIP call failed */
    RKMIPS_ERANGE = -4,   /* k outside [1, k_max], or magnitudes outside the exact range */
    RKMIPS_EBUSY = -5     /* result not ready / resource in use */
} rkmips_status;

/* Query-side switches (rkmips_params.flags at build time, or per call).  None of
 * them changes any returned set; they exist to prove that and to time the parts. */
enum {
    RKMIPS_FLAG_NO_BOUNDS = 1,      /* skip Cone-Tree pruning (Lemma 2 and Lemma 3 tests)   */
    RKMIPS_FLAG_FORCE_RECHECK = 2,  /* take every unpruned decision in canonical FP64       */
    RKMIPS_FLAG_NO_SAALSH = 4,      /* never run the SA-ALSH reject stage (overrides 32)     */
    RKMIPS_FLAG_NO_CERT = 8,        /* build: treat every top-k certificate as failed, so
                                       every lambda row comes from the full FP64 rescoring  */
    RKMIPS_FLAG_NO_VECTOR_BOUND = 16, /* skip only the per-user Lemma 3 test                 */
    RKMIPS_FLAG_SAALSH_FILTER = 32, /* run the SA-ALSH stage (Alg. 2) on the close calls
                                       before the FP64 recheck; its proven "no" answers
                                       skip the recheck.  Off by default: Alg. 2 scores
                                       ceil(beta |S_j|) candidates per pair, far more work
                                       than the O(d) FP64 recheck it can save.           */
    RKMIPS_FLAG_F32_MATRIX = 64,    /* build: score FP32 data on the FP32 matrix cores.
                                       By default FP32 rows with d <= 64 are scored as
                                       split BF16 products (h.h + l.h + h.l, h and l the
                                       BF16 head and tail of each value) with their own
                                       error bound; either way the exact path decides.   */
    RKMIPS_FLAG_POOL_LISTS = 128,   /* collect the answers in the result pool and sort
                                       the lists even when a batch's answer bits (one per
                                       query and user) fit the 64 MiB budget             */
    RKMIPS_FLAG_VERIFY_SIMPLE = 256 /* query: score with the one-group verify kernel
                                       (register-fed query tiles) where the two-group
                                       ring form would run (BF16 and FP8 indexes with
                                       padded rows of 128 or 256 values, FP32 indexes
                                       scored as split BF16 products); both take the
                                       same decisions                                     */
};

typedef struct {
    int32_t k_max;       /* largest k a query may use (Alg. 4 input); >= 1, <= 256     */
    int32_t leaf_size;   /* N0: most users in one Cone-Tree leaf (Alg. 3); 1..64       */
    int32_t num_hash;    /* K: sign-random-projection bits per code (Alg. 1); 32..256,
                            multiple of 32                                              */
    int32_t topk_slack;  /* s: approximate candidates kept per user beyond k_max       */
    float b;             /* interval ratio of the norm partitions (Alg. 1), 0 < b < 1  */
    float probe_frac;    /* beta: fraction of a partition probed by SimHash (Alg. 2)   */
    uint64_t seed;       /* seed of the Cone-Tree pivots (Alg. 3)                       */
    int32_t mode;        /* RKMIPS_MODE_EXACT, RKMIPS_MODE_SAH or RKMIPS_MODE_LAZY      */
    int32_t flags;       /* RKMIPS_FLAG_* defaults for every query of this index        */
    int32_t sah_items;   /* SAH and LAZY: |P'|, the items of largest norm whose exact
                            k_max-MIPS gives the lower-bound arrays L_u (Alg. 4); the
                            SA-ALSH index covers the other n - |P'|.  1 <= |P'| < n;
                            0 takes min(2 k_max, n - 1).  Ignored in exact mode.       */
} rkmips_params;

/* Query semantics of an index (rkmips_params.mode).
 *   EXACT: lambda_u is the exact k_max-MIPS over all of P; every answer set is the
 *          Definition 1 set (canonical FP64 scores).
 *   SAH:   the paper's approximate method.  L_u comes from P' only (Alg. 4) and the
 *          Alg. 5 decisions follow: s(u,q) < L_u^k -> no; s(u,q) >= ||u|| ||p_k||
 *          (p_k the k-th item in norm order, tested as s >= 0 and s^2 >= n2(u) n2(p_k)
 *          in FP64) -> yes; otherwise Alg. 2 over the SA-ALSH partitions of P \ P',
 *          its candidate set starting from u's scores on P' (phi = L_u^k).  Every "no"
 *          is proved, so each set contains the exact one; Alg. 2's "yes" may be wrong
 *          (false positives).  All scores are canonical FP64, so the sets do not
 *          depend on scheduling.  RKMIPS_FLAG_SAALSH_FILTER has no effect here.
 *   LAZY:  exact answers from the SAH index (only L_u over P' is built): the SAH steps
 *          with every item of each partition that Alg. 2 visits scored (probe_frac is
 *          set to 1).  A "no" is proved as in SAH; a "yes" after the last partition is
 *          exact because phi is then lambda_u^(k); the early "yes" (phi > mu_j) is exact
 *          because no unvisited item can score above mu_j < phi <= s(u,q).  This trades
 *          the 2mnd-FLOP lambda build for per-user work at query time. */
enum { RKMIPS_MODE_EXACT = 0, RKMIPS_MODE_SAH = 1, RKMIPS_MODE_LAZY = 2 };

/* Defaults: k_max 50, N0 64, K 128, s 14, b 0.5, beta 0.1, seed 221112751, exact mode,
 * sah_items 0. */
void rkmips_default_params(rkmips_params *p);

/*
 * Build the index (Alg. 4 with the lower-bound array made exact over all of P; in
 * RKMIPS_MODE_SAH over the |P'| items of largest norm, with the SA-ALSH index over the
 * rest).
 *   1. item norms and descending order (Alg. 4 first lines; Alg. 1 first line);
 *   2. lambda_u^(j), j = 1..k_max, for every user: a fused U.P^T matrix-core pass
 *      keeps k_max+s approximate candidates per user, FP64 rescoring sorts them
 *      and certifies the order; rows that fail are rescored in full in FP64;
 *   3. SA-ALSH index (Alg. 1): norm partitions, centroids, radii, the shifting-
 *      invariant transform (Eqn. 6) and K-bit sign-random-projection codes
 *      (Eqn. 1) for items, Eqn. 7 codes for users;
 *   4. Cone-Tree over user directions (Alg. 3); leaves are the user blocks, each
 *      with its centre, maximum angle and the per-block lower bounds L^j(B).
 * items [n x d], users [m x d]: device, see conventions; item_scales/user_scales:
 * device FP32 [n] / [m] for FP8 data, else NULL.  srp_proj: device FP32
 * [(d+1) x num_hash] row-major Gaussian projection matrix (column h is the vector a
 * of one hash function), or NULL to draw it from p->seed inside the library.
 * p: NULL for defaults.
 * Completion (stream-ordered, not synchronous): the call returns once every host-side
 * check is done and the rest of the build is queued on `stream` (the last part, FP64
 * refinement and block bounds, may still be running).  Work queued on `stream`
 * afterwards sees the complete index, query batches on other streams wait for it on the
 * device, and the host-side getters (info, stats, lambda, blocks, candidates, SA-ALSH
 * data) wait for it on the host.  rkmips_index_wait gives the synchronous form.  The
 * input arrays must stay valid until the build is complete.
 * Errors: EINVAL (null pointers, n, m, d < 1, d > 256, bad params, non-finite
 * values), ERANGE (max||u|| * max||p|| beyond 1e30 or a non-zero vector norm below
 * 1e-30, where FP32 bounds would lose exactness), ENOMEM, EDEVICE.
 */
rkmips_status rkmips_build_index(const void *items, const float *item_scales, int64_t n,
                                 const void *users, const float *user_scales, int64_t m,
                                 int32_t d, int32_t dtype, const float *srp_proj,
                                 const rkmips_params *p, void *stream, rkmips_index **out);

/* Wait on the host until the build of idx is complete (the synchronous form of
 * rkmips_build_index).  Errors: EINVAL (NULL), EDEVICE. */
rkmips_status rkmips_index_wait(rkmips_index *idx);

/*
 * Answer a batch of queries (Alg. 5 over all blocks: exact decisions, or the SAH
 * decisions of RKMIPS_MODE_SAH, see rkmips_params.mode).
 * queries: device [nq x d] in the index's dtype (query_scales: device FP32 [nq] for
 * FP8, else NULL).  ks: DEVICE int32 [nq], 1 <= ks[i] <= k_max.  flags: RKMIPS_FLAG_*
 * added to the index defaults for this call.  The host groups the queries by k, so the
 * call copies ks to the host in order on `stream` and waits for that copy (and so for
 * the stream's earlier work); the batch itself is then enqueued on `stream`, and *out
 * receives a result handle whose contents are valid after rkmips_result_wait.
 * nq = 0 is allowed (empty result).  Errors: EINVAL, ERANGE (a k out of range),
 * ENOMEM, EDEVICE.  Conditions that need the device data (a non-finite query value:
 * EINVAL; a query norm outside [1e-30, 1e30]: ERANGE) are returned by
 * rkmips_result_wait, and the result is then empty.
 */
rkmips_status rkmips_query_batch(rkmips_index *idx, const void *queries, const float *query_scales,
                                 int64_t nq, const int32_t *ks, int32_t flags, void *stream,
                                 rkmips_result **out);

/* rkmips_query_batch with ks in HOST memory (int32 [nq]): no host wait at all, the
 * batch queues behind the stream's earlier work (for example a build on the same
 * stream).  Same outputs and errors. */
rkmips_status rkmips_query_batch_hostk(rkmips_index *idx, const void *queries, const float *query_scales,
                                       int64_t nq, const int32_t *ks, int32_t flags, void *stream,
                                       rkmips_result **out);

/* Block until the batch is complete and its host-side outputs are filled. */
rkmips_status rkmips_result_wait(rkmips_result *r);

/* After wait: *nq = batch size; offsets: host int64 [nq+1]; ids: host int32
 * [offsets[nq]], the original user indices of query i at ids[offsets[i] ..
 * offsets[i+1]), ascending.  The arrays belong to r.  EBUSY before wait. */
rkmips_status rkmips_result_view(const rkmips_result *r, int64_t *nq, const int64_t **offsets,
                                 const int32_t **ids);

typedef struct {
    int64_t pairs_total;        /* nq * m                                              */
    int64_t pairs_block_pruned; /* removed by the node-level bound (Lemma 2)            */
    int64_t pairs_vector_pruned;/* removed by the vector-level bound (Lemma 3)          */
    int64_t pairs_scored;       /* inner products evaluated on the matrix cores        */
    int64_t pairs_rechecked;    /* decisions taken again in canonical FP64             */
    int64_t saalsh_checked;     /* pairs sent through the SA-ALSH stage                 */
    int64_t saalsh_rejects;     /* of those, rejected by phi (Alg. 2, "no")             */
    int64_t results;            /* sum of the answer sizes                              */
    double ms_total;            /* device time of the batch (events), milliseconds      */
} rkmips_query_stats;

/* Counters of a completed batch (after wait). */
rkmips_status rkmips_result_stats(const rkmips_result *r, rkmips_query_stats *out);

void rkmips_result_free(rkmips_result *r);

typedef struct {
    int64_t n, m;
    int32_t d, dtype, k_max, cand_per_user, num_hash, leaf_size;
    int32_t num_partitions;      /* t of Alg. 1                                          */
    int64_t num_blocks;          /* Cone-Tree leaves                                     */
    int64_t cert_failures;       /* users whose lambda row needed the full FP64 rescoring */
    double max_rel_err_raw;      /* max |s_fast - s64| / |s64| over the rescored candidates   */
    double max_rel_err_lambda32; /* max |lambda32 - lambda64| / |lambda64| after           */
    double ms_norms, ms_lambda, ms_refine, ms_saalsh, ms_cone, ms_total; /* device times   */
    int64_t device_bytes;        /* device memory held by the index                      */
    double ms_seed, ms_topk;     /* lambda build: threshold seed pass and fused top-k pass
                                    (both inside ms_lambda)                              */
    int32_t mma_dtype;           /* operand type of the lambda build's matrix cores
                                    (RKMIPS_BF16 for split FP32 data)                    */
    int32_t mma_terms;           /* products per stored coordinate (3 when split)       */
    double err_fast;             /* error bound of the fast scores / (||u|| ||p||)       */
    int32_t mode;                /* RKMIPS_MODE_*                                        */
    int32_t lambda_items;        /* items the lambda table covers: n, or |P'| (SAH)      */
} rkmips_index_info;

rkmips_status rkmips_get_info(const rkmips_index *idx, rkmips_index_info *out);

/* Statistics of the precision pattern: the fast (matrix-core) lambda before and after
 * the FP64 refinement, the certificate fallbacks of the build, and the counters of
 * every query batch of this index completed so far (summed over batches). */
typedef struct {
    double max_rel_err_raw;      /* max |s_fast - s64| / |s64| over the rescored candidates */
    double max_rel_err_lambda32; /* max |lambda32 - lambda64| / |lambda64| (refined)         */
    int64_t cert_failures;       /* users whose lambda row was rescored in full in FP64      */
    double fallback_rate;        /* cert_failures / m                                       */
    int64_t batches, queries;    /* completed batches and their queries                     */
    rkmips_query_stats query;    /* their counters, summed (ms_total: summed device time)   */
    double recheck_rate;         /* query.pairs_rechecked / query.pairs_scored              */
} rkmips_stats;

/* Waits for the build on the host.  Errors: EINVAL (NULL). */
rkmips_status rkmips_get_stats(const rkmips_index *idx, rkmips_stats *out);

/* lambda_u^(k) for every user in ORIGINAL order: host double [m] (k in 1..k_max). */
rkmips_status rkmips_get_lambda(const rkmips_index *idx, int32_t k, double *out_m);
/* The FP32 copy used by the fast decisions, RN(lambda64): host float [m]. */
rkmips_status rkmips_get_lambda32(const rkmips_index *idx, int32_t k, float *out_m);

/* Item order of step 1: host int64 [n] original item indices by descending norm
 * (equal squared norms by ascending index) and host double [n] their canonical
 * squared norms in that order. */
rkmips_status rkmips_get_item_order(const rkmips_index *idx, int64_t *order, double *norm2);

/* Approximate candidates of step 2 (before refining), per ORIGINAL user: host int32
 * [m x cand_per_user] item indices (-1 = empty slot), host float scores, and host
 * float [m] thresholds tau (every item that is not a candidate scored <= tau). */
rkmips_status rkmips_get_candidates(const rkmips_index *idx, int32_t *ids, float *scores,
                                    float *tau);

/* SA-ALSH index of step 3.  part_start: host int64 [t+1] positions in the item
 * order; centroid: host float [t x d]; radius: host float [t]; item_codes: host
 * uint32 [n x K/32] per ORIGINAL item; user_codes: host uint32 [m x K/32] per
 * ORIGINAL user.  Any pointer may be NULL to skip that array. */
rkmips_status rkmips_get_saalsh(const rkmips_index *idx, int64_t *part_start, float *centroid,
                                float *radius, uint32_t *item_codes, uint32_t *user_codes);

/* SA-ALSH query of Alg. 2 for explicit (query, user) pairs, as the paper states it:
 * partitions in order of M_j; yes if phi > M_j ||u||; SimHash probe of the
 * ceil(beta |S_j|) items whose K-bit codes agree most with the user's (equal counts:
 * earlier in the item order first); phi = k-th largest canonical inner product over all
 * candidates so far; no if <u,q> < phi; yes after the last partition.
 * queries: device [nq x d] (query_scales device [nq] for FP8); ks: host [nq];
 * pair_query / pair_user: host int64 [npairs] (query row, ORIGINAL user index);
 * phi_out: host double [npairs]; answer_out: host int32 [npairs] (1 yes, 0 no).
 * A "no" is exact (phi is a k-th largest over a subset of the items); a "yes" is the
 * paper's approximate decision.  Synchronous on `stream`.  Errors: EINVAL, ERANGE. */
rkmips_status rkmips_saalsh_probe(rkmips_index *idx, const void *queries, const float *query_scales,
                                  int64_t nq, const int32_t *ks, const int64_t *pair_query,
                                  const int64_t *pair_user, int64_t npairs, float probe_frac,
                                  void *stream, double *phi_out, int32_t *answer_out);

/* rkmips_saalsh_probe for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * results and errors; it calls no hipMalloc, hipFree or allocating library routine.  Its
 * staging (padded queries, k values, packed pairs, phi and answers) and Alg. 2's
 * candidate scratch come from one 64 MiB device array per GPU, held until the process
 * ends; a batch that does not fit (nq x row bytes + about 28 bytes per pair + one
 * candidate row of ceil(probe_frac n) + t + k_max + 1 doubles) is refused with ERANGE
 * before any device work.  All calls on one GPU share that array and it keeps the last
 * call's contents: calls that overlap on one GPU (other threads or streams) race and
 * must be serialised by the caller.  Synchronous on `stream`. */
rkmips_status rkmips_saalsh_probe_noalloc(rkmips_index *idx, const void *queries, const float *query_scales,
                                          int64_t nq, const int32_t *ks, const int64_t *pair_query,
                                          const int64_t *pair_user, int64_t npairs, float probe_frac,
                                          void *stream, double *phi_out, int32_t *answer_out);

/* Cone-Tree blocks of step 4.  leaf_users: host int32 [m] original user indices in
 * leaf order; block_start: host int64 [B+1]; center: host float [B x d] unit block
 * centres; cos_omega/sin_omega: host float [B] (bounds of the maximum angle); cos_theta
 * /sin_theta: host float [m] in leaf order; block_lb: host float [k_max x B] lower
 * bounds L^j(B) <= min over the block of lambda_u^(j)/||u|| (-inf = never prune).
 * Any pointer may be NULL. */
rkmips_status rkmips_get_blocks(const rkmips_index *idx, int32_t *leaf_users, int64_t *block_start,
                                float *center, float *cos_omega, float *sin_omega,
                                float *cos_theta, float *sin_theta, float *block_lb);

void rkmips_index_free(rkmips_index *idx);

/*
 * Insert n_new items into an exact-mode index (not a step of the paper, which builds its
 * index once; Definition 1 over the grown item set fixes the result).  items: device
 * [n_new x d] in the index's dtype (item_scales: device FP32 [n_new] for FP8, else NULL);
 * they receive the ids n, n + 1, ... .  Every user's lambda row takes the canonical scores
 * of the new items that rank among its k_max best; the item order, the sorted rows, the
 * SA-ALSH partitions, centroids, radii and codes (same projections) and the block lower
 * bounds are rebuilt over the grown set.  The result equals a build over the items
 * [old; new] with the same parameters and projections.  Synchronous on `stream`; no query
 * batch of the index may run meanwhile.  The raw candidates of the original build are
 * dropped (rkmips_get_candidates then fails).
 * Errors: EINVAL (null pointers, n_new < 0, an SAH or lazy index, n beyond 2^30,
 * non-finite values), ERANGE (magnitudes as in rkmips_build_index), ENOMEM, EDEVICE.
 */
rkmips_status rkmips_insert_items(rkmips_index *idx, const void *items, const float *item_scales, int64_t n_new,
                                  void *stream);

/*
 * SA-ALSH kMIPS (Alg. 2 run without a query, the search that SAH uses inside Alg. 5):
 * for each of the nu users users[i] (original ids, HOST int64), the k best scores that
 * the probes find.  Partitions are visited in norm order; each probes the
 * ceil(probe_frac |S_j|) items with the most equal code bits (ties: earlier in norm
 * order) and scores them in canonical FP64; the search stops before partition j once the
 * k-th best found exceeds mu_j = M_j ||u||.  Exact-mode index: the partitions cover all
 * of P and the search starts empty.  SAH and lazy indexes: they cover P \ P' and the
 * search starts from u's k best scores on P' (its lambda row), so k <= k_max.
 * scores_out: HOST double [nu x k], row i descending, -inf where fewer than k items were
 * scored.  probe_frac = 1 gives the exact k best scores (rkmips_get_lambda on an exact
 * index).  Synchronous on `stream`.
 * Errors: EINVAL (null pointers, user id out of range, probe_frac outside (0, 1]),
 * ERANGE (k outside [1, 256], or above k_max on an SAH or lazy index), ENOMEM, EDEVICE.
 */
rkmips_status rkmips_saalsh_kmips(rkmips_index *idx, const int64_t *users, int64_t nu, int32_t k,
                                  float probe_frac, void *stream, double *scores_out);

/*
 * Save a complete index to a file and load it back (not from the paper: the Alg. 4 index
 * is built once per item and user set, and a server can start from the file instead).
 * Save waits for the build, copies every array the queries and getters read, the build
 * statistics and the parameters to `path` (host byte order; the raw candidates of the
 * lambda build are not kept, so rkmips_get_candidates fails on a loaded index).  Load
 * reads such a file onto the current device; its arrays are ready when it returns, and
 * `stream` is the stream its buffers are recycled on.  A loaded index answers every
 * query exactly as the saved one.
 * Errors: EINVAL (null pointers, a file that cannot be opened, written or read, a wrong
 * magic or version, an inconsistent header or a missing array), ENOMEM, EDEVICE.  The
 * file checks happen before any device call.
 */
rkmips_status rkmips_index_save(const rkmips_index *idx, const char *path);
rkmips_status rkmips_index_load(const char *path, void *stream, rkmips_index **out);

/* Text of the last error on this thread ("" if none). */
const char *rkmips_last_error(void);

/*
 * Continuous-batching server replay (serving pattern: requests that arrive while
 * others are on the GPU are admitted as slots and memory free up, and their work
 * overlaps on the device).
 * queries: HOST [nq x d] in the index dtype (query_scales HOST [nq] for FP8);
 * ks: HOST [nq]; arrival_us: HOST int64 [nq], non-decreasing request times in
 * microseconds after the start.  A feeder thread releases each request at its time;
 * the dispatcher forms batches of up to max_batch arrived requests whenever one of
 * num_streams slots is free and the batch fits the memory budget, and runs each
 * batch on its slot's stream with the slot's preallocated buffers; a completion
 * thread records per-request latency (arrival to host-visible result).
 * latency_us: HOST double [nq] (out).  *out: the results in request order.
 */
typedef struct {
    int32_t max_batch;      /* <= 4096, e.g. 256                                          */
    int32_t num_streams;    /* in-flight batches, 1..8                                    */
    int64_t mem_budget;     /* bytes of device memory the slots may use; 0 = no limit     */
    int32_t flags;          /* RKMIPS_FLAG_* for every batch                               */
} rkmips_serve_params;

typedef struct {
    int64_t batches;
    int64_t max_inflight;   /* most batches on the device at once                          */
    int32_t slots;          /* slots admitted by the memory budget                         */
    double wall_ms;         /* first arrival to last completion                            */
    double p50_us, p99_us, mean_us;
} rkmips_serve_stats;

rkmips_status rkmips_serve_replay(rkmips_index *idx, const void *queries, const float *query_scales,
                                  int64_t nq, const int32_t *ks, const int64_t *arrival_us,
                                  const rkmips_serve_params *sp, double *latency_us,
                                  rkmips_serve_stats *stats, rkmips_result **out);

#ifdef __cplusplus
}
#endif

#endif /* RKMIPS_H */
