// Host-side declarations shared by the C-ABI implementation and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/rkmips.h"
#include "topk.h"

namespace rk {

// Thrown inside the library only; the C entry points convert it into a status code.
struct Error {
    rkmips_status st;
    std::string msg;
};
[[noreturn]] void fail(rkmips_status st, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define HIPC(x) ::rk::hip_check((x), #x)
// Waits on the host until event e has completed, polling it (a blocking wait can add tens
// of microseconds of wake-up latency to every host round trip).
void host_wait(hipEvent_t e);

// Throws EINVAL unless every build parameter is in its documented range.
void validate_params(const rkmips_params& p);

// Padded row length (elements) used for the stored copies of all vector sets.
int padded_dim(int d, int dtype);
int elt_bytes(int dtype);

// ---------------------------------------------------------------- prep (k_prep.hip)
// n2[r] = canonical FP64 <x_r, x_r>; sets *bad (device int) non-zero on a
// non-finite element/scale.  rows use leading dimension ld (elements).
void launch_norm_stats_init(unsigned long long* stats, hipStream_t s);
void launch_norm2(int dtype, const void* X, const float* scales, int64_t rows, int d, int ld,
                  double* n2, unsigned long long* stats, int slot, hipStream_t s);
// FP32 rows [rows x ld] -> BF16 rows [rows x 3 ld]: [h | l | h] (user_layout 0) against
// [h | h | l] (user_layout 1), whose BF16 dot product approximates the FP32 one within
// split_err_rel; user_layout 2 gives the pair rows [rows x 2 ld] = [h | l] that the top-k
// passes expand to the same three products.
void launch_split_bf16(const float* src, int64_t rows, int ld, uint16_t* dst, int user_layout, hipStream_t s);
// Matrix-core operand rows [rows x mma_ld] (BF16 bits) from stored rows [rows x ld]:
// split FP32 (see launch_split_bf16) or widened FP8 codes.
void launch_mma_operand(int mma_dtype, int dtype, const void* src, int64_t rows, int ld, uint16_t* dst,
                        int user_layout, hipStream_t s);
// Sort (key, val) pairs ascending by key then val, n <= 2^31.  keys/vals and the
// scratch arrays tmp_keys/tmp_vals hold cap >= n rounded up to min(2048, next power of
// two of n) entries; the sorted pairs end in keys/vals[0, n).
void sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* tmp_keys, uint32_t* tmp_vals, int64_t n, int64_t cap,
                hipStream_t s);
// dst[r] = src[perm[r]] row copy from leading dim ld_src to ld_dst (zero padded).
void launch_gather_rows(int dtype, const void* src, int ld_src, const float* src_scales,
                        const uint32_t* perm, int64_t rows, int d, void* dst, int ld_dst,
                        float* dst_scales, hipStream_t s);
// keys[i] = ~bits(n2[i]) (ascending = descending norm), vals[i] = i, padded to cap.
void launch_norm_keys(const double* n2, int64_t n, int64_t cap, uint64_t* keys, uint32_t* vals,
                      hipStream_t s);
void launch_permute_f64(const double* src, const uint32_t* perm, int64_t n, double* dst,
                        hipStream_t s);

// ---------------------------------------------------------------- lambda build
// (the fused top-k pass: topk.h)
constexpr int kErrSlots = 64;

struct RefineArgs {
    const void* items; const float* item_scales; int64_t n;
    const void* users; const float* user_scales; int64_t m;
    int d, ld, nseg, C, G, k_max;
    const uint2* buf; const int* cnt; const float* tau;
    const double* item_n2_sorted;   // canonical squared norms, sorted order
    int64_t seg_len;
    const double* user_n2;          // leaf order
    int force_fail;
    double* lam64;                  // [k_max x m]
    float* lam32;                   // [k_max x m]
    int* fail_list; int* fail_count;
    // build diagnostics as bits of non-negative doubles, kErrSlots slots each (fast-score
    // error, then lambda32 error): workgroup b takes slot b % kErrSlots, so that the
    // atomics of 10^5 waves do not all meet on one address; the host takes the maximum
    unsigned long long* max_raw_err_bits;
    double err_rel;                 // relative error bound of the fast scores
    int* spill; int* spill_count;   // [m] users with more candidates than the narrow pass holds
    const int* list; const int* list_count;   // users of a listed pass (null: all users)
    // split narrow pass: the kept candidates [m x C] (orderable key, item position) and per
    // user {count (-1: left to the wide pass), cut bits, largest threshold bits, 0}
    uint2* sel; int* sel_meta;
    // the block lower bounds' input, when given: lb_rows[leaf_of[u] x k_max + r] =
    // lambda_u^(r+1) / ||u|| (FP64), user-major in Cone-Tree leaf order, so that the
    // blocks (runs of leaf positions) read it contiguously
    double* lb_rows; const uint32_t* leaf_of;
};
void launch_refine(int dtype, const RefineArgs& a, hipStream_t s);
// Matrix-core accumulation probe (k_diag.hip): host arrays, synchronous.
void mma_probe(int kind, const uint8_t* a_host, const uint8_t* b_host, int K, float* c_host);
void fp8_decode(const uint8_t* codes_host, int n, float* out_host);
// Full FP64 rescoring of the users in fail_list (device count at fail_count, host copy nfail).
void launch_fallback(int dtype, const RefineArgs& a, double* scratch, int64_t scratch_rows, hipStream_t s);

// ---------------------------------------------------------------- cone tree
struct ConeLevelArgs {
    const uint16_t* unit;  // [m x ld] BF16 unit users (original order), or
    const uint8_t* codes;  // [m x ld] FP8 codes (original order) with
    const float* fac;      // [m] scale / ||u|| per user: the unit vector is fac x codes
    int ld, d;
    const uint32_t* perm;  // position -> user
    const int64_t* seg_start;  // [nseg+1] this level's segments (sorted, last = m)
    int64_t* next_start;       // [.. + 1] the next level's segments
    int64_t* ctl;              // [4] nseg of this level, nseg of the next, active segments of the next
    int ctl_cur;               // index of this level's nseg in ctl (0 or 1)
    int level, leaf;           // level number (pivot draws), N0
    uint64_t seed;
    int64_t m;
    const int* act;        // [nseg] active index of each segment (-1: leaf)
    int* next_act;         // the next level's
    unsigned long long* key1; unsigned long long* key2;  // [active x 8] argmin slots
    unsigned long long* next_key1; unsigned long long* next_key2;  // the next level's
    float* dot_l;          // [m] per position
    int* left;             // [m] per position
    int* nleft;            // [nseg] left count of each active segment
    int* degen;            // [nseg] split fell back to index halves
    const int* seg;        // [m] position -> segment of this level
    int* next_seg;         // [m] position -> segment of the next level (written by the scatter)
    int* next_index;       // [nseg] first next-level segment made from each segment
    int* lrank;            // [m] left flags before the position inside its 256-position block
    int* blk_cnt;          // [ceil(m/256)] left flags per block; exclusive prefix after k_cone_next
    // level-0 set-up only
    uint32_t* perm_init; int* seg_init; int64_t* seg_start_init; int* act_init;
};
struct LeafArgs {
    int dtype;
    const void* users;       // leaf order [m x ld]
    const float* user_scales;
    const double* user_n2;   // leaf order
    const uint32_t* perm;    // leaf position -> original user
    const int64_t* block_start;
    int64_t nblocks, m;
    int d, ld, k_max;
    const double* lam64;     // [k_max x m] original user order
    float* center;           // [nblocks x ld] unit centres
    float* cos_w; float* sin_w; int* block_ok;   // [nblocks]
    float* unorm; float* cos_t; float* sin_t;    // [m] leaf order
    int* user_block;                             // [m]
    float* block_lb;                             // [k_max x nblocks]
};

// ---------------------------------------------------------------- SA-ALSH
struct SaQueryArgs {
    int dtype;
    const void* items; const float* item_scales; int64_t n; int d, ld;   // sorted order
    const void* users; const float* user_scales;                          // leaf order
    const void* queries; const float* query_scales;                       // padded copy
    const double* item_n2; const double* user_n2;
    const int64_t* part_start; int t;
    const uint32_t* item_codes; const uint32_t* user_codes; int K;
    float beta;
    const unsigned long long* pairs; int64_t npairs;   // (query << 32) | leaf user
    const int* qk;                                     // k per query
    double* phi; int* answer;                          // per pair (k_saalsh_query)
    // SAH (launch_sah): the pair count on the device (npairs is its cap); u's scores on
    // P' start the candidate set -- the first entries of its lambda row (lam64
    // [k_max x m] by original user); a "yes" goes straight to the answers (bits, else
    // the pool as (caller query << 32) | original user), a "no" counts in *rejects
    const unsigned long long* npairs_dev;
    const double* lam64; const uint32_t* perm; int64_t m; int64_t n_init;
    uint32_t* bitmap; int64_t bm_words;
    unsigned long long* pool; unsigned long long* pool_count; int64_t pool_cap;
    const uint32_t* qorig;
    unsigned long long* rejects;
    // SAH: 1; LAZY: 1 + 2^-40, so that mu_j bounds every canonical FP64 score of the
    // partition despite the rounding of the scores and of mu_j itself
    double mu_scale;
    // Candidate appends past a workgroup's scratch row are not written: they set bit 4
    // of *overflow (if given) and the caller fails the call.  The launchers check the
    // sizes that make this impossible before every launch; the flag is the backstop.
    int64_t cand_cap;       // set by the launchers to scratch_stride
    int* overflow;
};
// Alg. 2 for each pair; scratch: grid x scratch_stride doubles (>= ceil(beta n) + t),
// scratch_bytes: its allocation (checked).
void launch_saalsh_query(const SaQueryArgs& a, double* scratch, size_t scratch_bytes, int64_t scratch_stride,
                         int grid, hipStream_t s);
// SAH (Alg. 5) for the listed pairs: slots for the users flagged in need[m] (slot,
// user_of_slot: int [m]; *nslots zeroed by the caller), per-user tables of kstar
// (>= every k of the pairs) scores after each partition, chunk slots at a time (tab:
// chunk x (t + 1) x kstar doubles), then the per-pair decisions; score[i]: s(u,q) of
// pair i.  scratch: grid x scratch_stride doubles (>= ceil(beta n) + t + 1 + kstar).
// SA-ALSH kMIPS for nu users (leaf positions user_of_slot, *nslots = nu on the device):
// tab [nu x (t + 1) x k] per-partition best-k rows, jlast [nu] the last row written.
void launch_saalsh_kmips(const SaQueryArgs& a, const int* user_of_slot, const int* nslots, int64_t nu, int k,
                         double* tab, int* jlast, double* scratch, size_t scratch_bytes, int64_t scratch_stride,
                         int grid, hipStream_t s);
void launch_sah(const SaQueryArgs& a, const unsigned char* need, int* slot, int* user_of_slot, int* nslots,
                const double* score, int kstar, double* tab, int64_t chunk, double* scratch, size_t scratch_bytes,
                int64_t scratch_stride, int grid, hipStream_t s);
constexpr int kSaalshOverflowBit = 4;

// ---------------------------------------------------------------- query
struct QueryArgs {
    int dtype;
    const void* users; const float* user_scales;     // leaf order [m x ld]
    int64_t m; int d, ld;
    const float* unorm; const float* cos_t; const float* sin_t;
    const int* user_block;
    const float* center; const float* cos_w; const float* sin_w; const int* block_ok;
    const uint16_t* center_mma;                      // [nblocks x 2 ld] BF16 [hi | lo], or null
    const float* block_lb; int64_t nblocks;
    const uint32_t* perm;                            // leaf -> original
    const float* lam32; const double* lam64; int k_max;   // [k_max x m], original user order
    const void* queries; const float* query_scales; int64_t nq;   // padded copy [nq x ld]
    // matrix-core operands of the inner-product test: the two arrays above, or their
    // split BF16 rows [x 3 ld] for FP32 data (users [h | h | l], queries [h | l | h])
    const void* mma_users; const void* mma_queries; int mma_dtype, mma_ld;
    const float* qnorm;                              // [nq]
    const float* cphi;                               // [nblocks x nq] cos of the query-centre angle
    // Lemma 2 prune words [nblocks x ntq]: bit i of word (b, T) is set when the block test
    // removes block b for query 32 T + i (written with the cosines; read by the ring form)
    uint32_t* prune; int64_t ntq;
    const int* qslot;                                // [nq] slot of the query's k
    const uint32_t* qorig;                           // [nq] k-sorted position -> caller index
    const int* qk;                                   // [nq] k of each (k-sorted) query
    int* bad;                                        // query validation flags
    const int* slot_k;                               // [nslots]
    int nslots;
    int flags;
    double err_rel;                                  // relative error bound of the fast score
    float err_phi;                                   // error bound of the FP32 cos(phi)
    float bound_slack;                               // relative slack of the bounds
    unsigned long long* pool; unsigned long long* pool_count; int64_t pool_cap;
    // yes answers as bits [nq x bm_words] by caller query and original user, in place of
    // the pool (null: the pool)
    uint32_t* bitmap; int64_t bm_words;
    unsigned long long* amb; unsigned long long* amb_count; int64_t amb_cap;
    unsigned long long* stats;                       // [8]
    // SAH mode (Alg. 5): the inner-product test hands every pair it does not reject to
    // the FP64 recheck, which answers yes when s >= ||u|| ||p_k|| and otherwise lists
    // the pair (same key as amb) for Alg. 2
    int sah;
    // relative widening of n2(u) n2(p_k) in that test: 0 in SAH mode (the paper's test);
    // 2^-40 in the exact lazy mode, where the canonical scores may exceed ||u|| ||p|| by
    // their rounding (below (d + 1) 2^-53 relative for d <= 256) and the squared-norm
    // products round too (both sides below 2^-43 in total)
    double norm_widen;
    const double* item_n2; int64_t n_items;          // sorted canonical squared norms
    const double* user_n2;                           // leaf order
    unsigned long long* sah_pairs; unsigned long long* sah_count;   // capacity amb_cap
    double* sah_score;                               // s(u,q) of each listed pair
    unsigned char* sah_need;                         // [m] leaf order: u has a listed pair
};
void launch_qnorm(int dtype, const void* Q, const float* qs, int64_t nq, int d, int ld,
                  float* qnorm, int* bad, hipStream_t s);
// cos(phi) per (block, query) into cphi (null: not stored) and the prune words a.prune
void launch_phi(const QueryArgs& a, float* cphi, hipStream_t s);
// true when launch_verify_range takes the ring form for this index (it reads the prune
// words only, not the cosines)
bool verify_uses_ring(const QueryArgs& a);
void launch_verify_range(const QueryArgs& a, int64_t q_begin, int64_t q_end, hipStream_t s);
void launch_recheck(const QueryArgs& a, int64_t namb, const int* reject, hipStream_t s);
// Item insertion: merge the canonical scores of n_new padded item rows into every user's
// lambda row (users, user_scales, perm: leaf order; lam64/lam32 [k_max x m] by original user).
void launch_insert_lambda(int dtype, const void* users, const float* user_scales, const uint32_t* perm, int64_t m,
                          int d, int ld, const void* items, const float* item_scales, int64_t n_new, double* lam64,
                          float* lam32, int k_max, unsigned long long* changed, hipStream_t s);
// Per-query ascending lists from the answer bits: counts, offsets (as launch_result_lists),
// then the ids (those past ids_cap are dropped: the caller checks offsets[nq]).
void launch_bitmap_lists(const uint32_t* bitmap, int64_t words, int64_t nq, int* cnt, int64_t* offsets,
                         long long* stat, int32_t* ids, int64_t ids_cap, hipStream_t s);
// the same with the close-call count kept on the device (pool tail cleared, span in ctr[5])
void launch_recheck_device(const QueryArgs& a, hipStream_t s);
// span_dev null: the pool span is `span`; otherwise it is read on the device and `span`
// is its upper bound
void launch_result_lists(const uint64_t* keys, int64_t span, const unsigned long long* span_dev, int64_t nq, int* cnt,
                         int64_t* offsets, long long* stat, int32_t* tmp, int32_t* ids, hipStream_t s);
void launch_result_merges(int64_t nq, int64_t max_count, const int64_t* offsets, int32_t* tmp, int32_t* ids,
                          hipStream_t s);

}  // namespace rk
