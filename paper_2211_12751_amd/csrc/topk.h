// Arguments and launchers of the fused top-k kernel (k_topk.hip), the first two passes
// of the exact lambda build.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rk {

struct TopkArgs {
    const void* items;      // sorted by norm, [n x ld]
    const float* item_scales;
    int64_t n;
    const void* users;      // original order, [m x ld]
    const float* user_scales;
    int64_t m;
    int d, ld;
    int64_t ns;             // seed pass: size of the stratified item sample (items then
                            // holds the gathered sample, n = ns)
    int64_t v0, v1;         // virtual item range of this launch
    int nseg;               // segments of this launch (grid.y)
    int seg_base;           // buffer segment of this launch's first segment
    int nseg_total;         // buffer segments per user
    int64_t seg_len;        // items per segment (multiple of the item tile)
    int C;                  // candidates kept per (user, segment)
    int G;                  // buffer capacity per (user, segment)
    const float* theta_init;  // per user starting threshold (stride theta_stride) or null
    int64_t theta_stride;
    uint2* buf;             // [m x nseg_total x G] {raw score bits, sorted item position}
    int* cnt;               // [m x nseg_total x 2] entries per buffer half
    float* tau;             // [m x nseg_total]
    float* theta_out;       // seed pass: [m] threshold estimates
};
enum { TK_MAIN = 0, TK_SEED = 1 };
constexpr int TK_T = 8;     // sample scores kept per lane by the seed pass
void launch_topk(int dtype, const TopkArgs& a, hipStream_t s);
void launch_topk_seed(int dtype, const TopkArgs& a, hipStream_t s);
int topk_users_per_block(int dtype, int ld);
// Bytes of one operand row of the top-k passes (ld elements of the operand form).
int topk_row_bytes(int dtype, int ld);
// The seed pass's stratified sample of ns of the n norm-sorted operand rows, gathered
// into dst [ns x row bytes] (and the scales into dscales when scales is given).
void launch_gather_sample(int dtype, const void* items, const float* scales, int64_t n, int64_t ns, int ld,
                          void* dst, float* dscales, hipStream_t s);
int topk_resident_blocks(int dtype, int ld, int G);


}  // namespace rk
