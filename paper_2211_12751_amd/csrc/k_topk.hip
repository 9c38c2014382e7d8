// lambda build: for every user u, lambda_u^(j), j = 1..k_max, the j-th largest inner
// product of u over all items (Definition 1; the lower-bound array of Alg. 4 taken
// over all of P instead of the top-norm subset P').
//
// Pass 1 (k_topk): fused U.P^T on the matrix cores with a streaming per-user top-C
//   (C = k_max + slack).  A workgroup keeps 128-256 users' operand fragments in
//   registers and streams item tiles (items in descending norm order, so the first
//   tile already holds the paper's P' and sets a high threshold early) through LDS.
//   Every MFMA output lane owns one user column; a score enters the user's candidate
//   buffer only if it beats the user's running threshold (register compare, ballot
//   gated).  When a buffer fills, the wave compacts it to its C best entries with a
//   wave-cooperative radix select and raises the threshold.  The threshold tau that
//   remains bounds every item left out.
// Pass 2 (k_refine): canonical FP64 rescoring of the candidates, ranking, and a
//   certificate: tau + eps(u) <= lambda64^(k_max) proves no left-out item can enter
//   the top k_max.  Users that fail get a full-row FP64 rescoring (k_fallback).
#include "common.h"
#include "internal.h"

namespace rk {

static constexpr int TK_WAVES = 4;
static constexpr int TK_IT = 64;  // items per LDS tile (two 32-row MFMA blocks)

// ------------------------------------------------------------------ wave radix select
// Compacts the `c` entries of a user's buffer (keys = orderable scores) to its C largest
// (ties at the threshold kept in buffer order) and returns the C-th largest key.
template <int GPL>
__device__ __forceinline__ uint32_t wave_select_compact(uint2* region, int c, int C, int* hist)
{
    const int l = lane_id();
    uint32_t key[GPL], id[GPL];
#pragma unroll
    for (int i = 0; i < GPL; i++) {
        const int idx = l + 64 * i;
        if (idx < c) {
            const unsigned long long raw = __hip_atomic_load((unsigned long long*)(region + idx),
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint2 w = make_uint2((uint32_t)raw, (uint32_t)(raw >> 32));
            key[i] = w.x;
            id[i] = w.y;
        } else {
            key[i] = 0u;
            id[i] = 0u;
        }
    }
    uint32_t prefix = 0u, pmask = 0u;
    int need = C;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = l; b < 256; b += 64) hist[b] = 0;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < GPL; i++)
            if (l + 64 * i < c && (key[i] & pmask) == prefix) atomicAdd(&hist[(key[i] >> shift) & 255u], 1);
        __builtin_amdgcn_wave_barrier();
        int h[4], x = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) { h[e] = hist[4 * l + e]; x += h[e]; }
        const int incl = wave_incl_scan(x);
        const int total = __shfl(incl, 63);
        int above = total - incl;  // keys whose digit lies in higher lanes' bins
        int sel = -1, sel_above = 0;
#pragma unroll
        for (int e = 3; e >= 0; e--) {
            if (sel < 0 && above < need && need <= above + h[e]) { sel = 4 * l + e; sel_above = above; }
            above += h[e];
        }
        const uint64_t bal = ballot64(sel >= 0);
        const int src = __builtin_ctzll(bal);
        const int dsel = __shfl(sel, src);
        const int dabove = __shfl(sel_above, src);
        prefix |= (uint32_t)dsel << shift;
        pmask |= 0xffu << shift;
        need -= dabove;
        __builtin_amdgcn_wave_barrier();
    }
    const uint32_t T = prefix;
    int eq_before = 0, kept_before = 0;
    int outpos[GPL];
#pragma unroll
    for (int i = 0; i < GPL; i++) {
        const bool valid = l + 64 * i < c;
        const bool gt = valid && key[i] > T;
        const bool eq = valid && key[i] == T;
        const uint64_t eb = ballot64(eq);
        const int rank_eq = eq_before + __popcll(eb & lanemask_lt());
        eq_before += __popcll(eb);
        const bool keep = gt || (eq && rank_eq < need);
        const uint64_t kb = ballot64(keep);
        outpos[i] = keep ? kept_before + __popcll(kb & lanemask_lt()) : -1;
        kept_before += __popcll(kb);
    }
#pragma unroll
    for (int i = 0; i < GPL; i++)
        if (outpos[i] >= 0) region[outpos[i]] = make_uint2(key[i], id[i]);
    return T;
}

// ------------------------------------------------------------------ fused GEMM + top-k
template <int DT, int DPT, int UBW, int GPL>
__global__ __launch_bounds__(256) void k_topk(TopkArgs a)
{
    constexpr int EB = Elt<DT>::bytes;
    constexpr int ROWB = DPT * EB;                // bytes of one stored row
    constexpr int LROW = ROWB + 16;               // padded LDS row (bank spread)
    constexpr int KSTEPS = ROWB / 32;             // 16-byte fragments per half row
    __shared__ __attribute__((aligned(16))) uint8_t tile[TK_IT * LROW];
    __shared__ float tscale[TK_IT];
    __shared__ int hist_all[TK_WAVES][256];

    const int l = lane_id();
    const int w = threadIdx.x >> 6;
    const int h = l >> 5;
    int* hist = hist_all[w];
    const int seg = blockIdx.y;
    const int64_t seg0 = (int64_t)seg * a.seg_len;
    int64_t seg1 = seg0 + a.seg_len;
    if (seg1 > a.n) seg1 = a.n;
    const int64_t user0 = (int64_t)blockIdx.x * (TK_WAVES * UBW * 32) + (int64_t)w * (UBW * 32);

    // ---- resident user fragments (the B operand), one user column per lane
    i32x4 bfrag[UBW][KSTEPS];
    float theta[UBW], su[UBW];
    int cnt[UBW];
    int64_t ug[UBW];
    uint2* region[UBW];
#pragma unroll
    for (int cb = 0; cb < UBW; cb++) {
        ug[cb] = user0 + cb * 32 + (l & 31);
        const bool ok = ug[cb] < a.m;
        const uint8_t* row = (const uint8_t*)a.users + (ok ? ug[cb] : 0) * ROWB;
#pragma unroll
        for (int t = 0; t < KSTEPS; t++) {
            i32x4 z = {0, 0, 0, 0};
            bfrag[cb][t] = ok ? *(const i32x4*)(row + t * 32 + h * 16) : z;
        }
        theta[cb] = ok ? -__builtin_inff() : __builtin_inff();   // +inf: nothing enters
        su[cb] = (DT == DT_FP8 && ok) ? a.user_scales[ug[cb]] : 1.0f;
        cnt[cb] = 0;
        region[cb] = a.buf + ((ok ? ug[cb] : 0) * a.nseg + seg) * (int64_t)a.G;
    }

    for (int64_t t0 = seg0; t0 < seg1; t0 += TK_IT) {
        // ---- stage the item tile
        __syncthreads();
        for (int c = threadIdx.x; c < TK_IT * (ROWB / 16); c += 256) {
            const int r = c / (ROWB / 16), c16 = c % (ROWB / 16);
            const int64_t p = t0 + r;
            i32x4 v = {0, 0, 0, 0};
            if (p < seg1) v = *(const i32x4*)((const uint8_t*)a.items + p * ROWB + c16 * 16);
            *(i32x4*)(tile + r * LROW + c16 * 16) = v;
        }
        if (DT == DT_FP8 && threadIdx.x < TK_IT) {
            const int64_t p = t0 + threadIdx.x;
            tscale[threadIdx.x] = p < seg1 ? a.item_scales[p] : 0.f;
        }
        __syncthreads();

#pragma unroll
        for (int rb = 0; rb < TK_IT / 32; rb++) {
            f32x16 acc[UBW];
#pragma unroll
            for (int cb = 0; cb < UBW; cb++)
#pragma unroll
                for (int r = 0; r < 16; r++) acc[cb][r] = 0.f;
            const uint8_t* arow = tile + (rb * 32 + (l & 31)) * LROW + h * 16;
#pragma unroll
            for (int t = 0; t < KSTEPS; t++) {
                const i32x4 af = *(const i32x4*)(arow + t * 32);
                if constexpr (DT == DT_F32) {
                    const f32x4 a4 = __builtin_bit_cast(f32x4, af);
#pragma unroll
                    for (int e = 0; e < 4; e++)
#pragma unroll
                        for (int cb = 0; cb < UBW; cb++) {
                            const f32x4 b4 = __builtin_bit_cast(f32x4, bfrag[cb][t]);
                            acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[e], b4[e], acc[cb], 0, 0, 0);
                        }
                } else if constexpr (DT == DT_BF16) {
                    const bf16x8 a8 = __builtin_bit_cast(bf16x8, af);
#pragma unroll
                    for (int cb = 0; cb < UBW; cb++)
                        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            a8, __builtin_bit_cast(bf16x8, bfrag[cb][t]), acc[cb], 0, 0, 0);
                } else {
                    // FP8 e4m3: 32x32x16 over 8 codes per lane and MFMA (two per fragment)
                    const long a0 = __builtin_bit_cast(long, (int __attribute__((ext_vector_type(2)))){af[0], af[1]});
                    const long a1 = __builtin_bit_cast(long, (int __attribute__((ext_vector_type(2)))){af[2], af[3]});
#pragma unroll
                    for (int cb = 0; cb < UBW; cb++) {
                        const i32x4 bf = bfrag[cb][t];
                        const long b0 = __builtin_bit_cast(long, (int __attribute__((ext_vector_type(2)))){bf[0], bf[1]});
                        const long b1 = __builtin_bit_cast(long, (int __attribute__((ext_vector_type(2)))){bf[2], bf[3]});
                        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a0, b0, acc[cb], 0, 0, 0);
                        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a1, b1, acc[cb], 0, 0, 0);
                    }
                }
            }

            // ---- epilogue: threshold filter, buffer append, compaction when full
#pragma unroll
            for (int cb = 0; cb < UBW; cb++) {
                float v[16];
                uint32_t pm = 0u;
#pragma unroll
                for (int r = 0; r < 16; r++) {
                    const int row = rb * 32 + mfma32_row(r, l);
                    float x = acc[cb][r];
                    if constexpr (DT == DT_FP8) x = (su[cb] * tscale[row]) * x;
                    v[r] = x;
                    if (t0 + row < seg1 && x > theta[cb]) pm |= 1u << r;
                }
                // every cross-lane read happens with the whole wave active: a permute
                // from an inactive lane returns 0
                int np = __popc(pm);
                int npo = __shfl_xor(np, 32);
                int tot = np + npo;
                uint64_t need = ballot64(cnt[cb] + tot > a.G) & 0xffffffffull;
                if (need) {
                    while (need) {
                        const int ul = __builtin_ctzll(need);
                        need &= need - 1;
                        const int c = __shfl(cnt[cb], ul);
                        const int64_t ugl = __shfl(ug[cb], ul);
                        uint2* rg = a.buf + (ugl * a.nseg + seg) * (int64_t)a.G;
                        const uint32_t T = wave_select_compact<GPL>(rg, c, a.C, hist);
                        if ((l & 31) == ul) {
                            theta[cb] = ord_f32(T);
                            cnt[cb] = a.C;
                        }
                    }
                    pm = 0u;
#pragma unroll
                    for (int r = 0; r < 16; r++) {
                        const int row = rb * 32 + mfma32_row(r, l);
                        if (t0 + row < seg1 && v[r] > theta[cb]) pm |= 1u << r;
                    }
                    np = __popc(pm);
                    npo = __shfl_xor(np, 32);
                    tot = np + npo;
                }
                if (tot) {
                    int pos = cnt[cb] + (h ? npo : 0);
#pragma unroll
                    for (int r = 0; r < 16; r++)
                        if (pm & (1u << r)) {
                            const int row = rb * 32 + mfma32_row(r, l);
                            region[cb][pos++] = make_uint2(f32_ord(v[r]), (uint32_t)(t0 + row));
                        }
                    cnt[cb] += tot;
                }
            }
        }
    }

    // ---- final compaction and outputs
#pragma unroll
    for (int cb = 0; cb < UBW; cb++) {
        uint64_t need = ballot64(cnt[cb] > a.C) & 0xffffffffull;
        while (need) {
            const int ul = __builtin_ctzll(need);
            need &= need - 1;
            const int c = __shfl(cnt[cb], ul);
            const int64_t ugl = __shfl(ug[cb], ul);
            uint2* rg = a.buf + (ugl * a.nseg + seg) * (int64_t)a.G;
            const uint32_t T = wave_select_compact<GPL>(rg, c, a.C, hist);
            if ((l & 31) == ul) {
                theta[cb] = ord_f32(T);
                cnt[cb] = a.C;
            }
        }
        if (l < 32 && ug[cb] < a.m) {
            a.cnt[ug[cb] * a.nseg + seg] = cnt[cb];
            a.tau[ug[cb] * a.nseg + seg] = theta[cb];
        }
    }
}

template <int DT, int DPT>
static void topk_dispatch_g(const TopkArgs& a, hipStream_t s)
{
    constexpr int UBW = (DT == DT_F32 && DPT >= 256) ? 1 : 2;
    dim3 grid((unsigned)((a.m + TK_WAVES * UBW * 32 - 1) / (TK_WAVES * UBW * 32)), (unsigned)a.nseg);
    const int gpl = a.G / 64;
    if (gpl == 2) hipLaunchKernelGGL((k_topk<DT, DPT, UBW, 2>), grid, dim3(256), 0, s, a);
    else if (gpl == 4) hipLaunchKernelGGL((k_topk<DT, DPT, UBW, 4>), grid, dim3(256), 0, s, a);
    else if (gpl == 8) hipLaunchKernelGGL((k_topk<DT, DPT, UBW, 8>), grid, dim3(256), 0, s, a);
    else fail(RKMIPS_EINVAL, "internal: unsupported candidate buffer size");
}

int topk_users_per_block(int dtype, int ld)
{
    const int ubw = (dtype == DT_F32 && ld >= 256) ? 1 : 2;
    return TK_WAVES * ubw * 32;
}

template <int DT>
static void topk_dispatch(const TopkArgs& a, hipStream_t s)
{
    switch (a.ld) {
    case 32: topk_dispatch_g<DT, 32>(a, s); break;
    case 64: topk_dispatch_g<DT, 64>(a, s); break;
    case 128: topk_dispatch_g<DT, 128>(a, s); break;
    case 256: topk_dispatch_g<DT, 256>(a, s); break;
    default: fail(RKMIPS_EINVAL, "internal: unsupported padded dimension");
    }
}

void launch_topk(int dtype, const TopkArgs& a, hipStream_t s)
{
    if (a.m <= 0 || a.n <= 0) return;
    if (dtype == DT_F32) topk_dispatch<DT_F32>(a, s);
    else if (dtype == DT_BF16) topk_dispatch<DT_BF16>(a, s);
    else topk_dispatch<DT_FP8>(a, s);
    HIPC(hipGetLastError());
}

// ------------------------------------------------------------------ FP64 refine + certificate
static constexpr int RF_MAXN = 512;  // candidates per user across segments

template <int DT>
__global__ __launch_bounds__(256) void k_refine(RefineArgs a)
{
    const double err_rel = a.err_rel;
    __shared__ uint32_t sid[4][RF_MAXN];
    __shared__ double s64[4][RF_MAXN];
    __shared__ float sraw[4][RF_MAXN];
    __shared__ double lam_row[4][256];
    __shared__ float raw_row[4][256];
    const int l = lane_id(), w = threadIdx.x >> 6;
    const int64_t u = (int64_t)blockIdx.x * 4 + w;
    if (u >= a.m) return;

    // gather candidates of all segments
    int N = 0;
    for (int s = 0; s < a.nseg; s++) {
        const int c = a.cnt[u * a.nseg + s];
        const uint2* rg = a.buf + (u * a.nseg + s) * (int64_t)a.G;
        for (int i = l; i < c; i += 64) {
            uint2 e = rg[i];
            sid[w][N + i] = e.y;
            sraw[w][N + i] = ord_f32(e.x);
        }
        N += c;
    }
    __builtin_amdgcn_wave_barrier();
    const float su = DT == DT_FP8 ? a.user_scales[u] : 1.f;
    for (int j = l; j < N; j += 64) {
        const int64_t p = sid[w][j];
        if (p >= a.n) {                  // never produced by k_topk; guards the load below
            s64[w][j] = -__builtin_inf();
            continue;
        }
        const float sp = DT == DT_FP8 ? a.item_scales[p] : 1.f;
        s64[w][j] = canon_dot<DT>(a.users, u, su, a.items, p, sp, a.d, a.ld);
    }
    __builtin_amdgcn_wave_barrier();
    for (int j = l; j < N; j += 64) {
        const double x = s64[w][j];
        const float y = sraw[w][j];
        int r64 = 0, rr = 0;
        for (int i = 0; i < N; i++) {
            const double xi = s64[w][i];
            const float yi = sraw[w][i];
            r64 += (xi > x) || (xi == x && i < j);
            rr += (yi > y) || (yi == y && i < j);
        }
        if (r64 < a.k_max) lam_row[w][r64] = x;
        if (rr < a.k_max) raw_row[w][rr] = y;
    }
    __builtin_amdgcn_wave_barrier();
    double worst = 0.0;
    for (int r = l; r < a.k_max; r += 64) {
        const double lv = r < N ? lam_row[w][r] : -__builtin_inf();
        a.lam64[(int64_t)r * a.m + u] = lv;
        a.lam32[(int64_t)r * a.m + u] = (float)lv;
        if (r < N && lv != 0.0) {
            const double e = fabs((double)raw_row[w][r] - lv) / fabs(lv);
            worst = e > worst ? e : worst;
        }
    }
    worst = wave_max(worst);
    if (l == 0 && worst > 0.0) atomicMax(a.max_raw_err_bits, (unsigned long long)__double_as_longlong(worst));

    // certificate: every item left out of segment s scored <= tau_s in the fast
    // arithmetic, hence <= tau_s + eps in exact arithmetic; it cannot enter the top
    // k_max if that is <= lambda64^(k_max).
    bool ok = !a.force_fail;
    if (ok && N < a.n) {
        const double un = sqrt(a.user_n2[u]);
        const double lk = N >= a.k_max ? lam_row[w][a.k_max - 1] : -__builtin_inf();
        for (int s = 0; s < a.nseg; s++) {
            const float t = a.tau[u * a.nseg + s];
            if (t == -__builtin_inff()) continue;   // every item of the segment is a candidate
            const int64_t first = (int64_t)s * a.seg_len;
            const double Ms = sqrt(a.item_n2_sorted[first]);
            const double bound = (double)t + err_rel * un * Ms + (double)a.d * 0x1p-125 * (un + Ms + 1.0);
            if (!(bound <= lk)) ok = false;
        }
    }
    if (!ok && l == 0) {
        const int pos = atomicAdd(a.fail_count, 1);
        a.fail_list[pos] = (int)u;
    }
}

void launch_refine(int dtype, const RefineArgs& a, hipStream_t s)
{
    if (a.m <= 0) return;
    if ((int64_t)a.nseg * a.C > RF_MAXN) fail(RKMIPS_EINVAL, "internal: too many candidates per user");
    dim3 g((unsigned)((a.m + 3) / 4)), b(256);
    if (dtype == DT_F32) hipLaunchKernelGGL(k_refine<DT_F32>, g, b, 0, s, a);
    else if (dtype == DT_BF16) hipLaunchKernelGGL(k_refine<DT_BF16>, g, b, 0, s, a);
    else hipLaunchKernelGGL(k_refine<DT_FP8>, g, b, 0, s, a);
    HIPC(hipGetLastError());
}

// ------------------------------------------------------------------ full FP64 fallback
template <int DT>
__global__ __launch_bounds__(256) void k_fallback(RefineArgs a, int64_t nfail, double* scratch,
                                                  int64_t scratch_rows)
{
    __shared__ int hist[256];
    __shared__ int s_sel, s_above;
    __shared__ double top[256];
    __shared__ int ntop;
    const int tid = threadIdx.x;
    for (int64_t fi = blockIdx.x; fi < nfail; fi += gridDim.x) {
        const int64_t u = a.fail_list[fi];
        double* sc = scratch + (int64_t)(blockIdx.x % scratch_rows) * a.n;
        const float su = DT == DT_FP8 ? a.user_scales[u] : 1.f;
        for (int64_t p = tid; p < a.n; p += 256) {
            const float sp = DT == DT_FP8 ? a.item_scales[p] : 1.f;
            sc[p] = canon_dot<DT>(a.users, u, su, a.items, p, sp, a.d, a.ld);
        }
        __syncthreads();
        const int want = (int)(a.n < a.k_max ? a.n : a.k_max);
        // radix select of the want-th largest (orderable 64-bit keys, 8 digits)
        uint64_t prefix = 0, pmask = 0;
        int need = want;
        for (int shift = 56; shift >= 0; shift -= 8) {
            hist[tid] = 0;
            __syncthreads();
            for (int64_t p = tid; p < a.n; p += 256) {
                const uint64_t k = f64_ord(sc[p]);
                if ((k & pmask) == prefix) atomicAdd(&hist[(k >> shift) & 255], 1);
            }
            __syncthreads();
            if (tid == 0) {
                int above = 0;
                for (int b = 255; b >= 0; b--) {
                    if (above < need && need <= above + hist[b]) { s_sel = b; s_above = above; break; }
                    above += hist[b];
                }
            }
            __syncthreads();
            prefix |= (uint64_t)s_sel << shift;
            pmask |= 0xffull << shift;
            need -= s_above;
            __syncthreads();
        }
        const double T = ord_f64(prefix);
        if (tid == 0) ntop = 0;
        __syncthreads();
        for (int64_t p = tid; p < a.n; p += 256)
            if (sc[p] > T) top[atomicAdd(&ntop, 1)] = sc[p];
        __syncthreads();
        const int ng = ntop;   // < want
        for (int j = tid; j < ng; j += 256) {
            int r = 0;
            for (int i = 0; i < ng; i++) r += (top[i] > top[j]) || (top[i] == top[j] && i < j);
            a.lam64[(int64_t)r * a.m + u] = top[j];
            a.lam32[(int64_t)r * a.m + u] = (float)top[j];
        }
        for (int r = ng + tid; r < a.k_max; r += 256) {
            const double v = r < want ? T : -__builtin_inf();
            a.lam64[(int64_t)r * a.m + u] = v;
            a.lam32[(int64_t)r * a.m + u] = (float)v;
        }
        __syncthreads();
    }
}

void launch_fallback(int dtype, const RefineArgs& a, int64_t nfail, double* scratch, int64_t scratch_rows,
                     hipStream_t s)
{
    if (nfail <= 0) return;
    const unsigned g = (unsigned)(nfail < scratch_rows ? nfail : scratch_rows);
    if (dtype == DT_F32) hipLaunchKernelGGL(k_fallback<DT_F32>, dim3(g), dim3(256), 0, s, a, nfail, scratch, scratch_rows);
    else if (dtype == DT_BF16) hipLaunchKernelGGL(k_fallback<DT_BF16>, dim3(g), dim3(256), 0, s, a, nfail, scratch, scratch_rows);
    else hipLaunchKernelGGL(k_fallback<DT_FP8>, dim3(g), dim3(256), 0, s, a, nfail, scratch, scratch_rows);
    HIPC(hipGetLastError());
}

__global__ void k_lam32_err(const double* lam64, const float* lam32, int64_t count, unsigned long long* out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < count) {
        const double x = lam64[i];
        if (x != 0.0 && x != -__builtin_inf()) e = fabs((double)lam32[i] - x) / fabs(x);
    }
    e = wave_max(e);
    if (lane_id() == 0 && e > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(e));
}

void launch_lambda32_err(const double* lam64, const float* lam32, int64_t count, unsigned long long* max_err_bits,
                         hipStream_t s)
{
    if (count <= 0) return;
    hipLaunchKernelGGL(k_lam32_err, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, lam64, lam32, count,
                       max_err_bits);
    HIPC(hipGetLastError());
}

}  // namespace rk
