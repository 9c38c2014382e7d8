// Index save and load.  The paper builds its index (Alg. 4) once per item and user set;
// this keeps a complete index in one file so that a server can start from it.
//
// File layout (host byte order):
//   8 bytes  magic "RKMIPSIX"
//   Header   (version, sizes, scalars, the build parameters)
//   for each array of arrays(), in order: uint64 byte count, then the bytes
// The raw candidates of the lambda build (inspection only) are not kept.
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "index.h"
#include "internal.h"
#include "mem.h"
#include "query.h"

namespace rk {

namespace {

constexpr char kMagic[8] = {'R', 'K', 'M', 'I', 'P', 'S', 'I', 'X'};
constexpr uint32_t kVersion = 2;

struct Header {
    uint32_t version;
    int32_t d, ld, dtype, mma_dtype, mma_ld, t, C, G, nseg, device_unused;
    int64_t n, m, n_lam, nblocks, ns, seg_len, cert_failures;
    double err_fast, max_item_norm, max_user_norm, max_rel_err_raw, max_rel_err_l32;
    double ms_norms, ms_lambda, ms_refine, ms_saalsh, ms_cone, ms_total, ms_seed, ms_topk;
    rkmips_params prm;
};
// A change of either layout must come with a new kVersion.
static_assert(sizeof(Header) == 256 && sizeof(rkmips_params) == 48, "index file layout changed: bump kVersion");

std::vector<DevBuf*> arrays(Index& x)
{
    return {&x.items, &x.item_scales, &x.item_order, &x.item_n2, &x.users, &x.user_scales, &x.users_mma,
            &x.user_perm, &x.user_n2, &x.unorm, &x.cos_t, &x.sin_t, &x.user_block, &x.block_start,
            &x.center, &x.cos_w, &x.sin_w, &x.block_ok, &x.block_lb, &x.lam64, &x.lam32, &x.part_start,
            &x.num_parts, &x.centroid, &x.radius, &x.srp, &x.item_codes, &x.user_codes};
}

struct File {
    std::FILE* f = nullptr;
    ~File()
    {
        if (f) std::fclose(f);
    }
};

void put(std::FILE* f, const void* p, size_t b)
{
    if (b && std::fwrite(p, 1, b, f) != b) fail(RKMIPS_EINVAL, "index file: write failed");
}

void get(std::FILE* f, void* p, size_t b)
{
    if (b && std::fread(p, 1, b, f) != b) fail(RKMIPS_EINVAL, "index file: truncated");
}

}  // namespace

void save_index(Index& x, const char* path)
{
    x.wait_ready();
    File fl;
    fl.f = std::fopen(path, "wb");
    if (!fl.f) fail(RKMIPS_EINVAL, std::string("cannot open ") + path + " for writing");
    Header h{};
    h.version = kVersion;
    h.d = x.d; h.ld = x.ld; h.dtype = x.dtype; h.mma_dtype = x.mma_dtype; h.mma_ld = x.mma_ld;
    h.t = x.t; h.C = x.C; h.G = x.G; h.nseg = x.nseg;
    h.n = x.n; h.m = x.m; h.n_lam = x.n_lam; h.nblocks = x.nblocks; h.ns = x.ns; h.seg_len = x.seg_len;
    h.cert_failures = x.cert_failures;
    h.err_fast = x.err_fast; h.max_item_norm = x.max_item_norm; h.max_user_norm = x.max_user_norm;
    h.max_rel_err_raw = x.max_rel_err_raw; h.max_rel_err_l32 = x.max_rel_err_l32;
    h.ms_norms = x.ms_norms; h.ms_lambda = x.ms_lambda; h.ms_refine = x.ms_refine; h.ms_saalsh = x.ms_saalsh;
    h.ms_cone = x.ms_cone; h.ms_total = x.ms_total; h.ms_seed = x.ms_seed; h.ms_topk = x.ms_topk;
    h.prm = x.prm;
    put(fl.f, kMagic, sizeof kMagic);
    put(fl.f, &h, sizeof h);
    std::vector<char> host;
    for (DevBuf* b : arrays(x)) {
        const uint64_t nb = b->p ? (uint64_t)b->bytes : 0;
        put(fl.f, &nb, sizeof nb);
        if (!nb) continue;
        host.resize(nb);
        HIPC(hipMemcpy(host.data(), b->p, nb, hipMemcpyDeviceToHost));
        put(fl.f, host.data(), nb);
    }
    if (std::fflush(fl.f) != 0) fail(RKMIPS_EINVAL, "index file: write failed");
}

// Byte count that the header implies for array i of arrays() (0: the array is absent).
static uint64_t expected_bytes(const Header& h, int i)
{
    const uint64_t n = (uint64_t)h.n, m = (uint64_t)h.m, ld = (uint64_t)h.ld, nb = (uint64_t)h.nblocks;
    const uint64_t km = (uint64_t)h.prm.k_max, t = (uint64_t)h.t;
    const uint64_t W = (uint64_t)h.prm.num_hash / 32, eb = (uint64_t)elt_bytes(h.dtype);
    const bool fp8 = h.dtype == RKMIPS_FP8_E4M3;
    switch (i) {
    case 0: return n * ld * eb;                                   // items
    case 1: return fp8 ? 4 * n : 0;                               // item_scales
    case 2: return 4 * n;                                         // item_order
    case 3: return 8 * n;                                         // item_n2
    case 4: return m * ld * eb;                                   // users
    case 5: return fp8 ? 4 * m : 0;                               // user_scales
    case 6: return h.mma_dtype != h.dtype ? 2 * m * (uint64_t)h.mma_ld : 0;   // users_mma
    case 7: return 4 * m;                                         // user_perm
    case 8: return 8 * m;                                         // user_n2
    case 9: case 10: case 11: case 12: return 4 * m;              // unorm, cos_t, sin_t, user_block
    case 13: return 8 * (m + 1);                                  // block_start
    case 14: return 4 * nb * ld;                                  // center
    case 15: case 16: case 17: return 4 * nb;                     // cos_w, sin_w, block_ok
    case 18: return 4 * nb * km;                                  // block_lb
    case 19: return 8 * km * m;                                   // lam64
    case 20: return 4 * km * m;                                   // lam32
    case 21: return 8 * (n + 2);                                  // part_start
    case 22: return 4;                                            // num_parts
    case 23: return 4 * t * ld;                                   // centroid
    case 24: return 4 * t;                                        // radius
    case 25: return 4 * ((uint64_t)h.d + 1) * (uint64_t)h.prm.num_hash;   // srp
    case 26: return 4 * n * W;                                    // item_codes
    default: return 4 * m * W;                                    // user_codes
    }
}

static bool is_permutation(const std::vector<char>& a, int64_t count)
{
    const uint32_t* v = (const uint32_t*)a.data();
    std::vector<char> seen((size_t)count, 0);
    for (int64_t i = 0; i < count; i++) {
        if (v[i] >= (uint64_t)count || seen[v[i]]) return false;
        seen[v[i]] = 1;
    }
    return true;
}

static void bad_file(const std::string& what) { fail(RKMIPS_EINVAL, "index file: " + what); }

Index* load_index(const char* path, hipStream_t s)
{
    // Everything is read and checked on the host first: the header against the build's own
    // rules, each array's byte count against the size the header implies, and the index
    // arrays that the kernels follow (orders, block and partition tables) for range and
    // consistency.  Only then does the device see the file.
    File fl;
    fl.f = std::fopen(path, "rb");
    if (!fl.f) fail(RKMIPS_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    get(fl.f, magic, sizeof magic);
    if (std::memcmp(magic, kMagic, sizeof magic) != 0) fail(RKMIPS_EINVAL, "not an index file");
    Header h{};
    get(fl.f, &h, sizeof h);
    if (h.version != kVersion) fail(RKMIPS_EINVAL, "index file version " + std::to_string(h.version));
    validate_params(h.prm);
    if (h.dtype != RKMIPS_F32 && h.dtype != RKMIPS_BF16 && h.dtype != RKMIPS_FP8_E4M3) bad_file("unknown dtype");
    if (h.n < 1 || h.n > ((int64_t)1 << 30) || h.m < 1 || h.m > ((int64_t)1 << 31) - 2 || h.d < 1 || h.d > 256 ||
        h.ld != padded_dim(h.d, h.dtype))
        bad_file("inconsistent sizes");
    // the matrix-core operand form follows from dtype, ld and the flags, as in the build
    const bool split = h.dtype == RKMIPS_F32 && h.ld <= 64 && !(h.prm.flags & RKMIPS_FLAG_F32_MATRIX);
    const int mma = split ? DT_SPLIT : (h.dtype == RKMIPS_FP8_E4M3 ? DT_FP8B : h.dtype);
    if (h.mma_dtype != mma || h.mma_ld != (split ? 2 * h.ld : h.ld)) bad_file("inconsistent operand form");
    if (h.prm.mode == RKMIPS_MODE_EXACT ? h.n_lam != h.n
                                        : (h.n_lam != h.prm.sah_items || h.n_lam < 1 || h.n_lam >= h.n))
        bad_file("inconsistent lambda item count");
    const int64_t n0 = h.prm.mode == RKMIPS_MODE_EXACT ? 0 : h.n_lam;   // first position of the partitions
    if (h.t < 1 || h.t > h.n - n0 || h.nblocks < 1 || h.nblocks > h.m) bad_file("inconsistent partition or block count");
    if (h.G < 0 || h.G > 4096 || h.nseg < 0 || h.nseg > 4096 || h.C < 0 || h.C > 4096) bad_file("inconsistent build sizes");

    std::vector<DevBuf*> bufs;
    std::unique_ptr<Index> x(new Index());
    bufs = arrays(*x);
    std::vector<std::vector<char>> host(bufs.size());
    for (size_t i = 0; i < bufs.size(); i++) {
        uint64_t nb = 0;
        get(fl.f, &nb, sizeof nb);
        const uint64_t want = expected_bytes(h, (int)i);
        if (nb != want)
            bad_file("array " + std::to_string(i) + " holds " + std::to_string(nb) + " bytes, the header implies " +
                     std::to_string(want));
        host[i].resize(nb);
        get(fl.f, host[i].data(), nb);
    }
    // orders and tables the kernels index with
    if (!is_permutation(host[2], h.n)) bad_file("item order is not a permutation");
    if (!is_permutation(host[7], h.m)) bad_file("user order is not a permutation");
    {
        const int64_t* bs = (const int64_t*)host[13].data();
        const int* ub = (const int*)host[12].data();
        if (bs[0] != 0 || bs[h.nblocks] != h.m) bad_file("block table does not cover the users");
        for (int64_t b = 0; b < h.nblocks; b++) {
            if (bs[b + 1] <= bs[b] || bs[b + 1] - bs[b] > h.prm.leaf_size) bad_file("block table out of range");
            for (int64_t u = bs[b]; u < bs[b + 1]; u++)
                if (ub[u] != b) bad_file("user block index out of range");
        }
    }
    {
        const int64_t* ps = (const int64_t*)host[21].data();
        if (ps[0] != n0 || ps[h.t] != h.n) bad_file("partitions do not cover the items");
        for (int j = 0; j < h.t; j++)
            if (ps[j + 1] <= ps[j]) bad_file("partition table out of range");
        if (*(const int*)host[22].data() != h.t) bad_file("partition count disagrees with the header");
    }

    x->d = h.d; x->ld = h.ld; x->dtype = h.dtype; x->mma_dtype = h.mma_dtype; x->mma_ld = h.mma_ld;
    x->t = h.t; x->C = h.C; x->G = h.G; x->nseg = h.nseg;
    x->n = h.n; x->m = h.m; x->n_lam = h.n_lam; x->nblocks = h.nblocks; x->ns = h.ns; x->seg_len = h.seg_len;
    x->cert_failures = h.cert_failures;
    // the error bound of the fast scores is the build's own function of the operand form
    x->err_fast = split ? split_err_rel(h.d) : fast_err_rel(h.d);
    x->max_item_norm = h.max_item_norm; x->max_user_norm = h.max_user_norm;
    x->max_rel_err_raw = h.max_rel_err_raw; x->max_rel_err_l32 = h.max_rel_err_l32;
    x->ms_norms = h.ms_norms; x->ms_lambda = h.ms_lambda; x->ms_refine = h.ms_refine; x->ms_saalsh = h.ms_saalsh;
    x->ms_cone = h.ms_cone; x->ms_total = h.ms_total; x->ms_seed = h.ms_seed; x->ms_topk = h.ms_topk;
    x->prm = h.prm;

    // device side
    HIPC(hipGetDevice(&x->device));
    hipDeviceProp_t prop;
    HIPC(hipGetDeviceProperties(&prop, x->device));
    x->num_cus = prop.multiProcessorCount;
    mem::StreamScope scope(s);
    for (size_t i = 0; i < bufs.size(); i++) {
        if (host[i].empty()) continue;
        bufs[i]->alloc(host[i].size());
        HIPC(hipMemcpy(bufs[i]->p, host[i].data(), host[i].size(), hipMemcpyHostToDevice));
    }
    // derived from the stored centres rather than kept in the file
    make_center_operand(*x, s);
    make_user_inverse(*x, s);
    HIPC(hipStreamSynchronize(s));
    return x.release();
}

}  // namespace rk

using namespace rk;

namespace rk {
rkmips_status guarded_call(void (*fn)(void*), void* ctx);
}

template <typename F>
static rkmips_status pguard(F&& f)
{
    struct Ctx { F* f; } c{&f};
    return rk::guarded_call([](void* p) { (*((Ctx*)p)->f)(); }, &c);
}

extern "C" {

rkmips_status rkmips_index_save(const rkmips_index* idx, const char* path)
{
    return pguard([&] {
        if (!idx || !path) fail(RKMIPS_EINVAL, "NULL argument");
        save_index(*(Index*)idx, path);
    });
}

rkmips_status rkmips_index_load(const char* path, void* stream, rkmips_index** out)
{
    return pguard([&] {
        if (!path || !out) fail(RKMIPS_EINVAL, "NULL argument");
        *out = nullptr;
        *out = (rkmips_index*)load_index(path, (hipStream_t)stream);
    });
}

}  // extern "C"
