// Index save and load.  The paper builds its index (Alg. 4) once per item and user set;
// this keeps a complete index in one file so that a server can start from it.
//
// File layout (host byte order):
//   8 bytes  magic "RKMIPSIX"
//   Header   (version, sizes, scalars, the build parameters)
//   for each array of kArrays, in order: uint64 byte count, then the bytes
// The raw candidates of the lambda build (inspection only) are not kept.
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "index.h"
#include "internal.h"
#include "mem.h"
#include "query.h"

namespace rk {

namespace {

constexpr char kMagic[8] = {'R', 'K', 'M', 'I', 'P', 'S', 'I', 'X'};
constexpr uint32_t kVersion = 1;

struct Header {
    uint32_t version;
    int32_t d, ld, dtype, mma_dtype, mma_ld, t, C, G, nseg, device_unused;
    int64_t n, m, n_lam, nblocks, ns, seg_len, cert_failures;
    double err_fast, max_item_norm, max_user_norm, max_rel_err_raw, max_rel_err_l32;
    double ms_norms, ms_lambda, ms_refine, ms_saalsh, ms_cone, ms_total, ms_seed, ms_topk;
    rkmips_params prm;
};

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

Index* load_index(const char* path, hipStream_t s)
{
    File fl;
    fl.f = std::fopen(path, "rb");
    if (!fl.f) fail(RKMIPS_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    get(fl.f, magic, sizeof magic);
    if (std::memcmp(magic, kMagic, sizeof magic) != 0) fail(RKMIPS_EINVAL, "not an index file");
    Header h{};
    get(fl.f, &h, sizeof h);
    if (h.version != kVersion) fail(RKMIPS_EINVAL, "index file version " + std::to_string(h.version));
    if (h.n < 1 || h.m < 1 || h.d < 1 || h.d > 256 || h.ld < h.d || h.t < 1 || h.nblocks < 1 ||
        h.n_lam < 1 || h.n_lam > h.n || h.prm.k_max < 1 || h.prm.k_max > 256)
        fail(RKMIPS_EINVAL, "index file: inconsistent header");
    std::unique_ptr<Index> x(new Index());
    x->d = h.d; x->ld = h.ld; x->dtype = h.dtype; x->mma_dtype = h.mma_dtype; x->mma_ld = h.mma_ld;
    x->t = h.t; x->C = h.C; x->G = h.G; x->nseg = h.nseg;
    x->n = h.n; x->m = h.m; x->n_lam = h.n_lam; x->nblocks = h.nblocks; x->ns = h.ns; x->seg_len = h.seg_len;
    x->cert_failures = h.cert_failures;
    x->err_fast = h.err_fast; x->max_item_norm = h.max_item_norm; x->max_user_norm = h.max_user_norm;
    x->max_rel_err_raw = h.max_rel_err_raw; x->max_rel_err_l32 = h.max_rel_err_l32;
    x->ms_norms = h.ms_norms; x->ms_lambda = h.ms_lambda; x->ms_refine = h.ms_refine; x->ms_saalsh = h.ms_saalsh;
    x->ms_cone = h.ms_cone; x->ms_total = h.ms_total; x->ms_seed = h.ms_seed; x->ms_topk = h.ms_topk;
    x->prm = h.prm;
    HIPC(hipGetDevice(&x->device));
    hipDeviceProp_t prop;
    HIPC(hipGetDeviceProperties(&prop, x->device));
    x->num_cus = prop.multiProcessorCount;
    mem::StreamScope scope(s);
    std::vector<char> host;
    for (DevBuf* b : arrays(*x)) {
        uint64_t nb = 0;
        get(fl.f, &nb, sizeof nb);
        if (!nb) continue;
        if (nb > (uint64_t)1 << 40) fail(RKMIPS_EINVAL, "index file: inconsistent array size");
        host.resize(nb);
        get(fl.f, host.data(), nb);
        b->alloc(nb);
        HIPC(hipMemcpy(b->p, host.data(), nb, hipMemcpyHostToDevice));
    }
    // the arrays the query path reads must all be there
    if (!x->items.p || !x->users.p || !x->lam64.p || !x->lam32.p || !x->block_start.p || !x->part_start.p ||
        !x->item_codes.p || !x->user_codes.p || x->lam64.bytes != sizeof(double) * (size_t)x->prm.k_max * x->m)
        fail(RKMIPS_EINVAL, "index file: missing arrays");
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
