"""ctypes binding of librkmips.so (include/rkmips.h), argument marshalling only.

Every computation runs in the HIP library; PyTorch only provides device memory
(tensor.data_ptr()) and streams.  torch is imported before the library is loaded so
that both share one HIP runtime.  If the library is not built this module raises at
import time: there is no fallback path.

The functions keep the C names (``rkmips_build_index`` ...).  ``Index`` is a small
owner object over the same calls for convenience.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (must precede the library: one HIP runtime per process)

_HERE = os.path.dirname(os.path.abspath(__file__))
# RKMIPS_LIB selects another build of the same library (the sanitized host build)
LIB_PATH = os.environ.get("RKMIPS_LIB") or os.path.join(_HERE, "lib", "librkmips.so")

F32, BF16, FP8_E4M3 = 0, 1, 2
DTYPES = {"f32": F32, "bf16": BF16, "fp8": FP8_E4M3}
FLAG_NO_BOUNDS, FLAG_FORCE_RECHECK, FLAG_NO_SAALSH, FLAG_NO_CERT, FLAG_NO_VECTOR_BOUND = 1, 2, 4, 8, 16
FLAG_SAALSH_FILTER = 32
FLAG_F32_MATRIX = 64
FLAG_POOL_LISTS = 128
FLAG_VERIFY_SIMPLE = 256
MODE_EXACT, MODE_SAH, MODE_LAZY = 0, 1, 2
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ERANGE", -5: "EBUSY"}


class RkmipsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class rkmips_params(C.Structure):
    _fields_ = [("k_max", C.c_int32), ("leaf_size", C.c_int32), ("num_hash", C.c_int32),
                ("topk_slack", C.c_int32), ("b", C.c_float), ("probe_frac", C.c_float),
                ("seed", C.c_uint64), ("mode", C.c_int32), ("flags", C.c_int32),
                ("sah_items", C.c_int32)]


class rkmips_query_stats(C.Structure):
    _fields_ = [("pairs_total", C.c_int64), ("pairs_block_pruned", C.c_int64),
                ("pairs_vector_pruned", C.c_int64), ("pairs_scored", C.c_int64),
                ("pairs_rechecked", C.c_int64), ("saalsh_checked", C.c_int64),
                ("saalsh_rejects", C.c_int64), ("results", C.c_int64), ("ms_total", C.c_double)]


class rkmips_index_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("d", C.c_int32), ("dtype", C.c_int32),
                ("k_max", C.c_int32), ("cand_per_user", C.c_int32), ("num_hash", C.c_int32),
                ("leaf_size", C.c_int32), ("num_partitions", C.c_int32), ("num_blocks", C.c_int64),
                ("cert_failures", C.c_int64), ("max_rel_err_raw", C.c_double),
                ("max_rel_err_lambda32", C.c_double), ("ms_norms", C.c_double),
                ("ms_lambda", C.c_double), ("ms_refine", C.c_double), ("ms_saalsh", C.c_double),
                ("ms_cone", C.c_double), ("ms_total", C.c_double), ("device_bytes", C.c_int64),
                ("ms_seed", C.c_double), ("ms_topk", C.c_double), ("mma_dtype", C.c_int32),
                ("mma_terms", C.c_int32), ("err_fast", C.c_double), ("mode", C.c_int32),
                ("lambda_items", C.c_int32)]


class rkmips_stats(C.Structure):
    _fields_ = [("max_rel_err_raw", C.c_double), ("max_rel_err_lambda32", C.c_double),
                ("cert_failures", C.c_int64), ("fallback_rate", C.c_double), ("batches", C.c_int64),
                ("queries", C.c_int64), ("query", rkmips_query_stats), ("recheck_rate", C.c_double)]


class rkmips_serve_params(C.Structure):
    _fields_ = [("max_batch", C.c_int32), ("num_streams", C.c_int32), ("mem_budget", C.c_int64),
                ("flags", C.c_int32)]


class rkmips_serve_stats(C.Structure):
    _fields_ = [("batches", C.c_int64), ("max_inflight", C.c_int64), ("slots", C.c_int32),
                ("wall_ms", C.c_double), ("p50_us", C.c_double), ("p99_us", C.c_double),
                ("mean_us", C.c_double)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc, gfx950)")
_lib = C.CDLL(LIB_PATH)
_P = C.c_void_p
_sig = {
    "rkmips_default_params": (None, [C.POINTER(rkmips_params)]),
    "rkmips_build_index": (C.c_int, [_P, _P, C.c_int64, _P, _P, C.c_int64, C.c_int32, C.c_int32, _P,
                                     C.POINTER(rkmips_params), _P, C.POINTER(_P)]),
    "rkmips_query_batch": (C.c_int, [_P, _P, _P, C.c_int64, _P, C.c_int32, _P, C.POINTER(_P)]),
    "rkmips_query_batch_hostk": (C.c_int, [_P, _P, _P, C.c_int64, _P, C.c_int32, _P, C.POINTER(_P)]),
    "rkmips_index_wait": (C.c_int, [_P]),
    "rkmips_get_stats": (C.c_int, [_P, C.POINTER(rkmips_stats)]),
    "rkmips_result_wait": (C.c_int, [_P]),
    "rkmips_result_view": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(_P), C.POINTER(_P)]),
    "rkmips_result_stats": (C.c_int, [_P, C.POINTER(rkmips_query_stats)]),
    "rkmips_result_free": (None, [_P]),
    "rkmips_get_info": (C.c_int, [_P, C.POINTER(rkmips_index_info)]),
    "rkmips_get_lambda": (C.c_int, [_P, C.c_int32, _P]),
    "rkmips_get_lambda32": (C.c_int, [_P, C.c_int32, _P]),
    "rkmips_get_item_order": (C.c_int, [_P, _P, _P]),
    "rkmips_get_candidates": (C.c_int, [_P, _P, _P, _P]),
    "rkmips_get_saalsh": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "rkmips_get_blocks": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "rkmips_saalsh_probe": (C.c_int, [_P, _P, _P, C.c_int64, _P, _P, _P, C.c_int64, C.c_float, _P, _P, _P]),
    "rkmips_saalsh_probe_noalloc": (C.c_int, [_P, _P, _P, C.c_int64, _P, _P, _P, C.c_int64, C.c_float, _P, _P, _P]),
    "rkmips_index_free": (None, [_P]),
    "rkmips_saalsh_kmips": (C.c_int, [_P, _P, C.c_int64, C.c_int32, C.c_float, _P, _P]),
    "rkmips_insert_items": (C.c_int, [_P, _P, _P, C.c_int64, _P]),
    "rkmips_index_save": (C.c_int, [_P, C.c_char_p]),
    "rkmips_index_load": (C.c_int, [C.c_char_p, _P, C.POINTER(_P)]),
    "rkmips_last_error": (C.c_char_p, []),
    "rkmips_diag_mma_probe": (C.c_int, [C.c_int32, _P, _P, C.c_int32, _P]),
    "rkmips_diag_fp8_decode": (C.c_int, [_P, C.c_int32, _P]),
    "rkmips_serve_replay": (C.c_int, [_P, _P, _P, C.c_int64, _P, _P, C.POINTER(rkmips_serve_params), _P,
                                      C.POINTER(rkmips_serve_stats), C.POINTER(_P)]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
EXPORTED = tuple(_sig)


def _check(st):
    if st != 0:
        raise RkmipsError(st, _lib.rkmips_last_error().decode())


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return _P(x.data_ptr())
    if isinstance(x, np.ndarray):
        return _P(x.ctypes.data)
    return _P(int(x))


def _stream(s):
    if s is None:
        return _P(torch.cuda.current_stream().cuda_stream)
    if isinstance(s, torch.cuda.Stream):
        return _P(s.cuda_stream)
    return _P(int(s))


# ------------------------------------------------------------------ C names
def rkmips_default_params():
    p = rkmips_params()
    _lib.rkmips_default_params(C.byref(p))
    return p


def rkmips_build_index(items, item_scales, n, users, user_scales, m, d, dtype, srp_proj, params, stream=None):
    h = _P()
    _check(_lib.rkmips_build_index(_ptr(items), _ptr(item_scales), n, _ptr(users), _ptr(user_scales), m, d,
                                   dtype, _ptr(srp_proj), C.byref(params) if params is not None else None,
                                   _stream(stream), C.byref(h)))
    return h


def rkmips_query_batch(idx, queries, query_scales, nq, ks, flags=0, stream=None):
    """ks: a device int32 tensor (the C call of this name), or host values (passed on to
    rkmips_query_batch_hostk)."""
    if not (isinstance(ks, torch.Tensor) and ks.is_cuda):
        return rkmips_query_batch_hostk(idx, queries, query_scales, nq, ks, flags, stream)
    if ks.dtype != torch.int32 or not ks.is_contiguous():
        raise ValueError("device ks must be a contiguous int32 tensor")
    h = _P()
    _check(_lib.rkmips_query_batch(idx, _ptr(queries), _ptr(query_scales), nq, _ptr(ks), flags,
                                   _stream(stream), C.byref(h)))
    return h


def rkmips_query_batch_hostk(idx, queries, query_scales, nq, ks, flags=0, stream=None):
    ks = np.ascontiguousarray(ks, dtype=np.int32)
    h = _P()
    _check(_lib.rkmips_query_batch_hostk(idx, _ptr(queries), _ptr(query_scales), nq, _ptr(ks), flags,
                                         _stream(stream), C.byref(h)))
    return h


def rkmips_index_wait(idx):
    _check(_lib.rkmips_index_wait(idx))


def rkmips_get_stats(idx):
    st = rkmips_stats()
    _check(_lib.rkmips_get_stats(idx, C.byref(st)))
    out = {f: getattr(st, f) for f, _ in rkmips_stats._fields_ if f != "query"}
    out["query"] = {f: getattr(st.query, f) for f, _ in rkmips_query_stats._fields_}
    return out


def rkmips_result_wait(r):
    _check(_lib.rkmips_result_wait(r))


def rkmips_result_view(r):
    """(offsets int64 [nq+1], ids int32 [total]) copied out of the result."""
    nq = C.c_int64()
    po, pi = _P(), _P()
    _check(_lib.rkmips_result_view(r, C.byref(nq), C.byref(po), C.byref(pi)))
    off = np.ctypeslib.as_array(C.cast(po, C.POINTER(C.c_int64)), shape=(nq.value + 1,)).copy()
    tot = int(off[-1])
    ids = (np.ctypeslib.as_array(C.cast(pi, C.POINTER(C.c_int32)), shape=(tot,)).copy()
           if tot else np.zeros(0, np.int32))
    return off, ids


def rkmips_result_stats(r):
    s = rkmips_query_stats()
    _check(_lib.rkmips_result_stats(r, C.byref(s)))
    return {f: getattr(s, f) for f, _ in rkmips_query_stats._fields_}


def rkmips_result_free(r):
    _lib.rkmips_result_free(r)


def rkmips_get_info(idx):
    s = rkmips_index_info()
    _check(_lib.rkmips_get_info(idx, C.byref(s)))
    return {f: getattr(s, f) for f, _ in rkmips_index_info._fields_}


def rkmips_get_lambda(idx, k, m):
    out = np.empty(m, np.float64)
    _check(_lib.rkmips_get_lambda(idx, k, _ptr(out)))
    return out


def rkmips_get_lambda32(idx, k, m):
    out = np.empty(m, np.float32)
    _check(_lib.rkmips_get_lambda32(idx, k, _ptr(out)))
    return out


def rkmips_get_item_order(idx, n):
    o = np.empty(n, np.int64)
    n2 = np.empty(n, np.float64)
    _check(_lib.rkmips_get_item_order(idx, _ptr(o), _ptr(n2)))
    return o, n2


def rkmips_get_candidates(idx, m, per_user):
    ids = np.empty((m, per_user), np.int32)
    sc = np.empty((m, per_user), np.float32)
    tau = np.empty(m, np.float32)
    _check(_lib.rkmips_get_candidates(idx, _ptr(ids), _ptr(sc), _ptr(tau)))
    return ids, sc, tau


def rkmips_get_saalsh(idx, n, m, d, t, K):
    ps = np.empty(t + 1, np.int64)
    cen = np.empty((t, d), np.float32)
    rad = np.empty(t, np.float32)
    ic = np.empty((n, K // 32), np.uint32)
    uc = np.empty((m, K // 32), np.uint32)
    _check(_lib.rkmips_get_saalsh(idx, _ptr(ps), _ptr(cen), _ptr(rad), _ptr(ic), _ptr(uc)))
    return ps, cen, rad, ic, uc


def rkmips_get_blocks(idx, m, d, nblocks, k_max):
    out = dict(leaf_users=np.empty(m, np.int32), block_start=np.empty(nblocks + 1, np.int64),
               center=np.empty((nblocks, d), np.float32), cos_omega=np.empty(nblocks, np.float32),
               sin_omega=np.empty(nblocks, np.float32), cos_theta=np.empty(m, np.float32),
               sin_theta=np.empty(m, np.float32), block_lb=np.empty((k_max, nblocks), np.float32))
    _check(_lib.rkmips_get_blocks(idx, *[_ptr(out[k]) for k in ("leaf_users", "block_start", "center",
                                                                  "cos_omega", "sin_omega", "cos_theta",
                                                                  "sin_theta", "block_lb")]))
    return out


def rkmips_saalsh_probe(idx, queries, query_scales, nq, ks, pair_query, pair_user, probe_frac, stream=None):
    ks = np.ascontiguousarray(ks, dtype=np.int32)
    pq = np.ascontiguousarray(pair_query, dtype=np.int64)
    pu = np.ascontiguousarray(pair_user, dtype=np.int64)
    phi = np.empty(len(pq), np.float64)
    ans = np.empty(len(pq), np.int32)
    _check(_lib.rkmips_saalsh_probe(idx, _ptr(queries), _ptr(query_scales), nq, _ptr(ks), _ptr(pq), _ptr(pu),
                                    len(pq), probe_frac, _stream(stream), _ptr(phi), _ptr(ans)))
    return phi, ans


def rkmips_saalsh_probe_noalloc(idx, queries, query_scales, nq, ks, pair_query, pair_user, probe_frac,
                                stream=None):
    ks = np.ascontiguousarray(ks, dtype=np.int32)
    pq = np.ascontiguousarray(pair_query, dtype=np.int64)
    pu = np.ascontiguousarray(pair_user, dtype=np.int64)
    phi = np.empty(len(pq), np.float64)
    ans = np.empty(len(pq), np.int32)
    _check(_lib.rkmips_saalsh_probe_noalloc(idx, _ptr(queries), _ptr(query_scales), nq, _ptr(ks), _ptr(pq),
                                            _ptr(pu), len(pq), probe_frac, _stream(stream), _ptr(phi), _ptr(ans)))
    return phi, ans


def rkmips_index_free(idx):
    _lib.rkmips_index_free(idx)


def rkmips_saalsh_kmips(idx, users, k, probe_frac, stream=None):
    users = np.ascontiguousarray(users, dtype=np.int64)
    out = np.empty((len(users), k), np.float64)
    _check(_lib.rkmips_saalsh_kmips(idx, _ptr(users), len(users), k, probe_frac, _stream(stream), _ptr(out)))
    return out


def rkmips_insert_items(idx, items, item_scales, n_new, stream=None):
    _check(_lib.rkmips_insert_items(idx, _ptr(items), _ptr(item_scales), n_new, _stream(stream)))


def rkmips_index_save(idx, path):
    _check(_lib.rkmips_index_save(idx, os.fsencode(path)))


def rkmips_index_load(path, stream=None):
    h = _P()
    _check(_lib.rkmips_index_load(os.fsencode(path), _stream(stream), C.byref(h)))
    return h


def rkmips_last_error():
    return _lib.rkmips_last_error().decode()


def rkmips_diag_mma_probe(kind, a_codes, b_codes):
    """One 32 x 32 block of e4m3 code products on the matrix cores (kind 0: codes widened
    to BF16; kind 1: FP8, 16-wide k steps; kind 2: FP8, 64-wide k steps, unit scales), FP32
    accumulation: float32 [32 x 32]."""
    a = np.ascontiguousarray(a_codes, dtype=np.uint8)
    b = np.ascontiguousarray(b_codes, dtype=np.uint8)
    if a.shape != b.shape or a.ndim != 2 or a.shape[0] != 32:
        raise ValueError("a_codes and b_codes must both be [32 x K]")
    out = np.empty((32, 32), np.float32)
    _check(_lib.rkmips_diag_mma_probe(int(kind), _ptr(a), _ptr(b), int(a.shape[1]), _ptr(out)))
    return out


def rkmips_diag_fp8_decode(codes):
    """e4m3 codes decoded by the hardware conversion instruction: float32 [n]."""
    c = np.ascontiguousarray(codes, dtype=np.uint8).ravel()
    out = np.empty(c.shape[0], np.float32)
    _check(_lib.rkmips_diag_fp8_decode(_ptr(c), int(c.shape[0]), _ptr(out)))
    return out


def rkmips_serve_replay(idx, queries_host, query_scales_host, nq, ks, arrival_us, sp):
    ks = np.ascontiguousarray(ks, dtype=np.int32)
    arr = np.ascontiguousarray(arrival_us, dtype=np.int64)
    lat = np.empty(nq, np.float64)
    st = rkmips_serve_stats()
    h = _P()
    _check(_lib.rkmips_serve_replay(idx, _ptr(queries_host), _ptr(query_scales_host), nq, _ptr(ks), _ptr(arr),
                                    C.byref(sp), _ptr(lat), C.byref(st), C.byref(h)))
    return h, lat, {f: getattr(st, f) for f, _ in rkmips_serve_stats._fields_}


# ------------------------------------------------------------------ owner object
def to_device(a, device="cuda"):
    """numpy storage array -> contiguous device tensor with the same bytes."""
    if a is None:
        return None
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a.view(np.int16) if a.dtype == np.uint16 else a)
    return t.to(device)


class Index:
    """Owns one rkmips_index built from numpy storage arrays (copied to the GPU)."""

    def __init__(self, items, item_scales, users, user_scales, dtype="f32", params=None, srp=None,
                 stream=None, **kw):
        p = params or rkmips_default_params()
        for k, v in kw.items():
            setattr(p, k, v)
        self.params = p
        self.dtype = DTYPES[dtype] if isinstance(dtype, str) else dtype
        self.n, self.d = items.shape
        self.m = users.shape[0]
        ti, tis = to_device(items), to_device(item_scales)
        tu, tus = to_device(users), to_device(user_scales)
        ts = to_device(srp) if srp is not None else None
        self.h = rkmips_build_index(ti, tis, self.n, tu, tus, self.m, self.d, self.dtype, ts, p, stream)
        torch.cuda.synchronize()
        self.info = rkmips_get_info(self.h)

    def query(self, queries, query_scales, ks, flags=0, stream=None, stats=False):
        """Per-query ascending original user IDs; queries: numpy storage array or device tensor."""
        q = queries if isinstance(queries, torch.Tensor) else to_device(queries)
        qs = query_scales if (query_scales is None or isinstance(query_scales, torch.Tensor)) else to_device(query_scales)
        nq = int(q.shape[0])
        dks = ks if isinstance(ks, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(ks, np.int32)).cuda()
        r = rkmips_query_batch(self.h, q, qs, nq, dks, flags, stream)
        try:
            rkmips_result_wait(r)
            off, ids = rkmips_result_view(r)
            st = rkmips_result_stats(r)
        finally:
            rkmips_result_free(r)
        lists = [ids[off[i]:off[i + 1]] for i in range(nq)]
        return (lists, st) if stats else lists

    def lam(self, k):
        return rkmips_get_lambda(self.h, k, self.m)

    def lam32(self, k):
        return rkmips_get_lambda32(self.h, k, self.m)

    def item_order(self):
        return rkmips_get_item_order(self.h, self.n)

    def candidates(self):
        return rkmips_get_candidates(self.h, self.m, self.info["cand_per_user"])

    def saalsh(self):
        return rkmips_get_saalsh(self.h, self.n, self.m, self.d, self.info["num_partitions"], self.params.num_hash)

    def blocks(self):
        return rkmips_get_blocks(self.h, self.m, self.d, self.info["num_blocks"], self.params.k_max)

    def serve(self, queries, query_scales, ks, arrival_us, max_batch=256, num_streams=4, mem_budget=0, flags=0):
        """Replay a timed request stream through the continuous-batching server.
        queries: host numpy storage array.  Returns (answers, latency_us, stats)."""
        q = np.ascontiguousarray(queries)
        q = q.view(np.int16) if q.dtype == np.uint16 else q
        qs = None if query_scales is None else np.ascontiguousarray(query_scales, dtype=np.float32)
        sp = rkmips_serve_params(max_batch, num_streams, mem_budget, flags)
        nq = int(q.shape[0])
        h, lat, st = rkmips_serve_replay(self.h, q, qs, nq, ks, arrival_us, sp)
        try:
            off, ids = rkmips_result_view(h)
        finally:
            rkmips_result_free(h)
        return [ids[off[i]:off[i + 1]] for i in range(nq)], lat, st

    def kmips(self, users, k, probe_frac, stream=None):
        """SA-ALSH kMIPS scores [len(users) x k] (descending, -inf padded)."""
        return rkmips_saalsh_kmips(self.h, users, k, probe_frac, stream)

    def insert(self, items, item_scales=None, stream=None):
        """Add items (numpy storage arrays or device tensors); they get the next ids."""
        ti = items if isinstance(items, torch.Tensor) else to_device(items)
        ts = item_scales if (item_scales is None or isinstance(item_scales, torch.Tensor)) else to_device(item_scales)
        rkmips_insert_items(self.h, ti, ts, int(ti.shape[0]), stream)
        self.info = rkmips_get_info(self.h)
        self.n = int(self.info["n"])

    def save(self, path):
        rkmips_index_save(self.h, path)

    @classmethod
    def load(cls, path, stream=None):
        """An Index object around an index read from a file written by save()."""
        self = cls.__new__(cls)
        self.h = rkmips_index_load(path, stream)
        self.info = rkmips_get_info(self.h)
        self.params = rkmips_default_params()
        self.params.k_max, self.params.num_hash = self.info["k_max"], self.info["num_hash"]
        self.params.leaf_size, self.params.mode = self.info["leaf_size"], self.info["mode"]
        self.dtype = int(self.info["dtype"])
        self.n, self.m, self.d = int(self.info["n"]), int(self.info["m"]), int(self.info["d"])
        return self

    def close(self):
        if getattr(self, "h", None):
            rkmips_index_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
