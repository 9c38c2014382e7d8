"""The C ABI library loads on a machine without a GPU, exports every entry point that
the headers under include/ declare, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        txt = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(rkmips_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def R():
    from paper_2211_12751_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    from paper_2211_12751_amd import rkmips
    return rkmips


def test_every_declared_symbol_is_exported(R):
    names = _declared()
    assert len(names) >= 17 and "rkmips_diag_mma_probe" in names
    for nm in names:
        assert hasattr(R._lib, nm), nm
        assert nm in R.EXPORTED, f"binding lacks {nm}"


def test_default_params(R):
    p = R.rkmips_default_params()
    assert (p.k_max, p.leaf_size, p.num_hash, p.topk_slack) == (50, 64, 128, 14)
    assert abs(p.b - 0.5) < 1e-7 and p.seed == 221112751
    # every field is set, whatever the struct held before (C callers may pass stack garbage)
    q = R.rkmips_params()
    C.memset(C.byref(q), 0x5A, C.sizeof(q))
    R._lib.rkmips_default_params(C.byref(q))
    assert (q.mode, q.flags, q.sah_items) == (R.MODE_EXACT, 0, 0)
    assert (q.k_max, q.leaf_size, q.num_hash, q.topk_slack) == (50, 64, 128, 14)


def test_argument_errors_before_device_work(R):
    p = R.rkmips_default_params()
    h = C.c_void_p()
    st = R._lib.rkmips_build_index(None, None, 10, None, None, 10, 8, 0, None, C.byref(p), None, C.byref(h))
    assert st == -1 and "NULL" in R.rkmips_last_error()
    dummy = C.c_void_p(16)
    for bad in (dict(n=0), dict(m=0), dict(d=0), dict(d=300), dict(dtype=7)):
        a = dict(n=10, m=10, d=8, dtype=0)
        a.update(bad)
        st = R._lib.rkmips_build_index(dummy, None, a["n"], dummy, None, a["m"], a["d"], a["dtype"], None,
                                       C.byref(p), None, C.byref(h))
        assert st == -1, bad
    for field, val in (("k_max", 0), ("k_max", 300), ("leaf_size", 65), ("num_hash", 48), ("b", 1.0),
                       ("probe_frac", 0.0), ("mode", 3), ("sah_items", -1)):
        q = R.rkmips_default_params()
        setattr(q, field, val)
        st = R._lib.rkmips_build_index(dummy, None, 10, dummy, None, 10, 8, 0, None, C.byref(q), None, C.byref(h))
        assert st == -1, field
    # SAH mode: P' must leave at least one item for the SA-ALSH index
    for n_prime in (10, 11):
        q = R.rkmips_default_params()
        q.mode, q.sah_items = R.MODE_SAH, n_prime
        st = R._lib.rkmips_build_index(dummy, None, 10, dummy, None, 10, 8, 0, None, C.byref(q), None, C.byref(h))
        assert st == -1 and "sah_items" in R.rkmips_last_error()
    # FP8 without scales, scales without FP8
    st = R._lib.rkmips_build_index(dummy, None, 10, dummy, None, 10, 8, 2, None, C.byref(p), None, C.byref(h))
    assert st == -1
    st = R._lib.rkmips_build_index(dummy, dummy, 10, dummy, None, 10, 8, 0, None, C.byref(p), None, C.byref(h))
    assert st == -1
    r = C.c_void_p()
    ks = np.ones(4, np.int32)
    st = R._lib.rkmips_query_batch(None, dummy, None, 4, ks.ctypes.data, 0, None, C.byref(r))
    assert st == -1
    assert R._lib.rkmips_result_wait(None) == -1
    assert R._lib.rkmips_result_view(None, None, None, None) == -1
    R._lib.rkmips_result_free(None)
    R._lib.rkmips_index_free(None)


def test_index_load_rejects_bad_files_before_device_work(R, tmp_path):
    h = C.c_void_p()
    st = R._lib.rkmips_index_load(str(tmp_path / "missing.idx").encode(), None, C.byref(h))
    assert st == -1 and "cannot open" in R.rkmips_last_error()
    bad = tmp_path / "bad.idx"
    bad.write_bytes(b"NOTANIDX" + b"\0" * 64)
    st = R._lib.rkmips_index_load(str(bad).encode(), None, C.byref(h))
    assert st == -1 and "not an index file" in R.rkmips_last_error()
    short = tmp_path / "short.idx"
    short.write_bytes(b"RKMIPSIX" + b"\1\0\0\0")
    st = R._lib.rkmips_index_load(str(short).encode(), None, C.byref(h))
    assert st == -1 and "truncated" in R.rkmips_last_error()
    st = R._lib.rkmips_index_save(None, str(bad).encode())
    assert st == -1


# ------------------------------------------------------------- index files, by hand
class _Header(C.Structure):
    """The index file header as the loader reads it (host byte order, natural alignment)."""
    _fields_ = ([("version", C.c_uint32)] + [(f, C.c_int32) for f in
                ("d", "ld", "dtype", "mma_dtype", "mma_ld", "t", "C", "G", "nseg", "device_unused")] +
                [(f, C.c_int64) for f in ("n", "m", "n_lam", "nblocks", "ns", "seg_len", "cert_failures")] +
                [(f, C.c_double) for f in ("err_fast", "max_item_norm", "max_user_norm", "max_rel_err_raw",
                                            "max_rel_err_l32", "ms_norms", "ms_lambda", "ms_refine", "ms_saalsh",
                                            "ms_cone", "ms_total", "ms_seed", "ms_topk")])


def _tiny_index(R, **edit):
    """Header and arrays of a consistent exact-mode FP32 index: n = 3 items, m = 2 users,
    d = 2 (rows padded to 32), one partition, one block, k_max = 1, K = 128."""
    class H(C.Structure):
        _fields_ = [("h", _Header), ("prm", R.rkmips_params)]
    x = H()
    p = R.rkmips_default_params()
    p.k_max = 1
    x.prm = p
    h = x.h
    h.version, h.d, h.ld, h.dtype, h.mma_dtype, h.mma_ld, h.t = 2, 2, 32, 0, 4, 64, 1
    h.n, h.m, h.n_lam, h.nblocks = 3, 2, 3, 1
    n, m, ld, W = 3, 2, 32, 4
    arr = [np.zeros(n * ld, np.float32), None, np.arange(n, dtype=np.uint32), np.ones(n),
           np.zeros(m * ld, np.float32), None, np.zeros(m * 2 * ld, np.uint16), np.arange(m, dtype=np.uint32),
           np.ones(m), np.ones(m, np.float32), np.ones(m, np.float32), np.zeros(m, np.float32),
           np.zeros(m, np.int32), np.array([0, m, 0], np.int64), np.zeros(ld, np.float32),
           np.zeros(1, np.float32), np.zeros(1, np.float32), np.ones(1, np.int32), np.zeros(1, np.float32),
           np.zeros(m), np.zeros(m, np.float32), np.array([0, n, 0, 0, 0], np.int64), np.ones(1, np.int32),
           np.zeros(ld, np.float32), np.zeros(1, np.float32), np.zeros(3 * 128, np.float32),
           np.zeros(n * W, np.uint32), np.zeros(m * W, np.uint32)]
    for k, v in edit.items():
        if k.startswith("prm_"):
            setattr(x.prm, k[4:], v)
        elif k.startswith("arr_"):
            arr[int(k[4:])] = v
        else:
            setattr(h, k, v)
    return x, arr


def _write(path, x, arr):
    with open(path, "wb") as f:
        f.write(b"RKMIPSIX")
        f.write(bytes(x))
        for a in arr:
            b = b"" if a is None else a.tobytes()
            f.write(np.uint64(len(b)).tobytes())
            f.write(b)


@pytest.mark.parametrize("edit, msg", [
    (dict(prm_num_hash=512), "num_hash"),
    (dict(prm_leaf_size=0), "leaf_size"),
    (dict(dtype=5), "unknown dtype"),
    (dict(mma_dtype=0), "operand form"),
    (dict(ld=64), "inconsistent sizes"),
    (dict(n_lam=2), "lambda item count"),
    (dict(t=4), "partition or block count"),
    (dict(arr_21=np.array([0, 3], np.int64)), "array 21"),             # short partition table
    (dict(arr_0=np.zeros(2 * 32, np.float32)), "array 0"),             # items of another n
    (dict(arr_1=np.ones(3, np.float32)), "array 1"),                   # scales without FP8
    (dict(arr_19=np.zeros(4)), "array 19"),                            # lambda of another k_max
    (dict(arr_2=np.array([0, 0, 2], np.uint32)), "item order"),
    (dict(arr_7=np.array([0, 5], np.uint32)), "user order"),
    (dict(arr_13=np.array([0, 1, 0], np.int64)), "block table"),
    (dict(arr_12=np.array([0, 1], np.int32)), "user block"),
    (dict(arr_21=np.array([0, 2, 0, 0, 0], np.int64)), "partitions do not cover"),
    (dict(arr_22=np.array([2], np.int32)), "partition count"),
])
def test_index_load_checks_every_array_before_device_work(R, tmp_path, edit, msg):
    x, arr = _tiny_index(R, **edit)
    f = tmp_path / "bad.idx"
    _write(f, x, arr)
    h = C.c_void_p()
    st = R._lib.rkmips_index_load(str(f).encode(), None, C.byref(h))
    assert st == -1 and msg in R.rkmips_last_error(), R.rkmips_last_error()


def test_index_load_passes_a_consistent_file_to_the_device(R, tmp_path):
    """The unedited tiny file passes every check; without a GPU the first device call
    then fails (EDEVICE), with one the index loads."""
    assert C.sizeof(_Header) + C.sizeof(R.rkmips_params) == 256
    x, arr = _tiny_index(R)
    f = tmp_path / "ok.idx"
    _write(f, x, arr)
    h = C.c_void_p()
    st = R._lib.rkmips_index_load(str(f).encode(), None, C.byref(h))
    assert st in (0, -3), R.rkmips_last_error()
    if st == 0:
        R._lib.rkmips_index_free(h)


def test_new_entry_points_check_arguments_first(R):
    dummy = C.c_void_p(16)
    r = C.c_void_p()
    ks = np.ones(4, np.int32)
    for fn in (R._lib.rkmips_query_batch, R._lib.rkmips_query_batch_hostk):
        assert fn(None, dummy, None, 4, ks.ctypes.data, 0, None, C.byref(r)) == -1
        assert fn(dummy, None, None, 4, ks.ctypes.data, 0, None, C.byref(r)) == -1
        assert fn(dummy, dummy, None, -1, ks.ctypes.data, 0, None, C.byref(r)) == -1
        assert fn(dummy, dummy, None, 4, None, 0, None, C.byref(r)) == -1
        assert fn(dummy, dummy, None, 4, ks.ctypes.data, 0, None, None) == -1
    assert R._lib.rkmips_index_wait(None) == -1
    assert R._lib.rkmips_get_stats(None, None) == -1


def test_mma_probe_rejects_bad_arguments(R):
    """The matrix-core probe validates on the host before any device call."""
    a = np.zeros((32, 24), np.uint8)
    with pytest.raises(R.RkmipsError) as e:
        R.rkmips_diag_mma_probe(0, a, a)          # K not a multiple of 16
    assert e.value.status == -1
    a = np.zeros((32, 16), np.uint8)
    with pytest.raises(R.RkmipsError):
        R.rkmips_diag_mma_probe(3, a, a)          # no such kind
    with pytest.raises(R.RkmipsError):
        R.rkmips_diag_mma_probe(2, a, a)          # 64-wide steps need K a multiple of 64
    a[0, 0] = 0x7f
    with pytest.raises(R.RkmipsError):
        R.rkmips_diag_mma_probe(1, a, a)          # NaN code


def test_fp8_decode_probe_rejects_bad_arguments(R):
    """The hardware-conversion probe validates on the host before any device call."""
    with pytest.raises(R.RkmipsError) as e:
        R.rkmips_diag_fp8_decode(np.zeros(6, np.uint8))      # n not a multiple of 4
    assert e.value.status == -1
    with pytest.raises(R.RkmipsError):
        R.rkmips_diag_fp8_decode(np.zeros(0, np.uint8))      # empty
    out = np.zeros(4, np.float32)
    assert R._lib.rkmips_diag_fp8_decode(None, 4, out.ctypes.data) == -1
