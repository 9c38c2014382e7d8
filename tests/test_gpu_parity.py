"""GPU parity of the HIP path against the CPU FP64 reference.

Every case states its inputs by seed and shape; sizes span several tiles and a ragged
tail.  lambda64 and result sets must be bit-exact; lambda32 must be RN32(lambda64)
(relative error <= 2^-24, well inside 1e-6).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_12751_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2211_12751_amd import rkmips
    return rkmips


def _lists_equal(a, b):
    assert len(a) == len(b)
    for i, (x, y) in enumerate(zip(a, b)):
        if not np.array_equal(np.asarray(x), np.asarray(y)):
            xs, ys = set(map(int, x)), set(map(int, y))
            raise AssertionError(f"query {i}: missing {sorted(ys - xs)[:10]} extra {sorted(xs - ys)[:10]}")


def _oracle_sets(w, ks, k_max, user_idx=None):
    lam = O.lambda_table(w.dtype, w.items, w.item_scales, w.users, w.user_scales, k_max, user_idx=user_idx)
    mem = O.member(w.dtype, w.users, w.user_scales, w.queries, w.query_scales, ks, lam, user_idx=user_idx)
    return lam, mem


def _build(R, w, k_max, **kw):
    print(f"\n[case] {w.name} n={w.n} m={w.m} d={w.d} dtype={w.dtype} k_max={k_max} {kw}", flush=True)
    return R.Index(w.items, w.item_scales, w.users, w.user_scales, dtype=w.dtype, k_max=k_max, **kw)


def _check_lambda(idx, lam, k_max):
    for k in range(1, k_max + 1):
        g64 = idx.lam(k)
        assert np.array_equal(g64, lam[k - 1]), f"lambda64 k={k}: {np.flatnonzero(g64 != lam[k - 1])[:10]}"
        g32 = idx.lam32(k)
        assert np.array_equal(g32, lam[k - 1].astype(np.float32))
        fin = np.isfinite(lam[k - 1]) & (lam[k - 1] != 0)
        assert (np.abs(g32[fin] - lam[k - 1][fin]) <= 1e-6 * np.abs(lam[k - 1][fin])).all()


def test_small_fp32_lambda_order_and_sets(R):
    w = I.make("c1", n=2000, m=5000, d=32, nq=100)
    k_max = 10
    ks = np.array([1, 10] * 50, np.int32)
    lam, mem = _oracle_sets(w, ks, k_max)
    idx = _build(R, w, k_max)
    try:
        n2, order = O.item_order("f32", w.items, None)
        go, gn2 = idx.item_order()
        assert np.array_equal(go, order) and np.array_equal(gn2, n2[order])
        _check_lambda(idx, lam, k_max)
        got, st = idx.query(w.queries, None, ks, stats=True)
        _lists_equal(got, [np.flatnonzero(r) for r in mem])
        print("stats", st, idx.info, flush=True)
    finally:
        idx.close()


def test_toggles_give_identical_sets(R):
    w = I.make("c1", n=1500, m=3000, d=32, nq=64, seed=7)
    k_max = 10
    ks = (np.arange(64) % 10 + 1).astype(np.int32)
    lam, mem = _oracle_sets(w, ks, k_max)
    ref = [np.flatnonzero(r) for r in mem]
    idx = _build(R, w, k_max)
    try:
        for fl in (0, R.FLAG_NO_BOUNDS, R.FLAG_FORCE_RECHECK, R.FLAG_NO_VECTOR_BOUND, R.FLAG_SAALSH_FILTER,
                   R.FLAG_SAALSH_FILTER | R.FLAG_FORCE_RECHECK, R.FLAG_POOL_LISTS,
                   R.FLAG_POOL_LISTS | R.FLAG_FORCE_RECHECK):
            print("flags", fl, flush=True)
            _lists_equal(idx.query(w.queries, None, ks, flags=fl), ref)
    finally:
        idx.close()
    # every lambda row from the full FP64 rescoring (certificates forced to fail)
    idx2 = _build(R, w, k_max, flags=R.FLAG_NO_CERT)
    try:
        assert idx2.info["cert_failures"] == w.m
        _check_lambda(idx2, lam, k_max)
        _lists_equal(idx2.query(w.queries, None, ks), ref)
    finally:
        idx2.close()
    # FP32 data scored on the FP32 matrix cores instead of split BF16 products
    idx4 = _build(R, w, k_max, flags=R.FLAG_F32_MATRIX)
    try:
        _check_lambda(idx4, lam, k_max)
        _lists_equal(idx4.query(w.queries, None, ks), ref)
    finally:
        idx4.close()
    # no slack: the certificate cannot hold, the fallback must give the same table
    idx3 = _build(R, w, k_max, topk_slack=0)
    try:
        _check_lambda(idx3, lam, k_max)
    finally:
        idx3.close()


@pytest.mark.parametrize("cfg, d, k_max", [("c2", 64, 120), ("c3", 100, 120), ("c5", 128, 100),
                                           ("c3", 64, 200), ("c5", 200, 210)])
def test_wide_refine_with_tied_scores(R, cfg, d, k_max):
    """C = k_max + slack above 64: the rescoring runs 64 candidates at a time and ranks up
    to 128 or 256 canonical scores with a sort across the wave.  Every item appears twice,
    so equal canonical scores occur throughout the lambda rows; the table must equal
    Definition 1's bit for bit."""
    w = I.make(cfg, n=380, m=900, d=d, nq=4, seed=k_max + d)
    items = np.concatenate([w.items, w.items[::-1]])
    isc = None if w.item_scales is None else np.concatenate([w.item_scales, w.item_scales[::-1]])
    print(f"\n[case] wide refine {cfg} dtype={w.dtype} n={len(items)} m={w.m} d={d} k_max={k_max}", flush=True)
    lam = O.lambda_table(w.dtype, items, isc, w.users, w.user_scales, k_max)
    idx = R.Index(items, isc, w.users, w.user_scales, dtype=w.dtype, k_max=k_max)
    try:
        assert idx.info["cert_failures"] < w.m   # the certified path ran
        _check_lambda(idx, lam, k_max)
    finally:
        idx.close()


@pytest.mark.parametrize("cfg, n, m, d, k_max", [("c5", 1 << 18, 2000, 32, 4), ("c3", 150_000, 1500, 32, 10),
                                                ("c2", 100_000, 1000, 16, 4), ("c2", 20_000, 300, 16, 2),
                                                ("c3", 30_000, 200, 64, 8), ("c5", 12_000, 100, 128, 1)])
def test_many_item_segments(R, cfg, n, m, d, k_max):
    """Few users and many items: the top-k pass splits the items into up to 16 segments to
    fill the GPU (small k gives small per-user buffers), and the refine must gather the
    candidates and thresholds of every segment.  (Reading only the first four once gave
    lambda values below Definition 1's, with the certificate passing.)"""
    w = I.make(cfg, n=n, m=m, d=d, nq=6, seed=n + k_max)
    ks = np.minimum(np.array([1, k_max, 2, k_max, 1, k_max], np.int32), k_max)
    lam, mem = _oracle_sets(w, ks, k_max)
    idx = _build(R, w, k_max)
    try:
        print("candidates per user", idx.info["cand_per_user"], "certificate failures", idx.info["cert_failures"],
              flush=True)
        assert idx.info["cert_failures"] < w.m   # the certified path ran
        _check_lambda(idx, lam, k_max)
        got = idx.query(w.queries, w.query_scales, ks)
        _lists_equal(got, [np.flatnonzero(mem[i]) for i in range(len(ks))])
    finally:
        idx.close()


@pytest.mark.parametrize("cfg, n, m, d, k_max, slack", [
    ("c5", 70_000, 300, 200, 3, 14),     # FP8 rows of 256 codes: the FP8 seed pass, many segments
    ("c5", 40_000, 500, 129, 60, 14),    # C = 74 > 64: the wide rescoring, two segments
    ("c3", 20_000, 700, 7, 1, 0),        # C = 1, no slack
    ("c3", 60_000, 90, 33, 17, 40),      # one user tile, the most segments
    ("c2", 9_000, 3000, 1, 5, 14),       # d = 1: scores are products of two numbers, many ties
    ("c2", 25_000, 1200, 64, 120, 14),   # C = 134 with the split FP32 operands
])
def test_config_sweep_lambda(R, cfg, n, m, d, k_max, slack):
    """Shapes across the top-k pass's structural thresholds (seed on or off, FP8 seed
    rows, candidate buffers of 128 to 1,024 entries, one to sixteen item segments, the
    narrow and wide rescoring): lambda64 and lambda32 equal Definition 1's."""
    w = I.make(cfg, n=n, m=m, d=d, nq=1, seed=7 * n + m + d)
    lam = O.lambda_table(w.dtype, w.items, w.item_scales, w.users, w.user_scales, k_max)
    idx = _build(R, w, k_max, topk_slack=slack)
    try:
        print("candidates per user", idx.info["cand_per_user"], "certificate failures", idx.info["cert_failures"],
              flush=True)
        _check_lambda(idx, lam, k_max)
    finally:
        idx.close()


@pytest.mark.parametrize("cfg, n, m, d, k_max, nq, flags", [
    ("c5", 3000, 5000, 256, 30, 1500, 0),    # FP8 rows of 256 codes, 30 distinct k (four launches)
    ("c3", 200, 100, 1, 5, 77, 0),           # fewer users than one workgroup's tile, d = 1
    ("c2", 5000, 4097, 64, 50, 33, 0),       # a ragged user tile, one k for every query
    ("c3", 4000, 2600, 128, 64, 300, 128),   # the pool list path
])
def test_query_sweep_sets(R, cfg, n, m, d, k_max, nq, flags):
    """Query batches across the verify pass's thresholds (user tiles, query tiles, k groups,
    the answer-bit and pool list paths): every list equals Definition 1's set."""
    w = I.make(cfg, n=n, m=m, d=d, nq=nq, seed=3 * n + m + nq)
    g = np.random.default_rng(nq + d)
    ks = (g.integers(0, k_max, nq) + 1).astype(np.int32) if nq != 33 else np.full(nq, k_max, np.int32)
    lam, mem = _oracle_sets(w, ks, k_max)
    idx = _build(R, w, k_max)
    try:
        got = idx.query(w.queries, w.query_scales, ks, flags=flags)
        _lists_equal(got, [np.flatnonzero(mem[i]) for i in range(nq)])
    finally:
        idx.close()


@pytest.mark.parametrize("n,m,d,k_max", [(7, 33, 20, 10), (1, 1, 1, 1), (300, 777, 64, 50), (129, 257, 100, 16)])
def test_ragged_and_degenerate_shapes(R, n, m, d, k_max):
    w = I.make("c2", n=n, m=m, d=d, nq=45, seed=n + m)
    ks = (np.arange(45) % k_max + 1).astype(np.int32)
    lam, mem = _oracle_sets(w, ks, k_max)
    idx = _build(R, w, k_max)
    try:
        _check_lambda(idx, lam, k_max)
        _lists_equal(idx.query(w.queries, None, ks), [np.flatnonzero(r) for r in mem])
    finally:
        idx.close()


def test_queries_equal_items_sum_identity(R):
    """Q = P: each user admits exactly k items, so the answer sizes sum to m*k."""
    w = I.make("c1", n=1000, m=2000, nq=1)
    idx = _build(R, w, 10)
    try:
        for k in (1, 5, 10):
            got = idx.query(w.items, None, np.full(w.n, k, np.int32))
            assert sum(len(g) for g in got) == w.m * k
    finally:
        idx.close()


def test_zero_and_duplicate_vectors(R):
    """Zero users (every item ties at 0: always in), a zero query, duplicated items."""
    w = I.make("c1", n=400, m=500, d=32, nq=40, seed=3)
    w.users[[0, 17, 499]] = 0
    w.items[5] = w.items[6]
    w.items[100:110] = w.items[100]
    w.queries[0] = 0
    w.queries[1] = w.items[100]
    ks = (np.arange(40) % 10 + 1).astype(np.int32)
    lam, mem = _oracle_sets(w, ks, 10)
    idx = _build(R, w, 10)
    try:
        _check_lambda(idx, lam, 10)
        _lists_equal(idx.query(w.queries, None, ks), [np.flatnonzero(r) for r in mem])
    finally:
        idx.close()


@pytest.mark.parametrize("n", [2049, 5000, 70001])
def test_item_order_merge_levels(R, n):
    """Item order past one sort chunk (2048): ragged runs, runs with no partner, equal
    norms (duplicated rows, ties by index) and zero rows (the largest key)."""
    w = I.make("c1", n=n, m=300, d=16, nq=1, seed=n)
    w.items[10:40] = w.items[9]
    w.items[n - 50:] = w.items[3]
    w.items[[0, 2048, n // 2]] = 0
    idx = _build(R, w, 5)
    try:
        n2, order = O.item_order("f32", w.items, None)
        go, gn2 = idx.item_order()
        assert np.array_equal(go, order) and np.array_equal(gn2, n2[order])
    finally:
        idx.close()


def test_mixed_k_more_than_eight_distinct(R):
    w = I.make("c1", n=500, m=900, nq=120, seed=11)
    k_max = 20
    ks = (np.arange(120) * 7 % k_max + 1).astype(np.int32)
    lam, mem = _oracle_sets(w, ks, k_max)
    idx = _build(R, w, k_max)
    try:
        _lists_equal(idx.query(w.queries, None, ks), [np.flatnonzero(r) for r in mem])
        _lists_equal(idx.query(w.queries[:0], None, ks[:0]), [])
    finally:
        idx.close()


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_low_precision_storage(R, dtype):
    w = I.make("c2", n=1200, m=2500, d=64, nq=80, dtype=dtype, seed=5)
    k_max = 20
    ks = (np.arange(80) % k_max + 1).astype(np.int32)
    lam, mem = _oracle_sets(w, ks, k_max)
    idx = _build(R, w, k_max)
    try:
        _check_lambda(idx, lam, k_max)
        _lists_equal(idx.query(w.queries, w.query_scales, ks), [np.flatnonzero(r) for r in mem])
        print("info", idx.info, flush=True)
    finally:
        idx.close()


def test_full_size_fp32_sampled(R):
    """The 20k x 100k x 64 FP32 workload, checked on a seeded sample of 1500 users for
    every query and k (lambda64 bit-exact, membership exact)."""
    w = I.make("c2")
    k_max = 50
    g = np.random.default_rng(2211)
    sample = np.sort(g.choice(w.m, 1500, replace=False))
    lam, mem = _oracle_sets(w, w.ks, k_max, user_idx=sample)
    idx = _build(R, w, k_max)
    try:
        for k in (1, 10, 50):
            assert np.array_equal(idx.lam(k)[sample], lam[k - 1])
        got, st = idx.query(w.queries, None, w.ks, stats=True)
        pos = {int(u): i for i, u in enumerate(sample)}
        for qi, lst in enumerate(got):
            mine = np.zeros(len(sample), np.uint8)
            for u in lst:
                j = pos.get(int(u))
                if j is not None:
                    mine[j] = 1
            assert np.array_equal(mine, mem[qi]), f"query {qi}"
        print("stats", st, idx.info, flush=True)
    finally:
        idx.close()
