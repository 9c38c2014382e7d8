"""The approximate SAH mode (Alg. 4 lower bounds from P', Alg. 5 decisions) on the GPU
against the CPU FP64 reference of the same method.

Every decision uses canonical FP64 scores, so the GPU sets equal the reference sets
when the sign-random-projection codes agree (GPU codes are signs of FP32 projections,
the reference's of FP64 ones; a bit can differ only where a projection is within
rounding of zero, which no fixed seed here has, and the tests assert the agreement).
Independently of the codes, each set must contain the exact Definition 1 set and lie inside the set that passes the
L_u^k test, and the lambda table must be the exact k_max-MIPS over P'.
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


def _f1(got, exact):
    tp = sum(len(np.intersect1d(a, b)) for a, b in zip(got, exact))
    ng, ne = sum(len(a) for a in got), sum(len(b) for b in exact)
    if ng == 0 and ne == 0:
        return 1.0
    return 2.0 * tp / (ng + ne)


CASES = [
    ("f32", 700, 900, 16, 30, 0.1, 0),
    ("bf16", 640, 1000, 32, 25, 0.15, 0),
    ("fp8", 600, 800, 48, 40, 0.1, 0),
    ("f32", 700, 900, 16, 0, 0.1, 0),                       # default |P'| = min(2 k_max, n - 1)
    ("f32", 700, 900, 16, 30, 0.1, 128),                    # pool lists instead of answer bits
]


@pytest.mark.parametrize("dtype, n, m, d, n_prime, beta, flags", CASES)
def test_sah_sets_match_reference(R, dtype, n, m, d, n_prime, beta, flags):
    w = I.make({"f32": "c2", "bf16": "c3", "fp8": "c5"}[dtype], n=n, m=m, d=d, nq=24, seed=51 + n_prime)
    k_max, K, b = 20, 64, 0.5
    ks = np.array([1, 5, 10, 20, 5, 1, 10, 20] * 3, np.int32)
    A = I.srp_matrix(w.d, K, seed=7)
    print(f"\n[case] sah dtype={dtype} n={n} m={m} d={d} n'={n_prime} beta={beta} flags={flags}", flush=True)
    idx = R.Index(w.items, w.item_scales, w.users, w.user_scales, dtype=dtype, k_max=k_max, num_hash=K, srp=A,
                  mode=R.MODE_SAH, sah_items=n_prime, b=b, probe_frac=beta)
    try:
        npr = n_prime or min(2 * k_max, n - 1)
        assert idx.info["mode"] == R.MODE_SAH and idx.info["lambda_items"] == npr
        got, st = idx.query(w.queries, w.query_scales, ks, flags=flags, stats=True)
        n2, order = O.item_order(dtype, w.items, w.item_scales)
        top = order[:npr]
        pps = None if w.item_scales is None else w.item_scales[top]
        lam_p = O.lambda_table(dtype, w.items[top], pps, w.users, w.user_scales, k_max)
        for k in (1, 7, k_max):
            assert np.array_equal(idx.lam(k), lam_p[k - 1]), f"lambda over P' k={k}"
        ps = O.partitions(n2, order, b, start=npr)
        _, _, icodes = O.saalsh_index(dtype, w.items, w.item_scales, order, ps, A)
        ucodes = O.user_codes(dtype, w.users, w.user_scales, A)
        gps, _, _, gic, guc = idx.saalsh()
        assert np.array_equal(gps, ps)
        inpart = np.zeros(n, bool)
        inpart[order[npr:]] = True
        # on these seeds no projection lies within rounding of zero, so the codes agree
        assert np.array_equal(icodes[inpart], gic[inpart]), "item SRP codes"
        assert np.array_equal(ucodes, guc), "user SRP codes"
        exact, _ = O.rkmips(dtype, w.items, w.item_scales, w.users, w.user_scales, w.queries, w.query_scales, ks,
                            k_max)
        surv = O.member(dtype, w.users, w.user_scales, w.queries, w.query_scales, ks, lam_p)
        for qi in range(len(ks)):
            g = set(np.asarray(got[qi]).tolist())
            assert set(exact[qi].tolist()) <= g, f"query {qi}: an exact answer is missing"
            assert g <= set(np.flatnonzero(surv[qi]).tolist()), f"query {qi}: an answer below L_u^k"
        ost = {}
        ref = O.sah_rkmips(dtype, w.items, w.item_scales, w.users, w.user_scales, w.queries, w.query_scales,
                           ks, k_max, npr, b, beta, A, stats=ost)
        for qi in range(len(ks)):
            assert np.array_equal(np.asarray(got[qi]), ref[qi]), f"query {qi}"
        print(f"F1 vs exact {_f1(got, exact):.4f} stats {st} oracle alg2 {ost['alg2']}", flush=True)
        assert st["saalsh_checked"] == ost["alg2"] > 0
    finally:
        idx.close()


def test_sah_full_probe_is_exact(R):
    """beta = 1: Alg. 2 scores every item of P minus P', so the sets are exact."""
    w = I.make("c2", n=500, m=600, d=16, nq=12, seed=61)
    ks = np.array([1, 5, 10, 20] * 3, np.int32)
    print("\n[case] sah beta=1", flush=True)
    idx = R.Index(w.items, None, w.users, None, dtype="f32", k_max=20, num_hash=64, mode=R.MODE_SAH,
                  sah_items=25, probe_frac=1.0)
    try:
        got = idx.query(w.queries, None, ks)
        exact, _ = O.rkmips("f32", w.items, None, w.users, None, w.queries, None, ks, 20)
        for a, b in zip(got, exact):
            assert np.array_equal(np.asarray(a), b)
    finally:
        idx.close()


def test_sah_rejects_bad_sizes(R):
    w = I.make("c2", n=50, m=60, d=8, nq=2, seed=62)
    print("\n[case] sah bad sizes", flush=True)
    for kw in (dict(sah_items=50), dict(sah_items=-1), dict(mode=3)):
        args = dict(mode=R.MODE_SAH)
        args.update(kw)
        with pytest.raises(R.RkmipsError) as e:
            R.Index(w.items, None, w.users, None, dtype="f32", k_max=10, **args)
        assert e.value.status == -1


@pytest.mark.parametrize("dtype, n, m, d, n_prime, flags", [
    ("f32", 700, 900, 16, 30, 0), ("bf16", 640, 1000, 32, 0, 0), ("fp8", 600, 800, 48, 40, 0),
    ("f32", 700, 900, 16, 30, 128),
])
def test_lazy_mode_is_exact(R, dtype, n, m, d, n_prime, flags):
    """The lazy mode builds only L_u over P' and decides the rest with Alg. 2 scoring every
    item of each visited partition: its sets are the Definition 1 sets."""
    w = I.make({"f32": "c2", "bf16": "c3", "fp8": "c5"}[dtype], n=n, m=m, d=d, nq=24, seed=71 + n_prime)
    ks = np.array([1, 5, 10, 20, 5, 1, 10, 20] * 3, np.int32)
    print(f"\n[case] lazy dtype={dtype} n={n} m={m} d={d} n'={n_prime} flags={flags}", flush=True)
    idx = R.Index(w.items, w.item_scales, w.users, w.user_scales, dtype=dtype, k_max=20, num_hash=64,
                  mode=R.MODE_LAZY, sah_items=n_prime, b=0.5, probe_frac=0.1)
    try:
        assert idx.info["mode"] == R.MODE_LAZY
        got, st = idx.query(w.queries, w.query_scales, ks, flags=flags, stats=True)
        exact, _ = O.rkmips(dtype, w.items, w.item_scales, w.users, w.user_scales, w.queries, w.query_scales, ks, 20)
        for qi in range(len(ks)):
            assert np.array_equal(np.asarray(got[qi]), exact[qi]), f"query {qi}"
        print(f"stats {st}", flush=True)
        assert st["saalsh_checked"] > 0
    finally:
        idx.close()


def test_lazy_mode_near_ties_with_the_norm_test(R):
    """Users that are power-of-two multiples of the largest-norm items, and queries equal to
    those items or one ulp away from them: s(u,q) sits at or next to ||u|| ||p_k||, where the
    lazy mode's norm test (Alg. 5) must not answer yes on rounding alone.  The sets must
    still be the Definition 1 sets."""
    g = np.random.default_rng(515)
    n, d = 300, 16
    P = g.standard_normal((n, d)).astype(np.float32)
    P *= np.exp(0.4 * g.standard_normal(n)).astype(np.float32)[:, None]
    top = np.argsort(-np.einsum("ij,ij->i", P.astype(np.float64), P.astype(np.float64)), kind="stable")[:6]
    users = [P[top[j]] * np.float32(2.0 ** e) for j in range(6) for e in (-3, -1, 0, 2)]
    users = np.concatenate([np.stack(users), g.standard_normal((200, d)).astype(np.float32)])
    qs = []
    for j in range(6):
        base = P[top[j]]
        qs.append(base.copy())
        for sgn in (1.0, -1.0):
            q = base.copy()
            i = int(np.argmax(np.abs(q)))
            q[i] = np.nextafter(q[i], np.float32(sgn * np.inf))
            qs.append(q)
    Q = np.stack(qs).astype(np.float32)
    ks = np.array([1, 2, 3, 5, 1, 2] * 3, np.int32)[:len(Q)]
    print("\n[case] lazy near ties with the norm test", flush=True)
    exact, _ = O.rkmips("f32", P, None, users, None, Q, None, ks, 5)
    idx = R.Index(P, None, users, None, dtype="f32", k_max=5, num_hash=64, mode=R.MODE_LAZY,
                  sah_items=3, b=0.5, probe_frac=0.1)
    try:
        got, st = idx.query(Q, None, ks, stats=True)
        for qi in range(len(ks)):
            assert np.array_equal(np.asarray(got[qi]), exact[qi]), f"query {qi}"
        print(f"stats {st}", flush=True)
        assert st["saalsh_checked"] > 0
    finally:
        idx.close()


def test_sah_small_p_prime_empty_batch_and_serving(R):
    """|P'| = 5 < k for most queries (L_u^k = -inf there, so every user reaches the norm
    test and Alg. 2 starts with phi = -inf), an empty batch, and the continuous-batching
    server on an SAH index, all against the reference."""
    w = I.make("c2", n=400, m=700, d=16, nq=20, seed=63)
    ks = np.array([1, 5, 10, 20] * 5, np.int32)
    A = I.srp_matrix(w.d, 64, seed=13)
    print("\n[case] sah n'=5, empty batch, serving", flush=True)
    idx = R.Index(w.items, None, w.users, None, dtype="f32", k_max=20, num_hash=64, srp=A, mode=R.MODE_SAH,
                  sah_items=5, probe_frac=0.1)
    try:
        assert idx.query(w.queries[:0], None, np.zeros(0, np.int32)) == []
        got = idx.query(w.queries, None, ks)
        n2, order = O.item_order("f32", w.items, None)
        ps = O.partitions(n2, order, 0.5, start=5)
        _, _, icodes = O.saalsh_index("f32", w.items, None, order, ps, A)
        gic, guc = idx.saalsh()[3], idx.saalsh()[4]
        inpart = np.zeros(w.n, bool)
        inpart[order[5:]] = True
        assert np.array_equal(icodes[inpart], gic[inpart]), "item SRP codes"
        assert np.array_equal(O.user_codes("f32", w.users, None, A), guc), "user SRP codes"
        ref = O.sah_rkmips("f32", w.items, None, w.users, None, w.queries, None, ks, 20, 5, 0.5, 0.1, A)
        for qi in range(len(ks)):
            assert np.array_equal(np.asarray(got[qi]), ref[qi]), f"query {qi}"
        arr = np.arange(len(ks), dtype=np.int64) * 50
        served, lat, st = idx.serve(w.queries, None, ks, arr, max_batch=8, num_streams=2)
        for qi in range(len(ks)):
            assert np.array_equal(np.asarray(served[qi]), np.asarray(got[qi])), f"served query {qi}"
    finally:
        idx.close()
