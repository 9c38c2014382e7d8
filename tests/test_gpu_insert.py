"""Item insertion: an index built on P and then given the items P_new equals an index
built on [P; P_new] with the same parameters and projections (lambda rows bit for bit,
item order, SA-ALSH data, blocks), and its answer sets are the Definition 1 sets."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_12751_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype, n0, n_new", [("f32", 400, 37), ("bf16", 300, 1), ("fp8", 500, 64), ("f32", 5, 60)])
def test_insert_equals_fresh_build(dtype, n0, n_new):
    from paper_2211_12751_amd import rkmips as R
    w = I.make({"f32": "c2", "bf16": "c3", "fp8": "c5"}[dtype], n=n0 + n_new, m=900, d=24, nq=30, seed=101 + n0)
    K, k_max = 64, 10
    A = I.srp_matrix(w.d, K, seed=11)
    sc = w.item_scales
    ks = np.array([1, 4, 10] * 10, np.int32)
    print(f"\n[case] insert dtype={dtype} n0={n0} n_new={n_new}", flush=True)
    a = R.Index(w.items[:n0], None if sc is None else sc[:n0], w.users, w.user_scales, dtype=dtype, k_max=k_max,
                num_hash=K, srp=A)
    b = R.Index(w.items, sc, w.users, w.user_scales, dtype=dtype, k_max=k_max, num_hash=K, srp=A)
    try:
        a.insert(w.items[n0:], None if sc is None else sc[n0:])
        assert a.info["n"] == n0 + n_new
        for k in range(1, k_max + 1):
            assert np.array_equal(a.lam(k), b.lam(k)), f"lambda k={k}"
            assert np.array_equal(a.lam32(k), b.lam32(k))
        assert np.array_equal(a.item_order(), b.item_order())
        ab, bb = a.blocks(), b.blocks()   # dicts of arrays: compare the arrays, key by key
        assert ab.keys() == bb.keys()
        for x, y in list(zip(a.saalsh(), b.saalsh())) + [(ab[k], bb[k]) for k in ab]:
            x, y = np.asarray(x), np.asarray(y)
            assert x.shape == y.shape and x.tobytes() == y.tobytes()
        lam = O.lambda_table(dtype, w.items, sc, w.users, w.user_scales, k_max)
        mem = O.member(dtype, w.users, w.user_scales, w.queries, w.query_scales, ks, lam)
        got = a.query(w.queries, w.query_scales, ks)
        for qi in range(len(ks)):
            assert np.array_equal(got[qi], np.flatnonzero(mem[qi])), f"query {qi}"
        with pytest.raises(R.RkmipsError):
            a.candidates()
    finally:
        a.close()
        b.close()


def test_insert_refuses_sah_index():
    from paper_2211_12751_amd import rkmips as R
    w = I.make("c2", n=200, m=300, d=16, nq=2, seed=102)
    print("\n[case] insert into SAH index", flush=True)
    a = R.Index(w.items, None, w.users, None, dtype="f32", k_max=10, mode=R.MODE_SAH)
    try:
        with pytest.raises(R.RkmipsError) as e:
            a.insert(w.items[:3])
        assert e.value.status == -1
    finally:
        a.close()
