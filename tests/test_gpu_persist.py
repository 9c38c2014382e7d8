"""Index save and load: a loaded index answers every query as the saved one and returns
the same lambda table, blocks and SA-ALSH data."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_12751_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype, mode", [("f32", 0), ("bf16", 1), ("fp8", 0)])
def test_save_load_round_trip(tmp_path, dtype, mode):
    from paper_2211_12751_amd import rkmips as R
    w = I.make({"f32": "c1", "bf16": "c3", "fp8": "c5"}[dtype], n=500, m=1200, d=40, nq=30, seed=81)
    ks = np.array([1, 3, 10] * 10, np.int32)
    print(f"\n[case] persist dtype={dtype} mode={mode}", flush=True)
    a = R.Index(w.items, w.item_scales, w.users, w.user_scales, dtype=dtype, k_max=10, mode=mode)
    path = str(tmp_path / "a.idx")
    try:
        a.save(path)
        b = R.Index.load(path)
        try:
            for key in ("n", "m", "d", "dtype", "k_max", "num_partitions", "num_blocks", "mode", "lambda_items",
                        "cert_failures", "err_fast"):
                assert a.info[key] == b.info[key], key
            ga, gb = a.query(w.queries, w.query_scales, ks), b.query(w.queries, w.query_scales, ks)
            for x, y in zip(ga, gb):
                assert np.array_equal(x, y)
            if mode == 0:
                lam = O.lambda_table(dtype, w.items, w.item_scales, w.users, w.user_scales, 10)
                mem = O.member(dtype, w.users, w.user_scales, w.queries, w.query_scales, ks, lam)
                for qi in range(len(ks)):
                    assert np.array_equal(gb[qi], np.flatnonzero(mem[qi]))
            for k in (1, 10):
                assert np.array_equal(a.lam(k), b.lam(k)) and np.array_equal(a.lam32(k), b.lam32(k))
            ab, bb = a.blocks(), b.blocks()   # dicts of arrays: compare the arrays, key by key
            assert ab.keys() == bb.keys()
            for x, y in [(ab[k], bb[k]) for k in ab] + list(zip(a.saalsh(), b.saalsh())):
                x, y = np.asarray(x), np.asarray(y)   # bit patterns (NaN centres of degenerate blocks)
                assert x.shape == y.shape and x.tobytes() == y.tobytes()
            assert np.array_equal(a.item_order(), b.item_order())
            with pytest.raises(R.RkmipsError):
                b.candidates()
        finally:
            b.close()
    finally:
        a.close()
