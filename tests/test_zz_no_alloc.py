"""rkmips_saalsh_probe_noalloc (Alg. 2 for explicit pairs, with its staging and candidate
scratch in the library's static per-GPU array) against rkmips_saalsh_probe on the same
pairs: identical phi values (bit for bit) and answers, on two calls in a row, the
second with a smaller input; and a batch that does not fit is refused."""
import numpy as np
import pytest
import torch

from paper_2211_12751_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype, mode", [("f32", 0), ("fp8", 0), ("bf16", 1)])
def test_noalloc_probe_equals_probe(dtype, mode):
    from paper_2211_12751_amd import rkmips as R
    name = {"f32": "c2", "bf16": "c3", "fp8": "c5"}[dtype]
    w = I.make(name, n=1500, m=900, d=40, nq=40, seed=401)
    print(f"\n[case] noalloc probe {dtype} mode={mode}", flush=True)
    p = R.rkmips_default_params()
    p.k_max, p.mode = 20, mode
    idx = R.Index(w.items, w.item_scales, w.users, w.user_scales, dtype=dtype, params=p)
    try:
        q = R.to_device(w.queries)
        qs = R.to_device(w.query_scales)
        g = np.random.default_rng(402)
        ks = g.integers(1, 21, w.nq).astype(np.int32)
        for npairs, nqu, beta in ((3000, w.nq, 0.1), (700, 17, 0.3)):
            pq = g.integers(0, nqu, npairs)
            pu = g.integers(0, w.m, npairs)
            a_phi, a_ans = R.rkmips_saalsh_probe(idx.h, q, qs, nqu, ks[:nqu], pq, pu, beta)
            b_phi, b_ans = R.rkmips_saalsh_probe_noalloc(idx.h, q, qs, nqu, ks[:nqu], pq, pu, beta)
            assert np.array_equal(a_phi.view(np.int64), b_phi.view(np.int64))
            assert np.array_equal(a_ans, b_ans)
        # too large for the 64 MiB array: refused before any device work
        big = 3_000_000
        with pytest.raises(R.RkmipsError) as e:
            R.rkmips_saalsh_probe_noalloc(idx.h, q, qs, w.nq, ks, np.zeros(big, np.int64), np.zeros(big, np.int64),
                                          0.1)
        assert e.value.status == -4 and "no-allocation" in str(e.value)
    finally:
        idx.close()
