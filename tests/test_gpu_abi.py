"""The C-ABI call shapes: device-side k values (rkmips_query_batch) against host-side
ones (rkmips_query_batch_hostk), the cumulative statistics (rkmips_get_stats) and the
synchronous wait for a build (rkmips_index_wait), with the answers checked against the
CPU FP64 reference (Definition 1)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2211_12751_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_device_and_host_ks_give_the_reference_sets():
    from paper_2211_12751_amd import rkmips as R
    w = I.make("c2", n=900, m=1700, d=40, nq=37, seed=301)
    k_max = 20
    ks = (np.arange(w.nq) * 7 % k_max + 1).astype(np.int32)
    print(f"\n[case] abi ks n={w.n} m={w.m} d={w.d} nq={w.nq}", flush=True)
    p = R.rkmips_default_params()
    p.k_max = k_max
    items, users, queries = R.to_device(w.items), R.to_device(w.users), R.to_device(w.queries)
    stream = torch.cuda.current_stream()
    h = R.rkmips_build_index(items, None, w.n, users, None, w.m, w.d, R.F32, None, p, stream)
    try:
        R.rkmips_index_wait(h)
        lam = O.lambda_table("f32", w.items, None, w.users, None, k_max)
        mem = O.member("f32", w.users, None, w.queries, None, ks, lam)
        dks = torch.from_numpy(ks).cuda()
        got = []
        for kind in ("device", "host"):
            r = (R.rkmips_query_batch(h, queries, None, w.nq, dks, 0, stream) if kind == "device"
                 else R.rkmips_query_batch_hostk(h, queries, None, w.nq, ks, 0, stream))
            R.rkmips_result_wait(r)
            off, ids = R.rkmips_result_view(r)
            R.rkmips_result_free(r)
            for qi in range(w.nq):
                assert np.array_equal(ids[off[qi]:off[qi + 1]], np.flatnonzero(mem[qi])), (kind, qi)
            got.append((off, ids))
        assert np.array_equal(got[0][0], got[1][0]) and np.array_equal(got[0][1], got[1][1])
        st = R.rkmips_get_stats(h)
        assert st["batches"] == 2 and st["queries"] == 2 * w.nq
        assert st["query"]["pairs_total"] == 2 * w.nq * w.m
        assert st["query"]["results"] == 2 * int(mem.sum())
        assert st["cert_failures"] == 0 and st["fallback_rate"] == 0.0
        assert 0.0 <= st["max_rel_err_lambda32"] <= 2.0 ** -24
        assert st["recheck_rate"] == st["query"]["pairs_rechecked"] / st["query"]["pairs_scored"]
        # a k out of range on the device side is refused like a host one
        bad = torch.from_numpy(np.where(np.arange(w.nq) == 5, k_max + 1, ks).astype(np.int32)).cuda()
        with pytest.raises(R.RkmipsError) as e:
            R.rkmips_query_batch(h, queries, None, w.nq, bad, 0, stream)
        assert e.value.status == -4
        assert R.rkmips_get_stats(h)["batches"] == 2
    finally:
        R.rkmips_index_free(h)
