"""Cone-Tree blocks (Alg. 3 leaves) and their bound data against the CPU reference.

The tree itself is one of many valid ones (its random points and split ties are the
library's), so the tests check that it is a valid blocking and compare everything that
is determined once the blocking is fixed: block centres, per-user angles to the stored
centres, the cone angle (which must bound every user's angle: it is what Lemma 2
prunes with) and the lower bounds L^j(B) (which must not exceed the exact minimum)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_12751_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype, n, m, d, k_max, cert", [("f32", 500, 3001, 24, 10, True),
                                                          ("bf16", 400, 2000, 64, 8, True),
                                                          ("fp8", 300, 1500, 40, 5, True),
                                                          ("bf16", 400, 1200, 64, 100, True),
                                                          ("fp8", 300, 900, 128, 70, False),
                                                          ("fp8", 1 << 18, 2000, 32, 4, True)])
def test_blocks_valid_and_bound_data_exact(dtype, n, m, d, k_max, cert):
    """k_max above 64 takes more than one column per lane in the bound pass; without the
    certificate every lambda row (and its bound row) comes from the full rescoring.  With
    2^18 items and more, FP8 builds split the tree on the users' padded code rows and
    per-user factors instead of BF16 unit rows."""
    from paper_2211_12751_amd import rkmips as R
    name = {"f32": "c1", "bf16": "c3", "fp8": "c5"}[dtype]
    w = I.make(name, n=n, m=m, d=d, nq=1, seed=m)
    w.users[[5, 77]] = 0 if dtype != "fp8" else w.users[[5, 77]]
    print(f"\n[case] cone {dtype} n={n} m={m} d={d} k_max={k_max} cert={cert}", flush=True)
    idx = R.Index(w.items, w.item_scales, w.users, w.user_scales, dtype=dtype, k_max=k_max,
                  flags=0 if cert else R.FLAG_NO_CERT)
    try:
        b = idx.blocks()
        leaf, bs = b["leaf_users"].astype(np.int64), b["block_start"]
        # a blocking: a permutation of the users cut into leaves of 1..N0 users
        assert np.array_equal(np.sort(leaf), np.arange(m))
        assert bs[0] == 0 and bs[-1] == m and np.all(np.diff(bs) >= 1) and np.all(np.diff(bs) <= 64)
        cen_o, _, _ = O.cone_block_stats(dtype, w.users, w.user_scales, leaf, bs)
        ok = ~np.isnan(cen_o[:, 0])
        assert np.allclose(b["center"][ok], cen_o[ok], atol=2e-6)
        # angles against the stored centres, and the cone angle bounds them all
        ct = O.cos_to_centres(dtype, w.users, w.user_scales, leaf, bs, b["center"].astype(np.float64))
        nb = len(bs) - 1
        for B in range(nb):
            sl = slice(bs[B], bs[B + 1])
            if b["cos_omega"][B] == -1.0 and b["sin_omega"][B] == 0.0:
                continue   # no usable cone: never pruned
            assert ok[B]
            assert np.allclose(b["cos_theta"][sl], ct[sl], atol=2e-7), B
            assert b["cos_omega"][B] <= ct[sl].min(), B
            assert b["cos_omega"][B] >= ct[sl].min() - 2e-6, B
            assert abs(b["sin_omega"][B] - np.sqrt(max(0.0, 1 - float(b["cos_omega"][B]) ** 2))) <= 1e-6
        st = b["sin_theta"].astype(np.float64)
        assert np.allclose(st, np.sqrt(np.maximum(0, 1 - b["cos_theta"].astype(np.float64) ** 2)), atol=1e-6)
        # lower bounds: L^j(B) rounded down to FP32 (one step at most), -inf without a cone
        lam = O.lambda_table(dtype, w.items, w.item_scales, w.users, w.user_scales, k_max)
        lb_o = O.block_lower_bounds(dtype, w.users, w.user_scales, lam, leaf, bs)
        lb = b["block_lb"].astype(np.float64)
        cone = ~((b["cos_omega"] == -1.0) & (b["sin_omega"] == 0.0))
        assert np.all(np.isneginf(lb[:, ~cone]))
        g, o = lb[:, cone], lb_o[:, cone]
        fin = np.isfinite(o)
        assert np.all(g[fin] <= o[fin])
        assert np.all(np.nextafter(g[fin].astype(np.float32), np.float32(np.inf)).astype(np.float64) >= o[fin])
        assert np.all(np.isneginf(g[~fin]))
    finally:
        idx.close()
