"""Candidates of the fused top-k pass (the streaming top-C before the FP64 refine),
checked against exact scores: every item whose exact score clears the user's final
threshold by more than the fast path's error bound must be a candidate, and every
candidate's score must be its exact score within that bound.  Both the split BF16
products (the FP32 default) and the FP32 matrix cores are covered."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_12751_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype, flags", [("f32", 0), ("f32", 64), ("bf16", 0), ("fp8", 0)])
def test_candidates_cover_and_score(dtype, flags):
    from paper_2211_12751_amd import rkmips as R
    name = {"f32": "c1", "bf16": "c3", "fp8": "c5"}[dtype]
    w = I.make(name, n=3000, m=700, d=48, nq=1, seed=51)
    k_max = 12
    print(f"\n[case] candidates {dtype} flags={flags}", flush=True)
    idx = R.Index(w.items, w.item_scales, w.users, w.user_scales, dtype=dtype, k_max=k_max, flags=flags)
    try:
        ids, sc, tau = idx.candidates()
        info = idx.info
        err = info["err_fast"]
        U = O.values(dtype, w.users, w.user_scales)
        P = O.values(dtype, w.items, w.item_scales)
        S = U @ P.T                                # exact up to 1e-15 relative
        un = np.linalg.norm(U, axis=1)
        pn = np.linalg.norm(P, axis=1)
        M = pn.max()
        slack = 1e-12 * (un[:, None] * pn[None, :]).max()
        for u in range(w.m):
            c = ids[u][ids[u] >= 0].astype(np.int64)
            assert len(c) == len(np.unique(c)), u
            must = np.flatnonzero(S[u] > tau[u] + err * un[u] * M + slack)
            assert np.isin(must, c).all(), (u, np.setdiff1d(must, c)[:5])
            s_u = sc[u][: len(c)].astype(np.float64)
            assert np.all(np.abs(s_u - S[u, c]) <= err * un[u] * pn[c] + 1e-30 + slack), u
            assert len(c) >= min(k_max, w.n) or info["cert_failures"] > 0
    finally:
        idx.close()
