"""The Cone-Tree bounds prune, and stay exact (Lemma 2, node level; Lemma 3, vector level;
Alg. 5 block and user tests).

Users come in a few tight direction clusters (plus some outliers that widen the cones of
the blocks they land in); items and queries are Gaussian.  Most (query, block) pairs
are then far apart in angle, so the bounds must remove many pairs.  The test checks:
- the answer sets equal the CPU FP64 reference (Definition 1) with the bounds on and off;
- the node-level bound prunes on the default path and the vector-level bound on the
  FP32 matrix-core path (where it is evaluated);
- the pruned counts lie within what the same bounds allow in FP64: Lemma 2 and Lemma 3
  evaluated exactly on the library's own leaf partition (cone data from the reference),
  and every pair those FP64 bounds remove is a true "no"."""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu


def clustered(seed, n=1800, m=2600, nq=90, d=16, nclusters=6, spread=0.04, outliers=0.03):
    g = np.random.default_rng(seed)
    cen = g.standard_normal((nclusters, d))
    cen /= np.linalg.norm(cen, axis=1, keepdims=True)
    lab = g.integers(0, nclusters, m)
    U = cen[lab] + spread * g.standard_normal((m, d))
    out = g.random(m) < outliers
    U[out] = g.standard_normal((int(out.sum()), d))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    U *= np.exp(0.5 * g.standard_normal(m))[:, None]
    P = g.standard_normal((n, d))
    Q = g.standard_normal((nq, d))
    return P.astype(np.float32), U.astype(np.float32), Q.astype(np.float32)


def fp64_prunable(P, U, Q, ks, lam, leaf, bs):
    """Pairs that Lemma 2 (whole block) and Lemma 3 (single user, block not pruned)
    remove when evaluated in FP64 on the given blocking."""
    cen, cos_t, cos_w = O.cone_block_stats("f32", U, None, leaf, bs)
    Uv, Qv = U.astype(np.float64), Q.astype(np.float64)
    un = np.linalg.norm(Uv, axis=1)
    qn = np.linalg.norm(Qv, axis=1)
    lb = O.block_lower_bounds("f32", U, None, lam, leaf, bs)
    node = np.zeros((len(Q), len(U)), bool)
    vec = np.zeros((len(Q), len(U)), bool)
    for b in range(len(bs) - 1):
        if np.isnan(cos_w[b]):
            continue
        idx = leaf[bs[b]:bs[b + 1]]
        om = np.arccos(np.clip(cos_w[b], -1, 1))
        phi = np.arccos(np.clip(Qv @ cen[b] / qn, -1, 1))
        ub = qn * np.cos(np.maximum(0.0, phi - om))
        th = np.arccos(np.clip(cos_t[bs[b]:bs[b + 1]], -1, 1))
        for qi in range(len(Q)):
            k = int(ks[qi])
            if ub[qi] < lb[k - 1, b]:
                node[qi, idx] = True
            else:
                ubv = un[idx] * qn[qi] * np.cos(np.abs(phi[qi] - th))
                vec[qi, idx] = ubv < lam[k - 1, idx]
    return node, vec


@pytest.mark.parametrize("seed", [11, 12])
def test_bounds_prune_and_stay_exact(seed):
    from paper_2211_12751_amd import rkmips as R
    P, U, Q = clustered(seed)
    k_max = 10
    ks = (np.arange(len(Q)) % k_max + 1).astype(np.int32)
    print(f"\n[case] bounds seed={seed} n={len(P)} m={len(U)} nq={len(Q)}", flush=True)
    lam = O.lambda_table("f32", P, None, U, None, k_max)
    mem = O.member("f32", U, None, Q, None, ks, lam)
    for flags_build in (0, R.FLAG_F32_MATRIX):
        p = R.rkmips_default_params()
        p.k_max, p.flags = k_max, flags_build
        idx = R.Index(P, None, U, None, dtype="f32", params=p)
        try:
            got, st = idx.query(Q, None, ks, stats=True)
            off, _ = idx.query(Q, None, ks, flags=R.FLAG_NO_BOUNDS, stats=True)
            for qi in range(len(Q)):
                assert np.array_equal(got[qi], np.flatnonzero(mem[qi])), (flags_build, qi)
                assert np.array_equal(off[qi], got[qi])
            b = idx.blocks()
            leaf, bs = b["leaf_users"].astype(np.int64), b["block_start"]
            node, vec = fp64_prunable(P, U, Q, ks, lam, leaf, bs)
            # Lemma 2 and 3 are sound on these data: every pair they remove is a "no"
            assert not np.any(mem.astype(bool) & (node | vec))
            nb, nv = int(st["pairs_block_pruned"]), int(st["pairs_vector_pruned"])
            print(f"flags={flags_build}: block pruned {nb} (fp64 {int(node.sum())}), "
                  f"vector pruned {nv} (fp64 {int(vec.sum())}) of {st['pairs_total']}", flush=True)
            assert 0 < nb <= int(node.sum())
            assert nb >= 0.9 * int(node.sum())      # the rounding slack costs little
            if flags_build == R.FLAG_F32_MATRIX:
                # evaluated only where it can skip FP32 products
                assert 0 < nv <= int(vec.sum()) + int(node.sum()) - nb
        finally:
            idx.close()
