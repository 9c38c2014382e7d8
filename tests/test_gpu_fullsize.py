"""Full-size workloads in the launch configuration the benchmark uses, checked against
the CPU FP64 oracle on the users that can be checked one by one.

For a user set S the oracle computes the exact lambda rows of S over all of P; then
every lambda64 entry of S must be bit-exact, lambda32 = RN32(lambda64), and for every
query of the batch the GPU answer restricted to S must equal the Definition 1 set
restricted to S (no returned user of S below its threshold, no member of S missing).

  c3: 100,000 x 1,000,000 x 128, BF16, 10,000 queries of k = 10, k_max = 50.
      S = every user returned by the first 200 queries + a seeded 1 % of all users.
  c4: the c3 index serving 2,000 Poisson requests (fresh item draws, k uniform over
      {1, 5, 10, 20, 50}) on four slots: each answer equals the answer of the same
      request alone, batches overlap on the device, and the answers restricted to
      S = the c3 seeded users + every user returned by the first 100 requests equal the
      oracle's.
  c5: 1,000,000 x 2,500,000 x 256, FP8 e4m3 + FP32 scales, 10,000 queries of
      k in {1, 10, 20, 50, 100}, k_max = 100.
      S = every user returned by the first 50 queries + 2,500 seeded users.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_12751_amd import inputs as I

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


class _Lambda:
    """Oracle lambda rows (all k <= k_max) of a workload, computed once per user."""

    def __init__(self, w):
        self.w = w
        self.rows = {}

    def get(self, users):
        w = self.w
        users = np.unique(np.asarray(users, np.int64))
        need = np.array([u for u in users.tolist() if u not in self.rows], np.int64)
        for c0 in range(0, len(need), 2048):   # in chunks, with a progress line each
            part = need[c0:c0 + 2048]
            lam = O.lambda_table(w.dtype, w.items, w.item_scales, w.users, w.user_scales, w.k_max, user_idx=part)
            for i, u in enumerate(part.tolist()):
                self.rows[u] = lam[:, i].copy()
            print(f"  oracle lambda rows {min(c0 + 2048, len(need))}/{len(need)}", flush=True)
        return users, np.stack([self.rows[u] for u in users.tolist()], axis=1)


def _check_lambda(idx, w, users, lam):
    for k in range(1, w.k_max + 1):
        assert np.array_equal(idx.lam(k)[users], lam[k - 1]), f"lambda64 k={k}"
        assert np.array_equal(idx.lam32(k)[users], lam[k - 1].astype(np.float32)), f"lambda32 k={k}"


def _check_sets(w, got, queries, q_scales, ks, users, lam, what):
    mem = O.member(w.dtype, w.users, w.user_scales, queries, q_scales, ks, lam, user_idx=users)
    pos = np.full(w.m, -1, np.int64)
    pos[users] = np.arange(len(users))
    for qi, lst in enumerate(got):
        mine = np.zeros(len(users), np.uint8)
        p = pos[np.asarray(lst, np.int64)]
        mine[p[p >= 0]] = 1
        if not np.array_equal(mine, mem[qi]):
            extra = users[(mine == 1) & (mem[qi] == 0)][:5]
            missing = users[(mine == 0) & (mem[qi] == 1)][:5]
            raise AssertionError(f"{what} {qi} (k={ks[qi]}): returned below threshold {extra}, missing {missing}")
    return int(mem.sum())


def _returned(got, count):
    parts = [np.asarray(got[i], np.int64) for i in range(min(count, len(got)))]
    return np.concatenate(parts) if parts else np.zeros(0, np.int64)


@pytest.fixture(scope="module")
def c3():
    from paper_2211_12751_amd import rkmips as R
    w = I.make("c3")
    print(f"\n[case] c3 n={w.n} m={w.m} d={w.d} dtype={w.dtype} k_max={w.k_max} nq={w.nq}", flush=True)
    idx = R.Index(w.items, w.item_scales, w.users, w.user_scales, dtype=w.dtype, k_max=w.k_max)
    seeded = np.random.default_rng(2212).choice(w.m, w.m // 100, replace=False)
    yield R, w, idx, _Lambda(w), seeded
    idx.close()


@pytest.mark.timeout(900)
def test_c3_returned_and_seeded_users(c3):
    R, w, idx, L, seeded = c3
    got = idx.query(w.queries, w.query_scales, w.ks)
    users, lam = L.get(np.concatenate([_returned(got, 200), seeded]))
    print(f"[c3] oracle users {len(users)} (returned by 200 queries + {len(seeded)} seeded)", flush=True)
    _check_lambda(idx, w, users, lam)
    hits = _check_sets(w, got, w.queries, w.query_scales, w.ks, users, lam, "query")
    assert hits >= len(_returned(got, 200)) > 0
    print(f"[c3] memberships checked {hits} over {w.nq} queries", flush=True)


@pytest.mark.timeout(900)
def test_c4_serving_on_c3_index(c3):
    R, w, idx, L, seeded = c3
    nreq, max_batch, streams = 2_000, 256, 4
    g = I.rng("queries", w.seed + 1)
    Qs = I.draw(I.CONFIGS["c4"]["items"], nreq, w.d, g)
    Qh = np.ascontiguousarray(I.bf16_bits(Qs))
    ks = I.k_draws(nreq, values=I.CONFIGS["c4"]["ks"], seed=w.seed + 1)
    # saturation rate of the server, then Poisson arrivals at 80 % of it
    _, _, st0 = idx.serve(Qh[:512], None, ks[:512], np.zeros(512, np.int64), max_batch=max_batch,
                          num_streams=streams)
    qps = 0.8 * 512 / (st0["wall_ms"] * 1e-3)
    arr = I.poisson_arrivals(nreq, qps, seed=w.seed + 5)
    print(f"[c4] {nreq} requests at {qps:.0f} qps", flush=True)
    got, lat, st = idx.serve(Qh, None, ks, arr, max_batch=max_batch, num_streams=streams)
    print(f"[c4] stats {st}", flush=True)
    assert st["max_inflight"] >= 2, "batches never overlapped on the device"
    assert (lat > 0).all() and st["p99_us"] >= st["p50_us"] > 0
    for i in range(nreq):
        alone = idx.query(Qh[i:i + 1], None, ks[i:i + 1])[0]
        assert np.array_equal(np.asarray(got[i]), np.asarray(alone)), f"request {i} differs from its lone answer"
    users, lam = L.get(np.concatenate([_returned(got, 100), seeded]))
    print(f"[c4] oracle users {len(users)}", flush=True)
    hits = _check_sets(w, got, Qh, None, ks, users, lam, "request")
    assert hits > 0
    print(f"[c4] memberships checked {hits} over {nreq} requests", flush=True)


@pytest.mark.timeout(900)
def test_c5_returned_and_seeded_users():
    from paper_2211_12751_amd import rkmips as R
    w = I.make("c5")
    print(f"\n[case] c5 n={w.n} m={w.m} d={w.d} dtype={w.dtype} k_max={w.k_max} nq={w.nq}", flush=True)
    idx = R.Index(w.items, w.item_scales, w.users, w.user_scales, dtype=w.dtype, k_max=w.k_max)
    try:
        got = idx.query(w.queries, w.query_scales, w.ks)
        seeded = np.random.default_rng(2213).choice(w.m, 2_500, replace=False)
        ret = _returned(got, 50)
        users, lam = _Lambda(w).get(np.concatenate([ret, seeded]))
        print(f"[c5] oracle users {len(users)} (returned by 50 queries: {len(np.unique(ret))})", flush=True)
        _check_lambda(idx, w, users, lam)
        hits = _check_sets(w, got, w.queries, w.query_scales, w.ks, users, lam, "query")
        assert hits >= len(ret) > 0
        print(f"[c5] memberships checked {hits} over {w.nq} queries", flush=True)
    finally:
        idx.close()
