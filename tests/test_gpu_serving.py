"""Continuous-batching server: every answer equals the answer of the same request
alone and the CPU FP64 reference, while batches of mixed k overlap on the device."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_12751_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    from paper_2211_12751_amd import rkmips as R
    w = I.make("c1", n=2000, m=5000, d=32, nq=600, seed=17)
    k_max = 10
    ks = I.k_draws(w.nq, values=(1, 5, 10), seed=17)
    lam = O.lambda_table("f32", w.items, None, w.users, None, k_max)
    mem = O.member("f32", w.users, None, w.queries, None, ks, lam)
    print(f"\n[case] serving n={w.n} m={w.m} d={w.d} nq={w.nq}", flush=True)
    idx = R.Index(w.items, None, w.users, None, dtype="f32", k_max=k_max)
    yield R, w, ks, mem, idx
    idx.close()


@pytest.fixture(scope="module")
def alone(setup):
    """Each request answered on its own, as a batch of one."""
    R, w, ks, mem, idx = setup
    return [idx.query(w.queries[i:i + 1], None, ks[i:i + 1])[0] for i in range(w.nq)]


@pytest.mark.parametrize("qps,max_batch,streams", [(20000.0, 32, 4), (5000.0, 256, 2), (1e6, 64, 1), (0.0, 16, 4)])
def test_serving_matches_alone_and_reference(setup, alone, qps, max_batch, streams):
    R, w, ks, mem, idx = setup
    # qps = 0: every request arrives at time 0, so the slots fill back to back
    arr = I.poisson_arrivals(w.nq, qps, seed=5) if qps > 0 else np.zeros(w.nq, np.int64)
    got, lat, st = idx.serve(w.queries, None, ks, arr, max_batch=max_batch, num_streams=streams)
    print("stats", st, flush=True)
    for i in range(w.nq):
        assert np.array_equal(got[i], np.flatnonzero(mem[i])), f"request {i}"
        assert np.array_equal(got[i], alone[i]), f"request {i} differs from its lone answer"
    assert st["batches"] >= (w.nq + max_batch - 1) // max_batch
    assert 1 <= st["max_inflight"] <= streams
    if qps == 0.0:
        assert st["max_inflight"] >= 2, "batches never overlapped on the device"
    assert (lat > 0).all() and st["p99_us"] >= st["p50_us"] > 0


def test_memory_budget_admission(setup):
    R, w, ks, mem, idx = setup
    arr = I.poisson_arrivals(w.nq, 50000.0, seed=6)
    with pytest.raises(R.RkmipsError) as e:
        idx.serve(w.queries, None, ks, arr, max_batch=64, num_streams=4, mem_budget=1024)
    assert e.value.status == -2
    # a budget of about two slots admits two of the four requested streams
    got, lat, st = idx.serve(w.queries, None, ks, arr, max_batch=64, num_streams=4, mem_budget=2_700_000)
    assert 1 <= st["slots"] <= 4
    for i in range(w.nq):
        assert np.array_equal(got[i], np.flatnonzero(mem[i]))
