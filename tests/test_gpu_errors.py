"""Error paths that the library can only detect on the device: non-finite values and
magnitudes outside the range where the FP32 fast path keeps its error model.  Every
case must return the stated status, and the library must keep working afterwards."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_12751_amd import inputs as I

pytestmark = pytest.mark.gpu

EINVAL, ERANGE = -1, -4


@pytest.fixture(scope="module")
def R():
    from paper_2211_12751_amd import rkmips
    return rkmips


def _small(seed=31):
    return I.make("c1", n=300, m=500, nq=20, seed=seed)


@pytest.mark.parametrize("where, value, status", [
    ("items", np.nan, EINVAL), ("users", np.inf, EINVAL),
    ("items", 1e20, ERANGE), ("users", 1e-35, ERANGE),
])
def test_build_rejects_bad_values(R, where, value, status):
    w = _small()
    items, users = w.items.copy(), w.users.copy()
    arr = items if where == "items" else users
    if np.isfinite(value) and value > 1e10:
        items[:] *= np.float32(1e18)
        users[:] *= np.float32(1e18)
    elif 0 < value < 1e-30:
        arr[7, :] = 0.0
        arr[7, 3] = np.float32(value)
    else:
        arr[5, 2] = value
    print(f"\n[case] build {where}={value}", flush=True)
    with pytest.raises(R.RkmipsError) as e:
        R.Index(items, None, users, None, dtype="f32", k_max=10)
    assert e.value.status == status


@pytest.mark.parametrize("value, status", [(np.nan, EINVAL), (1e-35, ERANGE)])
def test_query_rejects_bad_values_then_recovers(R, value, status):
    w = _small(seed=32)
    ks = np.full(w.nq, 5, np.int32)
    lam = O.lambda_table("f32", w.items, None, w.users, None, 10)
    mem = O.member("f32", w.users, None, w.queries, None, ks, lam)
    idx = R.Index(w.items, None, w.users, None, dtype="f32", k_max=10)
    try:
        q = w.queries.copy()
        if value < 1e-30:
            q[4, :] = 0.0
            q[4, 0] = np.float32(value)
        else:
            q[4, 1] = value
        print(f"\n[case] query value={value}", flush=True)
        with pytest.raises(R.RkmipsError) as e:
            idx.query(q, None, ks)
        assert e.value.status == status
        got = idx.query(w.queries, None, ks)
        for i in range(w.nq):
            assert np.array_equal(got[i], np.flatnonzero(mem[i]))
    finally:
        idx.close()


def test_empty_batch_and_long_lists(R):
    """nq = 0 gives an empty result; k = n makes every user qualify, so each list holds
    all m users (longer than one LDS sort chunk: the merge levels run).  With k = 64 > n
    every user qualifies (lambda = -inf)."""
    w = I.make("c1", n=63, m=9000, nq=6, seed=33)
    idx = R.Index(w.items, None, w.users, None, dtype="f32", k_max=64)
    try:
        assert idx.query(w.queries[:0], None, np.zeros(0, np.int32)) == []
        ks = np.array([64, 1, 64, 32, 64, 2], np.int32)
        lam = O.lambda_table("f32", w.items, None, w.users, None, 64)
        mem = O.member("f32", w.users, None, w.queries, None, ks, lam)
        got = idx.query(w.queries, None, ks)
        for i in range(len(ks)):
            assert np.array_equal(got[i], np.flatnonzero(mem[i]))
        assert len(got[0]) == w.m
    finally:
        idx.close()
