"""Seeded synthetic inputs for exact Reverse k-MIPS (RkMIPS).

This module only *draws* inputs and encodes them in their storage formats; it holds
none of the method's arithmetic (no inner products, norms used by the method,
top-k, bounds, hashing or membership tests).  Both the GPU path and the CPU
reference take their inputs from here, so it imports neither.

Workloads follow the matrix-factorisation shape of the paper's experiments
(Experiments, Setup; Appendix, dataset generation): item and user latent vectors
in R^d, queries drawn as fresh items.  The real datasets are not available, so
seeded synthetic vectors stand in for them:

* ``lndir(sigma)``  direction ~ N(0, I_d) normalised, norm ~ log-normal(0, sigma)
* ``shift(c)``      entries |N(0, 1)| + c (non-negative, not centred: the case the
                    shifting-invariant transform, Eqn. 6, is designed for)

Storage encodings:

* FP32 as is;
* BF16 as uint16 bit patterns, round-to-nearest-even from FP32;
* FP8 e4m3 (OCP "e4m3fn": bias 7, no infinities, max 448) as uint8 codes with
  one FP32 scale per vector, scale = amax / 448, codes round-to-nearest-even and
  saturating.
"""
from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np

BASE_SEED = 221112751
# independent counter streams of the base seed
STREAMS = {"items": 0, "users": 1, "queries": 2, "srp": 3, "tree": 4,
           "arrivals": 5, "kdraw": 6}

# name -> workload description (sizes and distributions)
CONFIGS = {
    # plain method, FP32
    "c1": dict(n=2_000, m=5_000, d=32, dtype="f32", ks=(1, 10), k_max=10, nq=100,
               items=("lndir", 0.5), users=("lndir", 0.5)),
    # FP32 path with SA-ALSH and Cone-Tree, shifted non-centred items
    "c2": dict(n=20_000, m=100_000, d=64, dtype="f32", ks=(1, 5, 10, 20, 50),
               k_max=50, nq=1_000, items=("shift", 0.3), users=("lndir", 0.7)),
    # precision: BF16 storage, same generators at d=128
    "c3": dict(n=100_000, m=1_000_000, d=128, dtype="bf16", ks=(10,), k_max=50,
               nq=10_000, items=("shift", 0.3), users=("lndir", 0.7)),
    # serving: the c3 index, Poisson arrivals, k ~ U{1,5,10,20,50}
    "c4": dict(n=100_000, m=1_000_000, d=128, dtype="bf16", ks=(1, 5, 10, 20, 50),
               k_max=50, nq=20_000, items=("shift", 0.3), users=("lndir", 0.7)),
    # large: FP8 e4m3 with per-vector scales
    "c5": dict(n=1_000_000, m=2_500_000, d=256, dtype="fp8", ks=(1, 10, 20, 50, 100),
               k_max=100, nq=10_000, items=("shift", 0.5), users=("lndir", 1.0)),
}

_CHUNK = 1 << 16


def rng(stream: str, seed: int = BASE_SEED) -> np.random.Generator:
    """Generator of one named stream of ``seed``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, STREAMS[stream]])))


def _workers() -> int:
    return max(1, min(8, os.cpu_count() or 1))


def draw(kind, rows: int, d: int, g: np.random.Generator) -> np.ndarray:
    """rows x d float32 matrix of the given kind, drawn in fixed-size row chunks.

    The random numbers are drawn chunk after chunk from the one generator (so any
    prefix of rows is reproducible); the per-chunk arithmetic that shapes them runs
    on worker threads."""
    name, par = kind
    if name not in ("lndir", "shift", "normal"):
        raise ValueError(f"unknown distribution {name!r}")
    out = np.empty((rows, d), dtype=np.float32)

    def shape(r0, x, rad):
        if name == "lndir":
            nrm = np.sqrt(np.einsum("ij,ij->i", x, x))
            nrm[nrm == 0] = 1.0
            out[r0:r0 + len(x)] = (x * (np.exp(par * rad) / nrm)[:, None]).astype(np.float32)
        elif name == "shift":
            out[r0:r0 + len(x)] = (np.abs(x) + par).astype(np.float32)
        else:
            out[r0:r0 + len(x)] = x.astype(np.float32)

    with cf.ThreadPoolExecutor(_workers()) as ex:
        futs = []
        for r0 in range(0, rows, _CHUNK):
            r1 = min(rows, r0 + _CHUNK)
            x = g.standard_normal((r1 - r0, d))
            rad = g.standard_normal(r1 - r0) if name == "lndir" else None
            futs.append(ex.submit(shape, r0, x, rad))
        for f in futs:
            f.result()
    return out


# ----------------------------------------------------------------------------------
# storage encodings
# ----------------------------------------------------------------------------------
def bf16_bits(x: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 bit patterns (uint16), round to nearest, ties to even."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_to_f32(bits: np.ndarray) -> np.ndarray:
    """BF16 bit patterns -> the FP32 values they denote (exact)."""
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def _e4m3_positive_table() -> np.ndarray:
    """Values of the 127 finite non-negative e4m3fn codes 0x00..0x7E, by code."""
    v = np.empty(127, dtype=np.float64)
    for c in range(127):
        e, mant = c >> 3, c & 7
        v[c] = mant * 2.0 ** -9 if e == 0 else (1 + mant / 8.0) * 2.0 ** (e - 7)
    return v


_E4M3_POS = _e4m3_positive_table()
E4M3_MAX = 448.0


def fp8_e4m3_codes(x: np.ndarray):
    """Per-row scaled FP8 e4m3fn encoding of a float32 matrix.

    Returns (codes uint8 [rows x d], scales float32 [rows]) with
    scale = amax/448 (1 for an all-zero row) and code = RNE(x/scale), saturating.
    The quotient y = |x|/scale is formed in float64; in the normal range
    (y >= 2^-6) its code is the float64 pattern rounded to three mantissa bits
    (round to nearest, ties to even, on the bits) and re-biased from 1023 to 7;
    below it the code is the subnormal count rint(y * 2^9).
    """
    x = np.asarray(x, dtype=np.float32)
    rows, d = x.shape
    codes = np.empty((rows, d), dtype=np.uint8)
    scales = np.empty(rows, dtype=np.float32)

    def enc(r0, r1):
        blk = x[r0:r1]
        amax = np.abs(blk).max(axis=1).astype(np.float64) if d else np.zeros(r1 - r0)
        sc = np.where(amax > 0, amax / E4M3_MAX, 1.0).astype(np.float32)
        scales[r0:r1] = sc
        y = np.abs(blk).astype(np.float64)
        y /= sc.astype(np.float64)[:, None]
        np.minimum(y, E4M3_MAX, out=y)
        b = y.view(np.uint64)
        r = (b + np.uint64((1 << 48) - 1) + ((b >> np.uint64(49)) & np.uint64(1))) >> np.uint64(49)
        normal = r.astype(np.int64) - ((1023 - 7) << 3)
        sub = np.rint(y * 512.0).astype(np.int64)
        c = np.where(y < 2.0 ** -6, sub, normal).astype(np.uint8)
        c |= ((blk < 0) & (c != 0)).astype(np.uint8) << 7
        codes[r0:r1] = c

    with cf.ThreadPoolExecutor(_workers()) as ex:
        for f in [ex.submit(enc, r0, min(rows, r0 + _CHUNK)) for r0 in range(0, rows, _CHUNK)]:
            f.result()
    return codes, scales


def fp8_e4m3_values(codes: np.ndarray, scales: np.ndarray) -> np.ndarray:
    """Decoded float64 values scale*value(code) of an encoded matrix (for checks)."""
    mag = _E4M3_POS[np.asarray(codes) & 0x7F]
    sgn = np.where(np.asarray(codes) & 0x80, -1.0, 1.0)
    return sgn * mag * np.asarray(scales, dtype=np.float64)[:, None]


# ----------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------
class Workload:
    """One synthetic workload: item, user and query matrices in storage format.

    ``items``/``users``/``queries`` are float32 (f32), uint16 (bf16) or uint8 (fp8)
    arrays; ``*_scales`` are float32 per-row scales for fp8, else None.
    ``ks`` holds one k per query (cycling through the configured k values).
    """

    def __init__(self, name, n, m, d, dtype, ks, k_max, nq, items, users,
                 seed=BASE_SEED):
        self.name, self.n, self.m, self.d = name, n, m, d
        self.dtype, self.k_values, self.k_max, self.nq = dtype, tuple(ks), k_max, nq
        self.seed = seed
        P = draw(items, n, d, rng("items", seed))
        U = draw(users, m, d, rng("users", seed))
        Q = draw(items, nq, d, rng("queries", seed))   # fresh draws of the item law
        self.items, self.item_scales = self._encode(P)
        self.users, self.user_scales = self._encode(U)
        self.queries, self.query_scales = self._encode(Q)
        self.ks = np.array([self.k_values[i % len(self.k_values)] for i in range(nq)],
                           dtype=np.int32)

    def _encode(self, x):
        if self.dtype == "f32":
            return np.ascontiguousarray(x), None
        if self.dtype == "bf16":
            return bf16_bits(x), None
        if self.dtype == "fp8":
            return fp8_e4m3_codes(x)
        raise ValueError(self.dtype)


def make(name: str, seed: int = BASE_SEED, **override) -> Workload:
    """Workload ``name`` (c1..c5) with optional size overrides (n, m, d, nq, ...)."""
    cfg = dict(CONFIGS[name])
    cfg.update(override)
    return Workload(name, seed=seed, **cfg)


def srp_matrix(d: int, K: int, seed: int = BASE_SEED) -> np.ndarray:
    """(d+1) x K matrix of i.i.d. N(0,1) entries: the K sign-random-projection
    vectors a of Eqn. 1 for the (d+1)-dimensional transformed space (float32)."""
    return rng("srp", seed).standard_normal((d + 1, K)).astype(np.float32)


def poisson_arrivals(nq: int, qps: float, seed: int = BASE_SEED) -> np.ndarray:
    """Arrival times in microseconds of a Poisson stream of ``nq`` requests."""
    gaps = rng("arrivals", seed).exponential(1.0 / qps, size=nq)
    return np.round(np.cumsum(gaps) * 1e6).astype(np.int64)


def k_draws(nq: int, values=(1, 5, 10, 20, 50), seed: int = BASE_SEED) -> np.ndarray:
    """k per request, uniform over ``values``."""
    return np.asarray(values, dtype=np.int32)[rng("kdraw", seed).integers(0, len(values), nq)]
