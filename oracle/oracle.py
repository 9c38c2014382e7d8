"""Python face of the CPU FP64 reference for exact Reverse k-MIPS.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's
CPU-baseline leg, never by the product path.  It shares no code with the GPU
library; it receives the same seeded input arrays and computes every result from
its definition (see rkmips_oracle.c for the definitions and the readings taken).

Functions (all inputs are numpy arrays in storage format: float32, uint16 BF16 bits
or uint8 FP8 e4m3 codes with float32 per-row scales):

* ``lambda_table``   lambda_u^(j), j = 1..k_max, per user (Def. 1; Alg. 4)
* ``fp8_scores``     canonical FP8 scores of a user set against a row set (exact)
* ``member``         membership of user u in R_k(q)   (Def. 1, ">=" tie reading)
* ``count_beating``  #{p : s(u,p) > s(u,q)}           (Def. 1, count form)
* ``item_order``     canonical squared norms and descending order (Alg. 4 / Alg. 1)
* ``partitions``, ``saalsh_index``, ``user_codes``, ``saalsh_decide``  (Alg. 1, 2)
* ``rkmips``         per-query ascending user-ID lists
* ``values``         stored rows widened to float64 (FP8: code value x row scale)
* ``cone_block_stats``, ``block_lower_bounds``  per-block cone data of a given
  partition of the users (Alg. 3 leaves; Lemmas 2 and 3; L^j(B) of Alg. 4)
* ``saalsh_kmips``   the k best scores Alg. 2's probes find for a user (no query)
* ``sah_rkmips``     the approximate SAH method: Alg. 4 with L_i from P' and the
  SA-ALSH index over P minus P', Alg. 5 per (query, user)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rkmips_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liborc.so")
# RKMIPS_ORACLE_SANITIZE=1: load an AddressSanitizer + UndefinedBehaviorSanitizer build
# instead (the process must preload gcc's libasan)
_SAN = os.environ.get("RKMIPS_ORACLE_SANITIZE", "") == "1"
_LIB_SAN = os.path.join(_HERE, "_build", "liborc_san.so")
_DT = {"f32": 0, "bf16": 1, "fp8": 2}
_lib = None



def _default_threads() -> int:
    """Threads for the parallel loops: RKMIPS_ORACLE_THREADS, else the CPUs this process
    may run on, capped by OMP_NUM_THREADS when that is set."""
    n = int(os.environ.get("RKMIPS_ORACLE_THREADS", "0") or 0)
    if n > 0:
        return n
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    omp = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return max(1, min(n, omp) if omp > 0 else n)


NTHREADS = _default_threads()


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile the reference with gcc (strict IEEE: no fast-math, no contraction);
    sanitize=True makes the AddressSanitizer + UndefinedBehaviorSanitizer build."""
    lib = _LIB_SAN if sanitize else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(lib), exist_ok=True)
        tmp = lib + f".tmp{os.getpid()}"
        extra = (["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                  "-fno-omit-frame-pointer"] if sanitize else ["-O2"])
        subprocess.check_call(["gcc", *extra, "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
                               "-std=c99", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, lib)
    return lib


def _L():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build(sanitize=_SAN))
        _lib.orc_e4m3_value.restype = C.c_double
        _lib.orc_e4m3_value.argtypes = [C.c_uint8]
        _lib.orc_score.restype = C.c_double
        _lib.orc_norm2.restype = C.c_double
    return _lib


def _p(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _c(a, dt=None):
    if a is None:
        return None
    return np.ascontiguousarray(a if dt is None else a.astype(dt, copy=False))


def _sel(user_idx, m):
    if user_idx is None:
        return None, m
    ui = _c(np.asarray(user_idx), np.int64)
    return ui, len(ui)


def e4m3_value(code: int) -> float:
    return _L().orc_e4m3_value(code)


def score(dtype, a, a_scales, ra, b, b_scales, rb) -> float:
    a, b = _c(a), _c(b)
    return _L().orc_score(_DT[dtype], a.shape[1], _p(a), _p(_c(a_scales, np.float32)), C.c_int64(ra),
                          _p(b), _p(_c(b_scales, np.float32)), C.c_int64(rb))


def _fp8_codes_f64(X):
    """Decoded e4m3 code values (unscaled) as float64, through the C decoder's table."""
    table = np.array([e4m3_value(c) for c in range(256)], dtype=np.float64)
    return table[np.asarray(X)]


def fp8_scores(U, U_scales, X, X_scales, user_idx=None, Xc=None):
    """Canonical FP8 scores s(u, x) = (s_u s_x) S(u, x) for the selected users (rows) and
    all rows x (columns), float64.  S, the sum of the decoded code products, is a sum of
    multiples of 2^-18 below 2^26 in magnitude, so every partial sum is exact in float64
    and a matrix product in any order gives S exactly; s_u s_x is exact too, so the one
    rounding is the final product, as in the canonical definition."""
    ui = np.arange(len(U)) if user_idx is None else np.asarray(user_idx, np.int64)
    Uc = _fp8_codes_f64(np.asarray(U)[ui])
    if Xc is None:
        Xc = _fp8_codes_f64(X)
    S = Uc @ Xc.T
    return (np.asarray(U_scales, np.float64)[ui][:, None] * np.asarray(X_scales, np.float64)[None, :]) * S


def lambda_table(dtype, P, P_scales, U, U_scales, k_max, user_idx=None, nthreads=None):
    """float64 [k_max x m_sel] (k-major): row j is lambda^(j+1) of each selected user.
    FP8 data: the scores come from fp8_scores (exact matrix product), the order statistics
    from a sort; other types: the C reference, one pair at a time."""
    if dtype == "fp8":
        return _lambda_fp8(P, P_scales, U, U_scales, k_max, user_idx)
    P, U = _c(P), _c(U)
    ui, ms = _sel(user_idx, U.shape[0])
    lam = np.empty((k_max, ms), dtype=np.float64)
    r = _L().orc_lambda(_DT[dtype], P.shape[1], _p(P), _p(_c(P_scales, np.float32)),
                        C.c_int64(P.shape[0]), _p(U), _p(_c(U_scales, np.float32)), _p(ui),
                        C.c_int64(ms), k_max, _p(lam), nthreads or NTHREADS)
    if r:
        raise MemoryError("oracle lambda table")
    return lam


def _lambda_fp8(P, P_scales, U, U_scales, k_max, user_idx, chunk_bytes=1 << 30):
    ui = np.arange(len(U)) if user_idx is None else np.asarray(user_idx, np.int64)
    n = len(P)
    lam = np.full((k_max, len(ui)), -np.inf)
    kk = min(k_max, n)
    rows = max(1, int(chunk_bytes // (8 * max(n, 1))))
    Pc = _fp8_codes_f64(P)   # decoded once
    for r0 in range(0, len(ui), rows):
        sc = fp8_scores(U, U_scales, P, P_scales, user_idx=ui[r0:r0 + rows], Xc=Pc)
        if kk < n:
            sc = np.partition(sc, n - kk, axis=1)[:, n - kk:]
        lam[:kk, r0:r0 + rows] = -np.sort(-sc, axis=1).T[:kk]
    return lam


def member(dtype, U, U_scales, Q, Q_scales, ks, lam, user_idx=None, nthreads=None):
    """uint8 [nq x m_sel]: 1 iff s(u,q) >= lambda_u^(k_q).  FP8 data: scores from
    fp8_scores (exact); other types: the C reference."""
    if dtype == "fp8":
        ks = np.asarray(ks, np.int64)
        if np.any(ks < 1) or np.any(ks > lam.shape[0]):
            raise ValueError("k outside [1, k_max]")
        sc = fp8_scores(U, U_scales, Q, Q_scales, user_idx=user_idx)            # [m_sel x nq]
        return (sc.T >= np.asarray(lam, np.float64)[ks - 1, :]).astype(np.uint8)
    U, Q = _c(U), _c(Q)
    ui, ms = _sel(user_idx, U.shape[0])
    ks = _c(np.asarray(ks), np.int32)
    lam = _c(lam, np.float64)
    out = np.empty((Q.shape[0], ms), dtype=np.uint8)
    r = _L().orc_member(_DT[dtype], U.shape[1], _p(U), _p(_c(U_scales, np.float32)), _p(ui),
                        C.c_int64(ms), _p(Q), _p(_c(Q_scales, np.float32)), C.c_int64(Q.shape[0]),
                        _p(ks), _p(lam), lam.shape[0], _p(out), nthreads or NTHREADS)
    if r == -1:
        raise ValueError("k outside [1, k_max]")
    if r:
        raise MemoryError("oracle membership")
    return out


def count_beating(dtype, P, P_scales, U, U_scales, Q, Q_scales, user_idx=None, nthreads=None):
    """int64 [nq x m_sel]: #{p in P : s(u,p) > s(u,q)}."""
    P, U, Q = _c(P), _c(U), _c(Q)
    ui, ms = _sel(user_idx, U.shape[0])
    out = np.empty((Q.shape[0], ms), dtype=np.int64)
    _L().orc_count_beating(_DT[dtype], P.shape[1], _p(P), _p(_c(P_scales, np.float32)),
                           C.c_int64(P.shape[0]), _p(U), _p(_c(U_scales, np.float32)), _p(ui),
                           C.c_int64(ms), _p(Q), _p(_c(Q_scales, np.float32)),
                           C.c_int64(Q.shape[0]), _p(out), nthreads or NTHREADS)
    return out


def rkmips(dtype, P, P_scales, U, U_scales, Q, Q_scales, ks, k_max, nthreads=None):
    """Per-query ascending user-ID lists plus the lambda table."""
    lam = lambda_table(dtype, P, P_scales, U, U_scales, k_max, nthreads=nthreads)
    mem = member(dtype, U, U_scales, Q, Q_scales, ks, lam, nthreads=nthreads)
    return [np.flatnonzero(row).astype(np.int32) for row in mem], lam


def item_order(dtype, P, P_scales):
    """(norm2 float64 [n], order int64 [n]): canonical n2 and descending order."""
    P = _c(P)
    n = P.shape[0]
    n2 = np.empty(n, dtype=np.float64)
    order = np.empty(n, dtype=np.int64)
    _L().orc_item_order(_DT[dtype], P.shape[1], _p(P), _p(_c(P_scales, np.float32)),
                        C.c_int64(n), _p(n2), _p(order))
    return n2, order


def partitions(norm2, order, b, start=0):
    """int64 partition starts into ``order`` (length t+1) of the items order[start:]
    (SAH leaves the first positions, P', out of the SA-ALSH index)."""
    norm2 = _c(norm2, np.float64)
    order = _c(np.asarray(order)[start:], np.int64)
    n = len(order)
    ps = np.empty(n + 2, dtype=np.int64)
    t = _L().orc_partitions(_p(norm2), _p(order), C.c_int64(n), C.c_float(b), _p(ps), n + 1)
    return ps[: t + 1].copy() + start


def saalsh_index(dtype, P, P_scales, order, part_start, A):
    """(centroid [t x d] f64, radius [t] f64, codes uint32 [n x K/32]) of Alg. 1."""
    P = _c(P)
    A = _c(A, np.float32)
    order, part_start = _c(order, np.int64), _c(part_start, np.int64)
    n, d = P.shape
    K = A.shape[1]
    t = len(part_start) - 1
    cen = np.empty((t, d), dtype=np.float64)
    rad = np.empty(t, dtype=np.float64)
    codes = np.zeros((n, K // 32), dtype=np.uint32)   # items outside every partition keep 0
    _L().orc_saalsh_index(_DT[dtype], d, _p(P), _p(_c(P_scales, np.float32)), C.c_int64(n),
                          _p(order), _p(part_start), t, _p(A), K, _p(cen), _p(rad), _p(codes))
    return cen, rad, codes


def user_codes(dtype, U, U_scales, A):
    U = _c(U)
    A = _c(A, np.float32)
    m, d = U.shape
    K = A.shape[1]
    codes = np.empty((m, K // 32), dtype=np.uint32)
    _L().orc_user_codes(_DT[dtype], d, _p(U), _p(_c(U_scales, np.float32)), C.c_int64(m),
                        _p(A), K, _p(codes))
    return codes


def saalsh_decide(dtype, P, P_scales, norm2, order, part_start, item_codes, ucode, beta,
                  U, U_scales, u, Q, Q_scales, qi, k, init=None):
    """(answer 0/1, phi) of Alg. 2 for user u, query qi and k.  ``init``: scores that
    are candidates before the first partition (SAH: u's scores on P')."""
    P, U, Q = _c(P), _c(U), _c(Q)
    init = _c(np.zeros(0) if init is None else np.asarray(init), np.float64)
    phi = C.c_double(0.0)
    ucode = _c(np.asarray(ucode), np.uint32)
    K = ucode.shape[-1] * 32
    r = _L().orc_saalsh_decide(_DT[dtype], P.shape[1], _p(P), _p(_c(P_scales, np.float32)),
                               _p(_c(norm2, np.float64)), _p(_c(order, np.int64)),
                               _p(_c(part_start, np.int64)), len(part_start) - 1,
                               _p(_c(item_codes, np.uint32)), _p(ucode), K, C.c_float(beta),
                               _p(U), _p(_c(U_scales, np.float32)), C.c_int64(u),
                               _p(Q), _p(_c(Q_scales, np.float32)), C.c_int64(qi), k,
                               _p(init), C.c_int64(len(init)), C.byref(phi))
    if r < 0:
        raise MemoryError("oracle saalsh_decide")
    return r, phi.value


def values(dtype, X, scales=None):
    """float64 [rows x d]: the stored rows as exact real numbers (BF16 widened, FP8
    e4m3 code value times the row's FP32 scale)."""
    X = np.asarray(X)
    if dtype == "f32":
        return X.astype(np.float64)
    if dtype == "bf16":
        return (X.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    table = np.array([e4m3_value(c) for c in range(256)], dtype=np.float64)
    return table[X] * np.asarray(scales, np.float64)[:, None]


def cone_block_stats(dtype, U, U_scales, leaf_users, block_start):
    """Cone data of the blocks of a given user partition (the leaves of Alg. 3).

    The users of block B are leaf_users[block_start[B]:block_start[B+1]].  Per block the
    centre c_B is the normalised mean of the unit user vectors (Fact 2 makes only the
    direction of u matter); theta_u is the angle between u and c_B (the vector-level
    bound of Lemma 3); the cone half-angle omega_B is the largest theta_u of the block
    (the node-level bound of Lemma 2).  Returns (centre [B x d], cos_theta [m] in leaf
    order, cos_omega [B]); a block whose mean vanishes, or that holds a zero user, gets
    a NaN centre row and NaN angles (no cone exists)."""
    V = values(dtype, U, U_scales)
    leaf_users = np.asarray(leaf_users, np.int64)
    block_start = np.asarray(block_start, np.int64)
    nb = len(block_start) - 1
    norms = np.sqrt(np.sum(V * V, axis=1))
    cen = np.full((nb, V.shape[1]), np.nan)
    cos_t = np.full(len(leaf_users), np.nan)
    cos_w = np.full(nb, np.nan)
    for b in range(nb):
        idx = leaf_users[block_start[b]:block_start[b + 1]]
        nrm = norms[idx]
        if np.any(nrm == 0):
            continue
        mean = np.mean(V[idx] / nrm[:, None], axis=0)
        mn = np.sqrt(np.sum(mean * mean))
        if mn == 0:
            continue
        c = mean / mn
        ct = (V[idx] @ c) / nrm
        cen[b] = c
        cos_t[block_start[b]:block_start[b + 1]] = ct
        cos_w[b] = np.min(ct)
    return cen, cos_t, cos_w


def cos_to_centres(dtype, U, U_scales, leaf_users, block_start, centres):
    """cos(theta_u) of every user (leaf order) against the given block centres."""
    V = values(dtype, U, U_scales)
    leaf_users = np.asarray(leaf_users, np.int64)
    block_start = np.asarray(block_start, np.int64)
    C_ = np.asarray(centres, np.float64)
    out = np.full(len(leaf_users), np.nan)
    for b in range(len(block_start) - 1):
        idx = leaf_users[block_start[b]:block_start[b + 1]]
        nrm = np.sqrt(np.sum(V[idx] * V[idx], axis=1))
        live = nrm > 0          # a zero user has no direction and no angle (NaN)
        out[block_start[b]:block_start[b + 1]][live] = (V[idx][live] @ C_[b]) / nrm[live]
    return out


def block_lower_bounds(dtype, U, U_scales, lam, leaf_users, block_start):
    """float64 [k_max x B]: L^j(B) = min over the users of B of lambda_u^(j) / ||u||
    (Alg. 4), with lam k-major in original user order.  A block that holds a zero user
    gets -inf: such a user has no direction, so no bound may prune its block."""
    V = values(dtype, U, U_scales)
    norms = np.sqrt(np.sum(V * V, axis=1))
    lam = np.asarray(lam, np.float64)
    leaf_users = np.asarray(leaf_users, np.int64)
    block_start = np.asarray(block_start, np.int64)
    nb = len(block_start) - 1
    out = np.empty((lam.shape[0], nb))
    for b in range(nb):
        idx = leaf_users[block_start[b]:block_start[b + 1]]
        if np.any(norms[idx] == 0):
            out[:, b] = -np.inf
            continue
        out[:, b] = np.min(lam[:, idx] / norms[idx][None, :], axis=1)
    return out


def sah_rkmips(dtype, P, P_scales, U, U_scales, Q, Q_scales, ks, k_max, n_prime, b, beta, A, stats=None):
    """The approximate SAH method, per query an ascending user-ID list.

    Index (Alg. 4): items in descending canonical norm; P' = the first ``n_prime`` of
    them; L_u^j = the j-th largest s(u, p) over P' (k_max-MIPS on P', exact); the
    SA-ALSH index (Alg. 1: partitions with ratio ``b``, centroids, radii, codes from the
    projection matrix ``A``) over P minus P'.  Query (Alg. 5), for every user u:
      s(u,q) < L_u^k                   -> no  (the block and angle tests of Alg. 5 are
                                              upper bounds of s(u,q): they only skip
                                              users this test rejects as well);
      s(u,q) >= ||u|| ||p_k||          -> yes (p_k the k-th item in norm order; taken
                                              as s >= 0 and s^2 >= n2(u) n2(p_k), with
                                              n2(p_k) = 0 when k > n);
      otherwise                        -> Alg. 2 over the partitions of P minus P', its
                                          candidates starting from u's scores on P'.
    ``stats`` (a dict, optional) receives how each surviving pair was decided:
    "norm_yes" and "alg2" are the pair counts, "norm_pairs" and "alg2_pairs" the
    (query, user) lists.
    """
    P, U, Q = _c(P), _c(U), _c(Q)
    n = P.shape[0]
    n2p, order = item_order(dtype, P, P_scales)
    n2u, _ = item_order(dtype, U, U_scales)
    top = order[:n_prime]
    Pp = P[top]
    Pps = None if P_scales is None else np.asarray(P_scales)[top]
    lam = lambda_table(dtype, Pp, Pps, U, U_scales, k_max)
    ps = partitions(n2p, order, b, start=n_prime)
    _, _, icodes = saalsh_index(dtype, P, P_scales, order, ps, A)
    ucodes = user_codes(dtype, U, U_scales, A)
    ks = np.asarray(ks)
    surv = member(dtype, U, U_scales, Q, Q_scales, ks, lam)
    norm_pairs, alg2_pairs = [], []
    out = []
    for qi in range(Q.shape[0]):
        k = int(ks[qi])
        pk2 = float(n2p[order[k - 1]]) if k <= n else 0.0
        keep = []
        for u in np.flatnonzero(surv[qi]):
            s = score(dtype, U, U_scales, int(u), Q, Q_scales, qi)
            if s >= 0.0 and s * s >= float(n2u[u]) * pk2:
                keep.append(u)
                norm_pairs.append((qi, int(u)))
                continue
            alg2_pairs.append((qi, int(u)))
            init = [score(dtype, U, U_scales, int(u), Pp, Pps, j) for j in range(len(top))]
            ans, _ = saalsh_decide(dtype, P, P_scales, n2p, order, ps, icodes, ucodes[u], beta,
                                   U, U_scales, int(u), Q, Q_scales, qi, k, init=init)
            if ans:
                keep.append(u)
        out.append(np.asarray(keep, dtype=np.int32))
    if stats is not None:
        stats.update(norm_yes=len(norm_pairs), alg2=len(alg2_pairs), norm_pairs=norm_pairs,
                     alg2_pairs=alg2_pairs)
    return out


def _popcount_rows(x):
    """Set bits per row of a uint32 matrix."""
    x = np.ascontiguousarray(x, dtype=np.uint32)
    return np.unpackbits(x.view(np.uint8), axis=1).sum(axis=1).astype(np.int64)


def saalsh_kmips(dtype, P, P_scales, norm2, order, part_start, item_codes, ucode, beta, U, U_scales, u, k,
                 init=None):
    """The k best scores that Alg. 2's probes find for user u without a query (float64
    [k], descending, -inf where fewer were scored).  Partitions in order; before
    partition j the search stops once the k-th best so far exceeds mu_j = M_j ||u||; each
    partition adds the ceil(beta |S_j|) items with the most equal code bits (equal counts:
    earlier in ``order`` first), scored canonically.  ``init``: scores that are candidates
    from the start (SAH: u's scores on P')."""
    import math
    K = np.asarray(ucode).shape[-1] * 32
    b = float(np.float32(beta))   # the library takes beta as a float
    unorm = math.sqrt(score(dtype, U, U_scales, u, U, U_scales, u))
    cand = [float(v) for v in (init if init is not None else [])]

    def kth():
        return sorted(cand, reverse=True)[k - 1] if len(cand) >= k else -math.inf

    for j in range(len(part_start) - 1):
        s0, s1 = int(part_start[j]), int(part_start[j + 1])
        if kth() > math.sqrt(float(norm2[order[s0]])) * unorm:
            break
        items = np.asarray(order[s0:s1])
        agree = K - _popcount_rows(np.asarray(item_codes)[items] ^ np.asarray(ucode, np.uint32)[None, :])
        sz = s1 - s0
        take = min(int(math.ceil(b * sz)), sz)
        sel = sorted(range(sz), key=lambda i: (-int(agree[i]), i))[:take]
        cand += [score(dtype, U, U_scales, u, P, P_scales, int(items[i])) for i in sel]
    top = sorted(cand, reverse=True)[:k]
    return np.array(top + [-math.inf] * (k - len(top)), dtype=np.float64)
