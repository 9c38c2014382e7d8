"""Benchmark of the exact RkMIPS hot path on one MI355X.

One step = the whole path over one batch: build the index from items and users that
are already resident in HBM (item norms and order, exact lambda table through the
fused U.P^T matrix-core pass + FP64 refine, SA-ALSH codes, Cone-Tree blocks), then
answer one batch of queries of mixed k (bounds, matrix-core inner products, FP64
recheck, sorted result lists) and free the index.

Default workload (the largest one-GPU configuration): 1,000,000 items x 2,500,000 users
x d = 256, FP8 e4m3 codes with one FP32 scale per vector; items |N(0,1)| + 0.5, users
N(0,I) directions with log-normal(0, 1) norms, 10,000 fresh item draws as queries with k
cycling through {1, 10, 20, 50, 100}, k_max = 100.

Prints one JSON line: value = queries/s of the whole step, the lambda-index TFLOP/s,
the roofline of the dominant kernel (the fused U.P^T + top-k pass, timed with HIP
events on its stream), the CPU FP64 reference timed on a bounded user sample and the
exactness of the GPU answers on a user sample plus every user some queries returned.
Side legs (skipped with --quick): the same build and batch on the FP32 matrix cores
(plain FP32 path), continuous-batching serving of Poisson streams on the
100,000 x 1,000,000 x 128 BF16 index at three offered loads, and the 20,000 x
100,000 x 64 FP32 workload with the paper's approximate SAH mode, the lazy exact mode
and the SA-ALSH kMIPS workloads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RkMIPS queries/s (exact set vs oracle) + λ_u index TFLOP/s + p99 latency"
PEAK_FP32_MFMA = 157.3   # TFLOP/s, dense
PEAK_BF16_MFMA = 2500.0
PEAK_FP8_MFMA = 5000.0
PEAK_HBM = 8000.0        # GB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--quick", action="store_true", help="headline only: no side legs")
    ap.add_argument("--cpu-sample-users", type=int, default=0,
                    help="users in the CPU reference sample (0: size it to ~12 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 matrix-core comparison")
    ap.add_argument("--no-sah", action="store_true", help="skip the SAH, lazy and kMIPS legs")
    ap.add_argument("--sah-sweep", action="store_true",
                    help="SAH leg over K in {64,128,256} x b in {0.3,0.5,0.7} x beta in {0.05,0.1,0.2}")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this size before timing (counter scale)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class Runner:
    """One workload resident on the device, with the step and its timings."""

    def __init__(self, name, w=None, f32_from=None):
        import torch
        from paper_2211_12751_amd import inputs as I
        from paper_2211_12751_amd import rkmips as R
        self.R, self.I, self.torch = R, I, torch
        t0 = time.perf_counter()
        self.w = w if w is not None else I.make(name)
        self.name = name
        w = self.w
        if f32_from is None:
            self.dtype_name = w.dtype
            items, users, queries = w.items, w.users, w.queries
            isc, usc, qsc = w.item_scales, w.user_scales, w.query_scales
        else:
            # the same vectors stored as FP32 (BF16 -> FP32 is exact; FP8 code x scale is
            # rounded once to FP32), scored on the FP32 matrix cores
            self.dtype_name = "f32"
            items, users, queries = (_widen(w.dtype, X, s).astype(np.float32) for X, s in
                                     ((w.items, w.item_scales), (w.users, w.user_scales),
                                      (w.queries, w.query_scales)))
            isc = usc = qsc = None
        self.items, self.users, self.queries = R.to_device(items), R.to_device(users), R.to_device(queries)
        self.isc, self.usc, self.qsc = R.to_device(isc), R.to_device(usc), R.to_device(qsc)
        self.ks = torch.from_numpy(np.ascontiguousarray(w.ks)).cuda()
        self.dtype = R.DTYPES[self.dtype_name]
        self.stream = torch.cuda.current_stream()
        self.prm = R.rkmips_default_params()
        self.prm.k_max = w.k_max
        if f32_from is not None:
            self.prm.flags = R.FLAG_F32_MATRIX
        log(f"{name}{' (FP32 copy)' if f32_from else ''}: inputs ready in {time.perf_counter() - t0:.1f} s")

    def build(self, prm=None):
        w, R = self.w, self.R
        return R.rkmips_build_index(self.items, self.isc, w.n, self.users, self.usc, w.m, w.d, self.dtype, None,
                                    prm or self.prm, self.stream)

    def step(self):
        """Build, answer the batch (device-side k values), read the lists, free."""
        R, w = self.R, self.w
        h = self.build()
        r = R.rkmips_query_batch(h, self.queries, self.qsc, w.nq, self.ks, 0, self.stream)
        R.rkmips_result_wait(r)
        info = R.rkmips_get_info(h)
        st = R.rkmips_result_stats(r)
        off, ids = R.rkmips_result_view(r)
        R.rkmips_result_free(r)
        R.rkmips_index_free(h)
        return info, st, off, ids

    def timed(self, steps, warmup):
        for i in range(warmup):
            self.step()
            log(f"{self.name}: warmup step {i} done")
        self.torch.cuda.synchronize()
        infos, sts = [], []
        t0 = time.perf_counter()
        for i in range(steps):
            info, st, off, ids = self.step()
            log(f"{self.name}: step {i}: build {info['ms_total']:.1f} ms, query {st['ms_total']:.1f} ms")
            infos.append(info)
            sts.append(st)
        self.torch.cuda.synchronize()
        t = time.perf_counter() - t0
        return summarize(self.w, infos, sts, t, steps), off, ids

    def batch_latency(self, reps=10):
        """Host wall time of one query batch on a complete index (submit to answers)."""
        R = self.R
        h = self.build()
        R.rkmips_index_wait(h)
        lat = []
        try:
            for _ in range(reps):
                t0 = time.perf_counter()
                r = R.rkmips_query_batch(h, self.queries, self.qsc, self.w.nq, self.ks, 0, self.stream)
                R.rkmips_result_wait(r)
                lat.append(time.perf_counter() - t0)
                R.rkmips_result_free(r)
        finally:
            R.rkmips_index_free(h)
        return lat

    def close(self):
        del self.items, self.users, self.queries, self.isc, self.usc, self.qsc
        self.torch.cuda.empty_cache()


def summarize(w, infos, sts, t_total, steps):
    flop = 2.0 * w.m * w.n * w.d
    ms_topk = float(np.mean([i["ms_topk"] for i in infos]))
    ms_build = float(np.mean([i["ms_total"] for i in infos]))
    ms_lambda = float(np.mean([i["ms_lambda"] for i in infos]))
    q_ms = float(np.mean([s["ms_total"] for s in sts]))
    mma = {0: "f32", 1: "bf16", 2: "fp8"}[int(infos[-1]["mma_dtype"])]
    return {
        "value": steps * w.nq / t_total,
        "ms_per_step": 1e3 * t_total / steps,
        "index_tflops": flop / (ms_build * 1e-3) / 1e12,
        "lambda_pass_tflops": flop / (ms_lambda * 1e-3) / 1e12,
        "topk_tflops": flop / (ms_topk * 1e-3) / 1e12,
        "ms_topk": ms_topk, "mma": mma, "mma_terms": int(infos[-1]["mma_terms"]),
        "query_ms": q_ms, "query_only_qps": w.nq / (q_ms * 1e-3),
        "phase_ms": {k: round(float(np.mean([i[k] for i in infos])), 4)
                     for k in ("ms_norms", "ms_cone", "ms_lambda", "ms_seed", "ms_topk", "ms_refine", "ms_saalsh",
                               "ms_total")},
        "query_stats": {k: int(sts[-1][k]) for k in ("pairs_total", "pairs_block_pruned", "pairs_vector_pruned",
                                                      "pairs_scored", "pairs_rechecked", "results")},
        "cert_failures": int(infos[-1]["cert_failures"]),
        "max_rel_err_raw": infos[-1]["max_rel_err_raw"],
        "max_rel_err_lambda32": infos[-1]["max_rel_err_lambda32"],
    }


def workload_desc(name, w):
    return (f"{name}: n={w.n} items, m={w.m} users, d={w.d}, {w.dtype}, {w.nq} queries, "
            f"k in {list(w.k_values)}, k_max={w.k_max}")


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on exactly one GPU; --gpus must be 1 "
              "(sharding over several GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)

    if args.calib_copy_mib:
        src = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    run = Runner(args.config)
    w = run.w
    head, off, ids = run.timed(args.steps, args.warmup)
    qlat = run.batch_latency()
    peak = {"f32": PEAK_FP32_MFMA, "bf16": PEAK_BF16_MFMA, "fp8": PEAK_FP8_MFMA}[head["mma"]]
    traffic = None
    tf = os.path.join(ROOT, "profiles", f"traffic_{args.config}.json")
    if os.path.exists(tf):
        with open(tf) as f:
            rec = json.load(f)
        # counters taken on another build of the kernel say nothing about this one
        if rec.get("source_sha256") == topk_source_hash():
            traffic = rec.get("k_topk_bytes_per_launch")
    line = {
        "metric": METRIC,
        "value": round(head["value"], 3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16": "bf16", "fp8": "fp8e4m3"}[w.dtype],
        "data": "synthetic",
        "config": {"workload": workload_desc(args.config, w), "n": w.n, "m": w.m, "d": w.d, "nq": w.nq,
                   "k_max": w.k_max},
        "index_tflops": round(head["index_tflops"], 3),
        "lambda_pass_tflops": round(head["lambda_pass_tflops"], 3),
        "query_only_qps": round(head["query_only_qps"], 1),
        "batch_latency_p99_ms": round(float(np.percentile(np.array(qlat) * 1e3, 99)), 4),
        "phase_ms": head["phase_ms"],
        "query_ms": round(head["query_ms"], 4),
        "query_stats": head["query_stats"],
        "cert_failures": head["cert_failures"],
        "max_rel_err_raw": head["max_rel_err_raw"],
        "max_rel_err_lambda32": head["max_rel_err_lambda32"],
        "roofline": {"bound": "mfma", "achieved": round(head["topk_tflops"], 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(head["topk_tflops"] / peak, 4), "traffic": traffic,
                     "kernel": "k_topk main pass (fused U.P^T + streaming top-k), one launch per build",
                     "flop_per_launch": 2.0 * w.m * w.n * w.d, "ms_per_launch": round(head["ms_topk"], 4),
                     "mma_dtype": head["mma"], "mma_terms": head["mma_terms"]},
    }
    run.close()

    if not args.quick and not args.no_fp32:
        line["fp32_path"] = fp32_leg(args, w, head, off, ids)
    if not args.quick and not args.no_serving:
        line["serving"] = serving_leg(args, w)
        line["p99_latency_ms"] = line["serving"]["loads"][-1]["p99_ms"]
    if not args.quick and args.config != "c2":
        line["c2"] = c2_leg(args)
    elif not args.quick and not args.no_sah:
        line.update(sah_legs(Runner("c2"), off, ids, args))
    if not args.no_cpu_baseline:
        log("cpu baseline and parity sample")
        line["cpu_baseline"], line["parity_sample"] = cpu_baseline(w, off, ids, args.cpu_sample_users)
        if not args.quick:
            line["cpu_single_thread"] = single_thread_oracle()
    print(json.dumps(line), flush=True)


# ----------------------------------------------------------------------------- legs
def fp32_leg(args, w, head, off, ids):
    """The plain FP32 GPU path on the same MI355X: the same vectors stored as FP32 and
    scored on the FP32 matrix cores.  At the precision workload (BF16 -> FP32 exactly)
    the answer lists must be the same; at the default FP8 workload FP32 rounds code x
    scale once, so only the times are compared."""
    from paper_2211_12751_amd import inputs as I
    out = {}
    legs = [("c3", 1, 1)] if args.config != "c3" else []
    legs.append((args.config, 1 if args.config == "c5" else 2, 0 if args.config == "c5" else 1))
    for name, steps, warm in legs:
        log(f"FP32 path: {name}")
        if name == args.config:
            ww, b_head, b_off, b_ids = w, head, off, ids
        else:
            base = Runner(name)
            b_head, b_off, b_ids = base.timed(2, 1)
            ww = base.w
            base.close()
        f32 = Runner(name, w=ww, f32_from=True)
        f_head, f_off, f_ids = f32.timed(steps, warm)
        f32.close()
        rec = {"workload": workload_desc(name, ww),
               "fp32_ms_per_step": round(f_head["ms_per_step"], 3),
               "fp32_index_tflops": round(f_head["index_tflops"], 3),
               "fp32_topk_tflops": round(f_head["topk_tflops"], 3),
               "fp32_query_only_qps": round(f_head["query_only_qps"], 1),
               "fp32_value": round(f_head["value"], 3),
               "native_ms_per_step": round(b_head["ms_per_step"], 3),
               "native_index_tflops": round(b_head["index_tflops"], 3),
               "native_topk_tflops": round(b_head["topk_tflops"], 3),
               "native_query_only_qps": round(b_head["query_only_qps"], 1),
               "native_value": round(b_head["value"], 3),
               "speedup_step": round(f_head["ms_per_step"] / b_head["ms_per_step"], 3)}
        if ww.dtype == "bf16":
            rec["lists_equal"] = bool(np.array_equal(f_off, b_off) and np.array_equal(f_ids, b_ids))
        out[name] = rec
    return out


def serving_leg(args, w):
    """Continuous batching on the 100,000 x 1,000,000 x 128 BF16 index: 20,000 Poisson
    requests (fresh item draws, k uniform over {1, 5, 10, 20, 50}) at 25, 50 and 80 % of
    the saturated throughput, measured first as the wall rate of back-to-back batches of
    256 on all slots (after untimed warm-up replays, one at time 0 and one paced)."""
    from paper_2211_12751_amd import inputs as I
    from paper_2211_12751_amd import rkmips as R
    log("serving: c4 (the c3 index)")
    run = Runner("c3")
    wc = run.w
    nreq, max_batch, streams = 20_000, 256, 4
    g = I.rng("queries", wc.seed + 1)
    Qs = I.draw(I.CONFIGS["c4"]["items"], nreq, wc.d, g)
    Qh = np.ascontiguousarray(I.bf16_bits(Qs)).view(np.int16)
    kk = I.k_draws(nreq, values=I.CONFIGS["c4"]["ks"], seed=wc.seed + 1)
    h = run.build()
    try:
        R.rkmips_index_wait(h)
        # saturation: every request at time 0, after one untimed replay of the whole request
        # set (the server's first call allocates its slot buffers and result space)
        sp = R.rkmips_serve_params(max_batch, streams, 0, 0)
        hr, lat, st = R.rkmips_serve_replay(h, Qh, None, nreq, kk, np.zeros(nreq, np.int64), sp)
        R.rkmips_result_free(hr)
        hr, lat, st = R.rkmips_serve_replay(h, Qh[:8192], None, 8192, kk[:8192], np.zeros(8192, np.int64), sp)
        R.rkmips_result_free(hr)
        sat = 8192 / (st["wall_ms"] * 1e-3)
        # one untimed paced replay too (the first paced replay of a process has shown a
        # stall of a few milliseconds)
        arr = I.poisson_arrivals(4096, 0.25 * sat, seed=wc.seed + 4)
        hr, lat, st = R.rkmips_serve_replay(h, Qh[:4096], None, 4096, kk[:4096], arr, sp)
        R.rkmips_result_free(hr)
        loads = []
        for frac in (0.25, 0.5, 0.8):
            arr = I.poisson_arrivals(nreq, frac * sat, seed=wc.seed + 5)
            hr, lat, st = R.rkmips_serve_replay(h, Qh, None, nreq, kk, arr, sp)
            R.rkmips_result_free(hr)
            loads.append({"offered_frac": frac, "offered_qps": round(frac * sat, 1),
                          "achieved_qps": round(nreq / (st["wall_ms"] * 1e-3), 1),
                          "p50_ms": round(st["p50_us"] * 1e-3, 4), "p99_ms": round(st["p99_us"] * 1e-3, 4),
                          "mean_ms": round(st["mean_us"] * 1e-3, 4), "batches": int(st["batches"]),
                          "max_inflight": int(st["max_inflight"])})
            log(f"serving at {frac:.2f} of {sat:.0f} qps: p99 {loads[-1]['p99_ms']} ms")
    finally:
        R.rkmips_index_free(h)
        run.close()
    return {"workload": "c4: the c3 index (n=100000, m=1000000, d=128, bf16), 20000 Poisson requests, "
                        "k uniform over {1, 5, 10, 20, 50}",
            "requests": nreq, "max_batch": max_batch, "streams": streams,
            "saturated_qps": round(sat, 1), "loads": loads}


def c2_leg(args):
    """The 20,000 x 100,000 x 64 FP32 workload: whole steps, plus the SAH, lazy and
    kMIPS legs on it."""
    run = Runner("c2")
    h2, off, ids = run.timed(5, 2)
    out = {"workload": workload_desc("c2", run.w), "value": round(h2["value"], 3),
           "ms_per_step": round(h2["ms_per_step"], 4), "index_tflops": round(h2["index_tflops"], 3),
           "topk_tflops": round(h2["topk_tflops"], 3), "query_ms": round(h2["query_ms"], 4),
           "phase_ms": h2["phase_ms"], "query_stats": h2["query_stats"],
           "roofline_frac_bf16": round(h2["topk_tflops"] / PEAK_BF16_MFMA, 4)}
    if not args.no_sah:
        out.update(sah_legs(run, off, ids, args))
    run.close()
    return out


def sah_legs(run, ex_off, ex_ids, args):
    R, w = run.R, run.w
    ks_host = np.ascontiguousarray(w.ks)
    k_max = w.k_max

    def sah_leg(grid):
        ex = [ex_ids[ex_off[i]:ex_off[i + 1]] for i in range(w.nq)]
        ne = int(ex_off[w.nq])
        out = []
        for K, b, beta in grid:
            q = R.rkmips_default_params()
            q.k_max, q.mode, q.num_hash, q.b, q.probe_frac = k_max, R.MODE_SAH, K, b, beta
            runs = []
            for _ in range(3):
                h = run.build(q)
                r = R.rkmips_query_batch(h, run.queries, run.qsc, w.nq, run.ks, 0, run.stream)
                R.rkmips_result_wait(r)
                info, st = R.rkmips_get_info(h), R.rkmips_result_stats(r)
                off, ids = R.rkmips_result_view(r)
                R.rkmips_result_free(r)
                R.rkmips_index_free(h)
                runs.append((info, st, off, ids))
            info, st, off, ids = runs[-1]
            tp = sum(len(np.intersect1d(ids[off[i]:off[i + 1]], ex[i], assume_unique=True)) for i in range(w.nq))
            ng = int(off[w.nq])
            out.append({"K": K, "b": b, "beta": beta, "p_prime": int(info["lambda_items"]),
                        "partitions": int(info["num_partitions"]),
                        "build_ms": round(float(np.median([x[0]["ms_total"] for x in runs])), 4),
                        "query_ms": round(float(np.median([x[1]["ms_total"] for x in runs])), 4),
                        "results": ng, "exact_results": ne,
                        "precision": round(tp / ng, 5) if ng else 1.0, "recall": round(tp / ne, 5) if ne else 1.0,
                        "f1": round(2.0 * tp / (ng + ne), 5) if ng + ne else 1.0,
                        "pairs_to_alg2": int(st["saalsh_checked"]), "alg2_no": int(st["saalsh_rejects"])})
        return out

    def lazy_leg():
        q = R.rkmips_default_params()
        q.k_max, q.mode = k_max, R.MODE_LAZY
        runs, same = [], True
        for _ in range(3):
            h = run.build(q)
            r = R.rkmips_query_batch(h, run.queries, run.qsc, w.nq, run.ks, 0, run.stream)
            R.rkmips_result_wait(r)
            info, st = R.rkmips_get_info(h), R.rkmips_result_stats(r)
            off, ids = R.rkmips_result_view(r)
            same = same and np.array_equal(off, ex_off) and np.array_equal(ids, ex_ids)
            R.rkmips_result_free(r)
            R.rkmips_index_free(h)
            runs.append((info, st))
        return {"p_prime": int(runs[-1][0]["lambda_items"]),
                "build_ms": round(float(np.median([x[0]["ms_total"] for x in runs])), 4),
                "query_ms": round(float(np.median([x[1]["ms_total"] for x in runs])), 4),
                "pairs_to_alg2": int(runs[-1][1]["saalsh_checked"]), "lists_equal_exact_mode": bool(same)}

    def kmips_leg():
        """(1) SA-ALSH kMIPS on a seeded sample of 5,000 users: recall@k of the k best
        scores found against the exact ones (the lambda rows) and the time per call.
        (2) F1 of each query's own kMIPS over the users (the k users with the largest
        <q, u>, numpy FP64 on the host, first 100 queries) against its RkMIPS list."""
        I = run.I
        h = run.build()
        out = {"recall": []}
        try:
            exact = np.stack([R.rkmips_get_lambda(h, k, w.m) for k in range(1, k_max + 1)])
            g = I.rng("queries", w.seed + 2)
            us = np.sort(g.choice(w.m, min(5000, w.m), replace=False))
            for beta in (0.05, 0.1, 0.2):
                for k in [k for k in (1, 5, 10, 20, 50) if k <= k_max]:
                    R.rkmips_saalsh_kmips(h, us[:64], k, beta, run.stream)
                    t0 = time.perf_counter()
                    sc = R.rkmips_saalsh_kmips(h, us, k, beta, run.stream)
                    dt = time.perf_counter() - t0
                    rec = float(np.mean([len(np.intersect1d(sc[i], exact[:k, u])) / k for i, u in enumerate(us)]))
                    out["recall"].append({"beta": beta, "k": k, "recall": round(rec, 5),
                                          "ms_per_call": round(dt * 1e3, 3), "users": int(len(us))})
        finally:
            R.rkmips_index_free(h)
        nqs = min(100, w.nq)
        S = _widen(w.dtype, w.queries[:nqs], None) @ _widen(w.dtype, w.users, None).T
        f1 = []
        for qi in range(nqs):
            k = int(ks_host[qi])
            top = np.argpartition(-S[qi], k - 1)[:k]
            rk = ex_ids[ex_off[qi]:ex_off[qi + 1]]
            f1.append(2.0 * len(np.intersect1d(top, rk)) / (k + len(rk)))
        out["kmips_as_rkmips_f1"] = round(float(np.mean(f1)), 5)
        out["kmips_as_rkmips_queries"] = nqs
        return out

    log("SAH, lazy and kMIPS legs")
    grid = ([(K, b, beta) for K in (64, 128, 256) for b in (0.3, 0.5, 0.7) for beta in (0.05, 0.1, 0.2)]
            if args.sah_sweep else [(128, 0.5, beta) for beta in (0.05, 0.1, 0.2)])
    return {"sah": sah_leg(grid), "lazy": lazy_leg(), "kmips": kmips_leg()}


# ----------------------------------------------------------------------------- helpers
def _widen(dtype, X, scales):
    """Stored rows as float64 (BF16 bit patterns, or FP8 e4m3 codes times the row scale)."""
    if dtype == "f32":
        return X.astype(np.float64)
    if dtype == "bf16":
        return (X.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    c = np.arange(256)
    e, m = (c >> 3) & 15, c & 7
    mag = np.where(e == 0, m / 8.0 * 2.0 ** -6, (1 + m / 8.0) * 2.0 ** (e - 7.0))
    table = np.where(c >= 128, -mag, mag)
    out = table[X]
    return out if scales is None else out * np.asarray(scales, np.float64)[:, None]


TOPK_SOURCES = ("k_topk.hip", "topk.h", "common.h")


def topk_source_hash():
    """Hash of the sources that fix the fused top-k kernel and its launch shape."""
    import hashlib
    h = hashlib.sha256()
    for f in TOPK_SOURCES:
        with open(os.path.join(ROOT, "paper_2211_12751_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _blas_threads():
    try:
        import threadpoolctl
        return max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info() if i.get("user_api") == "blas"]
                   or [1])
    except Exception:
        return 1


def cpu_baseline(w, off, ids, sample_users):
    """The CPU FP64 reference as it stands, on a seeded sample of users: lambda over all
    items plus membership for every query, extrapolated linearly in users.  Parity: the
    GPU lists are checked on that sample (every query) and on every user that the first
    queries returned (each such user's full membership row)."""
    from oracle import oracle as O
    threads = _blas_threads() if w.dtype == "fp8" else O.NTHREADS
    g = np.random.default_rng(20221)

    def oracle_rows(users):
        lam = O.lambda_table(w.dtype, w.items, w.item_scales, w.users, w.user_scales, w.k_max, user_idx=users)
        return O.member(w.dtype, w.users, w.user_scales, w.queries, w.query_scales, w.ks, lam, user_idx=users)

    if sample_users <= 0:
        cnt = 64 if w.m * w.n > 1e11 else 256
        cal = np.sort(g.choice(w.m, min(cnt, w.m), replace=False))
        t0 = time.perf_counter()
        oracle_rows(cal)
        per_user = max((time.perf_counter() - t0) / len(cal), 1e-9)
        sample_users = int(min(w.m, max(64, 12.0 / per_user)))
    sample = np.sort(g.choice(w.m, sample_users, replace=False))
    t0 = time.perf_counter()
    mem = oracle_rows(sample)
    t = time.perf_counter() - t0
    t_full = t * w.m / len(sample)

    def check(users, mem_rows):
        pos = np.full(w.m, -1, np.int64)
        pos[users] = np.arange(len(users))
        bad = 0
        for qi in range(w.nq):
            got = np.zeros(len(users), np.uint8)
            p = pos[ids[off[qi]:off[qi + 1]]]
            got[p[p >= 0]] = 1
            bad += int(np.count_nonzero(got != mem_rows[qi]))
        return bad

    bad_sample = check(sample, mem)
    # every user that the first queries returned: their whole membership rows
    nq_ret, ret = 0, np.zeros(0, np.int64)
    while nq_ret < w.nq and len(ret) < 1500:
        ret = np.union1d(ret, ids[off[nq_ret]:off[nq_ret + 1]])
        nq_ret += 1
    bad_ret = check(ret, oracle_rows(ret)) if len(ret) else 0
    base = {"value": round(w.nq / t_full, 6), "unit": "queries/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{len(sample)} of {w.m} users (seeded), lambda over all {w.n} items + membership "
                      f"for all {w.nq} queries; {t:.2f} s, extrapolated linearly in users "
                      f"(full job ~{t_full:.0f} s)"}
    par = {"sample_users": int(len(sample)), "returned_users": int(len(ret)),
           "returned_users_of_queries": int(nq_ret), "queries": int(w.nq),
           "pairs_checked": int((len(sample) + len(ret)) * w.nq), "mismatches": bad_sample + bad_ret,
           "exact_match": bad_sample + bad_ret == 0}
    return base, par


def single_thread_oracle():
    """The oracle on one thread, as the paper times its methods: the whole 2,000 x 5,000 x
    32 workload (100 queries), and the 20,000 x 100,000 x 64 one on a seeded 400-user
    sample extrapolated linearly in users (about a second each)."""
    from oracle import oracle as O
    from paper_2211_12751_amd import inputs as I
    out = {}
    for name, users in (("c1", None), ("c2", 400)):
        w = I.make(name)
        sel = None if users is None else np.sort(np.random.default_rng(20222).choice(w.m, users, replace=False))
        t0 = time.perf_counter()
        lam = O.lambda_table(w.dtype, w.items, w.item_scales, w.users, w.user_scales, w.k_max, user_idx=sel,
                             nthreads=1)
        O.member(w.dtype, w.users, w.user_scales, w.queries, w.query_scales, w.ks, lam, user_idx=sel, nthreads=1)
        t = time.perf_counter() - t0
        full = t * (w.m / len(sel) if sel is not None else 1.0)
        out[name] = {"workload": workload_desc(name, w), "threads": 1, "seconds": round(full, 3),
                     "queries_per_s": round(w.nq / full, 4),
                     "sample": "all users" if sel is None else f"{len(sel)} of {w.m} users, extrapolated"}
        log(f"single-thread oracle {name}: {full:.2f} s for {w.nq} queries")
    return out


if __name__ == "__main__":
    main()
