#!/usr/bin/env python3
"""Throughput of the SINDI search path on one MI355X.

One step = one ``sindi_search`` over the whole query set of the workload
(coarse accumulate over the mass-ratio-pruned window lists, per-query
candidate threshold, top-gamma, exact FP32 rerank, top-k), with the index
and the queries already resident in HBM.  Prints one JSON line.

Default workload: 8.8M synthetic SPLADE-shaped documents (vocabulary 30,522,
~125 non-zeros each), 7,000 queries (~35 non-zeros), alpha = 0.5,
lambda = 100,000, gamma = 500, k = 50, FP16 posting values.  The real
MS MARCO / SPLADE data is not used; the generator draws the same shapes.
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
CU_COUNT, CLOCK_HZ = 256, 2.4e9  # MI355X compute units, peak engine clock


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def batch_union_postings(qc, term_len, batch):
    """Sum over batches of B consecutive queries of sum_{j in union} |I'_j|."""
    tot = 0
    n = qc.n_rows
    for b0 in range(0, n, batch):
        a, b = int(qc.indptr[b0]), int(qc.indptr[min(n, b0 + batch)])
        u = np.unique(qc.indices[a:b])
        tot += int(term_len[u].sum())
    return tot


def per_query_postings(qc, term_len):
    return int(term_len[qc.indices].sum())


def coarse_queries(qc, beta):
    """The query terms a scoring pass reads: each row's beta-mass prefix (Sec. 4.1; entries
    by |q| descending, ties by term id, FP64 sums in that order, the shortest prefix reaching
    beta times the row's mass), as a CSR of term ids only.  beta = 1 keeps every term."""
    from types import SimpleNamespace
    if beta >= 1.0:
        return qc
    ptr, idx = [0], []
    for r in range(qc.n_rows):
        a, b = int(qc.indptr[r]), int(qc.indptr[r + 1])
        t, v = qc.indices[a:b], np.abs(qc.values[a:b].astype(np.float64))
        t, v = t[v > 0], v[v > 0]
        order = np.lexsort((t, -v))
        cs = np.cumsum(v[order])
        n = int(np.searchsorted(cs, beta * cs[-1], side="left")) + 1 if len(cs) else 0
        idx.append(np.sort(t[order[:n]]))
        ptr.append(ptr[-1] + n)
    return SimpleNamespace(n_rows=qc.n_rows, indptr=np.asarray(ptr, np.int64),
                           indices=np.concatenate(idx) if idx else np.zeros(0, np.int32))


def kernel_code_sha256(path):
    """sha256 of a source file without its comments, whitespace runs collapsed: edits to
    comments and layout leave a counter summary of the compiled code valid."""
    import hashlib
    import re
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = re.sub(r"\s+", " ", src).strip()
    return hashlib.sha256(src.encode()).hexdigest()


def probe_lds(stream=None):
    """LDS atomic-add rates of gfx950 (libsindi_probe.so): 32-bit integer adds with 64
    consecutive words per instruction (no bank shared), with the 4-word lane stride of a
    dense list read 4 postings per lane, and at pseudo-random words (the scatter of
    postings), plus FP32 adds at random words.  Adds per second, over 4,096 workgroups of
    512 threads (three per compute unit, as the scoring kernel's)."""
    from paper_2509_08395_amd import _lib
    lib = _lib.load_probe()
    out = {}
    for name, op, stride in (("int_conflict_free", 0, 1), ("int_stride4", 0, 4),
                             ("int_random", 0, 0), ("f32_random", 1, 0)):
        best = None
        for _ in range(3):
            ms, upd = _lib.probe_lds_add(lib, op, stride, 4096, 400 if op == 0 else 40)
            rate = upd / (ms * 1e-3)
            best = rate if best is None else max(best, rate)
        out[name] = round(best, 1)
    out["unit"] = "atomic adds/s (whole GPU)"
    out["per_cu_clock"] = {k: round(v / (CU_COUNT * CLOCK_HZ), 3) for k, v in out.items()
                           if isinstance(v, float)}
    return out


def measured_traffic(config):
    """HBM bytes per scoring launch from the committed rocprofv3 counter summary, if it was
    taken on this kernel code and configuration; else None."""
    src = os.path.join(ROOT, "paper_2509_08395_amd", "csrc", "sindi_kernels.hip")
    path = os.path.join(ROOT, "profiles",
                        f"k_accumulate1_queue_{config['workload']}_{config['value_storage']}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("    "):
            key, val = line.strip().split(":", 1)
            fields[key.strip()] = val.strip()
    sha = kernel_code_sha256(src)
    want = (f"batch={config['batch']} tile={config['tile']} value_storage={config['value_storage']} "
            f"n_queries={config['n_queries']} n_docs={config['n_docs']} alpha={config['alpha']} "
            f"beta={config['beta']}")
    if fields.get("kernel_code_sha256") != sha or fields.get("config") != want:
        return None
    return int(fields["fetch_bytes_per_launch"]) + int(fields["write_bytes_per_launch"])


def device_build_leg(sindi, torch, corpus, alpha, window, dtype, tile):
    """Wall time of the device index build (the index searched is the host build; the two are
    identical bit for bit): from the host CSR (upload included) and from a corpus already in
    HBM.  Each index is freed before the next."""
    out = {}
    torch.cuda.synchronize()
    t = time.time()
    ix = sindi.Index(corpus, alpha=alpha, window=window, value_dtype=dtype, tile=tile,
                     gpu_build=True)
    out["device_from_host_s"] = round(time.time() - t, 3)
    del ix
    dc = sindi.DeviceCsr.from_host(corpus)
    torch.cuda.synchronize()
    t = time.time()
    ix = sindi.Index(dc, alpha=alpha, window=window, value_dtype=dtype, tile=tile,
                     gpu_build=True)
    out["device_from_hbm_s"] = round(time.time() - t, 3)
    del ix, dc
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="splade-8.8m")
    ap.add_argument("--value-dtype", default=None, help="posting value storage f32/f16/bf16")
    ap.add_argument("--n-docs", type=int, default=0, help="override corpus size (development)")
    ap.add_argument("--vocab", type=int, default=0, help="override vocabulary size (sparsity sweeps)")
    ap.add_argument("--queries", type=int, default=0, help="override query count")
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--alpha", type=float, default=None)
    ap.add_argument("--gamma", type=int, default=0)
    ap.add_argument("--beta", type=float, default=None, help="query pruning (Sec. 4.1)")
    ap.add_argument("--recall-queries", type=int, default=0,
                    help="queries the live exact oracle scores (0: 16 to re-check the stored "
                         "exact top-k of every query, or 1,000 without it)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the alpha / gamma / beta / storage sweep")
    ap.add_argument("--no-shapes", action="store_true",
                    help="skip the second workload shapes and the pruning-rule comparison")
    ap.add_argument("--oracle-queries", type=int, default=7000)
    ap.add_argument("--no-oracle", action="store_true", help="skip recall and the CPU baseline")
    ap.add_argument("--serve-seconds", type=float, default=4.0,
                    help="open-loop serving run per arrival rate (0: skip serving)")
    ap.add_argument("--serve-rates", default="",
                    help="comma-separated arrival rates, queries/s (default: the serving workload's)")
    ap.add_argument("--serve-beta", type=float, default=0.8,
                    help="query mass ratio of the served searches' coarse stage (Sec. 4.1)")
    ap.add_argument("--serve-recall-queries", type=int, default=48,
                    help="serving-shaped queries checked against the exact oracle")
    ap.add_argument("--serve-inflight", type=int, default=3, help="server batch slots")
    ap.add_argument("--serve-max-batch", type=int, default=256, help="server batch cap")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the FP32 / BF16 posting-storage comparison")
    ap.add_argument("--no-diff", action="store_true",
                    help="skip the differentiation (score forward/backward) timing")
    ap.add_argument("--ablation", action="store_true",
                    help="only the pruning-rule comparison (MRP / VNP / LP / MRP+LP, Sec. 4.1): "
                         "Recall@10 and QPS on a 1M-document SPLADE-shaped corpus")
    ap.add_argument("--no-gpu-build", action="store_true",
                    help="skip timing the index build on the device")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))
        return

    if args.ablation:
        print(json.dumps(ablation(args)), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library does "
              "not shard the index across GPUs.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from synth.workloads import WORKLOADS
    import paper_2509_08395_amd as sindi
    from paper_2509_08395_amd import _lib

    wl = WORKLOADS[args.workload]
    if args.n_docs:
        wl = wl.scaled(args.n_docs)
    if args.vocab:
        from dataclasses import replace
        wl = replace(wl, vocab=args.vocab, name=f"{wl.name}-d{args.vocab}")
    n_q = args.queries or wl.n_queries
    dtype = args.value_dtype or wl.value_dtype
    alpha = wl.alpha if args.alpha is None else args.alpha
    gamma = args.gamma or wl.gamma
    beta = wl.beta if args.beta is None else args.beta
    k = wl.k

    t = time.time()
    corpus = wl.corpus()
    queries = wl.queries(n_q)
    gen_s = time.time() - t
    log(f"generated {corpus.n_rows} docs ({corpus.nnz} nnz), {queries.n_rows} queries in {gen_s:.1f}s")

    torch.cuda.init()
    t = time.time()
    idx = sindi.Index(corpus, alpha=alpha, window=wl.window, value_dtype=dtype, tile=args.tile)
    build_s = time.time() - t
    info = idx.info()
    log(f"built index in {build_s:.1f}s: {info}")
    build = {"host_s": round(build_s, 3)}
    if not args.no_gpu_build:
        build.update(device_build_leg(sindi, torch, corpus, alpha, wl.window, dtype, args.tile))
        log(f"device build: {build}")
    dq = sindi.DeviceCsr.from_host(queries)
    ids = torch.empty((n_q, k), dtype=torch.int64, device="cuda")
    scores = torch.empty((n_q, k), dtype=torch.float32, device="cuda")
    kw = dict(gamma=gamma, beta=beta, batch=args.batch, out=(ids, scores))

    for _ in range(args.warmup):
        idx.search(dq, k, **kw)
    torch.cuda.synchronize()
    log("warmup done")

    sindi.profile_enable(True)
    sindi.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        idx.search(dq, k, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sindi.profile_read(reset=True)
    sindi.profile_enable(False)
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    qps = n_q * args.steps / elapsed
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, {qps:.0f} QPS; kernels {prof}")

    # roofline of the dominant kernel (the scoring pass)
    term_len = idx.term_lengths()
    vbytes = {"f32": 4, "f16": 2, "bf16": 2}[dtype]
    bpp = 2 + vbytes
    batch = args.batch or 1
    cq = coarse_queries(queries, beta)
    union_post = batch_union_postings(cq, term_len, batch)
    query_post = per_query_postings(cq, term_len)
    offs_bytes = int(cq.indptr[-1]) * int(info["n_tiles"]) * 8
    algo_bytes = union_post * bpp + offs_bytes
    # one step may split the queries over several scoring launches (candidate memory)
    n_launch, acc_ms = prof["accumulate_score"]
    launches_per_step = max(n_launch // args.steps, 1)
    acc_ms_avg = acc_ms / max(n_launch, 1)
    launch_s = acc_ms_avg * 1e-3
    bytes_per_launch = algo_bytes // launches_per_step
    post_per_launch = query_post // launches_per_step
    config = {"workload": wl.name, "n_docs": corpus.n_rows, "vocab": wl.vocab,
              "n_queries": n_q, "value_storage": dtype, "alpha": alpha,
              "window": wl.window, "gamma": gamma, "k": k, "beta": beta,
              "batch": batch, "tile": info["tile_max"], "n_tiles": info["n_tiles"],
              "n_postings": info["n_postings"]}
    traffic = measured_traffic(config)
    achieved = traffic / launch_s / 1e9 if traffic and launch_s > 0 else None
    adds_per_s = post_per_launch / launch_s if launch_s > 0 else 0.0
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1) if achieved else None,
        "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None, "traffic": traffic,
        "achieved_is": "HBM bytes beyond L2 per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                       "copy-calibrated, profiles/) over the launch time by HIP events",
        "kernel": "k_accumulate1_queue (scoring pass, one persistent launch)",
        "launch_ms": round(acc_ms_avg, 3),
        "launches_per_step": launches_per_step, "batch": batch,
        "algorithmic_bytes_per_launch": bytes_per_launch,
        "algorithmic_GBs": round(bytes_per_launch / launch_s / 1e9, 1) if launch_s else None,
        "algorithmic_note": "every query's lists once (2 B id + value bytes per posting, 8 B of "
                            "list bounds per query term and tile); lists shared by queries "
                            "scoring the same tile at once are served from L2",
        "postings_per_launch": post_per_launch,
        "useful_postings_per_s": round(adds_per_s, 1),
        "paper_layout_8B_GBs": round(adds_per_s * 8 / 1e9, 1),
    }
    try:
        probe = probe_lds()
        roofline["lds"] = {
            "posting_adds_per_s": round(adds_per_s, 1),
            "conflict_free_adds_per_s": probe["int_conflict_free"],
            "random_adds_per_s": probe["int_random"],
            "frac": round(adds_per_s / probe["int_conflict_free"], 4),
            "frac_of_random_rate": round(adds_per_s / probe["int_random"], 4),
            "probe": probe}
        log(f"LDS probe: {probe}")
    except Exception as e:  # the probe library is measurement only
        log(f"LDS probe unavailable: {e}")

    result = {
        "metric": "QPS at Recall@50>=99% vs exact oracle, 8.8M docs; % HBM roofline; p99 ms",
        "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": config,
        "latency_ms_batch": round(ms_per_step, 3),
        "kernels_ms_per_step": {n: round(v[1] / args.steps, 3) for n, v in prof.items()},
        "build_s": round(build_s, 2),
        "build": build,
        "roofline": roofline,
    }

    if args.serve_seconds > 0 and dtype == "f16" and wl.name == "splade-8.8m":
        optional_leg(result, "serving", lambda: serving_leg(sindi, idx, args, corpus))
        if "rates" in result["serving"]:
            result["latency_p99_ms"] = {str(int(r["offered_qps"])): r["p99_ms"]
                                        for r in result["serving"]["rates"]}

    main_leg = wl.name == "splade-8.8m" and dtype == "f16"
    if not args.no_diff and main_leg:
        optional_leg(result, "differentiation", lambda: diff_leg(sindi))

    if not args.no_oracle:
        import oracle  # CPU baseline, recall and agreement only
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        gids = ids.cpu().numpy()
        stored = load_truth(wl, corpus, queries, k) if n_q == wl.n_queries else None
        n_rec = args.recall_queries or (16 if stored is not None else 1000)
        rsel = np.linspace(0, n_q - 1, min(n_rec, n_q)).astype(np.int64)
        qs = queries.take_rows(rsel)
        t = time.time()
        truth, _ = oracle.exact_topk(corpus, qs, k, threads=threads)
        exact_s = time.time() - t
        if stored is not None and not np.array_equal(stored[rsel], truth):
            log("stored exact top-k disagrees with the oracle on the sampled queries: not used")
            stored = None
        if stored is not None:
            tsel, truth_t = np.arange(n_q), stored
            rec_note = (f"all {n_q} queries; exact FP64 top-{k} written by the oracle "
                        f"(tests/golden, re-checked live on {len(rsel)} queries)")
        else:
            tsel, truth_t = rsel, truth
            rec_note = f"{len(rsel)} of {n_q} queries, evenly spaced; exact FP64 oracle"
        rec = oracle.recall_at_k(gids[tsel], truth_t)
        log(f"recall@{k} on {len(tsel)} queries: {rec:.5f} (live exact oracle {exact_s:.1f}s "
            f"for {len(rsel)})")
        osel = np.arange(min(args.oracle_queries, n_q))
        qo = queries.take_rows(osel)
        t = time.time()
        keep = oracle.mass_prune(corpus, alpha, threads=threads)
        oidx = oracle.build_index(corpus, wl.window, keep)
        oracle_build_s = time.time() - t
        pruned = oracle.apply_mask(corpus, keep) if not args.no_precision and main_leg else None
        del keep
        t = time.time()
        o_ids, _ = oracle.approx_search(oidx, corpus, qo, beta, gamma, k, threads=threads)
        oracle_s = time.time() - t
        agree = oracle.recall_at_k(gids[osel], o_ids)
        log(f"oracle Alg. 4 on {len(osel)} queries: {oracle_s:.1f}s (index {oracle_build_s:.1f}s), "
            f"GPU agreement {agree:.5f}")
        # single-thread figures, beside the paper's single-thread numbers
        n1 = min(100, n_q)
        t = time.time()
        oracle.approx_search(oidx, corpus, queries.take_rows(np.arange(n1)), beta, gamma, k,
                             threads=1)
        st_alg4 = n1 / (time.time() - t)
        ne = min(8, n_q)
        t = time.time()
        oracle.exact_topk(corpus, queries.take_rows(np.arange(ne)), k, threads=1)
        st_exact = ne / (time.time() - t)
        del oidx
        result["recall_at_k"] = round(rec, 5)
        result["recall_sample"] = rec_note
        result["alg4_agreement"] = round(agree, 5)
        result["alg4_agreement_sample"] = (f"{len(osel)} of {n_q} queries: share of the CPU "
                                           f"oracle's Alg. 4 top-{k} ids (FP64, same alpha, beta, "
                                           "gamma) found in the GPU's")
        result["cpu_baseline"] = {
            "value": round(len(osel) / oracle_s, 3), "unit": "queries/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {len(osel)} of {n_q} queries, FP64 Alg. 4 (same alpha, beta, gamma, "
                      f"k), {oracle_s:.1f}s on {threads} threads",
            "single_thread_alg4_qps": round(st_alg4, 3),
            "single_thread_alg4_sample": f"first {n1} queries",
            "exact_topk_qps": round(len(rsel) / exact_s, 3),
            "exact_topk_sample": f"{len(rsel)} evenly spaced queries on {threads} threads",
            "single_thread_exact_qps": round(st_exact, 4),
            "single_thread_exact_sample": f"first {ne} queries",
            "cpu": _cpu_model()}
        if rec < 0.99:
            result["note"] = f"recall {rec:.4f} below 0.99"
        if not args.no_precision and main_leg:
            dqs = sindi.DeviceCsr.from_host(qs)
            prec = {"f16": {"qps": result["value"], "ms_per_step": result["ms_per_step"],
                            "score_pass_ms": result["kernels_ms_per_step"]["accumulate_score"],
                            "recall_at_k": result["recall_at_k"], "bytes_per_posting": 4,
                            **coarse_error(idx, dqs, qs, pruned, k)}}
            try:
                prec.update(precision_leg(sindi, corpus, dq, wl, alpha, gamma, k, tsel, truth_t,
                                          n_q, dqs, qs, pruned, beta=beta))
            except Exception as e:  # noqa: BLE001 -- reported in the JSON line
                log(f"precision leg failed: {type(e).__name__}: {e}")
                prec["error"] = f"{type(e).__name__}: {e}"
            result["precision"] = prec
        if not args.no_shapes and main_leg:
            optional_leg(result, "shapes", lambda: shapes_leg(sindi))
            # one strength of each pruning rule at about the same kept fraction
            optional_leg(result, "ablation", lambda: ablation(args, gammas=(10, 30), grid=[
                ("mrp", dict(alpha=0.5)), ("vnp", dict(vn=22)), ("lp", dict(list_len=20_000)),
                ("mrp+lp", dict(alpha=0.5, list_len=20_000))]))
        if not args.no_sweep and main_leg:
            optional_leg(result, "layout",
                         lambda: layout_leg(sindi, corpus, dq, alpha, dtype, gamma, k, ids, scores,
                                            beta=beta))
            idx.close()  # room for the sweep's indexes
            optional_leg(result, "sweep",
                         lambda: sweep_leg(sindi, corpus, dq, wl, k, tsel, truth_t, rec_note))
            best = result["sweep"].get("best_at_recall_0.99", {}).get(dtype)
            if best:
                result["qps_best_at_recall_0.99"] = {**best, "note": "fastest sweep point with "
                                                     "Recall@50 >= 0.99 (value is the configuration "
                                                     "point: alpha 0.5, gamma 500, beta 1)"}
    print(json.dumps(result), flush=True)


def optional_leg(result, name, fn):
    """Run one secondary leg into result[name]; a failure is logged and recorded there, so the
    main measurement is never lost to it."""
    try:
        result[name] = fn()
    except Exception as e:  # noqa: BLE001 -- reported in the JSON line
        log(f"{name} leg failed: {type(e).__name__}: {e}")
        result[name] = {"error": f"{type(e).__name__}: {e}"}


def load_truth(wl, corpus, queries, k):
    """The exact top-k of every query of the workload as the oracle wrote it
    (tests/golden/make_exact_truth.py), if present and written for this very input (sizes,
    seed and a fingerprint of the generated arrays); else None."""
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import make_exact_truth as mt
    path = mt.truth_path(wl.name, k)
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
        ids = z["ids"].astype(np.int64)
    want = {"n_docs": corpus.n_rows, "vocab": wl.vocab, "n_queries": queries.n_rows, "k": k,
            "seed": wl.seed}
    if any(meta.get(key) != v for key, v in want.items()):
        return None
    if meta.get("fingerprint") != mt.fingerprint(corpus, queries):
        return None
    return ids


def sweep_leg(sindi, corpus, dq, wl, k, tsel, truth, rec_note, steps=3):
    """The parameters of Sec. 5.3 and Sec. 4.1 around the configuration point: alpha in {0.2,
    0.3, 0.4, 0.5}, gamma in {200, 500}, beta in {0.8, 1.0}, FP16 and FP32 posting values
    (each index built on the device), each searched over the whole query set: QPS and
    Recall@k, then per storage type the fastest point with Recall@k >= 0.99."""
    import torch
    import oracle
    n_q = dq.n_rows
    ids = torch.empty((n_q, k), dtype=torch.int64, device="cuda")
    sc = torch.empty((n_q, k), dtype=torch.float32, device="cuda")
    rows = []
    for dt in ("f16", "f32"):
        for a in (0.2, 0.3, 0.4, 0.5):
            idx = sindi.Index(corpus, alpha=a, window=wl.window, value_dtype=dt, gpu_build=True)
            for g in (200, 500):
                for b in (0.8, 1.0):
                    idx.search(dq, k, beta=b, gamma=g, out=(ids, sc))
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(steps):
                        idx.search(dq, k, beta=b, gamma=g, out=(ids, sc))
                    torch.cuda.synchronize()
                    el = time.perf_counter() - t0
                    rec = oracle.recall_at_k(ids.cpu().numpy()[tsel], truth)
                    rows.append({"value_storage": dt, "alpha": a, "gamma": g, "beta": b,
                                 "qps": round(n_q * steps / el, 1), "recall_at_k": round(rec, 5)})
                    log(f"sweep {rows[-1]}")
            idx.close()
            del idx
    best = {}
    for dt in ("f16", "f32"):
        ok = [r for r in rows if r["value_storage"] == dt and r["recall_at_k"] >= 0.99]
        best[dt] = max(ok, key=lambda r: r["qps"]) if ok else None
    cfg = {dt: next(r for r in rows if r["value_storage"] == dt and r["alpha"] == 0.5
                    and r["gamma"] == 500 and r["beta"] == 1.0) for dt in ("f16", "f32")}
    return {"grid": "alpha {0.2,0.3,0.4,0.5} x gamma {200,500} x beta {0.8,1.0} x {f16,f32}",
            "recall_sample": rec_note, "steps": steps, "config_point": cfg,
            "best_at_recall_0.99": best, "rows": rows}


def layout_leg(sindi, corpus, dq, alpha, dtype, gamma, k, ref_ids, ref_scores, beta=1.0,
               steps=3):
    """Window lambda and score tile T (the GPU's analog of Sec. 3.3.1's window size): tiles of at
    most T documents split each window equally, and one workgroup holds one tile's scores in
    LDS.  Each layout is built on the device and searched over the whole query set; Thm. 3.1
    makes the work, and the fixed-point sums make the results, the same in every layout, which
    the leg checks against the configuration point's ids and scores bit for bit."""
    import torch
    n_q = dq.n_rows
    ids = torch.empty_like(ref_ids)
    sc = torch.empty_like(ref_scores)
    rows = []
    for window, tile in ((100_000, 5_000), (100_000, 6_250), (100_000, 8_334), (100_000, 10_000),
                         (100_000, 12_500), (100_000, 14_286), (25_000, 12_500), (30_000, 12_500),
                         (1_000_000, 12_500), (corpus.n_rows, 12_500)):
        idx = sindi.Index(corpus, alpha=alpha, window=window, value_dtype=dtype, tile=tile,
                          gpu_build=True)
        info = idx.info()
        idx.search(dq, k, gamma=gamma, beta=beta, out=(ids, sc))
        torch.cuda.synchronize()
        sindi.profile_enable(True)
        sindi.profile_read(reset=True)
        t0 = time.perf_counter()
        for _ in range(steps):
            idx.search(dq, k, gamma=gamma, beta=beta, out=(ids, sc))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = sindi.profile_read(reset=True)
        sindi.profile_enable(False)
        n_launch, acc_ms = prof["accumulate_score"]
        rows.append({"window": window, "tile_max": info["tile_max"], "n_tiles": info["n_tiles"],
                     "qps": round(n_q * steps / el, 1),
                     "score_pass_ms": round(acc_ms / max(n_launch, 1), 3),
                     "same_results": bool(torch.equal(ids, ref_ids)
                                          and torch.equal(sc.view(torch.int32),
                                                          ref_scores.view(torch.int32)))})
        log(f"layout {rows[-1]}")
        idx.close()
        del idx
    return {"grid": "(window, tile) pairs, tiles splitting each window equally", "steps": steps,
            "rows": rows}


def coarse_error(idx, dqs, qs, pruned, k):
    """Relative error of the coarse scores (Alg. 2 over the index, no rerank) of the sampled
    queries' top-k against the FP64 inner products of the pruned vectors: max and 99th
    percentile over the returned (query, document) pairs."""
    import oracle
    ids, sc = idx.search_coarse(dqs, k)
    ids, sc = ids.cpu().numpy(), sc.cpu().numpy()
    r, c = np.nonzero(ids >= 0)
    exact = oracle.pair_scores(pruned, qs, r, ids[r, c])
    rel = np.abs(sc[r, c].astype(np.float64) - exact) / np.maximum(np.abs(exact), 1e-30)
    return {"coarse_rel_err_max": float(f"{rel.max():.3g}"),
            "coarse_rel_err_p99": float(f"{np.percentile(rel, 99):.3g}")}


def precision_leg(sindi, corpus, dq, wl, alpha, gamma, k, rsel, truth, n_q, dqs, qs, pruned,
                  beta=1.0, steps=3):
    """The same search with FP32 and BF16 posting values (each index built on its own):
    throughput, Recall@k and coarse-score error on the same sampled queries."""
    import torch
    import oracle
    out = {}
    for dt in ("f32", "bf16"):
        idx = sindi.Index(corpus, alpha=alpha, window=wl.window, value_dtype=dt, gpu_build=True)
        ids = torch.empty((n_q, k), dtype=torch.int64, device="cuda")
        sc = torch.empty((n_q, k), dtype=torch.float32, device="cuda")
        idx.search(dq, k, gamma=gamma, beta=beta, out=(ids, sc))
        torch.cuda.synchronize()
        sindi.profile_enable(True)
        sindi.profile_read(reset=True)
        t0 = time.perf_counter()
        for _ in range(steps):
            idx.search(dq, k, gamma=gamma, beta=beta, out=(ids, sc))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        pr = sindi.profile_read(reset=True)
        sindi.profile_enable(False)
        rec = oracle.recall_at_k(ids.cpu().numpy()[rsel], truth)
        out[dt] = {"qps": round(n_q * steps / el, 1), "ms_per_step": round(1e3 * el / steps, 3),
                   "score_pass_ms": round(pr["accumulate_score"][1] / steps, 3),
                   "recall_at_k": round(rec, 5), "bytes_per_posting": 6 if dt == "f32" else 4,
                   **coarse_error(idx, dqs, qs, pruned, k)}
        log(f"precision {dt}: {out[dt]}")
        idx.close()
        del idx, ids, sc
    return out


def diff_leg(sindi, steps=5):
    """Differentiation workload: exact top-100 candidates for 256 queries over 1M documents
    (vocabulary 250,002), then the pair scores and their gradient w.r.t. query and
    document values (score forward / backward kernels), timed with HIP events."""
    import torch
    from synth.workloads import WORKLOADS
    wl = WORKLOADS["diff-1m"]
    corpus, queries = wl.corpus(), wl.queries()
    corpus, _ = wl.plant_positives(corpus, queries)
    idx = sindi.Index(corpus, alpha=wl.alpha, window=wl.window)
    dq = sindi.DeviceCsr.from_host(queries)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    ids, _ = idx.search(dq, wl.k, gamma=wl.gamma)
    search_ms = timed(lambda: idx.search(dq, wl.k, gamma=wl.gamma))
    fwd_ms = timed(lambda: idx.score(dq, ids))
    G = torch.randn(ids.shape, device="cuda")
    gq = torch.zeros(queries.nnz, device="cuda")
    gx = torch.zeros(corpus.nnz, device="cuda")
    bwd_ms = timed(lambda: idx.score_backward(dq, ids, G, gq, gx))
    pairs = ids.numel()
    rec = {"workload": wl.name, "n_docs": corpus.n_rows, "vocab": wl.vocab,
           "n_queries": queries.n_rows, "candidates_per_query": wl.k,
           "exact_search_ms": round(search_ms, 3), "score_forward_ms": round(fwd_ms, 3),
           "score_backward_ms": round(bwd_ms, 3),
           "backward_pairs_per_s": round(pairs / (bwd_ms * 1e-3), 1)}
    log(f"differentiation {rec}")
    idx.close()
    return rec


def serving_leg(sindi, idx, args, corpus):
    """Open-loop Poisson arrivals at each rate into the continuous-batching server over the
    same index; latency = completion on the host minus scheduled arrival."""
    from synth.workloads import WORKLOADS
    wl = WORKLOADS["serving"]
    rates = ([float(x) for x in args.serve_rates.split(",")] if args.serve_rates
             else list(wl.extra["rates"]))
    out = []
    beta = args.serve_beta
    # the GPU's rate on this query mix with no request loop: one search call over 7,000
    # serving-shaped queries (k = 100), the ceiling the loop's batches approach, at the
    # serving beta and at beta 1; and Recall@100 of both against the exact oracle on a sample
    # (a request served in a batch gets exactly the search of its query alone)
    import torch
    import oracle
    qh = wl.queries(7_000, row0=1 << 40)
    qb = sindi.DeviceCsr.from_host(qh)
    ceiling, found = {}, {}
    for b in sorted({beta, 1.0}):
        ids, _ = idx.search(qb, 100, beta=b, gamma=wl.gamma)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            idx.search(qb, 100, beta=b, gamma=wl.gamma)
        torch.cuda.synchronize()
        ceiling[b] = 3 * 7_000 / (time.perf_counter() - t0)
        found[b] = ids.cpu().numpy()
    rsel = np.linspace(0, 6_999, args.serve_recall_queries).astype(np.int64)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    truth, _ = oracle.exact_topk(corpus, qh.take_rows(rsel), 100, threads=threads)
    recall = {b: oracle.recall_at_k(found[b][rsel], truth) for b in found}
    log(f"serving mix, one call of 7,000 queries: {ceiling} QPS; Recall@100 on {len(rsel)}: {recall}")
    del qb
    row0 = 0
    with sindi.Server(idx, max_inflight=args.serve_inflight, max_batch=args.serve_max_batch,
                      k_max=100, gamma=wl.gamma, beta=beta) as srv:
        for i, rate in enumerate(rates):
            n = max(1, int(rate * args.serve_seconds))
            q = wl.queries(n, row0=row0)
            ks = wl.request_ks(n, row0=row0)
            arr = wl.arrivals(rate, n, block=i)
            row0 += n
            st0 = srv.stats()
            ids, sc, lat = srv.replay(q, ks, arr)
            st1 = srv.stats()
            lat_ms = lat / 1e6
            # completion instants relative to the start of the replay
            span = float(np.max(arr + lat / 1e9))
            batches = st1["batches"] - st0["batches"]
            rec = {"offered_qps": rate, "requests": n, "achieved_qps": round(n / span, 1),
                   "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                   "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
                   "max_ms": round(float(lat_ms.max()), 3),
                   "mean_batch": round(n / max(batches, 1), 1),
                   "largest_batch": st1["largest_batch"],
                   "retried": st1["retried"] - st0["retried"],
                   "memory_waits": st1["memory_waits"] - st0["memory_waits"]}
            log(f"serving {rec}")
            out.append(rec)
    return {"workload": "serving", "query_nnz": "uniform 5..200", "k": "uniform {10, 50, 100}",
            "beta": beta,
            "batch_call_qps": {f"beta={b}": round(v, 1) for b, v in ceiling.items()},
            "recall_at_100": {f"beta={b}": round(v, 5) for b, v in recall.items()},
            "recall_sample": f"{len(rsel)} of 7,000 serving-shaped queries, exact FP64 oracle",
            "gamma": wl.gamma, "seconds_per_rate": args.serve_seconds,
            "max_inflight": args.serve_inflight, "max_batch": args.serve_max_batch,
            "arena_peak_bytes": st1["arena_peak_bytes"], "rates": out}


def shapes_leg(sindi, steps=3):
    """The second workload shapes on 1M documents: AntSparse-shaped (vocabulary 250,000, ~40
    non-zeros per document, ~6 per query, alpha 0.85, lambda 50,000) and RANDOM-shaped
    (uniform term ids and values, vocabulary 30,000, ~120 / ~50 non-zeros, alpha 0.5), FP16
    postings, gamma 500, k 50: QPS, and Recall@50 on all 1,000 queries against the exact
    oracle beside the oracle's own Alg. 4 recall (the method's loss, not the GPU's)."""
    import torch
    import oracle
    from synth.workloads import WORKLOADS
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = []
    for name in ("antsparse-1m", "random-1m"):
        wl = WORKLOADS[name]
        corpus, queries = wl.corpus(), wl.queries()
        idx = sindi.Index(corpus, alpha=wl.alpha, window=wl.window, value_dtype=wl.value_dtype,
                          gpu_build=True)
        dq = sindi.DeviceCsr.from_host(queries)
        ids, _ = idx.search(dq, wl.k, gamma=wl.gamma)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            idx.search(dq, wl.k, gamma=wl.gamma)
        torch.cuda.synchronize()
        qps = wl.n_queries * steps / (time.perf_counter() - t0)
        idx.close()
        truth, _ = oracle.exact_topk(corpus, queries, wl.k, threads=threads)
        oidx = oracle.build_index(corpus, wl.window, oracle.mass_prune(corpus, wl.alpha, threads=threads))
        o_ids, _ = oracle.approx_search(oidx, corpus, queries, wl.beta, wl.gamma, wl.k, threads=threads)
        rec = {"workload": name, "n_docs": wl.n_docs, "vocab": wl.vocab, "n_queries": wl.n_queries,
               "alpha": wl.alpha, "qps": round(qps, 1),
               "recall_at_k": round(oracle.recall_at_k(ids.cpu().numpy(), truth), 5),
               "oracle_alg4_recall_at_k": round(oracle.recall_at_k(o_ids, truth), 5),
               "alg4_agreement": round(oracle.recall_at_k(ids.cpu().numpy(), o_ids), 5)}
        log(f"shape {rec}")
        out.append(rec)
    return out


def ablation(args, n_docs=1_000_000, n_queries=1_000, gammas=(10, 30, 100), k=10, steps=3,
             grid=None):
    """The pruning rules of Sec. 4.1 at several strengths on the same corpus and queries,
    each searched with several rerank pools (a pool of k shows the coarse ranking alone)."""
    import torch
    import oracle
    import paper_2509_08395_amd as sindi
    from synth.workloads import WORKLOADS
    wl = WORKLOADS["splade-8.8m"].scaled(n_docs, n_queries)
    corpus, queries = wl.corpus(), wl.queries()
    sel = np.linspace(0, n_queries - 1, 200).astype(np.int64)
    truth, _ = oracle.exact_topk(corpus, queries.take_rows(sel), k)
    dq = sindi.DeviceCsr.from_host(queries)
    grid = grid or ([("mrp", dict(alpha=a)) for a in (0.3, 0.4, 0.5, 0.6, 0.7)] +
                    [("vnp", dict(vn=v)) for v in (8, 14, 22, 30, 45)] +
                    [("lp", dict(list_len=l)) for l in (2_000, 5_000, 10_000, 20_000, 50_000)] +
                    [("mrp+lp", dict(alpha=0.5, list_len=l)) for l in (5_000, 20_000, 50_000)])
    rows = []
    for prune, kw in grid:
        idx = sindi.Index(corpus, window=wl.window, value_dtype="f16", prune=prune, **kw)
        info = idx.info()
        row = {"prune": prune, **kw, "kept_fraction": round(info["n_postings"] / corpus.nnz, 4)}
        for gamma in gammas:
            ids, _ = idx.search(dq, k, gamma=gamma)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                ids, _ = idx.search(dq, k, gamma=gamma)
            torch.cuda.synchronize()
            row[f"qps_g{gamma}"] = round(n_queries * steps / (time.perf_counter() - t0), 1)
            row[f"recall_at_10_g{gamma}"] = round(oracle.recall_at_k(ids.cpu().numpy()[sel], truth), 4)
        log(f"ablation {row}")
        rows.append(row)
        idx.close()
    return {"ablation": "pruning rules (Sec. 4.1)", "workload": wl.name, "n_docs": n_docs,
            "n_queries": n_queries, "recall_sample": len(sel), "gammas": list(gammas), "k": k,
            "value_storage": "f16", "rows": rows}


def _cpu_model():
    """The host CPU as /proc/cpuinfo names it (model name, family/model/stepping, clock), with
    the logical CPUs this process may run on."""
    fields = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                key, val = (x.strip() for x in line.split(":", 1))
                if key in ("model name", "cpu family", "model", "stepping", "cpu MHz",
                           "vendor_id") and key not in fields:
                    fields[key] = val
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    name = fields.get("model name", "unknown")
    return (f"{name} (vendor {fields.get('vendor_id', '?')}, family {fields.get('cpu family', '?')} "
            f"model {fields.get('model', '?')} stepping {fields.get('stepping', '?')}, "
            f"{fields.get('cpu MHz', '?')} MHz; {usable} usable of {os.cpu_count()} logical CPUs)")


if __name__ == "__main__":
    main()
