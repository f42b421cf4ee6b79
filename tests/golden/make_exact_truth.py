#!/usr/bin/env python3
"""Write the exact top-k (FP64 inner products, Defs. 2-3) of every query of a synthetic
workload, computed by the CPU oracle alone, for bench.py's Recall@k over the whole query set.

    python tests/golden/make_exact_truth.py [workload] [--threads N]

Output: tests/golden/<workload>_exact_top<k>.npz with ids (int32 [n_queries, k]), scores
(the FP64 scores rounded to float32) and meta (JSON: the workload's sizes and seed, and a
fingerprint of the generated corpus and queries, which bench.py recomputes before it uses the
file).  Nothing here calls the GPU library.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def fingerprint(corpus, queries):
    """sha256 over strided samples of the generated arrays (cheap at 8.8M documents)."""
    import hashlib
    h = hashlib.sha256()
    for a in (corpus.indptr[::997], corpus.indices[::1009], corpus.values[::1013],
              queries.indptr, queries.indices, queries.values):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def truth_path(name, k):
    return os.path.join(HERE, f"{name}_exact_top{k}.npz")


def main():
    import oracle
    from synth.workloads import WORKLOADS
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", nargs="?", default="splade-8.8m")
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    args = ap.parse_args()
    wl = WORKLOADS[args.workload]
    corpus, queries = wl.corpus(), wl.queries()
    t = time.time()
    ids, sc = oracle.exact_topk(corpus, queries, wl.k, threads=args.threads)
    el = time.time() - t
    meta = {"workload": wl.name, "n_docs": wl.n_docs, "vocab": wl.vocab, "n_queries": wl.n_queries,
            "k": wl.k, "seed": wl.seed, "fingerprint": fingerprint(corpus, queries),
            "oracle": "exact_topk (FP64 term-at-a-time, ranking by score desc, id asc)",
            "seconds": round(el, 1), "threads": args.threads}
    np.savez_compressed(truth_path(wl.name, wl.k), ids=ids.astype(np.int32),
                        scores=sc.astype(np.float32), meta=json.dumps(meta))
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
