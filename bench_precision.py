#!/usr/bin/env python
"""Precision tiers on a large collection: the plain SFA scan, the BF16 prune
and the FP8 prune over batches of 4,096 queries at k = 10.

Collection: N x n z-normalised FP32 mix (even rows random walk, odd rows
8-sinusoid high-frequency; default 50M x 256, seed 3), generated on the host
in chunks of 1M rows and streamed to the GPU.  One index keeps the BF16 and
the FP8 copies.  Queries: noisy copies (sigma 0.1, same seed) of rows drawn
uniformly.

For each tier it reports queries/s (median of --steps calls after one
warm-up; one call for the plain scan), the stage times and the rows left to
the exact distance per query.  For the prune tiers it adds the tile kernel's
work: pairs computed and pairs its lists required, its rate in TFLOP/s (2n
flop per computed pair over the kernel's time) against the dense MFMA peak
of its type (BF16 2.5, FP8 5.0 PF/s), and the prune rate (the fraction of
(query, row) pairs never computed).  Bound slack: for --slack-queries
queries and --slack-rows rows drawn at random, each tier's batched-distance
bound (its own inspection kernel) against the FP64 squared distance
computed on the device: quantiles of bound / distance and the count of
bounds above the distance (must be zero).  The ids of every tier are
compared with each other; their parity with the FP64 oracle at this size is
the test `test_50M_precision_tiers`.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {1: 2500.0, 2: 5000.0}


def log(*a):
    print("[precision]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=50_000_000)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--slack-queries", type=int, default=8)
    ap.add_argument("--slack-rows", type=int, default=1_000_000)
    args = ap.parse_args()

    import torch
    from paper_2411_17483_amd import sofa
    import synth

    sofa.load()
    N, n, B, k = args.N, args.n, args.batch, args.k
    X = torch.empty((N, n), dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    for r0 in range(0, N, 1_000_000):
        m = min(1_000_000, N - r0)
        X[r0:r0 + m].copy_(torch.from_numpy(synth.collection(m, n, "mix", seed=args.seed, row0=r0)))
        if (r0 // 1_000_000) % 10 == 9:
            log(f"{r0 + m} rows generated, {time.perf_counter() - t0:.0f}s")
    src = synth.query_sources(N, B, args.seed)
    Q = synth.noisy_copies(X[torch.from_numpy(src).cuda()].cpu().numpy(), sigma=0.1, seed=args.seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bins = sofa.Bins.learn(X, N // 100)
    ix = sofa.Index(bins, X, leaf_size=256, precision=3)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    n_pad = ix.info()["n_pad"]
    log(f"bins and index with both copies: {t_build:.2f}s")
    Qd = torch.from_numpy(Q).cuda()

    tiers, ids_by = {}, {}
    for name, prune, steps in (("bf16", 1, args.steps), ("fp8", 2, args.steps), ("plain", 0, 1)):
        ix.knn(Qd, k, prune=prune)
        torch.cuda.synchronize()
        times = []
        for _ in range(steps):
            t0 = time.perf_counter()
            ids, _ = ix.knn(Qd, k, prune=prune)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        st = ix.stats()
        ms = float(np.median(times))
        r = {"queries_per_s": B / (ms * 1e-3), "ms_per_batch": ms,
             "stages_ms": {kk: st[kk] for kk in ("ms_prepare", "ms_leaf", "ms_seed", "ms_refine",
                                                  "ms_finalize", "ms_bf16_tiles", "ms_bf16_refine")},
             "rows_refined_per_query": st["series_refined"] / B,
             "fallbacks": {kk: st[kk] for kk in ("overflow_fallbacks", "overflow_retries", "overflow_band")}}
        if prune:
            pairs, needed = st["series_bf16_checked"], st["series_bf16_needed"]
            tflops = 2.0 * n_pad * pairs / (st["ms_bf16_tiles"] * 1e-3) / 1e12
            r["tile_kernel"] = {"pairs_computed": pairs, "pairs_needed": needed, "launches": st["prune_passes"],
                                "TFLOP_per_s": tflops, "peak_TFLOP_per_s": PEAK_TFLOPS[prune],
                                "frac": tflops / PEAK_TFLOPS[prune]}
            r["prune_rate"] = 1.0 - needed / (float(N) * B)
        tiers[name] = r
        ids_by[name] = ids.cpu().numpy()
        log(f"{name}: {r['queries_per_s']:.0f} queries/s ({ms:.2f} ms per batch of {B})")
    identical = all(np.array_equal(ids_by["plain"], v) for v in ids_by.values())
    log(f"ids identical across tiers: {identical}")

    # bound slack on a random sample of rows (leaf order, then original rows)
    S, R = args.slack_queries, args.slack_rows
    g = torch.Generator(device="cuda")
    g.manual_seed(args.seed)
    pos = torch.randint(0, N, (R,), device="cuda", generator=g)
    _, ids_leaf, _, _ = ix.export()
    rows = X[ids_leaf[pos].long()].double()
    q = Qd[:S].double()
    d2 = (q * q).sum(1)[:, None] + (rows * rows).sum(1)[None, :] - 2.0 * (q @ rows.T)
    slack = {}
    for name, fn in (("bf16", ix.bf16_lower_bounds), ("fp8", ix.fp8_lower_bounds)):
        lb = fn(Qd[:S].contiguous())[:, pos].double()
        ratio = (lb / d2.clamp_min(1e-30)).flatten().cpu().numpy()
        above = int(torch.sum(lb > d2 * (1 + 1e-12) + 1e-30).item())
        slack[name] = {"bound_over_distance": {f"p{p}": float(np.percentile(ratio, p)) for p in (1, 10, 50, 90, 99)},
                       "bounds_above_distance": above, "pairs": int(ratio.size)}
        log(f"{name} bound / d^2: median {slack[name]['bound_over_distance']['p50']:.4f}, above d^2: {above}")

    out = {"metric": f"precision tiers: queries/s at {N} x {n}, batches of {B}, k={k}",
           "config": {"N": N, "n": n, "batch": B, "k": k, "leaf_size": 256, "seed": args.seed,
                      "data": "synthetic mix, noisy-copy queries (sigma 0.1)"},
           "build_s": t_build, "tiers": tiers, "ids_identical_across_tiers": identical, "bound_slack": slack}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
