#!/usr/bin/env python
"""Serving benchmark: the request loop over three HBM-resident collections.

Collections (z-normalised FP32, even rows random walk, odd rows 8-sinusoid
high-frequency, generated on the host in chunks and streamed to the GPU):
100M x 128 (BF16 prune), 20M x 512 and 5M x 1024 (FP8 prune).  Requests
carry one noisy-copy query (sigma 0.1) of a uniformly chosen collection with
k uniform in {1, 10, 100}; arrivals are Poisson at a fixed offered rate.  For
each rate the run reports the achieved queries/s and the p50/p99 latency
from submission to result (measured by the server's own clock), plus the
batch sizes the loop formed and the HBM roofline fraction: the bytes the
batches' searches had to read (the server's hbm_bytes: each prune-copy chunk
with a non-empty query list once per pass, plus every exactly refined row)
over the level's wall time, against the 8 TB/s peak, and the same bytes over
the summed batch times (the rate of one batch while it runs).  A subset of requests is also answered one at
a time and checked to be identical to its answers in the mix.

Prints one JSON line.  `--scale` shrinks every collection (e.g. 0.05 for a
quick run); the defaults are the full sizes.
"""
import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


PEAK_HBM = 8.0e12  # B/s, MI355X published HBM3E bandwidth


def log(*a):
    print("[serve]", *a, file=sys.stderr, flush=True)


def build_collection(sofa, torch, N, n, seed, precision, chunk_rows):
    import synth
    dev = torch.device("cuda:0")
    X = torch.empty((N, n), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    for r0 in range(0, N, chunk_rows):
        m = min(chunk_rows, N - r0)
        X[r0:r0 + m].copy_(torch.from_numpy(synth.collection(m, n, "mix", seed=seed, row0=r0)))
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    bins = sofa.Bins.learn(X, max(1000, N // 100))
    ix = sofa.Index(bins, X, leaf_size=256, precision=precision)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    # noisy copies of stride-sampled rows as the query pool
    B = 4096
    src = (np.arange(B, dtype=np.int64) * (N // B)) % N
    rows = X[torch.from_numpy(src).to(dev)].cpu().numpy()
    Q = synth.noisy_copies(rows, sigma=0.1, seed=seed + 100)
    del X
    torch.cuda.empty_cache()
    return bins, ix, Q, t_gen, t_build


def run_level(srv, cids, pools, qps, duration, seed, ks=(1, 10, 100)):
    rng = np.random.default_rng(seed)
    n_req = max(1, int(qps * duration))
    gaps = rng.exponential(1.0 / qps, n_req)
    colls = rng.integers(len(cids), size=n_req)
    kk = rng.choice(ks, size=n_req)
    rows = [int(rng.integers(pools[c].shape[0])) for c in colls]
    tickets = [None] * n_req
    results = [None] * n_req
    ready = threading.Semaphore(0)

    def waiter():
        for i in range(n_req):
            ready.acquire()
            results[i] = srv.wait(tickets[i], int(kk[i]))

    th = threading.Thread(target=waiter)
    st0 = srv.stats()
    th.start()
    t_start = time.perf_counter()
    t_next = t_start
    for i in range(n_req):
        t_next += gaps[i]
        delay = t_next - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        c = int(colls[i])
        tickets[i] = srv.submit(cids[c], pools[c][rows[i]], int(kk[i]))
        ready.release()
    th.join()
    wall = time.perf_counter() - t_start
    st1 = srv.stats()
    dbytes = st1["hbm_bytes"] - st0["hbm_bytes"]
    dbusy = (st1["busy_ms"] - st0["busy_ms"]) * 1e-3
    lat = np.array([r[2][0] for r in results])
    queue = np.array([r[2][1] for r in results])
    batch = np.array([r[2][2] for r in results])
    per_k = {f"k{k}": {"p50_ms": float(np.percentile(lat[kk == k], 50)),
                       "p99_ms": float(np.percentile(lat[kk == k], 99))}
             for k in ks if np.any(kk == k)}
    per_c = {f"c{c}": {"p50_ms": float(np.percentile(lat[colls == c], 50)),
                       "p99_ms": float(np.percentile(lat[colls == c], 99))}
             for c in range(len(cids)) if np.any(colls == c)}
    return {"offered_qps": qps, "requests": n_req, "achieved_qps": n_req / wall,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "queue_p50_ms": float(np.percentile(queue, 50)),
            "mean_batch": float(np.mean(batch)), "max_batch": int(np.max(batch)),
            "hbm_bytes": dbytes, "hbm_gb_per_s": dbytes / wall / 1e9,
            "hbm_frac": dbytes / wall / PEAK_HBM,
            "hbm_frac_while_busy": dbytes / dbusy / PEAK_HBM if dbusy > 0 else None,
            "per_k": per_k, "per_collection": per_c}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--qps", default="100,400,1500,4000,8000,16000")
    ap.add_argument("--duration", type=float, default=6.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--max-batch", type=int, default=256)
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--per-collection", type=int, default=1,
                    help="batches of one collection in flight at once")
    ap.add_argument("--check", type=int, default=60, help="requests checked alone vs in the mix")
    args = ap.parse_args()

    import torch
    from paper_2411_17483_amd import sofa
    sofa.load()
    specs = [(100_000_000, 128, 6, 1, 1), (20_000_000, 512, 7, 2, 2), (5_000_000, 1024, 8, 2, 2)]
    colls, build = [], []
    for N, n, seed, prec, prune in specs:
        N = max(4096, int(N * args.scale))
        bins, ix, Q, t_gen, t_build = build_collection(sofa, torch, N, n, seed, prec, 5_000_000)
        colls.append((bins, ix, Q, prune))
        build.append({"N": N, "n": n, "prune": prune, "gen_s": t_gen, "build_s": t_build,
                      "index_gb": ix.info()["device_bytes"] / 1e9})
        log(f"collection {N}x{n}: generated {t_gen:.1f}s, built {t_build:.1f}s, "
            f"{ix.info()['device_bytes'] / 1e9:.1f} GB")

    srv = sofa.Server(slots=args.slots, max_batch=args.max_batch,
                      memory_budget=int(args.budget_gb * (1 << 30)), per_collection=args.per_collection)
    cids = [srv.add_collection(ix, prune) for _, ix, _, prune in colls]
    pools = [Q for _, _, Q, _ in colls]
    # warm-up: every (collection, k) once
    for c in range(len(cids)):
        for k in (1, 10, 100):
            srv.wait(srv.submit(cids[c], pools[c][0], k), k)
    log("warm")

    # alone vs mix on a subset
    rng = np.random.default_rng(9)
    sub = [(int(rng.integers(len(cids))), int(rng.choice([1, 10, 100])), int(rng.integers(4096)))
           for _ in range(args.check)]
    alone = [srv.wait(srv.submit(cids[c], pools[c][j], k), k) for c, k, j in sub]
    tick = [srv.submit(cids[c], pools[c][j], k) for c, k, j in sub]
    mix = [srv.wait(t, k) for t, (c, k, j) in zip(tick, sub)]
    same = all(np.array_equal(a[0], m[0]) and np.array_equal(a[1], m[1]) for a, m in zip(alone, mix))
    log(f"alone == mix on {len(sub)} requests: {same}")

    levels = []
    for qps in [float(x) for x in args.qps.split(",")]:
        res = run_level(srv, cids, pools, qps, args.duration, seed=int(qps))
        levels.append(res)
        log(f"offered {qps:.0f} q/s: achieved {res['achieved_qps']:.0f} q/s, p50 {res['p50_ms']:.2f} ms, "
            f"p99 {res['p99_ms']:.2f} ms, mean batch {res['mean_batch']:.1f}, HBM {res['hbm_gb_per_s']:.0f} GB/s "
            f"({res['hbm_frac']:.3f} of peak; {res['hbm_frac_while_busy'] or 0:.3f} per busy slot-second)")
    st = srv.stats()
    srv.close()
    out = {"metric": "serving p50/p99 latency and queries/s, 3 HBM-resident collections, "
                     "Poisson arrivals, k in {1,10,100}",
           "collections": build, "slots": args.slots, "max_batch": args.max_batch,
           "per_collection": args.per_collection,
           "memory_budget_gb": args.budget_gb, "alone_equals_mix": same, "checked": len(sub),
           "levels": levels, "server_stats": st}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
