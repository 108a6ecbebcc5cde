#!/usr/bin/env python
"""Summary ablation on synthetic collections: the GPU analogue of the paper's
TLB ablation (Section V-E: SFA with equi-depth or equi-width bins, with or
without variance selection, against iSAX, for alphabet sizes 4..256, l = 16)
and of its sampling study (Section V-C: the fraction of the collection the
bins are learned from).

For each collection kind (rw, hf, band, mix; N x n, z-normalised, own seed;
band: eight sinusoids of 4 to 16 cycles per series, which the 16-value
Fourier word holds and 16-sample segment means average away) and
each variant and alphabet size it reports:
  - TLB: the mean over (query, row) pairs of the word lower bound over the
    Euclidean distance (16 noisy-copy queries x 20,000 random rows; the bound
    is the library's own word bound, the distance is FP64 on the host);
  - the plain SFA/iSAX search at k = 10 over 200 queries: queries/s and the
    rows left to the exact distance per query (the pruning the bound buys).
The sampling sweep (mix, SFA EW + variance, alpha = 256) also times the BF16
prune.  Then, the analogue of the paper's index-creation and leaf-size
studies: `sofa_build` throughput on a `--build-N` x n mix collection (GB/s of
FP32 input, with and without the BF16 + FP8 copies), and queries/s of the
plain and BF16 paths against the leaf size on the mix collection.  Prints one
JSON line; `--N` shrinks the collections.
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


def log(*a):
    print("[ablation]", *a, file=sys.stderr, flush=True)


VARIANTS = {  # name: Bins.learn keywords
    "SFA ED+VAR": dict(binning=0, selection=0),
    "SFA EW+VAR": dict(binning=1, selection=0),
    "SFA ED": dict(binning=0, selection=1),
    "SFA EW": dict(binning=1, selection=1),
    "iSAX": dict(summary=1),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=1_000_000)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--queries", type=int, default=200)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--alphas", default="4,8,16,32,64,128,256")
    ap.add_argument("--kinds", default="rw,hf,band,mix")
    ap.add_argument("--rates", default="0.001,0.005,0.01,0.05,0.1,0.2")
    ap.add_argument("--leaves", default="64,128,256,512,1024,2048,4096")
    ap.add_argument("--build-N", type=int, default=10_000_000)
    args = ap.parse_args()

    import torch
    from paper_2411_17483_amd import sofa
    import synth
    sofa.load()
    dev = torch.device("cuda:0")
    N, n, B, k = args.N, args.n, args.queries, args.k
    alphas = [int(a) for a in args.alphas.split(",")]
    rng = np.random.default_rng(3)
    pos = np.sort(rng.choice(N, size=min(N, 20000), replace=False))
    tq = 16
    out = {"N": N, "n": n, "queries": B, "k": k, "l": 16, "tlb_sample": f"{tq} queries x {pos.size} rows",
           "tlb": {}, "plain": {}, "sampling": []}

    def measure(X, Q, Xd, Qd, bins, prunes=(0,)):
        ix = sofa.Index(bins, Xd, leaf_size=256, precision=1 if 1 in prunes else 0)
        _, ids_l, _, _ = ix.export()
        rows = ids_l.cpu().numpy()[pos]
        _, lbw = ix.lower_bounds(Qd[:tq].contiguous(), tables=False, lb=True)
        lbw = lbw[:, torch.from_numpy(pos).to(dev)].cpu().numpy().astype(np.float64)
        Xr = X[rows].astype(np.float64)
        d2 = np.stack([((Xr - Q[b].astype(np.float64)) ** 2).sum(-1) for b in range(tq)])
        tlb = float(np.mean(np.sqrt(np.maximum(lbw, 0.0)) / np.sqrt(np.maximum(d2, 1e-300))))
        res = {"tlb": tlb}
        for prune in prunes:
            ix.knn(Qd, k, prune=prune)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ix.knn(Qd, k, prune=prune)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            st = ix.stats()
            res[f"prune{prune}"] = {"queries_per_s": B / sec, "rows_refined_per_query": st["series_refined"] / B,
                                    "leaves_visited_per_query": st["leaves_visited"] / B}
        del ix
        return res

    for kind in args.kinds.split(","):
        X = synth.collection(N, n, kind, seed=11)
        Q, _ = synth.queries(X, B, sigma=0.1, seed=12)
        Xd = torch.from_numpy(X).to(dev)
        Qd = torch.from_numpy(Q).to(dev)
        out["tlb"][kind] = {}
        out["plain"][kind] = {}
        for name, kw in VARIANTS.items():
            tl, pl = [], []
            for a in alphas:
                bins = sofa.Bins.learn(Xd, max(1, N // 100), alpha=a, **kw)
                r = measure(X, Q, Xd, Qd, bins)
                tl.append(round(r["tlb"], 4))
                pl.append({"alpha": a, **r["prune0"]})
            out["tlb"][kind][name] = tl
            out["plain"][kind][name] = pl
            log(f"{kind} {name}: TLB " + " ".join(f"{t:.3f}" for t in tl) +
                f" | rows refined/query at alpha {alphas[-1]}: {pl[-1]['rows_refined_per_query']:.0f}")
        if kind == "mix":
            out["leaf_size"] = []
            bins = sofa.Bins.learn(Xd, max(1, N // 100), alpha=256, **VARIANTS["SFA EW+VAR"])
            for L in [int(x) for x in args.leaves.split(",")]:
                ix = sofa.Index(bins, Xd, leaf_size=L, precision=1 if L % 256 == 0 else 0)
                row = {"leaf_size": L}
                for prune in ((0, 1) if L % 256 == 0 else (0,)):
                    ix.knn(Qd, k, prune=prune)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    ix.knn(Qd, k, prune=prune)
                    torch.cuda.synchronize()
                    row[f"prune{prune}_queries_per_s"] = B / (time.perf_counter() - t0)
                    row[f"prune{prune}_leaves_visited_per_query"] = ix.stats()["leaves_visited"] / B
                out["leaf_size"].append(row)
                log(f"leaf {L}: " + ", ".join(f"{a} {b:.0f}" for a, b in row.items() if a.endswith("per_s")))
                del ix
            for rate in [float(r) for r in args.rates.split(",")]:
                bins = sofa.Bins.learn(Xd, max(1, int(N * rate)), alpha=256, **VARIANTS["SFA EW+VAR"])
                r = measure(X, Q, Xd, Qd, bins, prunes=(0, 1))
                out["sampling"].append({"rate": rate, **r})
                log(f"sampling {rate:.3%}: TLB {r['tlb']:.3f}, plain {r['prune0']['queries_per_s']:.0f} q/s, "
                    f"BF16 {r['prune1']['queries_per_s']:.0f} q/s")
        del Xd, Qd
        torch.cuda.empty_cache()
    # build throughput at full size
    if args.build_N > 0:
        Nb = args.build_N
        X = synth.collection(Nb, n, "mix", seed=13)
        Xd = torch.from_numpy(X).to(dev)
        del X
        bins = sofa.Bins.learn(Xd, max(1, Nb // 100))
        torch.cuda.synchronize()
        out["build"] = {"N": Nb, "n": n, "input_gb": Nb * n * 4 / 1e9}
        for prec, name in ((0, "sfa_only"), (3, "with_bf16_fp8")):
            sofa.Index(bins, Xd, leaf_size=256, precision=prec)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ix = sofa.Index(bins, Xd, leaf_size=256, precision=prec)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            out["build"][name] = {"seconds": sec, "input_gb_per_s": Nb * n * 4 / 1e9 / sec,
                                  "index_gb": ix.info()["device_bytes"] / 1e9}
            log(f"build {Nb}x{n} ({name}): {sec:.3f} s, {Nb * n * 4 / 1e9 / sec:.0f} GB/s of input")
            del ix
        del Xd
        torch.cuda.empty_cache()
    out["alphas"] = alphas
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
