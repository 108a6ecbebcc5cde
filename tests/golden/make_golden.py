#!/usr/bin/env python
"""Writes the stored expected values under tests/golden/ (run from the repo root).

Every value here comes from the FP64 CPU oracle (``oracle/``) applied to
seeded synthetic inputs (``synth/``); nothing comes from the GPU library.
The fixture pins the oracle and the generator against drift (a later change
to either must reproduce these bits or explain itself), and gives the GPU
tests expected answers that do not need the oracle at test time.

Case ``small_rw64``: 3,000 random-walk series of length 64 (seed 301), MCB
bins (Algorithm 1) on a 600-row stride sample with a pool of 16 complex
coefficients, l = 16, alpha = 16, equi-depth; SFA words (Algorithm 2) of the
first 32 rows; exact 5-NN (Section II-A, ties by row id) of 12 noisy-copy
queries (sigma 0.1, seed 302).
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

CASE = dict(name="small_rw64", N=3000, n=64, kind="rw", seed=301, B=12, sigma=0.1, qseed=302,
            m=600, P=16, l=16, alpha=16, binning=0, k=5, n_words=32)


def inputs(c):
    X = synth.collection(c["N"], c["n"], c["kind"], seed=c["seed"])
    Q, src = synth.queries(X, c["B"], sigma=c["sigma"], seed=c["qseed"])
    return X, Q, src


def compute(c):
    X, Q, src = inputs(c)
    var, sel, beta = oracle.learn_bins(X, c["m"], P=c["P"], l=c["l"], alpha=c["alpha"],
                                       binning=c["binning"])
    W, _ = oracle.words(X[:c["n_words"]], sel, beta, P=c["P"])
    ids, d2 = oracle.knn(X, Q, c["k"])
    return {
        "case": c,
        "sha256_X": hashlib.sha256(np.ascontiguousarray(X).tobytes()).hexdigest(),
        "sha256_Q": hashlib.sha256(np.ascontiguousarray(Q).tobytes()).hexdigest(),
        "query_sources": [int(s) for s in src],
        "sel": [int(s) for s in sel],
        "beta_hex": [[float(v).hex() for v in row] for row in beta],
        "words": W.astype(int).tolist(),
        "knn_ids": ids.tolist(),
        "knn_d2_hex": [[float(v).hex() for v in row] for row in d2],
    }


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), CASE["name"] + ".json")
    with open(out, "w") as f:
        json.dump(compute(CASE), f, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
