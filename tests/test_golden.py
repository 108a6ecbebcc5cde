"""The oracle and the input generator against their stored outputs (CPU).

tests/golden/small_rw64.json was written by tests/golden/make_golden.py from
the oracle alone.  These tests fail if the generator's bits, the MCB
breakpoints (Algorithm 1), the SFA words (Algorithm 2) or the exact k-NN
(Section II-A) of the oracle drift from the stored values.
"""
import hashlib
import json
import os

import numpy as np

import oracle
import synth

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "small_rw64.json")


def _load():
    with open(GOLD) as f:
        return json.load(f)


def _inputs(c):
    X = synth.collection(c["N"], c["n"], c["kind"], seed=c["seed"])
    Q, src = synth.queries(X, c["B"], sigma=c["sigma"], seed=c["qseed"])
    return X, Q, src


def test_generator_bits_match_golden():
    g = _load()
    X, Q, src = _inputs(g["case"])
    assert hashlib.sha256(np.ascontiguousarray(X).tobytes()).hexdigest() == g["sha256_X"]
    assert hashlib.sha256(np.ascontiguousarray(Q).tobytes()).hexdigest() == g["sha256_Q"]
    assert [int(s) for s in src] == g["query_sources"]


def test_oracle_bins_words_knn_match_golden():
    g = _load()
    c = g["case"]
    X, Q, _ = _inputs(c)
    _, sel, beta = oracle.learn_bins(X, c["m"], P=c["P"], l=c["l"], alpha=c["alpha"],
                                     binning=c["binning"])
    assert sel.tolist() == g["sel"]
    ref_beta = np.array([[float.fromhex(v) for v in row] for row in g["beta_hex"]])
    assert np.array_equal(beta, ref_beta)
    W, _ = oracle.words(X[:c["n_words"]], sel, beta, P=c["P"])
    assert W.astype(int).tolist() == g["words"]
    ids, d2 = oracle.knn(X, Q, c["k"])
    assert ids.tolist() == g["knn_ids"]
    ref_d2 = np.array([[float.fromhex(v) for v in row] for row in g["knn_d2_hex"]])
    assert np.array_equal(d2, ref_d2)
    # each noisy copy's nearest neighbour is its source row (sigma 0.1 << the
    # spacing of random walks of length 64)
    assert [r[0] for r in g["knn_ids"]] == g["query_sources"]
