"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (stated per test): breakpoints within 1e-12 relative and identical
selections; pool values within the projection bound eta * ||x||; symbols
valid for the exact value within that bound; lower bounds never above the
FP64 distance; neighbour ids bit-identical to the oracle's (distance, id)
ranking; distances within 1e-6 relative of sqrt(FP64 d^2).
"""
import os

import numpy as np
import pytest

import oracle
from tests import mlp_bound
import synth

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bins(sofa, X, m, **kw):
    return sofa.Bins.learn(_t(X), m, **kw)


# --------------------------------------------------------------------------- #
@pytest.mark.parametrize("binning", [0, 1])
@pytest.mark.parametrize("alpha", [4, 256])
def test_learn_bins_matches_oracle(gpu_lib, binning, alpha):
    X = synth.collection(20000, 256, "mix", seed=101)
    m = 3000
    b = _bins(gpu_lib, X, m, alpha=alpha, binning=binning).get()
    var, sel, beta = oracle.learn_bins(X, m, P=16, l=16, alpha=alpha, binning=binning)
    assert b["sel"].tolist() == sel.tolist()
    assert np.allclose(b["var"], var, rtol=1e-10, atol=0)
    scale = np.max(np.abs(beta))
    assert np.max(np.abs(b["beta"] - beta)) <= 1e-12 * scale


@pytest.mark.parametrize("binning", [0, 1])
def test_learn_bins_first_values_matches_oracle(gpu_lib, binning):
    """selection = 1: the first l pool values, with breakpoints learned on them."""
    X = synth.collection(20000, 256, "mix", seed=103)
    b = _bins(gpu_lib, X, 3000, alpha=64, binning=binning, selection=1).get()
    var, sel, beta = oracle.learn_bins(X, 3000, P=16, l=16, alpha=64, binning=binning, selection=1)
    assert b["selection"] == 1 and b["sel"].tolist() == list(range(16)) == sel.tolist()
    assert np.allclose(b["var"], var, rtol=1e-10, atol=0)
    assert np.max(np.abs(b["beta"] - beta)) <= 1e-12 * np.max(np.abs(beta))


def test_learn_bins_small_pool_and_l(gpu_lib):
    X = synth.collection(5000, 64, "hf", seed=5)
    b = _bins(gpu_lib, X, 5000, l=6, alpha=16, pool=8).get()
    var, sel, beta = oracle.learn_bins(X, 5000, P=8, l=6, alpha=16)
    assert b["sel"].tolist() == sel.tolist()
    assert np.max(np.abs(b["beta"] - beta)) <= 1e-12 * np.max(np.abs(beta))


@pytest.mark.parametrize("n", [64, 100, 256, 1024])
def test_transform_within_projection_bound(gpu_lib, n):
    P = min(16, n // 2 - 1)
    X = synth.collection(3001, n, "mix", seed=7 + n)
    bins = _bins(gpu_lib, X, 3001, pool=P)
    info = bins.get()
    pool, selv, words = bins.transform(_t(X))
    pool, selv, words = pool.cpu().numpy(), selv.cpu().numpy(), words.cpu().numpy()
    ref = oracle.dft_pool(X, P)
    norms = np.sqrt(np.sum(X.astype(np.float64) ** 2, axis=1))
    eta = bins.eta_per_norm * norms + 1e-30
    err = np.abs(pool.astype(np.float64) - ref)
    assert np.all(err <= eta[:, None]), float(np.max(err / eta[:, None]))
    sel, beta = info["sel"], info["beta"]
    l, am1 = beta.shape
    for j in range(l):
        c = ref[:, sel[j]]
        s = words[:, j].astype(np.int64)
        lo = np.where(s > 0, beta[j][np.maximum(s - 1, 0)], -np.inf)
        hi = np.where(s < am1, beta[j][np.minimum(s, am1 - 1)], np.inf)
        slack = eta + 2.0 ** -23 * np.abs(np.where(np.isfinite(lo), lo, 0)) + 1e-12
        assert np.all(lo - slack <= c), j
        slack_hi = eta + 2.0 ** -23 * np.abs(np.where(np.isfinite(hi), hi, 0)) + 1e-12
        assert np.all(c < hi + slack_hi), j
        assert np.array_equal(selv[:, j], pool[:, sel[j]])
    # symbols equal to the oracle's wherever the exact value is clear of every
    # breakpoint by more than the projection bound (rows of the sample sit on
    # breakpoints, where either neighbouring symbol is valid)
    W, C = oracle.words(X[:300], sel, beta, P=P)
    for j in range(l):
        gap = np.min(np.abs(C[:, j][:, None] - beta[j][None, :]), axis=1)
        clear = gap > eta[:300] + 2.0 ** -23 * np.max(np.abs(beta[j])) + 1e-12
        assert np.array_equal(W[clear, j], words[:300, j][clear]), j
        assert np.mean(clear) > 0.5


def test_index_layout_properties(gpu_lib):
    import torch
    N, n, L = 10000 + 37, 128, 128
    X = synth.collection(N, n, "mix", seed=9)
    bins = _bins(gpu_lib, X, 2000)
    ix = gpu_lib.Index(bins, _t(X), leaf_size=L, key_scheme=1)
    W, ids, env, keys = (t.cpu().numpy() for t in ix.export())
    info = ix.info()
    assert info["n_leaves"] == (N + L - 1) // L
    assert np.array_equal(np.sort(ids), np.arange(N))
    _, _, W0 = bins.transform(_t(X))
    assert np.array_equal(W, W0.cpu().numpy()[ids])
    # key = interleave (MSB first) of the top 4 bits of each symbol, word order
    s8 = W.astype(np.uint64)
    k = np.zeros(N, dtype=np.uint64)
    for b in range(7, 3, -1):
        for j in range(16):
            k = (k << np.uint64(1)) | ((s8[:, j] >> np.uint64(b)) & np.uint64(1))
    ku = keys.view(np.uint64)
    assert np.array_equal(ku, k)
    assert np.all(ku[1:] >= ku[:-1])
    # stable: equal keys keep increasing row ids
    same = ku[1:] == ku[:-1]
    assert np.all(ids[1:][same] > ids[:-1][same])
    for leaf in range(info["n_leaves"]):
        blk = W[leaf * L:(leaf + 1) * L]
        assert np.array_equal(env[leaf, :16], blk.min(axis=0))
        assert np.array_equal(env[leaf, 16:], blk.max(axis=0))
    # default scheme: 8 bits for positions 0-3, 4 for 4-7, 2 for 8-15
    ix0 = gpu_lib.Index(bins, _t(X), leaf_size=L)
    W0l, ids0, _, keys0 = (t.cpu().numpy() for t in ix0.export())
    nb = [8] * 4 + [4] * 4 + [2] * 8
    s8 = W0l.astype(np.uint64)
    k = np.zeros(N, dtype=np.uint64)
    for b in range(7, -1, -1):
        for j in range(16):
            if b >= 8 - nb[j]:
                k = (k << np.uint64(1)) | ((s8[:, j] >> np.uint64(b)) & np.uint64(1))
    assert np.array_equal(keys0.view(np.uint64), k)
    assert np.all(keys0.view(np.uint64)[1:] >= keys0.view(np.uint64)[:-1])


@pytest.mark.parametrize("B", [1, 2, 3, 5])
def test_word_scan_equals_table_sums(gpu_lib, B):
    """The word scan writes, for each query and leaf-order row, the sum over
    word positions of the query's table at the row's symbol (Eq. 3 summed as
    in Eq. 2): recomputed here from the exported words and tables."""
    N, n = 5000 + 13, 256
    X = synth.collection(N, n, "mix", seed=15)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=16)
    bins = _bins(gpu_lib, X, 2000)
    ix = gpu_lib.Index(bins, _t(X), leaf_size=256)
    T, LB, ms = ix.lower_bounds(_t(Q), timed=True)
    assert ms > 0.0
    T, LB = T.cpu().numpy().astype(np.float64), LB.cpu().numpy().astype(np.float64)
    words, _, _, _ = ix.export()
    W = words.cpu().numpy().reshape(N, 16).astype(np.int64)
    for b in range(B):
        ref = T[b][np.arange(16)[None, :], W].sum(axis=1)
        assert np.all(np.abs(LB[b] - ref) <= 1e-5 * ref + 1e-6), b


@pytest.mark.parametrize("binning", [0, 1])
def test_lower_bounds_never_exceed_distance(gpu_lib, binning):
    N, n, B = 3000, 256, 24
    X = synth.collection(N, n, "mix", seed=13)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=14)
    Q[:4] = synth.collection(4, n, "hf", seed=99)  # unrelated queries too
    bins = _bins(gpu_lib, X, N, binning=binning)
    ix = gpu_lib.Index(bins, _t(X), leaf_size=64)
    T, LB = ix.lower_bounds(_t(Q))
    T, LB = T.cpu().numpy().astype(np.float64), LB.cpu().numpy().astype(np.float64)
    _, ids, _, _ = ix.export()
    ids = ids.cpu().numpy()
    info = bins.get()
    sel, beta = info["sel"], info["beta"]
    Xd = X.astype(np.float64)
    for b in range(B):
        d2 = np.sum((Xd[ids] - Q[b].astype(np.float64)) ** 2, axis=1)
        assert np.all(LB[b] <= d2 * (1 + 1e-12)), b
    # tables: never above 2*mind^2 of the exact query values (Eq. 3), and no
    # lower than that gap shrunk by the projection bounds of data and query
    # plus the FP32 rounding of the breakpoints
    qv = oracle.dft_pool(Q, 16)[:, sel]
    # (the table widens by eta_x + eta_q around the GPU's own query value, which
    # is itself within eta_q of the exact one)
    eta = ix.info()["eta_x"] + 2 * bins.eta_per_norm * np.sqrt(np.sum(Q.astype(np.float64) ** 2, 1))
    for b in range(B):
        for j in range(16):
            shrink = 1.01 * eta[b] + 2.0 ** -23 * np.max(np.abs(beta[j]))
            for s in range(0, 256, 3):
                m = oracle.mind(qv[b, j], s, beta[j])
                assert T[b, j, s] <= 2.0 * m * m * (1 + 1e-12) + 1e-30
                lo = 2.0 * max(0.0, m - shrink) ** 2 * (1 - 1e-6)
                assert T[b, j, s] >= lo - 1e-12, (b, j, s, T[b, j, s], lo)


def _check_knn(ids, d, ref_ids, ref_d2):
    assert np.array_equal(ids, ref_ids)
    ref = np.sqrt(ref_d2)
    assert np.all(np.abs(d.astype(np.float64) - ref) <= 1e-6 * np.maximum(ref, 1e-30))


@pytest.mark.parametrize("k", [1, 10, 100])
def test_knn_matches_oracle_mix(gpu_lib, k):
    N, n, B = 30000 + 11, 256, 48
    X = synth.collection(N, n, "mix", seed=21)
    X[1000] = X[20]            # exact duplicates: ties go to the lower row id
    X[29000] = X[20]
    Q, src = synth.queries(X, B, sigma=0.1, seed=22)
    Q[0] = X[20]               # query equal to three rows
    Q[1] = synth.collection(1, n, "hf", seed=1234)[0]   # a far query
    bins = _bins(gpu_lib, X, 3000)
    ix = gpu_lib.Index(bins, _t(X))
    ids, d = ix.knn(_t(Q), k)
    ref_ids, ref_d2 = oracle.knn(X, Q, k)
    _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    if k >= 3:
        assert ids[0, :3].cpu().tolist() == [20, 1000, 29000]


def test_knn_small_config_plain(gpu_lib):
    """100,000 random walks x 256, bins from a 10,000-row stride sample,
    100 noisy-copy queries (sigma 0.1), exact 1-NN."""
    N, n = 100000, 256
    X = synth.collection(N, n, "rw", seed=1)
    Q, src = synth.queries(X, 100, sigma=0.1, seed=2)
    bins = _bins(gpu_lib, X, 10000)
    ix = gpu_lib.Index(bins, _t(X))
    ids, d = ix.knn(_t(Q), 1)
    ref_ids, ref_d2 = oracle.knn(X, Q, 1)
    _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    st = ix.stats()
    assert st["leaves_visited"] < st["leaves_total"]


@pytest.mark.parametrize("n,L,N", [(100, 64, 5000 + 3), (64, 512, 9000 + 1), (512, 256, 4000 + 5),
                                   (1024, 64, 2000 + 7)])
def test_knn_ragged_shapes(gpu_lib, n, L, N):
    P = min(16, n // 2 - 1)
    X = synth.collection(N, n, "mix", seed=31 + n)
    Q, _ = synth.queries(X, 16, sigma=0.1, seed=32)
    bins = _bins(gpu_lib, X, min(N, 2000), pool=P)
    ix = gpu_lib.Index(bins, _t(X), leaf_size=L)
    for k in (1, 7, 70):
        ids, d = ix.knn(_t(Q), k)
        ref_ids, ref_d2 = oracle.knn(X, Q, k)
        _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)


@pytest.mark.parametrize("N", [1, 5, 64, 65, 257])
def test_knn_degenerate_sizes(gpu_lib, N):
    """Collections smaller than a leaf or a 256-row chunk, a single row, and
    k up to N (every row returned): ids equal to the oracle's on the plain
    scan and on both batched-distance tiers, with bins from all N rows."""
    n = 64
    X = synth.collection(N, n, "mix", seed=281 + N)
    Q = np.empty((6, n), dtype=np.float32)
    Q[:4], _ = synth.queries(X, 4, sigma=0.1, seed=282)
    Q[4] = X[N - 1]                                           # exact copy
    Q[5] = synth.collection(1, n, "hf", seed=283)[0]          # unrelated series
    bins = _bins(gpu_lib, X, N)
    ix = gpu_lib.Index(bins, _t(X), leaf_size=256, precision=3)
    ix64 = gpu_lib.Index(bins, _t(X), leaf_size=64)
    for k in sorted({1, min(N, 5), min(N, 100)}):
        ref_ids, ref_d2 = oracle.knn(X, Q, k)
        for index, prune in ((ix64, 0), (ix, 0), (ix, 1), (ix, 2)):
            ids, d = index.knn(_t(Q), k, prune=prune)
            _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)


@pytest.mark.parametrize("alpha", [1, 2])
def test_knn_alphabet_of_one_and_two(gpu_lib, alpha):
    """Degenerate alphabets: with one symbol every word bound is 0, so the
    plain scan visits every leaf; with two, one breakpoint per value.  The
    answer is still the oracle's on the plain scan and both prune tiers."""
    N, n, B = 3000 + 3, 128, 10
    X = synth.collection(N, n, "mix", seed=291)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=292)
    bins = _bins(gpu_lib, X, 1000, alpha=alpha)
    ix = gpu_lib.Index(bins, _t(X), leaf_size=256, precision=3)
    ref_ids, ref_d2 = oracle.knn(X, Q, 10)
    for prune in (0, 1, 2):
        ids, d = ix.knn(_t(Q), 10, prune=prune)
        _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
        st = ix.stats()  # the last call's counters
        if alpha == 1 and prune == 0:
            assert st["leaves_visited"] == st["leaves_total"]


def test_knn_constant_series(gpu_lib):
    """A constant series z-normalises to zeros (population sigma 0).  A zero
    query is at d^2 = |x|^2 (= n up to the FP32 rounding of each row) from
    every row, so every row falls inside the FP32 band and the order comes
    from the FP64 ranking alone; zero rows in the collection sit at |q|^2
    from every query.  Plain scan and both prune tiers against the oracle."""
    N, n = 5000 + 3, 64
    X = synth.collection(N, n, "mix", seed=301)
    X[[10, 2000, 4999]] = 0.0
    Q = np.empty((4, n), dtype=np.float32)
    Q[0] = 0.0
    Q[1] = X[7]
    Q[2:], _ = synth.queries(X, 2, sigma=0.1, seed=302)
    bins = _bins(gpu_lib, X, 2000)
    ix = gpu_lib.Index(bins, _t(X), leaf_size=256, precision=3)
    for k in (1, 10, 100):
        ref_ids, ref_d2 = oracle.knn(X, Q, k)
        for prune in (0, 1, 2):
            ids, d = ix.knn(_t(Q), k, prune=prune)
            _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)


def test_knn_radius_paths_are_exact(gpu_lib):
    import torch
    N, n, B, k = 20000, 256, 32, 10
    X = synth.collection(N, n, "mix", seed=41)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=42)
    bins = _bins(gpu_lib, X, 2000)
    ix = gpu_lib.Index(bins, _t(X))
    ref_ids, ref_d2 = oracle.knn(X, Q, k)
    kth = np.sqrt(ref_d2[:, -1]).astype(np.float32)
    for radius in (np.full(B, 1e-3, np.float32),          # every query misses -> fallback
                   np.full(B, 1e3, np.float32),           # loose
                   kth * np.float32(1.001),               # just outside the k-th
                   kth * np.float32(0.999)):              # just inside: fallback
        ids, d = ix.knn(_t(Q), k, radius=_t(radius))
        _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    ids, d = ix.knn(_t(Q), k, radius=_t(np.full(B, 1e-3, np.float32)))
    assert ix.stats()["radius_fallbacks"] == B


def test_knn_many_exact_ties_take_exhaustive_pass(gpu_lib):
    N, n = 8000, 128
    X = synth.collection(N, n, "rw", seed=51)
    dup = np.sort(np.random.default_rng(0).choice(np.arange(1, N), 300, replace=False))
    X[dup] = X[0]
    Q = np.stack([X[0], X[5]])
    bins = _bins(gpu_lib, X, 2000)
    ix = gpu_lib.Index(bins, _t(X), leaf_size=64)
    for k in (1, 5, 90):
        ids, d = ix.knn(_t(Q), k)
        ref_ids, ref_d2 = oracle.knn(X, Q, k)
        _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)


def test_knn_band_overflow_ranked_from_refined_rows(gpu_lib):
    """1,500 copies of one row: more rows tie inside the final band than the
    finalize ranks in one workgroup (1,024).  The BF16 path keeps every
    in-band candidate in the query's list of refined rows, so the band is
    ranked in FP64 from that list, with no exhaustive pass.  The plain
    path's per-wave lists evict tied rows, and the eviction sends the query
    to the exhaustive pass.  Both answers are the oracle's."""
    N, n = 12000, 128
    X = synth.collection(N, n, "rw", seed=53)
    dup = np.sort(np.random.default_rng(1).choice(np.arange(1, N), 1500, replace=False))
    X[dup] = X[0]
    Q = np.stack([X[0], X[7]])
    bins = _bins(gpu_lib, X, 2000)
    ix = gpu_lib.Index(bins, _t(X), leaf_size=256, precision=1)
    for prune in (0, 1):
        for k in (1, 10, 100):
            ids, d = ix.knn(_t(Q), k, prune=prune)
            ref_ids, ref_d2 = oracle.knn(X, Q, k)
            _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
            st = ix.stats()
            if prune == 1:
                assert st["overflow_band"] == 1 and st["overflow_fallbacks"] == 0, (k, st)
            else:
                assert st["overflow_evicted"] == 1 and st["overflow_fallbacks"] == 1, (k, st)


@pytest.mark.parametrize("n,prec", [(64, 1), (1024, 2)])
def test_finalize_ranks_bands_over_several_batches(gpu_lib, n, prec):
    """The finalize stages the in-band rows in LDS a batch at a time: 64
    rows at n = 64 and 4 at n = 1024. Query 0 has 180 exact copies, so its
    final band holds 181 rows at distance zero. That spans 3 batches at
    n = 64 and 46 at n = 1024. Ids (ties to the lower row id) and distances
    are the oracle's on the plain path and on the prune tier of the index's
    copy: BF16 at n = 64, FP8 at n = 1024."""
    N = 4000 + 3
    X = synth.collection(N, n, "rw", seed=61 + n)
    dup = np.sort(np.random.default_rng(2).choice(np.arange(1, N), 180, replace=False))
    X[dup] = X[0]
    Q = np.stack([X[0], X[11]])
    bins = _bins(gpu_lib, X, 2000)
    ix = gpu_lib.Index(bins, _t(X), leaf_size=256, precision=prec)
    for prune in (0, prec):
        for k in (10, 100):
            ids, d = ix.knn(_t(Q), k, prune=prune)
            ref_ids, ref_d2 = oracle.knn(X, Q, k)
            _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)


def test_knn_tiny_candidate_capacity_stays_exact(gpu_lib):
    N, n, B = 20000, 256, 24
    X = synth.collection(N, n, "mix", seed=81)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=82)
    bins = _bins(gpu_lib, X, 2000)
    ix = gpu_lib.Index(bins, _t(X))
    for k, cap in ((1, 1), (10, 4), (10, 40)):
        ids, d = ix.knn(_t(Q), k, candidate_capacity=cap)
        ref_ids, ref_d2 = oracle.knn(X, Q, k)
        _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    assert ix.stats()["overflow_fallbacks"] > 0


def test_knn_counters_consistent(gpu_lib):
    N, n, B, L = 20000 + 5, 256, 16, 64
    X = synth.collection(N, n, "mix", seed=91)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=92)
    bins = _bins(gpu_lib, X, 2000)
    ix = gpu_lib.Index(bins, _t(X), leaf_size=L)
    for k in (1, 10):
        ix.knn(_t(Q), k)
        st = ix.stats()
        nl = ix.info()["n_leaves"]
        assert st["leaves_total"] == B * nl
        assert 0 < st["leaves_visited"] <= st["leaves_total"]
        assert st["series_refined"] <= st["series_lb_checked"] <= st["leaves_visited"] * L
        assert st["series_refined"] >= k * B
        assert st["overflow_fallbacks"] == 0
    # with no bound at all every row of every query is refined
    ix.knn(_t(Q[:2]), 1, radius=None, no_seed_leaf=True)


def test_knn_no_seed_and_repeatable(gpu_lib):
    N, n = 15000, 256
    X = synth.collection(N, n, "mix", seed=61)
    Q, _ = synth.queries(X, 20, sigma=0.1, seed=62)
    bins = _bins(gpu_lib, X, 2000)
    ix = gpu_lib.Index(bins, _t(X))
    a_ids, a_d = ix.knn(_t(Q), 5)
    b_ids, b_d = ix.knn(_t(Q), 5, no_seed_leaf=True)
    c_ids, c_d = ix.knn(_t(Q), 5)
    assert np.array_equal(a_ids.cpu().numpy(), b_ids.cpu().numpy())
    assert np.array_equal(a_ids.cpu().numpy(), c_ids.cpu().numpy())
    assert np.array_equal(a_d.cpu().numpy(), c_d.cpu().numpy())


def test_errors_are_reported(gpu_lib):
    import torch
    N, n = 2000, 64
    X = synth.collection(N, n, "rw", seed=71)
    bins = _bins(gpu_lib, X, 500, pool=8)
    ix = gpu_lib.Index(bins, _t(X), leaf_size=64)
    Q = X[:3].copy()
    Q[1, 5] = np.nan
    with pytest.raises(gpu_lib.SofaError) as e:
        ix.knn(_t(Q), 1)
    assert e.value.status == gpu_lib.SOFA_EINVAL
    with pytest.raises(gpu_lib.SofaError):
        ix.knn(_t(X[:2]), 0)
    with pytest.raises(gpu_lib.SofaError):
        ix.knn(_t(X[:2]), 101)
    Xb = X.copy()
    Xb[7, 3] = np.inf
    with pytest.raises(gpu_lib.SofaError):
        gpu_lib.Index(bins, _t(Xb))
    ids, d = ix.knn(_t(X[:0]), 3)
    assert ids.shape == (0, 3)
    ws = gpu_lib.Workspace(max_bytes=1024)
    with pytest.raises(gpu_lib.SofaError) as e:
        ix.knn(_t(X[:4]), 1, ws=ws)
    assert e.value.status == gpu_lib.SOFA_ENOMEM


# --------------------------------------------------------------------------- #
# BF16 batched-distance prune
def _bf16_index(gpu_lib, X, m=2000, L=256):
    bins = _bins(gpu_lib, X, m)
    return bins, gpu_lib.Index(bins, _t(X), leaf_size=L, precision=1)


def test_bf16_lower_bounds_never_exceed_distance(gpu_lib):
    """The MFMA bound is below the FP64 distance on every pair, including
    near-duplicates, rows far from unit scale and values on BF16 ties."""
    N, n, B = 4096 + 17, 256, 40
    X = synth.collection(N, n, "mix", seed=201)
    rng = np.random.default_rng(5)
    X[10] *= np.float32(300.0)                       # large magnitude
    X[11] *= np.float32(1e-3)                        # small magnitude
    X[12] = (np.round(X[12] * 128) / 128 + 2.0 ** -9).astype(np.float32)  # BF16 ties
    Q, _ = synth.queries(X, B, sigma=0.1, seed=202)
    Q[0] = X[7]                                                  # exact copy
    Q[1] = X[8] + np.float32(1e-4) * rng.standard_normal(n).astype(np.float32)  # near copy
    Q[2] = X[10] * np.float32(1.0001)                            # near the large row
    Q[3] = X[12]
    Q[4] = X[11]
    bins, ix = _bf16_index(gpu_lib, X)
    LB = ix.bf16_lower_bounds(_t(Q)).cpu().numpy().astype(np.float64)
    _, ids, _, _ = ix.export()
    ids = ids.cpu().numpy()
    Xd = X.astype(np.float64)[ids]
    rel = []
    for b in range(B):
        d2 = np.sum((Xd - Q[b].astype(np.float64)) ** 2, axis=1)
        assert np.all(LB[b] <= d2 * (1 + 1e-12) + 1e-30), (b, float(np.max(LB[b] - d2)))
        rel.append((d2 - LB[b]) / np.maximum(d2, 1.0))
    # useful on typical pairs (the leaf holding the scaled row is loose by design:
    # its bound uses the leaf's largest BF16 residual)
    assert np.median(np.concatenate(rel)) < 0.02


@pytest.mark.parametrize("k", [1, 10, 100])
def test_bf16_knn_matches_oracle(gpu_lib, k):
    N, n, B = 30000 + 11, 256, 48
    X = synth.collection(N, n, "mix", seed=211)
    X[1000] = X[20]
    X[29000] = X[20]
    Q, _ = synth.queries(X, B, sigma=0.1, seed=212)
    Q[0] = X[20]
    Q[1] = synth.collection(1, n, "hf", seed=4321)[0]
    bins, ix = _bf16_index(gpu_lib, X)
    ids, d = ix.knn(_t(Q), k, prune=1)
    ref_ids, ref_d2 = oracle.knn(X, Q, k)
    _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    st = ix.stats()
    assert st["series_bf16_checked"] > 0
    assert st["overflow_fallbacks"] == 0


def test_bf16_knn_radius_and_capacity_paths(gpu_lib):
    N, n, B, k = 40000, 256, 40, 10
    X = synth.collection(N, n, "mix", seed=221)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=222)
    bins, ix = _bf16_index(gpu_lib, X, L=512)
    ref_ids, ref_d2 = oracle.knn(X, Q, k)
    kth = np.sqrt(ref_d2[:, -1]).astype(np.float32)
    for radius in (None, np.full(B, 1e-3, np.float32), np.full(B, 1e3, np.float32),
                   kth * np.float32(1.0005), kth * np.float32(0.999)):
        ids, d = ix.knn(_t(Q), k, prune=1, radius=None if radius is None else _t(radius))
        _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    ids, d = ix.knn(_t(Q), k, prune=1, radius=_t(kth * np.float32(1.0005)))
    tight = ix.stats()
    ids, d = ix.knn(_t(Q), k, prune=1)
    loose = ix.stats()
    assert tight["radius_fallbacks"] == 0
    assert tight["series_refined"] <= loose["series_refined"]
    ids, d = ix.knn(_t(Q), k, prune=1, candidate_capacity=8)
    _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    assert ix.stats()["overflow_fallbacks"] > 0


def test_bf16_small_n_and_ragged(gpu_lib):
    for n, N in ((64, 9000 + 7), (128, 7000 + 3)):
        X = synth.collection(N, n, "mix", seed=231 + n)
        Q, _ = synth.queries(X, 20, sigma=0.1, seed=232)
        bins = _bins(gpu_lib, X, 2000, pool=min(16, n // 2 - 1))
        ix = gpu_lib.Index(bins, _t(X), leaf_size=256, precision=1)
        for k in (1, 9):
            ids, d = ix.knn(_t(Q), k, prune=1)
            ref_ids, ref_d2 = oracle.knn(X, Q, k)
            _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)


def test_bf16_argument_errors(gpu_lib):
    X = synth.collection(3000, 256, "rw", seed=241)
    bins = _bins(gpu_lib, X, 1000)
    plain = gpu_lib.Index(bins, _t(X))
    with pytest.raises(gpu_lib.SofaError):
        plain.knn(_t(X[:2]), 1, prune=1)
    with pytest.raises(gpu_lib.SofaError):
        gpu_lib.Index(bins, _t(X), leaf_size=64, precision=1)
    X5 = synth.collection(3000, 512, "rw", seed=242)
    b5 = _bins(gpu_lib, X5, 1000)
    with pytest.raises(gpu_lib.SofaError):
        gpu_lib.Index(b5, _t(X5), precision=1)


# --------------------------------------------------------------------------- #
# stored oracle answers (tests/golden, written from the oracle alone)
def test_golden_small_rw64(gpu_lib):
    import json
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "small_rw64.json")) as f:
        g = json.load(f)
    c = g["case"]
    X = synth.collection(c["N"], c["n"], c["kind"], seed=c["seed"])
    Q, _ = synth.queries(X, c["B"], sigma=c["sigma"], seed=c["qseed"])
    bins = _bins(gpu_lib, X, c["m"], alpha=c["alpha"], binning=c["binning"], pool=c["P"])
    info = bins.get()
    assert info["sel"].tolist() == g["sel"]
    ref_beta = np.array([[float.fromhex(v) for v in row] for row in g["beta_hex"]])
    assert np.max(np.abs(info["beta"] - ref_beta)) <= 1e-12 * np.max(np.abs(ref_beta))
    ref_d = np.sqrt(np.array([[float.fromhex(v) for v in row] for row in g["knn_d2_hex"]]))
    for prec, prune in ((0, 0), (3, 1), (3, 2)):
        ix = gpu_lib.Index(bins, _t(X), leaf_size=256, precision=prec)
        ids, d = ix.knn(_t(Q), c["k"], prune=prune)
        assert ids.cpu().numpy().tolist() == g["knn_ids"], prune
        assert np.all(np.abs(d.cpu().numpy() - ref_d) <= 1e-6 * ref_d)


# --------------------------------------------------------------------------- #
# FP8 (e4m3) tier
def _fp8_index(gpu_lib, X, m=2000, L=256, precision=2):
    bins = _bins(gpu_lib, X, m)
    return bins, gpu_lib.Index(bins, _t(X), leaf_size=L, precision=precision)


def test_fp8_lower_bounds_never_exceed_distance(gpu_lib):
    """The FP8 MFMA bound is below the FP64 distance on every pair: near
    copies, a row that sets its chunk's scale, rows in the e4m3 subnormal
    range, values half-way between e4m3 codes."""
    N, n, B = 4096 + 17, 256, 40
    X = synth.collection(N, n, "mix", seed=251)
    rng = np.random.default_rng(6)
    X[10] *= np.float32(300.0)                       # sets chunk 0's scale
    X[11] *= np.float32(1e-5)                        # subnormal after scaling
    X[300] *= np.float32(2e-3)
    # half-way values of the e4m3 grid (for a unit scale): 1 + 1/16 lies
    # between the codes 1 and 1 + 1/8
    X[600] = np.where(np.arange(n) % 2 == 0, 1.0625, -1.0625).astype(np.float32)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=252)
    Q[0] = X[7]
    Q[1] = X[8] + np.float32(1e-4) * rng.standard_normal(n).astype(np.float32)
    Q[2] = X[10] * np.float32(1.0001)
    Q[3] = X[11]
    Q[4] = X[600]
    Q[5] = X[300] * np.float32(1e3)
    bins, ix = _fp8_index(gpu_lib, X)
    assert ix.info()["has_fp8"] == 1
    LB = ix.fp8_lower_bounds(_t(Q)).cpu().numpy().astype(np.float64)
    _, ids, _, _ = ix.export()
    ids = ids.cpu().numpy()
    Xd = X.astype(np.float64)[ids]
    rel = []
    for b in range(B):
        d2 = np.sum((Xd - Q[b].astype(np.float64)) ** 2, axis=1)
        assert np.all(LB[b] <= d2 * (1 + 1e-12) + 1e-30), (b, float(np.max(LB[b] - d2)))
        rel.append((d2 - LB[b]) / np.maximum(d2, 1.0))
    # e4m3 keeps 3 fraction bits: the slack is a few percent of |q||x| on
    # typical pairs, far below the distance between unrelated series
    assert np.median(np.concatenate(rel)) < 0.2


@pytest.mark.parametrize("k", [1, 10, 100])
def test_fp8_knn_matches_oracle(gpu_lib, k):
    N, n, B = 30000 + 11, 256, 48
    X = synth.collection(N, n, "mix", seed=261)
    X[1000] = X[20]
    X[29000] = X[20]
    Q, _ = synth.queries(X, B, sigma=0.1, seed=262)
    Q[0] = X[20]
    Q[1] = synth.collection(1, n, "hf", seed=4331)[0]
    bins, ix = _fp8_index(gpu_lib, X, precision=3)
    ids, d = ix.knn(_t(Q), k, prune=2)
    ref_ids, ref_d2 = oracle.knn(X, Q, k)
    _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    st = ix.stats()
    assert st["series_bf16_checked"] > 0
    assert st["overflow_fallbacks"] == 0
    # the BF16 tier of the same index gives the same answer
    ids1, d1 = ix.knn(_t(Q), k, prune=1)
    assert np.array_equal(ids1.cpu().numpy(), ids.cpu().numpy())


def test_fp8_knn_radius_and_capacity_paths(gpu_lib):
    N, n, B, k = 40000, 256, 40, 10
    X = synth.collection(N, n, "mix", seed=271)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=272)
    bins, ix = _fp8_index(gpu_lib, X, L=512)
    ref_ids, ref_d2 = oracle.knn(X, Q, k)
    kth = np.sqrt(ref_d2[:, -1]).astype(np.float32)
    for radius in (None, np.full(B, 1e-3, np.float32), np.full(B, 1e3, np.float32),
                   kth * np.float32(1.0005), kth * np.float32(0.999)):
        for sampling in (0, 2):
            ids, d = ix.knn(_t(Q), k, prune=2, sampling=sampling,
                            radius=None if radius is None else _t(radius))
            _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    ids, d = ix.knn(_t(Q), k, prune=2, candidate_capacity=8)
    _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    assert ix.stats()["overflow_fallbacks"] > 0


def test_fp8_lower_bounds_never_exceed_distance_1024(gpu_lib):
    """Rows of 1024 values (16 K steps, one wave per SIMD): the FP8 bound
    stays below the FP64 distance on every pair."""
    N, n, B = 2048 + 9, 1024, 24
    X = synth.collection(N, n, "mix", seed=255)
    X[5] *= np.float32(200.0)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=256)
    Q[0] = X[3]
    Q[1] = X[5] * np.float32(1.0001)
    bins, ix = _fp8_index(gpu_lib, X)
    LB = ix.fp8_lower_bounds(_t(Q)).cpu().numpy().astype(np.float64)
    _, ids, _, _ = ix.export()
    Xd = X.astype(np.float64)[ids.cpu().numpy()]
    for b in range(B):
        d2 = np.sum((Xd - Q[b].astype(np.float64)) ** 2, axis=1)
        assert np.all(LB[b] <= d2 * (1 + 1e-12) + 1e-30), (b, float(np.max(LB[b] - d2)))


def test_prune_bounds_fuzz_ten_million_pairs(gpu_lib):
    """Both batched-distance bounds (BF16 and FP8, one index holding both
    copies) stay below the FP64 distance on 12.6M pairs: 262,157 rows, one
    in 509 of them scaled by 1e-4 to 316 (log-uniform), so that FP8 chunk
    scales vary and small rows fall into the e4m3 subnormal range, rows on
    BF16 ties, and 48 queries: noisy copies, near and exact copies (also of
    scaled rows) and unrelated series."""
    N, n = (1 << 18) + 13, 256
    X = synth.collection(N, n, "mix", seed=271)
    rng = np.random.default_rng(272)
    scaled = np.arange(0, N, 509)
    X[scaled] *= (10.0 ** rng.uniform(-4.0, 2.5, scaled.size)).astype(np.float32)[:, None]
    X[3:7] = (np.round(X[3:7] * 128) / 128 + 2.0 ** -9).astype(np.float32)
    Q = np.empty((48, n), dtype=np.float32)
    Q[:16], _ = synth.queries(X, 16, sigma=0.1, seed=273)
    near = rng.integers(0, N, 8)
    Q[16:24] = X[near] + np.float32(1e-4) * rng.standard_normal((8, n)).astype(np.float32)
    Q[24:28] = X[rng.integers(0, N, 4)]                       # exact copies
    Q[28:32] = X[scaled[rng.integers(0, scaled.size, 4)]]     # exact copies of scaled rows
    Q[32:40] = X[scaled[rng.integers(0, scaled.size, 8)]] * np.float32(1.0001)
    Q[40:44] = X[3:7]                                         # rows on BF16 ties
    Q[44:48] = synth.collection(4, n, "mix", seed=274)        # unrelated series
    bins, ix = _fp8_index(gpu_lib, X, m=4000, precision=3)
    Qd = _t(Q)
    LBb = ix.bf16_lower_bounds(Qd).cpu().numpy().astype(np.float64)
    LBf = ix.fp8_lower_bounds(Qd).cpu().numpy().astype(np.float64)
    _, ids, _, _ = ix.export()
    Xd = X.astype(np.float64)[ids.cpu().numpy()]
    for b in range(Q.shape[0]):
        d2 = np.sum((Xd - Q[b].astype(np.float64)) ** 2, axis=1)
        lim = d2 * (1 + 1e-12) + 1e-30
        assert np.all(LBb[b] <= lim), ("bf16", b, float(np.max(LBb[b] - d2)))
        assert np.all(LBf[b] <= lim), ("fp8", b, float(np.max(LBf[b] - d2)))


def test_fp8_lengths_64_to_1024(gpu_lib):
    for n, N in ((64, 9000 + 7), (128, 7000 + 3), (512, 6000 + 5), (1024, 5000 + 3)):
        X = synth.collection(N, n, "mix", seed=281 + n)
        Q, _ = synth.queries(X, 20, sigma=0.1, seed=282)
        bins = _bins(gpu_lib, X, 2000, pool=min(16, n // 2 - 1))
        ix = gpu_lib.Index(bins, _t(X), leaf_size=256, precision=2)
        for k in (1, 9):
            ids, d = ix.knn(_t(Q), k, prune=2)
            ref_ids, ref_d2 = oracle.knn(X, Q, k)
            _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)


def test_fp8_argument_errors(gpu_lib):
    X = synth.collection(3000, 256, "rw", seed=291)
    bins = _bins(gpu_lib, X, 1000)
    bf = gpu_lib.Index(bins, _t(X), precision=1)
    with pytest.raises(gpu_lib.SofaError):
        bf.knn(_t(X[:2]), 1, prune=2)
    with pytest.raises(gpu_lib.SofaError):
        bf.fp8_lower_bounds(_t(X[:2]))
    with pytest.raises(gpu_lib.SofaError):
        bf.knn(_t(X[:2]), 1, prune=3)
    with pytest.raises(gpu_lib.SofaError):
        gpu_lib.Index(bins, _t(X), leaf_size=64, precision=2)
    # every supported length (n <= 1024) has the FP8 tier; longer series
    # are rejected when the bins are learned
    X20 = synth.collection(1000, 2048, "rw", seed=292)
    with pytest.raises(gpu_lib.SofaError):
        _bins(gpu_lib, X20, 500)


# --------------------------------------------------------------------------- #
# learned radius network
def _mlp_params(seed, D=32, H1=256, H2=256):
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((H1, D)) * np.sqrt(2.0 / D)
    b1 = rng.standard_normal(H1) * 0.1
    W2 = rng.standard_normal((H2, H1)) * np.sqrt(2.0 / H1)
    b2 = rng.standard_normal(H2) * 0.1
    W3 = rng.standard_normal(H2) * np.sqrt(1.0 / H2)
    b3 = 0.7
    flat = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, [b3]]).astype(np.float32)
    return flat


def _unflat(flat, D=32, H1=256, H2=256, bf16=True):
    f = flat.astype(np.float64)
    o = 0
    W1 = f[o:o + H1 * D].reshape(H1, D); o += H1 * D
    b1 = f[o:o + H1]; o += H1
    W2 = f[o:o + H2 * H1].reshape(H2, H1); o += H2 * H1
    b2 = f[o:o + H2]; o += H2
    W3 = f[o:o + H2]; o += H2
    b3 = f[o]
    if bf16:
        W1, W2, W3 = oracle.to_bf16(W1), oracle.to_bf16(W2), oracle.to_bf16(W3)
    return oracle.MLPParams(W1, b1, W2, b2, W3, b3)


def _mlp_data(seed, B, D=32):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, D)).astype(np.float32)
    t = (rng.standard_normal(B) * 0.5 + 1.0).astype(np.float32)
    return x, t


def test_mlp_forward_matches_oracle(gpu_lib):
    """Forward pass against the FP64 oracle, element by element, within the
    FP32 error bound of tests/mlp_bound.py (8 sigma of the rounding-error
    model, propagated through both layers)."""
    flat = _mlp_params(1)
    m = gpu_lib.RadiusModel(k=10)
    m.set(params=flat, mu=np.zeros(32), sd=np.ones(32), margin=0.0)
    x, _ = _mlp_data(2, 300)
    y = m.forward(_t(x)).cpu().numpy().astype(np.float64)
    ref = oracle.mlp_forward(_unflat(flat), x)
    _, bound, _ = mlp_bound.forward_bound(_unflat(flat), x)
    assert np.all(np.abs(y - ref) <= bound), np.max(np.abs(y - ref) / bound)
    # standardisation: (x - mu) / sd applied to the inputs (formed in FP32 on
    # both sides; the bound allows each input four roundings)
    mu = np.linspace(-1, 1, 32).astype(np.float32)
    sd = np.linspace(0.5, 2, 32).astype(np.float32)
    m.set(mu=mu, sd=sd)
    y2 = m.forward(_t(x)).cpu().numpy().astype(np.float64)
    xs = ((x - mu) / sd).astype(np.float32)
    ref2 = oracle.mlp_forward(_unflat(flat), xs)
    _, bound2, _ = mlp_bound.forward_bound(_unflat(flat), xs, xs_rounded=True)
    assert np.all(np.abs(y2 - ref2) <= bound2), np.max(np.abs(y2 - ref2) / bound2)


def test_radius_predict_is_forward_plus_margin(gpu_lib):
    """The radii of sofa_radius_predict come from one fused kernel (the one
    a search uses for its radii) that repeats the forward kernels'
    operations in their order: they are exp(y + margin) of sofa_radius_forward's
    y bit for bit, with standardisation, on 301 rows (not a multiple of the
    kernel's 4 rows per workgroup) and on a single row."""
    flat = _mlp_params(1)
    m = gpu_lib.RadiusModel(k=10)
    mu = np.linspace(-1, 1, 32).astype(np.float32)
    sd = np.linspace(0.5, 2, 32).astype(np.float32)
    m.set(params=flat, mu=mu, sd=sd, margin=0.1875)
    for B in (301, 1):
        x, _ = _mlp_data(6 + B, B)
        y = m.forward(_t(x)).cpu().numpy()
        r = m.predict(_t(x)).cpu().numpy()
        ref = np.exp(y.astype(np.float64) + 0.1875).astype(np.float32)
        assert np.array_equal(r, ref), np.max(np.abs(r / ref - 1))


def test_mlp_gradients_match_oracle(gpu_lib):
    """Every gradient element and the loss against the FP64 oracle, within
    the element-wise FP32 error bound of tests/mlp_bound.py."""
    flat = _mlp_params(3)
    m = gpu_lib.RadiusModel(k=10)
    m.set(params=flat, mu=np.zeros(32), sd=np.ones(32))
    x, t = _mlp_data(4, 257)
    g, loss = m.gradients(_t(x), _t(t))
    g = g.cpu().numpy().astype(np.float64)
    ref_loss, rg = oracle.mlp_backward(_unflat(flat), x, t)
    ref = np.concatenate([rg["W1"].ravel(), rg["b1"], rg["W2"].ravel(), rg["b2"], rg["W3"], rg["b3"]])
    _, bound, _, loss_bound = mlp_bound.gradient_bound(_unflat(flat), x, t)
    assert abs(float(loss.cpu()[0]) - ref_loss) <= loss_bound
    bad = np.abs(g - ref) > bound
    assert not bad.any(), (np.flatnonzero(bad)[:10], np.max(np.abs(g - ref) / bound))


def test_mlp_adam_steps_match_oracle(gpu_lib):
    flat = _mlp_params(5)
    lr = 1e-3
    m = gpu_lib.RadiusModel(k=1, lr=lr)
    m.set(params=flat, mu=np.zeros(32), sd=np.ones(32))
    p = flat.astype(np.float64).copy()
    mom, vel = np.zeros_like(p), np.zeros_like(p)
    for step in (1, 2):
        x, t = _mlp_data(10 + step, 200)
        m.train_step(_t(x), _t(t))
        _, rg = oracle.mlp_backward(_unflat(p.astype(np.float32)), x, t)
        g = np.concatenate([rg["W1"].ravel(), rg["b1"], rg["W2"].ravel(), rg["b2"], rg["W3"], rg["b3"]])
        oracle.adam(p, g, mom, vel, step, lr=lr)
        got = m.get()["params"].astype(np.float64)
        assert m.get()["step"] == step
        # elements whose gradient is clear of zero move exactly as the oracle's
        clear = np.abs(g) > 1e-3 * np.max(np.abs(g))
        assert np.max(np.abs(got - p)[clear]) <= 2e-6
        assert np.mean(np.abs(got - p) <= 2.5 * lr) == 1.0


def test_learned_radius_search_is_exact(gpu_lib):
    import torch
    N, n, k = 40000, 256, 10
    X = synth.collection(N, n, "mix", seed=301)
    bins, ix = _bf16_index(gpu_lib, X)
    Qtr, _ = synth.queries(X, 3000, sigma=0.1, seed=302)
    Qte, _ = synth.queries(X, 64, sigma=0.1, seed=303)
    ids_tr, d_tr = ix.knn(_t(Qtr), k)                   # labels from the plain path
    target = torch.log(d_tr[:, -1]).contiguous()
    feat, _, _ = bins.transform(_t(Qtr), sel=False, words=False)
    m = gpu_lib.RadiusModel(k=k, seed=7)
    m.standardize(feat)
    losses = m.fit(feat[:2500].contiguous(), target[:2500].contiguous(), epochs=30, batch=250)
    assert losses[-1] < losses[0]
    m.calibrate(feat[2500:].contiguous(), target[2500:].contiguous(), 0.99)
    ref_ids, ref_d2 = oracle.knn(X, Qte, k)
    for prune in (0, 1):
        ids, d = ix.knn(_t(Qte), k, prune=prune, model=m)
        _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    st = ix.stats()
    assert st["radius_fallbacks"] <= 16
    m1 = gpu_lib.RadiusModel(k=1)
    with pytest.raises(gpu_lib.SofaError):
        ix.knn(_t(Qte), k, model=m1)


def test_learned_radius_gains_over_the_search_without_it(gpu_lib):
    """What the trained network buys: with the predicted radius seeding the
    bound, the same exact answers need fewer exact distances (FP32 refine)
    than the search seeded by the best leaf alone, on both the plain SFA scan
    and the BF16 prune.  Trained on the GPU by the library's own kernels."""
    import torch
    N, n = 60000, 256
    X = synth.collection(N, n, "mix", seed=311)
    bins, ix = _bf16_index(gpu_lib, X)
    Qtr, _ = synth.queries(X, 4000, sigma=0.1, seed=312)
    Qte, _ = synth.queries(X, 96, sigma=0.1, seed=313)
    feat, _, _ = bins.transform(_t(Qtr), sel=False, words=False)
    gains = {}
    for k in (1, 10):
        _, d_tr = ix.knn(_t(Qtr), k, prune=1)
        target = torch.log(d_tr[:, -1]).contiguous()
        m = gpu_lib.RadiusModel(k=k, seed=17)
        m.standardize(feat)
        m.fit(feat[:3500].contiguous(), target[:3500].contiguous(), epochs=40, batch=250)
        m.calibrate(feat[3500:].contiguous(), target[3500:].contiguous(), 0.999)
        ref_ids, ref_d2 = oracle.knn(X, Qte, k)
        for prune in (0, 1):
            ids0, d0 = ix.knn(_t(Qte), k, prune=prune)
            base = ix.stats()
            ids1, d1 = ix.knn(_t(Qte), k, prune=prune, model=m)
            learned = ix.stats()
            _check_knn(ids0.cpu().numpy(), d0.cpu().numpy(), ref_ids, ref_d2)
            _check_knn(ids1.cpu().numpy(), d1.cpu().numpy(), ref_ids, ref_d2)
            gains[(k, prune)] = (base["series_refined"], learned["series_refined"],
                                 learned["radius_fallbacks"])
    for key, (b, l, fb) in gains.items():
        assert l < b, (key, gains)
    # the seed alone leaves far more exact work at k = 1 on the BF16 prune
    b, l, _ = gains[(1, 1)]
    assert l * 2 <= b, gains


def test_tile_pair_counters(gpu_lib):
    """The tile kernel's pair counters on a k = 10 search without a radius
    (five sampled passes, the lists rebuilt before the last two): the pairs it
    had to evaluate (rows of each listed leaf times the leaf's queries) never
    exceed the pairs whose leaf passed the first envelope bound, and the pairs
    computed in whole 64-query groups exceed them by less than one group per
    leaf."""
    N, n, L = 60000 + 77, 256, 256
    X = synth.collection(N, n, "mix", seed=321)
    bins, ix = _bf16_index(gpu_lib, X)
    Q, _ = synth.queries(X, 150, sigma=0.1, seed=322)
    ref_ids, ref_d2 = oracle.knn(X, Q, 10)
    ids, d = ix.knn(_t(Q), 10, prune=1)
    _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    st = ix.stats()
    need, done = st["series_bf16_needed"], st["series_bf16_checked"]
    n_leaves = (N + L - 1) // L
    assert 0 < need <= st["leaves_visited"] * L, st
    assert need <= done < need + n_leaves * 64 * L, st


@pytest.mark.parametrize("k", [1, 10])
def test_prune_batch_above_1024_queries(gpu_lib, k):
    """A batch of 1,500 queries (1,536 slots, 24 query groups per leaf at
    most) on both prune tiers, with and without list rebuilds (k = 10 rebuilds before its last two passes, k = 1
    without a radius before its last), against the oracle."""
    N, n, B = 12000 + 13, 64, 1500
    X = synth.collection(N, n, "mix", seed=341)
    bins, ix = _fp8_index(gpu_lib, X, precision=3)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=342)
    ref_ids, ref_d2 = oracle.knn(X, Q, k)
    for prune in (1, 2):
        ids, d = ix.knn(_t(Q), k, prune=prune)
        _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
        st = ix.stats()
        assert 0 < st["series_bf16_needed"] <= st["series_bf16_checked"], (prune, st)


@pytest.mark.parametrize("n", [36, 100, 200])
def test_prune_lengths_with_padding(gpu_lib, n):
    """Lengths that are not a multiple of 64 (padded to 64, 128 and 256 with
    zeros in both operands) on both prune tiers against the oracle."""
    N, B = 3000 + 5, 16
    X = synth.collection(N, n, "mix", seed=371 + n)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=372)
    bins, ix = _fp8_index(gpu_lib, X, precision=3)
    for k in (1, 10):
        ref_ids, ref_d2 = oracle.knn(X, Q, k)
        for prune in (1, 2):
            ids, d = ix.knn(_t(Q), k, prune=prune)
            _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)


def test_largest_batch(gpu_lib):
    """The largest batch a call takes, 65,535 queries (65,536 slots: the
    list builds stage each sub-block's survivor bits in 16 pieces of 4,096
    slots, twice), on the plain scan and both prune tiers
    against the oracle; one more query is refused."""
    N, n, B = 2000 + 3, 64, 65535
    X = synth.collection(N, n, "mix", seed=351)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=352)
    bins, ix = _fp8_index(gpu_lib, X, precision=3)
    ref_ids, ref_d2 = oracle.knn(X, Q, 3)
    Qd = _t(Q)
    for prune in (0, 1, 2):
        ids, d = ix.knn(Qd, 3, prune=prune)
        _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    with pytest.raises(gpu_lib.SofaError) as e:
        ix.knn(_t(np.concatenate([Q, Q[:1]])), 3)
    assert e.value.status == gpu_lib.SOFA_EINVAL


@pytest.mark.parametrize("L", [512, 1024])
def test_prune_large_leaves(gpu_lib, L):
    """Leaves of several 256-row chunks: every chunk of a leaf runs the leaf's
    query list; both prune tiers against the oracle, k = 10."""
    N, n, B = 20000 + 29, 128, 60
    X = synth.collection(N, n, "mix", seed=361)
    bins = _bins(gpu_lib, X, 2000)
    ix = gpu_lib.Index(bins, _t(X), leaf_size=L, precision=3)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=362)
    ref_ids, ref_d2 = oracle.knn(X, Q, 10)
    for prune in (0, 1, 2):
        ids, d = ix.knn(_t(Q), 10, prune=prune)
        _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)


def test_approximate_search(gpu_lib):
    """approx_leaves = M scans the M leaves of smallest envelope bound per
    query (no exactness guarantee).  With M at least the number of leaves it
    is the exact search; for any M every returned distance is the true
    distance of its id, ranked by (distance, id); recall does not fall as M
    grows; out-of-range M is an error."""
    N, n, B, k, L = 3000 + 7, 128, 50, 10, 64
    X = synth.collection(N, n, "mix", seed=371)
    bins = _bins(gpu_lib, X, N)
    ix = gpu_lib.Index(bins, _t(X), leaf_size=L)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=372)
    ref_ids, ref_d2 = oracle.knn(X, Q, k)
    n_leaves = ix.info()["n_leaves"]
    assert n_leaves <= 64
    ids, d = ix.knn(_t(Q), k, approx_leaves=64)
    _check_knn(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    recalls = []
    for M in (1, 2, 4, 8, 16):
        ids, d = ix.knn(_t(Q), k, approx_leaves=M)
        ids, d = ids.cpu().numpy(), d.cpu().numpy().astype(np.float64)
        for b in range(B):
            got = ids[b][ids[b] >= 0]
            assert got.size == min(k, M * L)
            d2 = oracle.dist2_rows(X, Q[b], got)
            assert np.all(np.abs(d[b][:got.size] - np.sqrt(d2)) <= 1e-6 * np.maximum(np.sqrt(d2), 1e-30))
            key = list(zip(d2.tolist(), got.tolist()))
            assert key == sorted(key)
        recalls.append(np.mean([len(set(ids[b]) & set(ref_ids[b])) / k for b in range(B)]))
    assert all(r1 <= r2 + 1e-12 for r1, r2 in zip(recalls, recalls[1:])), recalls
    assert recalls[-1] > recalls[0], recalls
    with pytest.raises(gpu_lib.SofaError):
        ix.knn(_t(Q), k, approx_leaves=65)
