"""GPU parity at the full sizes of the benchmark workloads, on sampled outputs.

The collections are too large for a brute-force check of every query, so:

- every collection is generated on the host in chunks of 1M rows (the
  generator is counter-based per row) and copied into its slice of one
  device tensor;
- during the same pass, the oracle computes the exact k nearest rows of each
  chunk for a sample of the queries, and the chunks' lists are merged by
  (d^2, id): the sampled queries get the oracle's full answer, and the GPU
  must return exactly those ids (distances within 1e-6 relative of
  sqrt(FP64 d^2));
- every query of the batch (sampled or not) must return k distinct valid ids
  ranked by (d, id), each distance matching the FP64 distance of its row
  recomputed one by one.

Workloads (k-NN over z-normalised mix collections: even rows random walk,
odd rows eight sinusoids plus noise; queries are noisy copies, sigma 0.1):

- 10M x 256, 1,000 queries, k = 10 and 1, the learned radius with the BF16
  prune, in the launch configuration the benchmark times; and the learned
  radius evaluated on 10,000 further queries (network trained here on
  100,000 queries, fewer than the benchmark's 1,000,000);
- 50M x 256 with BF16 and FP8 copies, batches of 4,096 queries, k = 10,
  plain scan, BF16 prune and FP8 prune;
- 70M x 64 with both copies: past 2^26 rows, where a launch of one wave per
  row would exceed the 2^32 work-items a dispatch can count (every row must
  reach the index: the exported ids form a permutation);
- three HBM-resident collections served together (100M x 128 on the BF16
  tier, 20M x 512 and 5M x 1024 on the FP8 tier), requests of k in
  {1, 10, 100}, each answer the same alone and in the mix.
"""
import gc
import sys
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

CHUNK = 1_000_000
SIGMA = 0.1


def _log(*a):
    print("[workload]", *a, file=sys.stderr, flush=True)


def _first_queries(n, seed, qseed, src, s):
    """The first s noisy-copy queries (noise seed qseed) of a batch over the
    collection of seed `seed`, from their source rows alone: the same values
    as synth.queries over the whole collection."""
    rows = np.concatenate([synth.collection(1, n, "mix", seed=seed, row0=int(j)) for j in src[:s]])
    return synth.noisy_copies(rows, sigma=SIGMA, seed=qseed)


def _merge(a, b, k):
    ids = np.concatenate([a[0], b[0]], axis=1)
    d2 = np.concatenate([a[1], b[1]], axis=1)
    out_i = np.empty((ids.shape[0], k), np.int64)
    out_d = np.empty((ids.shape[0], k), np.float64)
    for r in range(ids.shape[0]):
        o = np.lexsort((ids[r], d2[r]))[:k]
        out_i[r], out_d[r] = ids[r][o], d2[r][o]
    return out_i, out_d


def _stream(N, n, seed, probes, k):
    """Device copy of the mix collection (N, n, seed) and the oracle's exact
    k-NN of each probe array, merged over the chunks."""
    import torch
    X = torch.empty((N, n), dtype=torch.float32, device="cuda")
    best = [None] * len(probes)
    t0 = time.perf_counter()
    for r0 in range(0, N, CHUNK):
        m = min(CHUNK, N - r0)
        Xc = synth.collection(m, n, "mix", seed=seed, row0=r0)
        X[r0:r0 + m].copy_(torch.from_numpy(Xc))
        for i, P in enumerate(probes):
            ids, d2 = oracle.knn(Xc, P, min(k, m))
            part = (ids + r0, d2)
            best[i] = part if best[i] is None else _merge(best[i], part, k)
        if (r0 // CHUNK) % 10 == 9:
            _log(f"{N}x{n}: {r0 + m} rows generated, {time.perf_counter() - t0:.0f}s")
    torch.cuda.synchronize()
    return X, best


def _batch_queries(X, src, seed):
    import torch
    rows = X[torch.from_numpy(np.asarray(src, np.int64)).cuda()].cpu().numpy()
    return synth.noisy_copies(rows, sigma=SIGMA, seed=seed)


def _check_sampled(ids, d, ref_ids, ref_d2, what):
    s, k = ref_ids.shape
    got_i, got_d = ids[:s, :k], d[:s, :k].astype(np.float64)
    for r in range(s):
        assert np.array_equal(got_i[r], ref_ids[r]), (what, r, got_i[r], ref_ids[r])
    ref = np.sqrt(ref_d2)
    assert np.all(np.abs(got_d - ref) <= 1e-6 * np.maximum(ref, 1e-30)), what


def _check_all(X, Q, ids, d, what):
    """Every row: k distinct ids in range, ranked by (d, id), each distance the
    FP64 distance of its row (recomputed one by one) within 1e-6 relative."""
    import torch
    B, k = ids.shape
    N = X.shape[0]
    assert np.all((ids >= 0) & (ids < N)), what
    rows = X[torch.from_numpy(ids.reshape(-1)).cuda()].cpu().numpy().reshape(B, k, -1)
    for r in range(B):
        assert len(set(ids[r].tolist())) == k, (what, r)
        d2 = oracle.dist2_rows(rows[r], Q[r], np.arange(k))
        ref = np.sqrt(d2)
        assert np.all(np.abs(d[r].astype(np.float64) - ref) <= 1e-6 * np.maximum(ref, 1e-30)), (what, r)
        order = np.lexsort((ids[r], d2))
        assert np.array_equal(order, np.arange(k)), (what, r)


def _release():
    """Return what the deleted objects held to the device."""
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _train_radius(sofa, torch, bins, ix, X, k, seed, ntr):
    """A radius network for k, trained as the benchmark trains it, on ntr
    noisy-copy queries labelled by the BF16-prune search."""
    src = synth.query_sources(X.shape[0], ntr, seed)
    Qtr = torch.from_numpy(_batch_queries(X, src, seed)).cuda()
    feat, _, _ = bins.transform(Qtr, sel=False, words=False)
    lab = []
    for i in range(0, ntr, 4096):
        _, dd = ix.knn(Qtr[i:i + 4096].contiguous(), k, prune=1)
        lab.append(torch.log(dd[:, -1]))
    target = torch.cat(lab).contiguous()
    n_fit = ntr - ntr // 10
    m = sofa.RadiusModel(k=k, seed=11 + k)
    m.standardize(feat[:n_fit].contiguous())
    m.fit(feat[:n_fit].contiguous(), target[:n_fit].contiguous(), epochs=8, batch=1024)
    m.calibrate(feat[n_fit:].contiguous(), target[n_fit:].contiguous(), 0.9999)
    return m


# --------------------------------------------------------------------------- #
def test_10M_learned_radius_bf16(gpu_lib):
    import torch
    sofa = gpu_lib
    N, n, B, seed = 10_000_000, 256, 1000, 2
    n_eval, eval_seed = 10_000, 5
    src = synth.query_sources(N, B, seed)
    src_ev = synth.query_sources(N, n_eval, eval_seed)
    _release()
    Qs = _first_queries(n, seed, seed, src, 8)
    Qes = _first_queries(n, seed, eval_seed, src_ev, 4)
    X, (ref, ref_ev) = _stream(N, n, seed, [Qs, Qes], 10)
    Q = _batch_queries(X, src, seed)
    Qe = _batch_queries(X, src_ev, eval_seed)
    assert np.array_equal(Q[:8], Qs) and np.array_equal(Qe[:4], Qes)
    bins = sofa.Bins.learn(X, N // 100)
    ix = sofa.Index(bins, X, leaf_size=256, precision=1)
    models = {k: _train_radius(sofa, torch, bins, ix, X, k, 4, 100_000) for k in (10, 1)}
    _log("10M x 256: index built, radius networks trained")
    Qd, Qed = torch.from_numpy(Q).cuda(), torch.from_numpy(Qe).cuda()
    for k in (10, 1):
        # the benchmark's call: 1,000 queries, learned radius, BF16 prune, sampled passes
        ids, d = ix.knn(Qd, k, prune=1, model=models[k], sampling=1)
        ids, d = ids.cpu().numpy(), d.cpu().numpy()
        _check_sampled(ids, d, ref[0][:, :k], ref[1][:, :k], f"10M k={k}")
        _check_all(X, Q, ids, d, f"10M k={k}")
        # the learned radius on 10,000 held-out queries, fallbacks included
        ids, d = ix.knn(Qed, k, prune=1, model=models[k], sampling=1)
        st = ix.stats()
        ids, d = ids.cpu().numpy(), d.cpu().numpy()
        _check_sampled(ids, d, ref_ev[0][:, :k], ref_ev[1][:, :k], f"10M eval k={k}")
        _check_all(X, Qe, ids, d, f"10M eval k={k}")
        _log(f"10M eval k={k}: radius fallbacks {st['radius_fallbacks']} of {n_eval}")
    del ix, bins, X, Qd, Qed, models
    _release()


def test_50M_precision_tiers(gpu_lib):
    import torch
    sofa = gpu_lib
    N, n, B, seed, k = 50_000_000, 256, 4096, 3, 10
    _release()
    src = synth.query_sources(N, B, seed)
    Qs = _first_queries(n, seed, seed, src, 4)
    X, (ref,) = _stream(N, n, seed, [Qs], k)
    Q = _batch_queries(X, src, seed)
    assert np.array_equal(Q[:4], Qs)
    bins = sofa.Bins.learn(X, N // 100)
    ix = sofa.Index(bins, X, leaf_size=256, precision=3)
    Qd = torch.from_numpy(Q).cuda()
    for prune in (1, 2, 0):
        ids, d = ix.knn(Qd, k, prune=prune)
        ids, d = ids.cpu().numpy(), d.cpu().numpy()
        _check_sampled(ids, d, ref[0], ref[1], f"50M prune={prune}")
        _check_all(X, Q, ids, d, f"50M prune={prune}")
        _log(f"50M x 256, 4096 queries, prune={prune}: checked")
    del ix, bins, X, Qd
    _release()


def test_layout_beyond_2_pow_26_rows(gpu_lib):
    """70M x 64 rows with BF16 and FP8 copies: launches with one wave per row
    would pass 2^32 work-items here; every row must reach the index."""
    import torch
    sofa = gpu_lib
    _release()
    N, n, seed, k = 70_000_000, 64, 9, 10
    src = synth.query_sources(N, 64, seed + 100)
    Qs = _first_queries(n, seed, seed + 100, src, 8)
    X, (ref,) = _stream(N, n, seed, [Qs], k)
    bins = sofa.Bins.learn(X, N // 100)
    ix = sofa.Index(bins, X, leaf_size=256, precision=3)
    W, ids, env, _ = ix.export()
    s_ids, _ = torch.sort(ids.long())
    assert torch.equal(s_ids, torch.arange(N, device="cuda"))
    del s_ids
    lo = env[:, :16].repeat_interleave(256, 0)[:N]
    hi = env[:, 16:].repeat_interleave(256, 0)[:N]
    assert not bool(((W < lo) | (W > hi)).any().item())
    del W, ids, env, lo, hi
    Qd = torch.from_numpy(Qs).cuda()
    for prune in (0, 1, 2):
        got, d = ix.knn(Qd, k, prune=prune)
        got, d = got.cpu().numpy(), d.cpu().numpy()
        _check_sampled(got, d, ref[0], ref[1], f"70M prune={prune}")
        _check_all(X, Qs, got, d, f"70M prune={prune}")
    _log("70M x 64: permutation, envelopes and sampled searches checked")
    del ix, bins, X, Qd
    _release()


def test_serving_three_collections(gpu_lib):
    sofa = gpu_lib
    _release()
    specs = [  # (N, n, collection seed, copies built, prune tier served)
        (100_000_000, 128, 6, 1, 1),
        (20_000_000, 512, 7, 2, 2),
        (5_000_000, 1024, 8, 2, 2),
    ]
    pool, s = 64, 3
    colls = []
    for N, n, seed, prec, prune in specs:
        qseed = seed + 100
        src = synth.query_sources(N, pool, qseed)
        Qs = _first_queries(n, seed, qseed, src, s)
        X, (ref,) = _stream(N, n, seed, [Qs], 100)
        Q = _batch_queries(X, src, qseed)
        assert np.array_equal(Q[:s], Qs)
        bins = sofa.Bins.learn(X, max(1000, N // 100))
        ix = sofa.Index(bins, X, leaf_size=256, precision=prec)
        del X
        _release()
        colls.append(dict(bins=bins, ix=ix, Q=Q, ref=ref, prune=prune))
        _log(f"{N}x{n}: index built")
    srv = sofa.Server(slots=4, max_batch=256)
    cids = [srv.add_collection(c["ix"], c["prune"]) for c in colls]
    # the sampled queries of every collection at k = 1, 10 and 100, alone
    reqs = [(c, k, j) for c in range(len(colls)) for k in (1, 10, 100) for j in range(s)]
    alone = [srv.wait(srv.submit(cids[c], colls[c]["Q"][j], k), k) for c, k, j in reqs]
    # then the same requests in a mix with 96 others, all in flight together
    rng = np.random.default_rng(17)
    extra = [(int(rng.integers(len(colls))), int(rng.choice([1, 10, 100])), int(rng.integers(pool)))
             for _ in range(96)]
    order = list(range(len(reqs) + len(extra)))
    rng.shuffle(order)
    allreq = reqs + extra
    tickets = {i: srv.submit(cids[allreq[i][0]], colls[allreq[i][0]]["Q"][allreq[i][2]], allreq[i][1])
               for i in order}
    mix = {i: srv.wait(tickets[i], allreq[i][1]) for i in order}
    st = srv.stats()
    assert st["completed"] == st["submitted"] == len(reqs) + len(allreq)
    assert st["max_batch"] > 1
    for i, (c, k, j) in enumerate(reqs):
        ia, da, _ = alone[i]
        im, dm, _ = mix[i]
        assert np.array_equal(ia, im) and np.array_equal(da, dm), (c, k, j)
        ref_ids, ref_d2 = colls[c]["ref"]
        assert np.array_equal(im, ref_ids[j, :k]), (c, k, j)
        ref = np.sqrt(ref_d2[j, :k])
        assert np.all(np.abs(dm.astype(np.float64) - ref) <= 1e-6 * np.maximum(ref, 1e-30)), (c, k, j)
    _log(f"serving: {len(reqs)} sampled requests equal alone, in the mix and to the oracle; "
         f"largest batch {st['max_batch']}")
    srv.close()
    del srv, colls
    _release()
