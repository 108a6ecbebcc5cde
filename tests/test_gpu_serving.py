"""GPU tests of the request loop (sofa_server_*): continuous batching over
several HBM-resident collections gives each request the same answer alone
and in the mix, and that answer is the oracle's.  Memory admission shrinks
or delays batches, and rejects a query that cannot fit on its own."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _collections(sofa):
    specs = [  # (N, n, build precision, prune)
        (20000 + 3, 128, 1, 1),
        (6000 + 5, 512, 2, 2),
        (3000 + 1, 1024, 0, 0),
    ]
    out = []
    for i, (N, n, prec, prune) in enumerate(specs):
        X = synth.collection(N, n, "mix", seed=501 + i)
        bins = sofa.Bins.learn(_t(X), 1500, pool=16)
        ix = sofa.Index(bins, _t(X), leaf_size=256, precision=prec)
        Q, _ = synth.queries(X, 24, sigma=0.1, seed=511 + i)
        out.append(dict(X=X, Q=Q, bins=bins, ix=ix, prune=prune))
    return out


def _requests(colls, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        c = int(rng.integers(len(colls)))
        k = int(rng.choice([1, 10, 100]))
        j = int(rng.integers(colls[c]["Q"].shape[0]))
        reqs.append((c, k, j))
    return reqs


def test_serving_alone_equals_mix_equals_oracle(gpu_lib):
    colls = _collections(gpu_lib)
    srv = gpu_lib.Server(slots=4, max_batch=32)
    cids = [srv.add_collection(c["ix"], c["prune"]) for c in colls]
    reqs = _requests(colls, 72, seed=7)
    # alone: one request in the system at a time
    alone = []
    for c, k, j in reqs:
        t = srv.submit(cids[c], colls[c]["Q"][j], k)
        ids, d, tm = srv.wait(t, k)
        assert tm[2] == 1
        alone.append((ids, d))
    # mix: everything submitted before anything is waited for
    tickets = [srv.submit(cids[c], colls[c]["Q"][j], k) for c, k, j in reqs]
    mix = [srv.wait(t, k) for t, (c, k, j) in zip(tickets, reqs)]
    st = srv.stats()
    assert st["completed"] == st["submitted"] == 2 * len(reqs)
    assert st["max_batch"] > 1            # the mix was batched
    for (c, k, j), (ia, da), (im, dm, _) in zip(reqs, alone, mix):
        assert np.array_equal(ia, im) and np.array_equal(da, dm), (c, k, j)
    # and the answer is the oracle's
    for ci, col in enumerate(colls):
        for k in (1, 10, 100):
            sel = [i for i, r in enumerate(reqs) if r[0] == ci and r[1] == k]
            if not sel:
                continue
            Q = col["Q"][[reqs[i][2] for i in sel]]
            ref_ids, ref_d2 = oracle.knn(col["X"], Q, k)
            for row, i in enumerate(sel):
                assert np.array_equal(mix[i][0], ref_ids[row]), (ci, k, i)
                ref = np.sqrt(ref_d2[row])
                assert np.all(np.abs(mix[i][1].astype(np.float64) - ref) <= 1e-6 * np.maximum(ref, 1e-30))
    srv.close()


def test_serving_memory_admission(gpu_lib):
    colls = _collections(gpu_lib)[:1]
    ix = colls[0]["ix"]
    one = ix.workspace_bytes(1, 100, prune=1)
    many = ix.workspace_bytes(32, 100, prune=1)
    assert many > 2 * one
    # room for a few queries at a time: batches are halved or wait, and all finish
    srv = gpu_lib.Server(slots=4, max_batch=32, memory_budget=int(one * 2.5))
    cid = srv.add_collection(ix, 1)
    Q = colls[0]["Q"]
    tickets = [srv.submit(cid, Q[j % Q.shape[0]], 100) for j in range(40)]
    res = [srv.wait(t, 100) for t in tickets]
    st = srv.stats()
    assert st["completed"] == 40 and st["memory_waits"] > 0
    assert st["in_flight_bytes_peak"] <= int(one * 2.5)
    ref_ids, _ = oracle.knn(colls[0]["X"], Q, 100)
    for j, (ids, _, _) in enumerate(res):
        assert np.array_equal(ids, ref_ids[j % Q.shape[0]])
    srv.close()
    # a budget below one query's workspace: that request fails, the server lives on
    srv = gpu_lib.Server(slots=2, max_batch=8, memory_budget=max(1, one // 2))
    cid = srv.add_collection(ix, 1)
    t = srv.submit(cid, Q[0], 100)
    with pytest.raises(gpu_lib.SofaError):
        srv.wait(t, 100)
    srv.close()


def test_serving_device_memory_within_budget(gpu_lib):
    """The server's real device memory (hipMemGetInfo, sampled while a
    mixed-k stream of requests runs) stays within its budget: the staging
    buffers and every slot's workspace, which keeps the capacity of its
    largest batch and its reserved fall-back buffers, are charged, and idle
    slots give their memory back when a batch needs it."""
    import threading
    import torch
    colls = _collections(gpu_lib)[:1]
    ix = colls[0]["ix"]
    many = ix.workspace_bytes(32, 100, prune=1)
    # room for one and a half of the largest batches: four slots that each
    # kept their largest workspace would need 4x that
    budget = int(1.5 * many)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, _ = torch.cuda.mem_get_info()
    low = [free0]
    done = threading.Event()

    def sample():
        while not done.is_set():
            low[0] = min(low[0], torch.cuda.mem_get_info()[0])

    srv = gpu_lib.Server(slots=4, max_batch=32, memory_budget=budget)
    cid = srv.add_collection(ix, 1)
    Q = colls[0]["Q"]
    rng = np.random.default_rng(91)
    ks = [int(rng.choice([1, 10, 100])) for _ in range(96)]
    th = threading.Thread(target=sample)
    th.start()
    try:
        tickets = [srv.submit(cid, Q[j % Q.shape[0]], k) for j, k in enumerate(ks)]
        res = [srv.wait(t, k) for t, k in zip(tickets, ks)]
        low[0] = min(low[0], torch.cuda.mem_get_info()[0])
    finally:
        done.set()
        th.join()
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(ks)
    assert st["in_flight_bytes_peak"] <= budget
    # allocation granularity: at most 2 MiB per buffer (5 per slot)
    slack = 4 * 5 * (2 << 20)
    assert free0 - low[0] <= budget + slack, (free0 - low[0], budget)
    for k in (1, 10, 100):
        sel = [j for j, kk in enumerate(ks) if kk == k]
        ref_ids, _ = oracle.knn(colls[0]["X"], Q[[j % Q.shape[0] for j in sel]], k)
        for row, j in enumerate(sel):
            assert np.array_equal(res[j][0], ref_ids[row]), (k, j)


def test_serving_argument_errors(gpu_lib):
    colls = _collections(gpu_lib)[:1]
    srv = gpu_lib.Server(slots=1, max_batch=4)
    with pytest.raises(gpu_lib.SofaError):
        srv.add_collection(colls[0]["ix"], 2)   # the index has no FP8 copy
    cid = srv.add_collection(colls[0]["ix"], 1)
    with pytest.raises(gpu_lib.SofaError):
        srv.submit(cid, colls[0]["Q"][0], 101)
    with pytest.raises(gpu_lib.SofaError):
        srv.submit(cid + 5, colls[0]["Q"][0], 1)
    with pytest.raises(ValueError):
        srv.submit(cid, colls[0]["Q"][0][:10], 1)
    srv.close()
