"""GPU test of sofa_knn_noalloc, the search for callers that cannot allocate
device memory, through the C ABI: on two calls in a row (the second with a
smaller batch) it returns what sofa_knn returns on the same inputs, ids
identical and distances equal, for the three refine paths, with forced
fall-backs (dropped candidates, radius misses) and query z-normalisation;
it takes nothing from the allocator hook nor from the device's free memory;
batches above its scratch are refused before any device work."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _outputs(B, k):
    import torch
    ids = torch.full((B, k), -7, dtype=torch.int64, device="cuda")
    d = torch.full((B, k), -1.0, dtype=torch.float32, device="cuda")
    return ids, d


def _noalloc(ix, Q, k, **kw):
    ids, d = _outputs(Q.shape[0], k)
    return ix.knn_noalloc(Q, k, ids, d, **kw)


def test_noalloc_equals_knn(gpu_lib):
    import torch
    N, n, k = 30000 + 17, 256, 10
    X = synth.collection(N, n, "mix", seed=801)
    Q, _ = synth.queries(X, 40, sigma=0.1, seed=802)
    bins = gpu_lib.Bins.learn(_t(X), 3000)
    ix = gpu_lib.Index(bins, _t(X), precision=3)
    ref_ids, ref_d2 = oracle.knn(X, Q, k)
    # radii below the k-th distance for every other query: those miss and
    # are searched again without a radius
    dk = np.sqrt(ref_d2[:, k - 1])
    radius = _t((dk * np.where(np.arange(len(dk)) % 2 == 0, 0.9, 1.1)).astype(np.float32))
    Qd = _t(Q)
    cases = [dict(prune=p) for p in (0, 1, 2)]
    cases += [dict(prune=1, candidate_capacity=64), dict(prune=2, candidate_capacity=64),
              dict(prune=1, radius=radius), dict(prune=0, radius=radius), dict(prune=0, znormalise=True)]
    _noalloc(ix, Qd[:2], k)   # the first call looks up the array's device address
    torch.cuda.synchronize()
    alloc = gpu_lib.TorchAllocator()
    for kw in cases:
        for B in (40, 23):     # two calls in a row, the second smaller
            kw = dict(kw, radius=kw["radius"][:B]) if "radius" in kw else kw
            want_ids, want_d = ix.knn(Qd[:B], k, **kw)
            got_ids, got_d = _outputs(B, k)
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            gpu_lib.set_allocator(alloc)
            try:
                ix.knn_noalloc(Qd[:B], k, got_ids, got_d, **kw)
            finally:
                gpu_lib.set_allocator(None)
            torch.cuda.synchronize()
            assert torch.cuda.mem_get_info()[0] == free0, kw
            assert alloc.allocs == 0, kw
            assert torch.equal(got_ids, want_ids), (kw, B)
            assert torch.equal(got_d, want_d), (kw, B)
            assert np.array_equal(got_ids.cpu().numpy(), ref_ids[:B]), (kw, B)
            ref = np.sqrt(ref_d2[:B])
            assert np.all(np.abs(got_d.cpu().numpy() - ref) <= 1e-6 * ref), (kw, B)


def test_noalloc_refuses_batches_above_its_scratch(gpu_lib):
    import torch
    N, n = 3000, 128
    X = synth.collection(N, n, "mix", seed=803)
    bins = gpu_lib.Bins.learn(_t(X), 500)
    ix = gpu_lib.Index(bins, _t(X), precision=1)
    Q = torch.zeros((4097, n), dtype=torch.float32, device="cuda")
    with pytest.raises(gpu_lib.SofaError) as e:       # more queries than the read-back holds
        _noalloc(ix, Q, 10)
    assert e.value.status == gpu_lib.SOFA_ENOMEM
    # 4096 queries at k = 100: about 2 GiB of result lists, far above the array
    assert ix.workspace_bytes(4096, 100, prune=1) > (128 << 20)
    with pytest.raises(gpu_lib.SofaError) as e:
        _noalloc(ix, Q[:4096], 100, prune=1)
    assert e.value.status == gpu_lib.SOFA_ENOMEM
    assert "scratch" in str(e.value)
    with pytest.raises(gpu_lib.SofaError) as e:       # no workspace on this entry point
        ws = gpu_lib.Workspace()
        from paper_2411_17483_amd.sofa import KnnParams, _check, _dev, _stream, load
        import ctypes
        ids = torch.empty((4, 10), dtype=torch.int64, device="cuda")
        d = torch.empty((4, 10), dtype=torch.float32, device="cuda")
        p = KnnParams(0, None, None, 0, ws._h, 0, 0, 0, 0)
        _check(load().sofa_knn_noalloc(ix._h, _dev(Q), 4, 10, ctypes.byref(p), _dev(ids), _dev(d), _stream()))
    assert e.value.status == gpu_lib.SOFA_EINVAL
    # the library still answers after the refusals
    Xq = _t(synth.queries(X, 5, sigma=0.1, seed=804)[0])
    ids, d = _noalloc(ix, Xq, 3, prune=1)
    want_ids, want_d = ix.knn(Xq, 3, prune=1)
    assert torch.equal(ids, want_ids) and torch.equal(d, want_d)
