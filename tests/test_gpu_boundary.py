"""GPU tests of the boundary's device-memory hook and of device
z-normalisation (Section II), through the C ABI.

z-normalisation bar (derived in the design notes): the device forms the mean
and the population standard deviation in FP64 and rounds (x - mean)/sd to
FP32 once; the oracle does the same arithmetic in FP64 in another summation
order.  Each FP64 side is within (n + 8) 2^-53 (M/sd + |z|) of the exact
value (M = max |x_t|: the error of the mean, scaled by 1/sd, and the relative
error of sd and the quotient), so every output is within
2^-24 |z_ref| + 2 (n + 8) 2^-53 (M/sd + |z_ref|) (1 + 2^-20) of the oracle's
FP64 value z_ref.  Constant rows give exact zeros on both sides.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _raw_rows(m, n, seed):
    """Rows of the mix recipe, each scaled and shifted (scale 10^U(-3, 3),
    offset up to 1e4 times the scale), plus constant rows and a spike."""
    rng = np.random.default_rng(seed)
    X = synth.collection(m, n, "mix", seed=seed).astype(np.float64)
    a = 10.0 ** rng.uniform(-3, 3, size=(m, 1))
    b = rng.uniform(-1e4, 1e4, size=(m, 1)) * a
    R = (X * a + b).astype(np.float32)
    R[3] = 7.25                      # constant row: all zeros out
    R[5] = 0.0
    R[8] = 0.0
    R[8, n // 3] = 1.0               # one spike
    return R


def _znorm_bound(R, ref):
    n = R.shape[1]
    R64 = R.astype(np.float64)
    sd = R64.std(axis=1, keepdims=True)
    M = np.abs(R64).max(axis=1, keepdims=True)
    ratio = np.where(sd > 0, M / np.where(sd > 0, sd, 1.0), 0.0)
    return (2.0 ** -24 * np.abs(ref) + 2 * (n + 8) * 2.0 ** -53 * (ratio + np.abs(ref))) * (1 + 2.0 ** -20)


@pytest.mark.parametrize("n", [64, 100, 256, 1000])
def test_znormalise_matches_oracle(gpu_lib, n):
    R = _raw_rows(3001, n, seed=700 + n)
    out = gpu_lib.znormalise(_t(R)).cpu().numpy()
    ref = np.stack([oracle.znorm(r) for r in R])
    bound = _znorm_bound(R, ref)
    assert np.all(np.abs(out.astype(np.float64) - ref) <= bound), np.max(np.abs(out - ref) / bound)
    assert np.all(out[3] == 0.0) and np.all(out[5] == 0.0)
    # in place gives the same bits
    Rd = _t(R)
    gpu_lib.znormalise(Rd, out=Rd)
    assert np.array_equal(Rd.cpu().numpy(), out)


def test_znormalise_empty_and_bad_arguments(gpu_lib):
    import torch
    X = torch.zeros((0, 64), dtype=torch.float32, device="cuda")
    assert gpu_lib.znormalise(X).shape == (0, 64)
    L = gpu_lib.load()
    assert L.sofa_znormalise(None, 4, 64, None, None) == gpu_lib.SOFA_EINVAL
    assert L.sofa_znormalise(None, 4, 0, None, None) == gpu_lib.SOFA_EINVAL


def _check_knn_near_ties(ids, d, ref_ids, ref_d2, tol=1e-5):
    """ids/dists of a search over data normalised on the device against the
    oracle's search over data it normalised itself.  The two copies of the
    data differ by an FP32 rounding here and there, which moves distances by
    about 1e-6 relative, so: the distance at every rank matches within tol,
    and the ids match wherever the oracle's distance at that rank is
    separated from its neighbours by more than 2 tol."""
    ref = np.sqrt(ref_d2)
    assert np.all(np.abs(d.astype(np.float64) - ref) <= tol * np.maximum(ref, 1e-30))
    gap = np.full(ref.shape, np.inf)
    rel = np.diff(ref, axis=1) / np.maximum(ref[:, 1:], 1e-30)
    gap[:, 1:] = np.minimum(gap[:, 1:], rel)
    gap[:, :-1] = np.minimum(gap[:, :-1], rel)
    clear = gap > 2 * tol
    assert np.array_equal(ids[clear], ref_ids[clear])
    assert clear.mean() > 0.9


def test_build_and_search_with_znormalise(gpu_lib):
    """Raw (scaled and shifted) rows and queries: bins, index and search with
    device z-normalisation against the oracle's k-NN over the rows and
    queries it z-normalised itself (Section II)."""
    N, n, B, k = 20000, 256, 40, 5
    R = _raw_rows(N, n, seed=711)
    R[3] = R[4]  # no constant rows here: a query near one would have all distances equal
    R[5] = R[6]
    R[8] = R[9]
    Z = np.stack([oracle.znorm(r) for r in R]).astype(np.float32)
    Qz, _ = synth.queries(Z, B, sigma=0.1, seed=712)
    rng = np.random.default_rng(713)
    Qraw = (Qz.astype(np.float64) * 10.0 ** rng.uniform(-2, 2, (B, 1)) + rng.uniform(-50, 50, (B, 1))
            ).astype(np.float32)
    Qref = np.stack([oracle.znorm(q) for q in Qraw]).astype(np.float32)
    ref_ids, ref_d2 = oracle.knn(Z, Qref, k)
    bins = gpu_lib.Bins.learn(_t(R), 2000, znormalise=1)
    ix = gpu_lib.Index(bins, _t(R), precision=1, znormalise=1)
    Qd = _t(Qraw)
    for prune in (0, 1):
        ids, d = ix.knn(Qd, k, prune=prune, znormalise=True)
        _check_knn_near_ties(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_d2)
    assert np.array_equal(Qd.cpu().numpy(), Qraw)   # the caller's queries are left as they were
    # bins learned on raw rows with the flag equal bins learned on normalised rows
    bz = gpu_lib.Bins.learn(gpu_lib.znormalise(_t(R)), 2000).get()
    br = bins.get()
    assert np.array_equal(bz["sel"], br["sel"])
    assert np.array_equal(bz["beta"], br["beta"])


def test_search_with_torch_allocator(gpu_lib):
    """sofa_set_allocator with PyTorch's caching allocator: every device
    buffer of the bins, the index, the searches (three paths, with
    fall-backs forced by a tiny candidate list) and a network comes from the
    torch pool and goes back to it; the answers equal the oracle's."""
    import torch
    N, n, B, k = 30000, 256, 32, 10
    X = synth.collection(N, n, "mix", seed=721)
    Q, _ = synth.queries(X, B, sigma=0.1, seed=722)
    ref_ids, ref_d2 = oracle.knn(X, Q, k)
    alloc = gpu_lib.TorchAllocator()
    gpu_lib.set_allocator(alloc)
    try:
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        bins = gpu_lib.Bins.learn(_t(X), 3000)
        ix = gpu_lib.Index(bins, _t(X), precision=3)
        ws = gpu_lib.Workspace()
        m = gpu_lib.RadiusModel(k=k, seed=3)
        for prune in (0, 1, 2):
            for cap in (0, 64):
                ids, d = ix.knn(_t(Q), k, prune=prune, ws=ws, candidate_capacity=cap)
                assert np.array_equal(ids.cpu().numpy(), ref_ids), (prune, cap)
                ref = np.sqrt(ref_d2)
                assert np.all(np.abs(d.cpu().numpy() - ref) <= 1e-6 * ref)
        feat, _, _ = bins.transform(_t(Q), sel=False, words=False)
        y = m.forward(feat.contiguous())
        assert torch.isfinite(y).all()
        assert alloc.allocs >= 10 and alloc.live_bytes > 0
        assert torch.cuda.memory_allocated() >= before + ix.info()["device_bytes"]
        del ix, bins, ws, m, feat, y
        import gc
        gc.collect()
        torch.cuda.synchronize()
        assert alloc.live_bytes == 0 and alloc.frees == alloc.allocs
    finally:
        gpu_lib.set_allocator(None)
    # after restoring hipMalloc the library works as before
    bins = gpu_lib.Bins.learn(_t(X), 3000)
    ix = gpu_lib.Index(bins, _t(X))
    ids, _ = ix.knn(_t(Q), k)
    assert np.array_equal(ids.cpu().numpy(), ref_ids)
    import ctypes
    L = gpu_lib.load()
    assert L.sofa_set_allocator(ctypes.cast(alloc._alloc, ctypes.c_void_p), None, None) == gpu_lib.SOFA_EINVAL
