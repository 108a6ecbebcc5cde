"""Thin ctypes binding of libsofa.so (the C ABI declared in include/sofa.h).

Argument marshalling only: every step of the search runs in the library's HIP
kernels.  torch tensors supply device memory and the current stream.  The
binding refuses to run without the compiled library: there is no CPU path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsofa.so")
_lib = None

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64

SOFA_OK, SOFA_EINVAL, SOFA_ENOMEM, SOFA_EDEVICE, SOFA_EBUSY, SOFA_EINTERNAL = range(6)
EXPORTED = [
    "sofa_last_error", "sofa_learn_bins", "sofa_bins_create", "sofa_bins_get", "sofa_bins_free",
    "sofa_transform", "sofa_bins_eta_per_norm", "sofa_build", "sofa_index_get_info",
    "sofa_index_export", "sofa_index_free", "sofa_workspace_create", "sofa_workspace_bytes_for",
    "sofa_workspace_free", "sofa_knn", "sofa_knn_get_stats", "sofa_lower_bounds",
    "sofa_bf16_lower_bounds", "sofa_fp8_lower_bounds", "sofa_radius_create", "sofa_radius_free", "sofa_radius_num_params",
    "sofa_radius_get", "sofa_radius_set", "sofa_radius_standardize", "sofa_radius_gradients",
    "sofa_radius_train_step", "sofa_radius_fit", "sofa_radius_forward", "sofa_radius_calibrate",
    "sofa_radius_predict", "sofa_server_create", "sofa_server_add_collection",
    "sofa_server_set_model", "sofa_server_submit", "sofa_server_wait", "sofa_server_get_stats",
    "sofa_server_free", "sofa_set_allocator", "sofa_znormalise", "sofa_knn_noalloc",
]


class SofaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"sofa status {status}: {msg}")
        self.status = status


class BinParams(ctypes.Structure):
    _fields_ = [("l", _i32), ("alpha", _i32), ("pool", _i32), ("binning", _i32), ("summary", _i32),
                ("selection", _i32), ("znormalise", _i32)]


class BuildParams(ctypes.Structure):
    _fields_ = [("leaf_size", _i32), ("precision", _i32), ("key_scheme", _i32), ("znormalise", _i32)]


class IndexInfo(ctypes.Structure):
    _fields_ = [("N", _i64), ("n", _i32), ("n_pad", _i32), ("leaf_size", _i32), ("l", _i32),
                ("alpha", _i32), ("n_leaves", _i64), ("device_bytes", _i64), ("eta_x", ctypes.c_double),
                ("has_bf16", _i32), ("has_fp8", _i32)]


class KnnParams(ctypes.Structure):
    _fields_ = [("prune", _i32), ("d_radius", _vp), ("radius_model", _vp), ("no_seed_leaf", _i32),
                ("ws", _vp), ("candidate_capacity", _i32), ("sampling", _i32),
                ("approx_leaves", _i32), ("znormalise", _i32)]


class RadiusParams(ctypes.Structure):
    _fields_ = [("in_dim", _i32), ("hidden1", _i32), ("hidden2", _i32), ("k", _i32),
                ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("seed", ctypes.c_uint64)]


class KnnStats(ctypes.Structure):
    _fields_ = [("queries", _i64), ("leaves_total", _i64), ("leaves_visited", _i64),
                ("series_lb_checked", _i64), ("series_refined", _i64),
                ("series_bf16_checked", _i64), ("radius_fallbacks", _i64),
                ("overflow_fallbacks", _i64), ("ms_total", ctypes.c_double),
                ("ms_prepare", ctypes.c_double), ("ms_leaf", ctypes.c_double),
                ("ms_seed", ctypes.c_double), ("ms_refine", ctypes.c_double),
                ("ms_finalize", ctypes.c_double), ("ms_bf16_tiles", ctypes.c_double),
                ("ms_bf16_refine", ctypes.c_double), ("overflow_evicted", _i64),
                ("overflow_bf16_drop", _i64), ("overflow_band", _i64), ("max_candidates", _i64),
                ("overflow_retries", _i64), ("series_bf16_needed", _i64),
                ("prune_passes", _i64), ("prune_rows_streamed", _i64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerParams(ctypes.Structure):
    _fields_ = [("slots", _i32), ("max_batch", _i32), ("memory_budget", _i64),
                ("per_collection", _i32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", _i64), ("completed", _i64), ("batches", _i64), ("max_batch", _i64),
                ("in_flight_bytes_peak", _i64), ("memory_waits", _i64), ("busy_ms", ctypes.c_double),
                ("hbm_bytes", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def load():
    """Load libsofa.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2411_17483_amd/build.py "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    L.sofa_last_error.restype = ctypes.c_char_p
    L.sofa_learn_bins.argtypes = [_vp, _i64, _i32, _i64, ctypes.POINTER(BinParams), _vp,
                                  ctypes.POINTER(_vp)]
    L.sofa_bins_create.argtypes = [_i32, ctypes.POINTER(BinParams), _vp, _vp, _vp, ctypes.POINTER(_vp)]
    L.sofa_bins_get.argtypes = [_vp, ctypes.POINTER(BinParams), ctypes.POINTER(_i32), _vp, _vp, _vp]
    L.sofa_bins_free.argtypes = [_vp]
    L.sofa_bins_free.restype = None
    L.sofa_transform.argtypes = [_vp, _vp, _i64, _vp, _vp, _vp, _vp]
    L.sofa_bins_eta_per_norm.argtypes = [_vp]
    L.sofa_bins_eta_per_norm.restype = ctypes.c_double
    L.sofa_build.argtypes = [_vp, _vp, _i64, _i32, ctypes.POINTER(BuildParams), _vp, ctypes.POINTER(_vp)]
    L.sofa_index_get_info.argtypes = [_vp, ctypes.POINTER(IndexInfo)]
    L.sofa_index_export.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    L.sofa_index_free.argtypes = [_vp]
    L.sofa_index_free.restype = None
    L.sofa_workspace_create.argtypes = [_i64, ctypes.POINTER(_vp)]
    L.sofa_workspace_bytes_for.argtypes = [_vp, _i64, _i32, _i32, ctypes.POINTER(_i64)]
    L.sofa_workspace_free.argtypes = [_vp]
    L.sofa_workspace_free.restype = None
    L.sofa_knn.argtypes = [_vp, _vp, _i64, _i32, ctypes.POINTER(KnnParams), _vp, _vp, _vp]
    L.sofa_knn_noalloc.argtypes = [_vp, _vp, _i64, _i32, ctypes.POINTER(KnnParams), _vp, _vp, _vp]
    L.sofa_knn_get_stats.argtypes = [_vp, _vp, ctypes.POINTER(KnnStats)]
    L.sofa_lower_bounds.argtypes = [_vp, _vp, _i64, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)]
    L.sofa_bf16_lower_bounds.argtypes = [_vp, _vp, _i64, _vp, _vp]
    L.sofa_fp8_lower_bounds.argtypes = [_vp, _vp, _i64, _vp, _vp]
    L.sofa_server_create.argtypes = [ctypes.POINTER(ServerParams), ctypes.POINTER(_vp)]
    L.sofa_server_add_collection.argtypes = [_vp, _vp, _i32, ctypes.POINTER(_i32)]
    L.sofa_server_set_model.argtypes = [_vp, _i32, _vp]
    L.sofa_server_submit.argtypes = [_vp, _i32, _vp, _i32, ctypes.POINTER(_i64)]
    L.sofa_server_wait.argtypes = [_vp, _i64, _vp, _vp, _vp, _i32]
    L.sofa_server_get_stats.argtypes = [_vp, ctypes.POINTER(ServerStats)]
    L.sofa_server_free.argtypes = [_vp]
    L.sofa_server_free.restype = None
    L.sofa_radius_create.argtypes = [ctypes.POINTER(RadiusParams), ctypes.POINTER(_vp)]
    L.sofa_radius_free.argtypes = [_vp]
    L.sofa_radius_free.restype = None
    L.sofa_radius_num_params.argtypes = [_vp]
    L.sofa_radius_num_params.restype = _i64
    L.sofa_radius_get.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    L.sofa_radius_set.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    L.sofa_radius_standardize.argtypes = [_vp, _vp, _i64, _vp]
    L.sofa_radius_gradients.argtypes = [_vp, _vp, _vp, _i64, _vp, _vp, _vp]
    L.sofa_radius_train_step.argtypes = [_vp, _vp, _vp, _i64, _vp, _vp]
    L.sofa_radius_fit.argtypes = [_vp, _vp, _vp, _i64, _i32, _i32, _vp, _vp]
    L.sofa_radius_forward.argtypes = [_vp, _vp, _i64, _vp, _vp]
    L.sofa_radius_calibrate.argtypes = [_vp, _vp, _vp, _i64, ctypes.c_double, _vp]
    L.sofa_radius_predict.argtypes = [_vp, _vp, _i64, _vp, _vp]
    L.sofa_set_allocator.argtypes = [_vp, _vp, _vp]
    L.sofa_znormalise.argtypes = [_vp, _i64, _i32, _vp, _vp]
    _lib = L
    return L


def _check(st):
    if st != SOFA_OK:
        raise SofaError(st, load().sofa_last_error().decode())


def _stream():
    import torch
    return _vp(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype=None):
    import torch
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return _vp(t.data_ptr())


_ALLOC_FN = ctypes.CFUNCTYPE(_vp, ctypes.c_size_t, _vp, _vp)
_FREE_FN = ctypes.CFUNCTYPE(None, _vp, _vp, _vp)
_allocator = None


class TorchAllocator:
    """sofa_set_allocator backed by PyTorch's caching allocator: the library's
    device memory comes from (and goes back to) torch's pool.  Counts the
    calls and the bytes outstanding."""

    def __init__(self, device=None):
        import torch
        self.device = torch.cuda.current_device() if device is None else device
        self.allocs = self.frees = 0
        self.live = {}

        def alloc(nbytes, stream, ctx):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream or 0)
            except RuntimeError:
                return None
            self.allocs += 1
            self.live[p] = int(nbytes)
            return p

        def free(p, stream, ctx):
            self.frees += 1
            self.live.pop(p, None)
            torch.cuda.caching_allocator_delete(p)

        self._alloc, self._free = _ALLOC_FN(alloc), _FREE_FN(free)

    @property
    def live_bytes(self):
        return sum(self.live.values())


def set_allocator(allocator):
    """Install a TorchAllocator (or None for hipMalloc/hipFree).  The object
    is kept alive here while installed; buffers taken from it must be freed
    before it is dropped."""
    global _allocator
    if allocator is None:
        _check(load().sofa_set_allocator(None, None, None))
    else:
        _check(load().sofa_set_allocator(ctypes.cast(allocator._alloc, _vp), ctypes.cast(allocator._free, _vp),
                                         None))
    _allocator = allocator


def znormalise(X, out=None):
    """Rows of X (m x n FP32 device tensor) z-normalised on the device
    (sofa_znormalise); out may be X itself."""
    import torch
    out = torch.empty_like(X) if out is None else out
    m, n = X.shape
    _check(load().sofa_znormalise(_dev(X, torch.float32), m, n, _dev(out, torch.float32), _stream()))
    return out


# --------------------------------------------------------------------------- #
class Bins:
    """Word quantisation (sofa_learn_bins / sofa_bins_create): learned SFA
    (summary 0) or iSAX (summary 1: PAA means, N(0,1) breakpoints)."""

    def __init__(self, handle):
        self._h = _vp(handle)

    @classmethod
    def learn(cls, X, m, l=16, alpha=256, pool=16, binning=0, summary=0, selection=0, znormalise=0):
        import torch
        L = load()
        N, n = X.shape
        h = _vp()
        p = BinParams(l, alpha, pool, binning, summary, selection, int(znormalise))
        _check(L.sofa_learn_bins(_dev(X, torch.float32), N, n, m, ctypes.byref(p), _stream(),
                                 ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def create(cls, n, sel, beta, var=None, pool=16, binning=0, summary=0):
        L = load()
        sel = np.ascontiguousarray(sel, dtype=np.int32)
        beta = np.ascontiguousarray(beta, dtype=np.float64)
        l, am1 = beta.shape
        p = BinParams(l, am1 + 1, pool, binning, summary)
        v = None if var is None else np.ascontiguousarray(var, dtype=np.float64)
        h = _vp()
        _check(L.sofa_bins_create(n, ctypes.byref(p), sel.ctypes.data, beta.ctypes.data,
                                  None if v is None else v.ctypes.data, ctypes.byref(h)))
        return cls(h.value)

    def get(self):
        L = load()
        p = BinParams()
        n = _i32()
        _check(L.sofa_bins_get(self._h, ctypes.byref(p), ctypes.byref(n), None, None, None))
        sel = np.zeros(p.l, dtype=np.int32)
        beta = np.zeros((p.l, max(p.alpha - 1, 0)), dtype=np.float64)
        var = np.zeros(2 * p.pool, dtype=np.float64)
        _check(L.sofa_bins_get(self._h, None, None, sel.ctypes.data,
                               beta.ctypes.data if beta.size else None, var.ctypes.data))
        return {"n": n.value, "l": p.l, "alpha": p.alpha, "pool": p.pool, "binning": p.binning,
                "summary": p.summary, "selection": p.selection, "sel": sel, "beta": beta, "var": var}

    @property
    def eta_per_norm(self):
        return load().sofa_bins_eta_per_norm(self._h)

    def transform(self, X, pool=True, sel=True, words=True):
        """(pool values m x 2P, kept values m x 16, words m x 16 uint8) as device tensors."""
        import torch
        info = self.get()
        m = X.shape[0]
        dev = X.device
        P = torch.empty((m, 2 * info["pool"]), dtype=torch.float32, device=dev) if pool else None
        S = torch.empty((m, 16), dtype=torch.float32, device=dev) if sel else None
        W = torch.empty((m, 16), dtype=torch.uint8, device=dev) if words else None
        _check(load().sofa_transform(self._h, _dev(X, torch.float32), m,
                                     None if P is None else _dev(P), None if S is None else _dev(S),
                                     None if W is None else _dev(W), _stream()))
        return P, S, W

    def __del__(self):
        if _lib is not None and getattr(self, "_h", None) and self._h.value:
            _lib.sofa_bins_free(self._h)
            self._h = _vp()


class Workspace:
    def __init__(self, max_bytes=0):
        h = _vp()
        _check(load().sofa_workspace_create(int(max_bytes), ctypes.byref(h)))
        self._h = h

    def stats(self):
        s = KnnStats()
        _check(load().sofa_knn_get_stats(self._h, None, ctypes.byref(s)))
        return s.as_dict()

    def __del__(self):
        if _lib is not None and getattr(self, "_h", None) and self._h.value:
            _lib.sofa_workspace_free(self._h)
            self._h = _vp()


class Index:
    """A built index (sofa_build) and exact k-NN queries (sofa_knn)."""

    def __init__(self, bins, X, leaf_size=256, precision=0, key_scheme=0, znormalise=0):
        import torch
        L = load()
        N, n = X.shape
        h = _vp()
        p = BuildParams(leaf_size, precision, key_scheme, int(znormalise))
        _check(L.sofa_build(bins._h, _dev(X, torch.float32), N, n, ctypes.byref(p), _stream(),
                            ctypes.byref(h)))
        self._h = h
        self.bins = bins

    def info(self):
        i = IndexInfo()
        _check(load().sofa_index_get_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in i._fields_}

    def export(self):
        import torch
        info = self.info()
        N, nl = info["N"], info["n_leaves"]
        W = torch.empty((N, 16), dtype=torch.uint8, device="cuda")
        ids = torch.empty(N, dtype=torch.int32, device="cuda")
        env = torch.empty((nl, 32), dtype=torch.uint8, device="cuda")
        keys = torch.empty(N, dtype=torch.int64, device="cuda")
        _check(load().sofa_index_export(self._h, _dev(W), _dev(ids), _dev(env), _dev(keys), _stream()))
        return W, ids, env, keys

    def knn(self, Q, k, radius=None, prune=0, no_seed_leaf=False, ws=None, candidate_capacity=0,
            model=None, sampling=0, approx_leaves=0, znormalise=False):
        """Exact k-NN of the rows of Q: (ids B x k int64, dists B x k float32) device tensors.
        approx_leaves > 0: approximate search over that many leaves per query."""
        import torch
        B = Q.shape[0]
        ids = torch.empty((B, k), dtype=torch.int64, device=Q.device)
        d = torch.empty((B, k), dtype=torch.float32, device=Q.device)
        p = KnnParams(prune, None if radius is None else _dev(radius, torch.float32),
                      None if model is None else model._h, 1 if no_seed_leaf else 0,
                      None if ws is None else ws._h, int(candidate_capacity), int(sampling),
                      int(approx_leaves), 1 if znormalise else 0)
        _check(load().sofa_knn(self._h, _dev(Q, torch.float32), B, k, ctypes.byref(p), _dev(ids),
                               _dev(d), _stream()))
        return ids, d

    def knn_noalloc(self, Q, k, ids, d, radius=None, prune=0, candidate_capacity=0, model=None,
                    sampling=0, znormalise=False):
        """sofa_knn_noalloc into the caller's ids (B x k int64) and d (B x k
        float32) device tensors: the library allocates nothing."""
        import torch
        B = Q.shape[0]
        p = KnnParams(prune, None if radius is None else _dev(radius, torch.float32),
                      None if model is None else model._h, 0, None, int(candidate_capacity), int(sampling),
                      0, 1 if znormalise else 0)
        _check(load().sofa_knn_noalloc(self._h, _dev(Q, torch.float32), B, k, ctypes.byref(p), _dev(ids),
                                       _dev(d), _stream()))
        return ids, d

    def stats(self, ws=None):
        s = KnnStats()
        _check(load().sofa_knn_get_stats(None if ws is None else ws._h, self._h, ctypes.byref(s)))
        return s.as_dict()

    def workspace_bytes(self, B, k, prune=0):
        b = _i64()
        _check(load().sofa_workspace_bytes_for(self._h, B, k, prune, ctypes.byref(b)))
        return b.value

    def lower_bounds(self, Q, tables=True, lb=True, timed=False):
        """(tables B x 16 x 256, word bounds B x N in leaf order) as device
        tensors; with timed=True also the word-scan kernel's duration in ms."""
        import torch
        B = Q.shape[0]
        N = self.info()["N"]
        T = torch.empty((B, 16, 256), dtype=torch.float32, device=Q.device) if tables else None
        LB = torch.empty((B, N), dtype=torch.float32, device=Q.device) if lb else None
        ms = ctypes.c_double(0.0)
        _check(load().sofa_lower_bounds(self._h, _dev(Q, torch.float32), B,
                                        None if T is None else _dev(T),
                                        None if LB is None else _dev(LB), _stream(),
                                        ctypes.byref(ms) if timed else None))
        return (T, LB, ms.value) if timed else (T, LB)

    def bf16_lower_bounds(self, Q):
        """B x N batched-distance lower bounds (leaf order) from the BF16 MFMA kernel."""
        return self._prune_lower_bounds(Q, load().sofa_bf16_lower_bounds)

    def fp8_lower_bounds(self, Q):
        """B x N batched-distance lower bounds (leaf order) from the FP8 MFMA kernel."""
        return self._prune_lower_bounds(Q, load().sofa_fp8_lower_bounds)

    def _prune_lower_bounds(self, Q, fn):
        import torch
        B = Q.shape[0]
        N = self.info()["N"]
        LB = torch.empty((B, N), dtype=torch.float32, device=Q.device)
        _check(fn(self._h, _dev(Q, torch.float32), B, _dev(LB), _stream()))
        return LB

    def __del__(self):
        if _lib is not None and getattr(self, "_h", None) and self._h.value:
            _lib.sofa_index_free(self._h)
            self._h = _vp()


class RadiusModel:
    """The learned-radius network (sofa_radius_*): predicts ln d_k from a
    query's Fourier pool values; trained with the library's own kernels."""

    def __init__(self, k, in_dim=32, hidden1=256, hidden2=256, lr=1e-3, seed=0):
        h = _vp()
        p = RadiusParams(in_dim, hidden1, hidden2, k, lr, 0.9, 0.999, 1e-8, seed)
        _check(load().sofa_radius_create(ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self.k, self.in_dim = k, in_dim

    @property
    def num_params(self):
        return load().sofa_radius_num_params(self._h)

    def get(self):
        P = self.num_params
        params = np.zeros(P, dtype=np.float32)
        mu = np.zeros(self.in_dim, dtype=np.float32)
        sd = np.zeros(self.in_dim, dtype=np.float32)
        margin = ctypes.c_float()
        step = _i64()
        _check(load().sofa_radius_get(self._h, params.ctypes.data, mu.ctypes.data, sd.ctypes.data,
                                      ctypes.byref(margin), ctypes.byref(step)))
        return {"params": params, "mu": mu, "sd": sd, "margin": margin.value, "step": step.value}

    def set(self, params=None, mu=None, sd=None, margin=None, step=None):
        def f32(a):
            return None if a is None else np.ascontiguousarray(a, dtype=np.float32)
        params, mu, sd = f32(params), f32(mu), f32(sd)
        mg = None if margin is None else ctypes.byref(ctypes.c_float(margin))
        sp = None if step is None else ctypes.byref(_i64(step))
        _check(load().sofa_radius_set(self._h, None if params is None else params.ctypes.data,
                                      None if mu is None else mu.ctypes.data,
                                      None if sd is None else sd.ctypes.data, mg, sp))

    def standardize(self, feat):
        _check(load().sofa_radius_standardize(self._h, _dev(feat), feat.shape[0], _stream()))

    def gradients(self, feat, target):
        import torch
        g = torch.empty(self.num_params, dtype=torch.float32, device=feat.device)
        loss = torch.empty(1, dtype=torch.float32, device=feat.device)
        _check(load().sofa_radius_gradients(self._h, _dev(feat), _dev(target), feat.shape[0], _dev(g),
                                            _dev(loss), _stream()))
        return g, loss

    def train_step(self, feat, target):
        import torch
        loss = torch.empty(1, dtype=torch.float32, device=feat.device)
        _check(load().sofa_radius_train_step(self._h, _dev(feat), _dev(target), feat.shape[0],
                                             _dev(loss), _stream()))
        return loss

    def fit(self, feat, target, epochs, batch):
        losses = np.zeros(epochs, dtype=np.float32)
        _check(load().sofa_radius_fit(self._h, _dev(feat), _dev(target), feat.shape[0], epochs, batch,
                                      losses.ctypes.data, _stream()))
        return losses

    def forward(self, feat):
        import torch
        y = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device)
        _check(load().sofa_radius_forward(self._h, _dev(feat), feat.shape[0], _dev(y), _stream()))
        return y

    def calibrate(self, feat, target, quantile):
        _check(load().sofa_radius_calibrate(self._h, _dev(feat), _dev(target), feat.shape[0],
                                            float(quantile), _stream()))

    def predict(self, feat):
        import torch
        r = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device)
        _check(load().sofa_radius_predict(self._h, _dev(feat), feat.shape[0], _dev(r), _stream()))
        return r

    def __del__(self):
        if _lib is not None and getattr(self, "_h", None) and self._h.value:
            _lib.sofa_radius_free(self._h)
            self._h = _vp()


class Server:
    """The request loop (sofa_server_*): continuous batching of single-query
    requests over registered indexes, admitted by workspace memory, run on
    `slots` streams.  Keeps references to the indexes and models it serves."""

    def __init__(self, slots=4, max_batch=256, memory_budget=8 << 30, per_collection=1):
        h = _vp()
        p = ServerParams(int(slots), int(max_batch), int(memory_budget), int(per_collection))
        _check(load().sofa_server_create(ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self._keep = []
        self._n = []

    def add_collection(self, index, prune=0):
        cid = _i32()
        _check(load().sofa_server_add_collection(self._h, index._h, int(prune), ctypes.byref(cid)))
        self._keep.append(index)
        self._n.append(index.info()["n"])
        return cid.value

    def set_model(self, collection, model):
        _check(load().sofa_server_set_model(self._h, int(collection), model._h))
        self._keep.append(model)

    def submit(self, collection, query, k):
        """query: n FP32 values (host array).  Returns a ticket."""
        q = np.ascontiguousarray(query, dtype=np.float32)
        if 0 <= collection < len(self._n) and q.shape != (self._n[collection],):
            raise ValueError(f"query must have {self._n[collection]} values")
        t = _i64()
        _check(load().sofa_server_submit(self._h, int(collection), q.ctypes.data, int(k),
                                         ctypes.byref(t)))
        return t.value

    def wait(self, ticket, k, timeout_ms=-1):
        """(ids int64[k], dists float32[k], (latency_ms, queue_ms, batch_size))."""
        ids = np.empty(k, dtype=np.int64)
        d = np.empty(k, dtype=np.float32)
        tm = np.zeros(3, dtype=np.float64)
        _check(load().sofa_server_wait(self._h, int(ticket), ids.ctypes.data, d.ctypes.data,
                                       tm.ctypes.data, int(timeout_ms)))
        return ids, d, (float(tm[0]), float(tm[1]), int(tm[2]))

    def stats(self):
        s = ServerStats()
        _check(load().sofa_server_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if _lib is not None and getattr(self, "_h", None) and self._h.value:
            _lib.sofa_server_free(self._h)
            self._h = _vp()

    def __del__(self):
        self.close()
