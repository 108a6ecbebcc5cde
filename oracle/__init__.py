"""FP64 CPU oracle for exact k-NN search with the SFA summary.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this package; the GPU library never does.  The
arithmetic lives in ``sofa_oracle.c`` (plain C, FP64, no fused multiply-add);
this module compiles it with gcc and wraps it with ctypes and numpy.  It
shares no code with the GPU path.

Functions and the passages they follow (arXiv 2411.17483):
  znorm              Section II, z-normalised Euclidean distance (population sigma)
  dist2              Section II, squared distance, sequential FP64 sum
  dft_pool           Section IV-E, orthonormal DFT; pool = Re/Im of k = 1..P
  learn_bins         Algorithm 1 (MCB): stride sample, variance selection,
                     equi-depth or equi-width breakpoints
  words              Algorithm 2 (SFA transform), quantisation into half-open bins
  sfa_lb2            Eq. 2 and Eq. 3 (SFA lower bound, DC term omitted)
  dft_lb2            Eq. 1 (DFT lower bound)
  knn                Section II similarity search, k-NN extension (Section IV-C);
                     ranking key (FP64 distance, row id)
  mlp_forward / mlp_backward / adam
                     learned-radius network (not in the paper): FP64 forward,
                     chain-rule gradients and Adam (Kingma & Ba 2015)
  to_bf16 / to_e4m3  round-to-nearest-even onto the BF16 and OCP E4M3 grids
  tlb                Section V-E tightness of lower bound (a diagnostic)
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sofa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


def build():
    """Compile liboracle.so with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_znorm.argtypes = [_vp, ctypes.c_int, _vp]
        L.orc_dist2.argtypes = [_vp, _vp, ctypes.c_int]
        L.orc_dist2.restype = ctypes.c_double
        L.orc_dft_pool.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp]
        L.orc_dft_coef.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.orc_weight.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_weight.restype = ctypes.c_double
        L.orc_breakpoints.argtypes = [_vp, ctypes.c_long, ctypes.c_int, ctypes.c_int, _vp]
        L.orc_select.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp]
        L.orc_learn_bins.argtypes = [_vp, ctypes.c_long, ctypes.c_int, ctypes.c_long, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
        L.orc_symbol.argtypes = [ctypes.c_double, _vp, ctypes.c_int]
        L.orc_symbol.restype = ctypes.c_int
        L.orc_sfa_word.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   _vp, _vp, _vp, _vp]
        L.orc_mind.argtypes = [ctypes.c_double, ctypes.c_int, _vp, ctypes.c_int]
        L.orc_mind.restype = ctypes.c_double
        L.orc_sfa_lb2.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int]
        L.orc_sfa_lb2.restype = ctypes.c_double
        L.orc_dft_lb2.argtypes = [_vp, _vp, _vp, ctypes.c_int]
        L.orc_paa.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp]
        L.orc_paa.restype = None
        L.orc_isax_breakpoints.argtypes = [ctypes.c_int, _vp]
        L.orc_isax_breakpoints.restype = None
        L.orc_isax_word.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
        L.orc_isax_word.restype = None
        L.orc_isax_lb2.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_isax_lb2.restype = ctypes.c_double
        L.orc_paa_dist2.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_int]
        L.orc_paa_dist2.restype = ctypes.c_double
        L.orc_dft_lb2.restype = ctypes.c_double
        L.orc_knn.argtypes = [_vp, ctypes.c_long, ctypes.c_int, _vp, ctypes.c_long, ctypes.c_int,
                              _vp, _vp, ctypes.c_int]
        L.orc_dist2_rows.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_long, _vp]
        L.orc_tlb.argtypes = [_vp, _vp, ctypes.c_long]
        L.orc_tlb.restype = ctypes.c_double
        L.orc_mlp_forward.argtypes = [_vp, ctypes.c_long, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      _vp, _vp, _vp, _vp, _vp, ctypes.c_double, _vp]
        L.orc_mlp_backward.argtypes = [_vp, _vp, ctypes.c_long, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, _vp, _vp, _vp, _vp, _vp, ctypes.c_double,
                                       _vp, _vp, _vp, _vp, _vp, _vp]
        L.orc_mlp_backward.restype = ctypes.c_double
        L.orc_adam.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_long, ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_to_bf16.argtypes = [ctypes.c_double]
        L.orc_to_bf16.restype = ctypes.c_double
        L.orc_to_e4m3.argtypes = [ctypes.c_double]
        L.orc_to_e4m3.restype = ctypes.c_double
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _threads(nthreads):
    if nthreads:
        return int(nthreads)
    env = os.environ.get("OMP_NUM_THREADS")
    return int(env) if env else (os.cpu_count() or 1)


# --------------------------------------------------------------------------- #
def znorm(x):
    """z-normalise one series (population sigma) in FP64."""
    x = _f64(x)
    out = np.empty_like(x)
    _load().orc_znorm(x.ctypes.data, x.shape[0], out.ctypes.data)
    return out


def dist2(q, x):
    """Squared distance of two FP32 series, FP64 sequential sum."""
    q, x = _f32(q), _f32(x)
    return _load().orc_dist2(q.ctypes.data, x.ctypes.data, q.shape[0])


def dft_pool(X, P):
    """Pool of Fourier values of each row: (m, 2P) FP64, Re/Im of k = 1..P."""
    X = _f32(np.atleast_2d(X))
    m, n = X.shape
    out = np.empty((m, 2 * P), dtype=np.float64)
    L = _load()
    for i in range(m):
        L.orc_dft_pool(X[i].ctypes.data, n, P, out[i].ctypes.data)
    return out


def dft_coef(x, k):
    x = _f32(x)
    re, im = ctypes.c_double(), ctypes.c_double()
    _load().orc_dft_coef(x.ctypes.data, x.shape[0], k, ctypes.byref(re), ctypes.byref(im))
    return re.value, im.value


def weight(k, n):
    return _load().orc_weight(k, n)


def breakpoints(vals, alpha, binning=0):
    vals = _f64(vals)
    beta = np.empty(alpha - 1, dtype=np.float64)
    _load().orc_breakpoints(vals.ctypes.data, vals.shape[0], alpha, binning, beta.ctypes.data)
    return beta


def select(var, l):
    var = _f64(var)
    sel = np.empty(l, dtype=np.int32)
    _load().orc_select(var.ctypes.data, var.shape[0], l, sel.ctypes.data)
    return sel


def learn_bins(X, m, P=16, l=16, alpha=256, binning=0, selection=0):
    """Algorithm 1 on the stride sample of m rows: returns (var, sel, beta[l, alpha-1]).
    selection=1 keeps the first l pool values instead of the l of largest variance."""
    X = _f32(X)
    N, n = X.shape
    var = np.empty(2 * P, dtype=np.float64)
    sel = np.empty(l, dtype=np.int32)
    beta = np.empty((l, alpha - 1), dtype=np.float64)
    _load().orc_learn_bins(X.ctypes.data, N, n, m, P, l, alpha, binning, int(selection),
                           var.ctypes.data, sel.ctypes.data, beta.ctypes.data)
    return var, sel, beta


def words(X, sel, beta, P=16):
    """SFA words (m, l) uint8 and the selected Fourier values (m, l) FP64."""
    X = _f32(np.atleast_2d(X))
    m, n = X.shape
    sel = np.ascontiguousarray(sel, dtype=np.int32)
    beta = _f64(beta)
    l, am1 = beta.shape
    W = np.empty((m, l), dtype=np.uint8)
    C = np.empty((m, l), dtype=np.float64)
    L = _load()
    for i in range(m):
        L.orc_sfa_word(X[i].ctypes.data, n, P, l, am1 + 1, sel.ctypes.data, beta.ctypes.data,
                       W[i].ctypes.data, C[i].ctypes.data)
    return W, C


def symbol(c, beta_j):
    beta_j = _f64(beta_j)
    return _load().orc_symbol(float(c), beta_j.ctypes.data, beta_j.shape[0] + 1)


def mind(v, s, beta_j):
    beta_j = _f64(beta_j)
    return _load().orc_mind(float(v), int(s), beta_j.ctypes.data, beta_j.shape[0] + 1)


def sfa_lb2(qsel, word, beta, w=None):
    """Squared SFA lower bound of one query's selected values against one word."""
    qsel = _f64(qsel)
    word = np.ascontiguousarray(word, dtype=np.uint8)
    beta = _f64(beta)
    l, am1 = beta.shape
    w = _f64(np.full(l, 2.0) if w is None else w)
    return _load().orc_sfa_lb2(qsel.ctypes.data, word.ctypes.data, beta.ctypes.data,
                               w.ctypes.data, l, am1 + 1)


def paa(x, l):
    """PAA means of one series over l equal segments (Section IV-D)."""
    x = _f32(x)
    out = np.zeros(l, dtype=np.float64)
    _load().orc_paa(x.ctypes.data, x.shape[0], l, out.ctypes.data)
    return out


def isax_breakpoints(alpha):
    """The alpha-1 equal-depth breakpoints of N(0,1)."""
    out = np.zeros(max(alpha - 1, 1), dtype=np.float64)
    _load().orc_isax_breakpoints(alpha, out.ctypes.data)
    return out[:alpha - 1]


def isax_words(X, l, alpha):
    """(words m x l uint8, PAA means m x l) of the rows of X."""
    X = _f32(np.atleast_2d(X))
    m, n = X.shape
    beta = _f64(np.append(isax_breakpoints(alpha), 0.0))
    W = np.zeros((m, l), dtype=np.uint8)
    M = np.zeros((m, l), dtype=np.float64)
    L = _load()
    for i in range(m):
        L.orc_isax_word(X[i].ctypes.data, n, l, alpha, beta.ctypes.data, W[i].ctypes.data,
                        M[i].ctypes.data)
    return W, M


def isax_lb2(qpaa, word, n, alpha):
    """Squared iSAX lower bound of one query's PAA means against one word."""
    qpaa = _f64(qpaa)
    word = np.ascontiguousarray(word, dtype=np.uint8)
    beta = _f64(np.append(isax_breakpoints(alpha), 0.0))
    return _load().orc_isax_lb2(qpaa.ctypes.data, word.ctypes.data, beta.ctypes.data, n,
                                qpaa.shape[0], alpha)


def paa_dist2(q, x, l):
    """Squared PAA distance n/l * sum (mean_j(q) - mean_j(x))^2."""
    q, x = _f32(q), _f32(x)
    return _load().orc_paa_dist2(q.ctypes.data, x.ctypes.data, q.shape[0], l)


def dft_lb2(a, b, w):
    a, b, w = _f64(a), _f64(b), _f64(w)
    return _load().orc_dft_lb2(a.ctypes.data, b.ctypes.data, w.ctypes.data, a.shape[0])


def knn(X, Q, k, nthreads=0):
    """Brute-force exact k-NN: (ids (B, k) int64, d2 (B, k) FP64), ranked by (d2, id)."""
    X, Q = _f32(X), _f32(np.atleast_2d(Q))
    N, n = X.shape
    B = Q.shape[0]
    ids = np.empty((B, k), dtype=np.int64)
    d2 = np.empty((B, k), dtype=np.float64)
    _load().orc_knn(X.ctypes.data, N, n, Q.ctypes.data, B, k, ids.ctypes.data, d2.ctypes.data,
                    _threads(nthreads))
    return ids, d2


def dist2_rows(X, q, rows):
    X, q = _f32(X), _f32(q)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(rows.shape[0], dtype=np.float64)
    _load().orc_dist2_rows(X.ctypes.data, X.shape[1], q.ctypes.data, rows.ctypes.data,
                           rows.shape[0], out.ctypes.data)
    return out


def tlb(lb2, d2):
    lb2, d2 = _f64(lb2), _f64(d2)
    return _load().orc_tlb(lb2.ctypes.data, d2.ctypes.data, lb2.shape[0])


# --------------------------------------------------------------------------- #
class MLPParams:
    """FP64 parameters of the 32 -> 256 -> 256 -> 1 radius network."""

    def __init__(self, W1, b1, W2, b2, W3, b3):
        self.W1, self.b1, self.W2, self.b2, self.W3 = (_f64(a) for a in (W1, b1, W2, b2, W3))
        self.b3 = float(b3)

    @property
    def dims(self):
        H1, D = self.W1.shape
        return D, H1, self.W2.shape[0]


def mlp_forward(p, x):
    x = _f32(x)
    D, H1, H2 = p.dims
    y = np.empty(x.shape[0], dtype=np.float64)
    _load().orc_mlp_forward(x.ctypes.data, x.shape[0], D, H1, H2, p.W1.ctypes.data,
                            p.b1.ctypes.data, p.W2.ctypes.data, p.b2.ctypes.data,
                            p.W3.ctypes.data, p.b3, y.ctypes.data)
    return y


def mlp_backward(p, x, t):
    """Returns (loss, grads dict with keys W1 b1 W2 b2 W3 b3)."""
    x, t = _f32(x), _f32(t)
    D, H1, H2 = p.dims
    g = {"W1": np.empty((H1, D)), "b1": np.empty(H1), "W2": np.empty((H2, H1)),
         "b2": np.empty(H2), "W3": np.empty(H2)}
    gb3 = ctypes.c_double()
    loss = _load().orc_mlp_backward(x.ctypes.data, t.ctypes.data, x.shape[0], D, H1, H2,
                                    p.W1.ctypes.data, p.b1.ctypes.data, p.W2.ctypes.data,
                                    p.b2.ctypes.data, p.W3.ctypes.data, p.b3,
                                    g["W1"].ctypes.data, g["b1"].ctypes.data,
                                    g["W2"].ctypes.data, g["b2"].ctypes.data,
                                    g["W3"].ctypes.data, ctypes.byref(gb3))
    g["b3"] = np.array([gb3.value])
    return loss, g


def adam(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step on flat FP64 arrays p, m, v with gradient g."""
    for a in (p, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _load().orc_adam(p.ctypes.data, g.ctypes.data, m.ctypes.data, v.ctypes.data, p.shape[0],
                     int(step), lr, beta1, beta2, eps)


def to_bf16(a):
    f = _load().orc_to_bf16
    return np.array([f(float(v)) for v in np.ravel(a)]).reshape(np.shape(a))


def to_e4m3(a):
    f = _load().orc_to_e4m3
    return np.array([f(float(v)) for v in np.ravel(a)]).reshape(np.shape(a))
