"""Seeded synthetic data series (inputs only; none of the method's arithmetic).

The C source ``synth.c`` does the work; this module compiles it with gcc and
exposes it through ctypes.  Both the CPU oracle checks and the GPU library's
tests and benchmark take their inputs from here, so both sides read exactly
the same FP32 bits.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None

RW, HF, MIX, BAND = 0, 1, 2, 3
KINDS = {"rw": RW, "hf": HF, "mix": MIX, "band": BAND}


def build():
    """Compile libsynth.so (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.syn_generate.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_longlong,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_ulonglong, ctypes.c_int]
        lib.syn_queries.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_int,
                                    ctypes.c_longlong, ctypes.c_double, ctypes.c_ulonglong,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.syn_query_sources.argtypes = [ctypes.c_longlong, ctypes.c_longlong,
                                          ctypes.c_ulonglong, ctypes.c_void_p]
        lib.syn_noisy_copies.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_ulonglong, ctypes.c_void_p]
        _lib = lib
    return _lib


def _threads(nthreads):
    if nthreads:
        return int(nthreads)
    env = os.environ.get("OMP_NUM_THREADS")
    return int(env) if env else (os.cpu_count() or 1)


def collection(N, n, kind="rw", seed=1, row0=0, out=None, nthreads=0):
    """Rows [row0, row0+N) of a z-normalised FP32 collection, shape (N, n)."""
    k = KINDS[kind] if isinstance(kind, str) else int(kind)
    if out is None:
        out = np.empty((N, n), dtype=np.float32)
    assert out.shape == (N, n) and out.dtype == np.float32 and out.flags.c_contiguous
    if N > 0:
        _load().syn_generate(out.ctypes.data, row0, N, n, k, seed, _threads(nthreads))
    return out


def queries(X, B, sigma=0.1, seed=1, nthreads=0):
    """Noisy-copy queries of a host collection X: returns (Q (B, n) FP32, src (B,) int64)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    N, n = X.shape
    Q = np.empty((B, n), dtype=np.float32)
    src = np.empty(B, dtype=np.int64)
    if B > 0:
        _load().syn_queries(X.ctypes.data, N, n, B, float(sigma), seed, Q.ctypes.data,
                            src.ctypes.data, _threads(nthreads))
    return Q, src


def query_sources(N, B, seed=1):
    src = np.empty(B, dtype=np.int64)
    if B > 0:
        _load().syn_query_sources(N, B, seed, src.ctypes.data)
    return src


def noisy_copies(rows, sigma=0.1, seed=1):
    rows = np.ascontiguousarray(rows, dtype=np.float32)
    B, n = rows.shape
    Q = np.empty((B, n), dtype=np.float32)
    if B > 0:
        _load().syn_noisy_copies(rows.ctypes.data, B, n, float(sigma), seed, Q.ctypes.data)
    return Q
