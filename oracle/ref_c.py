"""ctypes access to the plain FP64 C oracle (``rg_ref.c``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  ``build()`` compiles
``rg_ref.c`` with gcc into ``oracle/librg_ref.so``; ``load()`` only loads it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rg_ref.c")
_LIB = os.path.join(_HERE, "librg_ref.so")
_lib = None

_p = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)


def build():
    """Compile the C oracle (always rebuilds)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    global _lib
    _lib = None
    return _LIB


def build_from_source(src_text, out_path):
    """Compile C oracle source text (e.g. a copy with a mistake planted by a
    mutation test) into ``out_path``; returns the path."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", src, "-o", out_path, "-lm"])
    return out_path


def source():
    with open(_SRC) as f:
        return f.read()


_other = {}


def load(lib_path=None):
    """Load the oracle library (``lib_path``: another build of the same source,
    such as a mutated copy)."""
    global _lib
    if lib_path is not None:
        if lib_path not in _other:
            _other[lib_path] = _bind(ctypes.CDLL(lib_path))
        return _other[lib_path]
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    lib.rgo_new.restype = _p
    lib.rgo_new.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double]
    lib.rgo_free.argtypes = [_p]
    lib.rgo_push.restype = ctypes.c_int
    lib.rgo_push.argtypes = [_p, _p, _p, ctypes.c_int64, _p]
    lib.rgo_rank.restype = ctypes.c_int
    lib.rgo_rank.argtypes = [_p]
    lib.rgo_get.argtypes = [_p, _p, _p, _p, _p]
    lib.rgo_solve_batch.restype = ctypes.c_int
    lib.rgo_solve_batch.argtypes = [ctypes.c_int, _p, _p, _p, _p, _p, _p, ctypes.c_double, _p, _p, _p, _p, _p,
                                    ctypes.c_int]
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class Stream:
    """One recursive least-squares stream kept by the C oracle."""

    def __init__(self, m, cap=None, eps=-1.0, lib_path=None):
        self._lib = load(lib_path)
        self.m = int(m)
        self.cap = int(cap if cap is not None else m)
        self._h = self._lib.rgo_new(self.m, self.cap, float(eps))
        if not self._h:
            raise MemoryError("rgo_new failed")

    def push(self, A, Y, decisions=False):
        A = np.ascontiguousarray(A, dtype=np.float64).reshape(-1, self.m)
        Y = np.ascontiguousarray(Y, dtype=np.float64).reshape(-1)
        assert A.shape[0] == Y.shape[0]
        dec = np.zeros(A.shape[0], dtype=np.uint8) if decisions else None
        rc = self._lib.rgo_push(self._h, _ptr(A), _ptr(Y), A.shape[0], _ptr(dec))
        if rc != 0:
            raise OverflowError("rank capacity exceeded")
        return dec

    @property
    def rank(self):
        return self._lib.rgo_rank(self._h)

    def state(self):
        r = self.rank
        X = np.zeros(self.m)
        C = np.zeros((r, self.m))
        Ct = np.zeros((r, self.m))
        P = np.zeros((r, r))
        self._lib.rgo_get(self._h, _ptr(X), _ptr(C), _ptr(Ct), _ptr(P))
        return X, C, Ct, P

    @property
    def x(self):
        return self.state()[0]

    def close(self):
        if self._h:
            self._lib.rgo_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(A, Y, eps=-1.0, cap=None, decisions=False, lib_path=None):
    """Solve one stream from scratch; returns (x, r, C, Ct, Pinv[, decisions])."""
    A = np.asarray(A, dtype=np.float64)
    s = Stream(A.shape[1], cap, eps, lib_path)
    dec = s.push(A, Y, decisions)
    X, C, Ct, P = s.state()
    r = s.rank
    s.close()
    return (X, r, C, Ct, P, dec) if decisions else (X, r, C, Ct, P)


def solve_batch(ms, row_ptr, a_off, A, Y, eps=-1.0, caps=None, order=None, nthreads=None):
    """Solve B independent streams on a thread pool.  Returns (X packed,
    x_off, rank, status, threads_used)."""
    lib = load()
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    B = ms.shape[0]
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    a_off = np.ascontiguousarray(a_off, dtype=np.int64)
    A = np.ascontiguousarray(A, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    caps = None if caps is None else np.ascontiguousarray(caps, dtype=np.int32)
    order = None if order is None else np.ascontiguousarray(order, dtype=np.int64)
    x_off = np.zeros(B, dtype=np.int64)
    if B > 1:
        x_off[1:] = np.cumsum(ms[:-1].astype(np.int64))
    X = np.zeros(int(ms.astype(np.int64).sum()), dtype=np.float64)
    rank = np.zeros(B, dtype=np.int32)
    status = np.zeros(B, dtype=np.int32)
    nth = nthreads or os.cpu_count() or 1
    used = lib.rgo_solve_batch(B, _ptr(ms), _ptr(caps), _ptr(row_ptr), _ptr(a_off), _ptr(A), _ptr(Y),
                               float(eps), _ptr(order), _ptr(x_off), _ptr(X), _ptr(rank), _ptr(status), int(nth))
    return X, x_off, rank, status, used
