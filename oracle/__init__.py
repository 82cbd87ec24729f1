"""CPU FP64 oracle for exact reverse k-MIPS.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP path: it is plain C (``rk_oracle.c``, double precision, sequential
inner products) behind ctypes, plus numpy glue.  See ``rk_oracle.c`` for the
definition it implements (Definition 2 of the paper, ties go to q) and the
pre-processing steps of Algorithm 1 (norms, norm sort, lower-bound arrays,
block minima).

Pins: every function here is checked in ``tests/test_oracle_pins.py``
against things other than itself: the paper's Example 1 (Table 1), exact
rational arithmetic on integer-valued vectors, the textbook argmax form at
k = 1, the order-statistic identity between the brute and table forms, the
counting invariant sum_q |R(q, k)| = k * n, scaling and permutation
covariance, and the textbook error bound of a recursive double sum.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile rk_oracle.c into liboracle.so with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    lib.ork_dot.argtypes = [f32p, f32p, i32]
    lib.ork_dot.restype = ctypes.c_double
    lib.ork_brute.argtypes = [f32p, i64, f32p, i64, i32, f32p, i32, u8p]
    lib.ork_brute.restype = i64
    lib.ork_theta.argtypes = [f32p, i64, f32p, i64, i32, i32, f64p]
    lib.ork_theta.restype = None
    lib.ork_theta_query.argtypes = [f64p, i32, f32p, i64, i32, f32p, i32, u8p]
    lib.ork_theta_query.restype = i64
    lib.ork_pair_dots.argtypes = [f32p, f32p, i32, i64p, i64p, i64, f64p]
    lib.ork_pair_dots.restype = None
    lib.ork_sqnorms.argtypes = [f32p, i64, i32, f64p]
    lib.ork_sqnorms.restype = None
    lib.ork_sort_desc.argtypes = [f64p, i64, i32p]
    lib.ork_sort_desc.restype = None
    lib.ork_lower_bounds.argtypes = [f32p, i64, f32p, i64, i32, i32p, i32p, i32, i64, f64p]
    lib.ork_lower_bounds.restype = None
    lib.ork_block_min.argtypes = [f64p, i64, i32, i32, f64p]
    lib.ork_block_min.restype = i64
    lib.ork_num_threads.argtypes = []
    lib.ork_num_threads.restype = i32
    lib.ork_set_threads.argtypes = [i32]
    lib.ork_set_threads.restype = None
    _lib = lib
    return lib


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a


def _rows(a, d):
    a = _f32(a)
    return a.reshape(-1, d) if a.size else np.zeros((0, d), np.float32)


def dot(x, y) -> float:
    """f(x, y): double sum of float32 products in index order."""
    x, y = _f32(x).ravel(), _f32(y).ravel()
    return _load().ork_dot(x, y, x.shape[0])


def pair_dots(A, B, ia, ib) -> np.ndarray:
    A = _f32(A)
    d = A.shape[1]
    B = _rows(B, d)
    ia = np.ascontiguousarray(ia, np.int64)
    ib = np.ascontiguousarray(ib, np.int64)
    out = np.empty(ia.shape[0], np.float64)
    _load().ork_pair_dots(A, B, d, ia, ib, ia.shape[0], out)
    return out


def brute_mask(Q, P, q, k: int) -> np.ndarray:
    """Definition 2 evaluated literally; boolean membership per user."""
    Q = _f32(Q)
    n, d = Q.shape
    P = _rows(P, d)
    q = _f32(q).ravel()
    assert q.shape[0] == d and k >= 1
    mask = np.zeros(n, np.uint8)
    _load().ork_brute(Q, n, P, P.shape[0], d, q, int(k), mask)
    return mask.astype(bool)


def brute(Q, P, q, k: int) -> np.ndarray:
    """Reverse k-MIPS result as ascending user ids (int32)."""
    return np.nonzero(brute_mask(Q, P, q, k))[0].astype(np.int32)


def theta(Q, P, kmax: int) -> np.ndarray:
    """[n, kmax] float64: descending top-kmax values of f(p, u) over P."""
    Q = _f32(Q)
    n, d = Q.shape
    P = _rows(P, d)
    out = np.empty((n, kmax), np.float64)
    _load().ork_theta(Q, n, P, P.shape[0], d, int(kmax), out)
    return out


def theta_query(th, Q, q, k: int) -> np.ndarray:
    """Membership via the exact table (k <= kmax); ascending user ids."""
    th = np.ascontiguousarray(th, np.float64)
    Q = _f32(Q)
    n, d = Q.shape
    kmax = th.shape[1]
    assert 1 <= k <= kmax
    mask = np.zeros(n, np.uint8)
    _load().ork_theta_query(th, kmax, Q, n, d, _f32(q).ravel(), int(k), mask)
    return np.nonzero(mask)[0].astype(np.int32)


def sqnorms(X) -> np.ndarray:
    X = _f32(X)
    out = np.empty(X.shape[0], np.float64)
    _load().ork_sqnorms(X, X.shape[0], X.shape[1], out)
    return out


def sort_desc(key) -> np.ndarray:
    key = np.ascontiguousarray(key, np.float64)
    perm = np.empty(key.shape[0], np.int32)
    _load().ork_sort_desc(key, key.shape[0], perm)
    return perm


def preprocess(Q, P, kmax: int, lb_items: int, b: int = 64) -> dict:
    """Algorithm 1: norms, descending norm sort of Q and P, lower-bound
    arrays over P' = first lb_items sorted items, and block minima.

    Returns permQ/permP (int32), s2Q/s2P (squared norms, original order),
    L [kmax, n] (sorted user order) and LB [kmax, nB]."""
    Q = _f32(Q)
    n, d = Q.shape
    P = _rows(P, d)
    m = P.shape[0]
    s2Q, s2P = sqnorms(Q), sqnorms(P)
    permQ, permP = sort_desc(s2Q), sort_desc(s2P)
    L = np.empty((kmax, n), np.float64)
    lib = _load()
    lib.ork_lower_bounds(Q, n, P, m, d, permQ, permP, int(kmax), int(lb_items), L)
    nB = (n + b - 1) // b
    LB = np.empty((kmax, max(nB, 0)), np.float64)
    if n:
        lib.ork_block_min(L, n, int(kmax), int(b), LB)
    return dict(permQ=permQ, permP=permP, s2Q=s2Q, s2P=s2P, L=L, LB=LB, nB=nB)


def num_threads() -> int:
    return int(_load().ork_num_threads())


def set_threads(t: int) -> None:
    _load().ork_set_threads(int(t))
