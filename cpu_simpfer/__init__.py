"""Simpfer on the host CPU, as the paper designs it (Algorithms 1-3, OpenMP
over blocks): a comparison baseline for the benchmark, not part of the GPU
library and sharing no code with it or with the oracle.  See simpfer.c for
the readings taken where the algorithms are silent.

    from cpu_simpfer import CpuSimpfer
    s = CpuSimpfer(Q, P, k_max)          # Algorithm 1
    ids = s.query(q, k)                  # Algorithm 3, ascending original ids
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "simpfer.c")
_LIB = os.path.join(_HERE, "libcpusimpfer.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile simpfer.c with gcc -O3 and OpenMP (as the paper's g++ -O3 build)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O3", "-fopenmp", "-fno-fast-math", "-ffp-contract=off", "-fPIC",
                        "-shared", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("blocks", "blocks_pruned", "users", "lemma1_no",
                                              "lemma2_yes", "scans", "scan_items", "results")]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    L = ctypes.CDLL(_LIB)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.cs_build.argtypes = [vp, i64, vp, i64, i32, i32, i32, i32]
    L.cs_build.restype = vp
    L.cs_rebuild.argtypes = [vp, i32]
    L.cs_rebuild.restype = None
    L.cs_free.argtypes = [vp]
    L.cs_free.restype = None
    L.cs_query.argtypes = [vp, vp, i32, vp, ctypes.POINTER(Stats)]
    L.cs_query.restype = i64
    L.cs_threads.argtypes = []
    L.cs_threads.restype = i32
    L.cs_set_threads.argtypes = [i32]
    L.cs_set_threads.restype = None
    _lib = L
    return L


def threads() -> int:
    return int(_load().cs_threads())


def set_threads(t: int) -> None:
    _load().cs_set_threads(int(t))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


class CpuSimpfer:
    def __init__(self, Q, P, k_max: int, lb_items: int = 0, block_size: int = 0):
        self.Q = np.ascontiguousarray(Q, np.float32)
        self.P = np.ascontiguousarray(P, np.float32)
        self.n, self.d = self.Q.shape
        self.m = self.P.reshape(-1, self.d).shape[0]
        self.k_max = int(k_max)
        self._h = _load().cs_build(_ptr(self.Q), self.n, _ptr(self.P), self.m, self.d, self.k_max,
                                   int(lb_items), int(block_size))
        if not self._h:
            raise ValueError("cs_build: bad sizes")
        self.last_stats = {}

    def query(self, q, k: int) -> np.ndarray:
        q = np.ascontiguousarray(q, np.float32).ravel()
        if k < 1:
            raise ValueError("k must be >= 1")
        if self.k_max < k <= self.m:  # the paper's rule: rebuild the lower-bound arrays
            _load().cs_rebuild(self._h, int(k))
            self.k_max = int(k)
        ids = np.empty(max(self.n, 1), np.int32)
        st = Stats()
        c = _load().cs_query(self._h, _ptr(q), int(k), _ptr(ids), ctypes.byref(st))
        if c < 0:
            raise RuntimeError("cs_query failed")
        self.last_stats = st.as_dict()
        return ids[:c].copy()

    def free(self):
        if self._h:
            _load().cs_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
