"""Thin ctypes binding of librkmips.so (C ABI in include/rkmips.h).

Argument marshalling only: every step of the query and build path runs in the
HIP library.  There is no fallback: if the library is missing or fails to
load, every call raises.  Names follow the C entry points.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librkmips.so")

RK_OK, RK_E_INVAL, RK_E_KMAX, RK_E_NOMEM, RK_E_TRUNC, RK_E_DEVICE, RK_E_BUSY = range(7)
RK_FP32, RK_BF16 = 0, 1
(RK_F_PERM_Q, RK_F_PERM_P, RK_F_SQNORM_Q, RK_F_SQNORM_P, RK_F_NORM_Q, RK_F_NORM_P,
 RK_F_L64, RK_F_L32, RK_F_LB, RK_F_BNORM) = range(10)
(RK_C_BLOCK_NO, RK_C_LEMMA1_NO, RK_C_LEMMA2_YES, RK_C_TABLE_YES, RK_C_SCAN_NO,
 RK_C_SCAN_YES, RK_C_RECHECK_NO, RK_C_RECHECK_YES) = range(8)

# Every exported symbol the header declares.
EXPORTS = [
    "rk_build_opts_default", "rk_build_index", "rk_build_index_dev", "rk_reverse_kmips",
    "rk_reverse_kmips_dev", "rk_reverse_kmips_batch", "rk_reverse_kmips_batch_dev",
    "rk_reverse_kmips_trace", "rk_index_set_timing", "rk_index_kernel_times",
    "rk_reverse_kmips_batch_dev_noalloc",
    "rk_index_set_counting", "rk_index_stats",
    "rk_index_reset_counters", "rk_index_export", "rk_index_rebuild", "rk_index_footprint",
    "rk_index_add_items", "rk_index_add_users",
    "rk_index_free", "rk_last_error",
    "rk_server_opts_default", "rk_server_create", "rk_server_add_catalog", "rk_server_submit",
    "rk_server_poll", "rk_server_inflight", "rk_server_used_bytes", "rk_server_free",
    "rk_server_submit_many", "rk_server_now_ms", "rk_server_catalog_state",
]


class RkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rk status {status}: {msg}")
        self.status = status


class BuildOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("lb_items", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("device", ctypes.c_int32),
                ("margin_rel", ctypes.c_double), ("cand_cap", ctypes.c_int32),
                ("auto_rebuild", ctypes.c_int32), ("pair_cap", ctypes.c_int32),
                ("handoff_tiles", ctypes.c_int32), ("no_blocks", ctypes.c_int32),
                ("verify_tiles", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("d", ctypes.c_int32), ("k_max", ctypes.c_int32), ("lb_items", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("n_blocks", ctypes.c_int32),
                ("precision", ctypes.c_int32),
                ("footprint_bytes", ctypes.c_int64), ("build_ms", ctypes.c_double),
                ("build_cand_total", ctypes.c_int64), ("build_cand_overflow_users", ctypes.c_int64),
                ("rebuilds", ctypes.c_int64), ("queries", ctypes.c_int64),
                ("blocks_visited", ctypes.c_int64), ("blocks_pruned", ctypes.c_int64),
                ("users_evaluated", ctypes.c_int64), ("lemma1_no", ctypes.c_int64),
                ("lemma2_yes", ctypes.c_int64), ("table_yes", ctypes.c_int64),
                ("survivors", ctypes.c_int64), ("scan_items", ctypes.c_int64),
                ("rechecks", ctypes.c_int64), ("results", ctypes.c_int64),
                ("scan_long", ctypes.c_int64), ("scan_full_f64", ctypes.c_int64),
                ("scan_handoff", ctypes.c_int64), ("scan_quarters", ctypes.c_int64),
                ("scan_valu_tiles", ctypes.c_int64), ("updates", ctypes.c_int64),
                ("reserved", ctypes.c_int64 * 2)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class ServerOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("max_wait_us", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("hbm_budget", ctypes.c_int64), ("max_queue", ctypes.c_int64),
                ("reserved", ctypes.c_int64 * 5)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("catalog", ctypes.c_int32), ("status", ctypes.c_int32),
                ("count", ctypes.c_int64), ("ids_offset", ctypes.c_int64),
                ("submit_ms", ctypes.c_double), ("done_ms", ctypes.c_double)]


_lib = None


def lib():
    """Load librkmips.so (raises if it has not been built).

    PyTorch is imported first: its HIP runtime (libamdhip64.so.7) is then the
    one the library binds to, so device pointers, streams and device-wide
    synchronisation are shared with torch in one runtime.  Loading the
    library before torch would bring in a second HIP/HSA runtime."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pidx = ctypes.POINTER(ctypes.c_void_p)
    L.rk_build_opts_default.argtypes = [ctypes.POINTER(BuildOpts)]
    L.rk_build_opts_default.restype = None
    for name in ("rk_build_index", "rk_build_index_dev"):
        f = getattr(L, name)
        f.argtypes = [vp, i64, vp, i64, i32, i32, ctypes.POINTER(BuildOpts), pidx]
        f.restype = ctypes.c_int
    L.rk_reverse_kmips.argtypes = [vp, vp, i32, vp, i64, ctypes.POINTER(i64)]
    L.rk_reverse_kmips.restype = ctypes.c_int
    L.rk_reverse_kmips_dev.argtypes = [vp, vp, i32, vp, i64, vp, vp]
    L.rk_reverse_kmips_dev.restype = ctypes.c_int
    L.rk_reverse_kmips_batch.argtypes = [vp, vp, i64, vp, vp, vp, i64]
    L.rk_reverse_kmips_batch.restype = ctypes.c_int
    L.rk_reverse_kmips_batch_dev.argtypes = [vp, vp, i64, vp, vp, vp, i64, vp]
    L.rk_reverse_kmips_batch_dev.restype = ctypes.c_int
    L.rk_reverse_kmips_batch_dev_noalloc.argtypes = [vp, vp, i64, vp, vp, vp, i64, vp]
    L.rk_reverse_kmips_batch_dev_noalloc.restype = ctypes.c_int
    L.rk_reverse_kmips_trace.argtypes = [vp, vp, i32, vp, vp]
    L.rk_reverse_kmips_trace.restype = ctypes.c_int
    L.rk_index_set_timing.argtypes = [vp, i32]
    L.rk_index_set_timing.restype = ctypes.c_int
    L.rk_index_kernel_times.argtypes = [vp, vp, vp, i32]
    L.rk_index_kernel_times.restype = ctypes.c_int
    L.rk_index_set_counting.argtypes = [vp, i32]
    L.rk_index_set_counting.restype = ctypes.c_int
    L.rk_index_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.rk_index_stats.restype = ctypes.c_int
    L.rk_index_reset_counters.argtypes = [vp]
    L.rk_index_reset_counters.restype = ctypes.c_int
    L.rk_index_export.argtypes = [vp, i32, vp, i64]
    L.rk_index_export.restype = ctypes.c_int
    L.rk_index_rebuild.argtypes = [vp, i32]
    L.rk_index_rebuild.restype = ctypes.c_int
    for f in (L.rk_index_add_items, L.rk_index_add_users):
        f.argtypes = [vp, vp, i64]
        f.restype = ctypes.c_int
    L.rk_index_footprint.argtypes = [i64, i64, i32, i32, ctypes.POINTER(BuildOpts)]
    L.rk_index_footprint.restype = i64
    L.rk_index_free.argtypes = [vp]
    L.rk_index_free.restype = None
    L.rk_last_error.argtypes = []
    L.rk_last_error.restype = ctypes.c_char_p
    L.rk_server_opts_default.argtypes = [ctypes.POINTER(ServerOpts)]
    L.rk_server_opts_default.restype = None
    L.rk_server_create.argtypes = [ctypes.POINTER(ServerOpts), pidx]
    L.rk_server_create.restype = ctypes.c_int
    L.rk_server_add_catalog.argtypes = [vp, vp, ctypes.POINTER(i32)]
    L.rk_server_add_catalog.restype = ctypes.c_int
    L.rk_server_submit.argtypes = [vp, i32, vp, i32, i64]
    L.rk_server_submit.restype = ctypes.c_int
    L.rk_server_poll.argtypes = [vp, ctypes.POINTER(Completion), i64, vp, i64, i32]
    L.rk_server_poll.restype = i64
    L.rk_server_inflight.argtypes = [vp]
    L.rk_server_inflight.restype = i64
    L.rk_server_used_bytes.argtypes = [vp]
    L.rk_server_used_bytes.restype = i64
    L.rk_server_free.argtypes = [vp]
    L.rk_server_free.restype = None
    L.rk_server_submit_many.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    L.rk_server_submit_many.restype = ctypes.c_int
    L.rk_server_now_ms.argtypes = [vp]
    L.rk_server_now_ms.restype = f64
    L.rk_server_catalog_state.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.rk_server_catalog_state.restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != RK_OK:
        raise RkError(status, lib().rk_last_error().decode())


def build_opts(precision="fp32", lb_items=0, device=0, margin_rel=0.0, cand_cap=0,
               auto_rebuild=False, pair_cap=0, handoff_tiles=0, block_size=0,
               no_blocks=False, verify_tiles=0) -> BuildOpts:
    o = BuildOpts()
    lib().rk_build_opts_default(ctypes.byref(o))
    o.precision = {"fp32": RK_FP32, "bf16": RK_BF16}[precision] if isinstance(precision, str) else int(precision)
    o.lb_items = int(lb_items)
    o.device = int(device)
    o.margin_rel = float(margin_rel)
    o.cand_cap = int(cand_cap)
    o.auto_rebuild = 1 if auto_rebuild else 0
    o.pair_cap = int(pair_cap)
    o.handoff_tiles = int(handoff_tiles)
    o.block_size = int(block_size)
    o.no_blocks = 1 if no_blocks else 0
    o.verify_tiles = int(verify_tiles)
    return o


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def index_footprint(n, m, d, k_max, **opts) -> int:
    return int(lib().rk_index_footprint(n, m, d, k_max, ctypes.byref(build_opts(**opts))))


class Index:
    """A device-resident reverse k-MIPS index (rk_index)."""

    def __init__(self, handle, n, m, d, k_max):
        self._h = handle
        self.n, self.m, self.d, self.k_max = n, m, d, k_max

    # -- construction ------------------------------------------------------
    @classmethod
    def build(cls, Q, P, k_max: int, **opts) -> "Index":
        Q, P = _f32(Q), _f32(P)
        d = Q.shape[1] if Q.ndim == 2 else P.shape[1]
        if P.size == 0:
            P = P.reshape(0, d)
        h = ctypes.c_void_p()
        _check(lib().rk_build_index(_ptr(Q), Q.shape[0], _ptr(P), P.shape[0], d, int(k_max),
                                    ctypes.byref(build_opts(**opts)), ctypes.byref(h)))
        return cls(h, Q.shape[0], P.shape[0], d, int(k_max))

    @classmethod
    def build_dev(cls, Q_dev, P_dev, k_max: int, **opts) -> "Index":
        """Q_dev, P_dev: contiguous float32 torch tensors on the device."""
        n, d = Q_dev.shape
        m = P_dev.shape[0]
        h = ctypes.c_void_p()
        _check(lib().rk_build_index_dev(ctypes.c_void_p(Q_dev.data_ptr()), n,
                                        ctypes.c_void_p(P_dev.data_ptr()), m, d, int(k_max),
                                        ctypes.byref(build_opts(**opts)), ctypes.byref(h)))
        return cls(h, n, m, d, int(k_max))

    def free(self):
        if self._h:
            lib().rk_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # -- queries -------------------------------------------------------------
    def reverse_kmips(self, q, k: int) -> np.ndarray:
        q = _f32(q).ravel()
        ids = np.empty(max(self.n, 1), np.int32)
        cnt = ctypes.c_int64()
        _check(lib().rk_reverse_kmips(self._h, _ptr(q), int(k), _ptr(ids), ids.shape[0],
                                      ctypes.byref(cnt)))
        return ids[:cnt.value].copy()

    def reverse_kmips_batch(self, qs, ks, cap: int | None = None):
        """Returns (offsets int64 [nq+1], ids int32)."""
        qs = _f32(qs).reshape(-1, self.d)
        ks = np.ascontiguousarray(ks, np.int32)
        nq = qs.shape[0]
        offsets = np.zeros(nq + 1, np.int64)
        cap = int(cap if cap is not None else max(1, min(nq * self.n, 1 << 26)))
        ids = np.empty(max(cap, 1), np.int32)
        st = lib().rk_reverse_kmips_batch(self._h, _ptr(qs), nq, _ptr(ks), _ptr(offsets),
                                          _ptr(ids), cap)
        if st == RK_E_TRUNC:
            ids = np.empty(int(offsets[-1]), np.int32)
            st = lib().rk_reverse_kmips_batch(self._h, _ptr(qs), nq, _ptr(ks), _ptr(offsets),
                                              _ptr(ids), ids.shape[0])
        _check(st)
        return offsets, ids[:offsets[-1]].copy()

    def trace(self, q, k: int):
        """Per-user decision classes (rk_class) and bulk u.q, by original id."""
        q = _f32(q).ravel()
        cls_ = np.empty(max(self.n, 1), np.uint8)
        shat = np.empty(max(self.n, 1), np.float32)
        _check(lib().rk_reverse_kmips_trace(self._h, _ptr(q), int(k), _ptr(cls_), _ptr(shat)))
        return cls_[:self.n], shat[:self.n]

    def reverse_kmips_dev(self, q_dev, k: int, ids_dev, count_dev, stream=None):
        """Device tensors: q_dev float32 [d], ids_dev int32 [cap], count_dev int64 [1]."""
        _check(lib().rk_reverse_kmips_dev(self._h, ctypes.c_void_p(q_dev.data_ptr()), int(k),
                                          ctypes.c_void_p(ids_dev.data_ptr()), ids_dev.numel(),
                                          ctypes.c_void_p(count_dev.data_ptr()),
                                          ctypes.c_void_p(stream) if stream else None))

    def reverse_kmips_batch_dev(self, qs_dev, ks_host, offsets_dev, ids_dev, stream=None):
        ks = np.ascontiguousarray(ks_host, np.int32)
        _check(lib().rk_reverse_kmips_batch_dev(
            self._h, ctypes.c_void_p(qs_dev.data_ptr()), qs_dev.shape[0], _ptr(ks),
            ctypes.c_void_p(offsets_dev.data_ptr()), ctypes.c_void_p(ids_dev.data_ptr()),
            ids_dev.numel(), ctypes.c_void_p(stream) if stream else None))

    def reverse_kmips_batch_dev_noalloc(self, qs_dev, ks_host, offsets_dev, ids_dev, stream=None):
        """As reverse_kmips_batch_dev, with the library's static workspace
        (no allocation); keep ks_host alive until the stream passes the call."""
        ks = np.ascontiguousarray(ks_host, np.int32)
        self._noalloc_ks = ks
        _check(lib().rk_reverse_kmips_batch_dev_noalloc(
            self._h, ctypes.c_void_p(qs_dev.data_ptr()), qs_dev.shape[0], _ptr(ks),
            ctypes.c_void_p(offsets_dev.data_ptr()), ctypes.c_void_p(ids_dev.data_ptr()),
            ids_dev.numel(), ctypes.c_void_p(stream) if stream else None))

    # -- introspection --------------------------------------------------------
    KERNEL_CLASSES = ("filter", "verify", "recheck", "finalize", "fill_all",
                      "batch_prep", "batch_filter", "batch_pairs", "batch_assemble")

    def set_timing(self, max_launches: int):
        _check(lib().rk_index_set_timing(self._h, int(max_launches)))

    def kernel_times(self) -> dict:
        """{class: (total_ms, launches)} of the launches timed since set_timing."""
        nc = len(self.KERNEL_CLASSES)
        ms = np.zeros(nc, np.float64)
        cnt = np.zeros(nc, np.int64)
        _check(lib().rk_index_kernel_times(self._h, _ptr(ms), _ptr(cnt), nc))
        return {c: (float(ms[i]), int(cnt[i])) for i, c in enumerate(self.KERNEL_CLASSES) if cnt[i]}

    def set_counting(self, on: bool = True):
        _check(lib().rk_index_set_counting(self._h, 1 if on else 0))

    def reset_counters(self):
        _check(lib().rk_index_reset_counters(self._h))

    def stats(self) -> dict:
        s = Stats()
        _check(lib().rk_index_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def rebuild(self, k_max: int):
        _check(lib().rk_index_rebuild(self._h, int(k_max)))
        self.k_max = int(k_max)

    def add_items(self, P):
        """Append items (ids continue from m); see rk_index_add_items."""
        P = _f32(P).reshape(-1, self.d)
        _check(lib().rk_index_add_items(self._h, _ptr(P), P.shape[0]))
        self.m += P.shape[0]

    def add_users(self, Q):
        """Append users (ids continue from n); see rk_index_add_users."""
        Q = _f32(Q).reshape(-1, self.d)
        _check(lib().rk_index_add_users(self._h, _ptr(Q), Q.shape[0]))
        self.n += Q.shape[0]

    def export(self, field: int) -> np.ndarray:
        st = self.stats()
        n, m, kmax, nB = st["n"], st["m"], st["k_max"], st["n_blocks"]
        spec = {
            RK_F_PERM_Q: (np.int32, (n,)), RK_F_PERM_P: (np.int32, (m,)),
            RK_F_SQNORM_Q: (np.float64, (n,)), RK_F_SQNORM_P: (np.float64, (m,)),
            RK_F_NORM_Q: (np.float32, (n,)), RK_F_NORM_P: (np.float32, (m,)),
            RK_F_L64: (np.float64, (kmax, n)), RK_F_L32: (np.float32, (kmax, n)),
            RK_F_LB: (np.float32, (kmax, nB)), RK_F_BNORM: (np.float32, (nB,)),
        }[field]
        out = np.empty(spec[1], spec[0])
        _check(lib().rk_index_export(self._h, int(field), _ptr(out) or ctypes.c_void_p(1),
                                     out.nbytes))
        return out


class Server:
    """Continuous-batching server over resident catalogs (rk_server_*): per
    catalog, `slots` launches in flight, each taking the queued requests when
    it is free.

    The indices added as catalogs are borrowed: keep them alive and do not
    query them directly while the server runs (this object holds references).
    """

    def __init__(self, max_batch: int = 1024, max_wait_us: int = 0, hbm_budget: int = 0,
                 device: int = 0, slots: int = 0, max_queue: int = 0):
        o = ServerOpts()
        lib().rk_server_opts_default(ctypes.byref(o))
        o.device, o.max_batch, o.max_wait_us, o.hbm_budget = device, max_batch, max_wait_us, hbm_budget
        o.slots, o.max_queue = slots, max_queue
        h = ctypes.c_void_p()
        _check(lib().rk_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._indices = []
        self._cap = 1 << 16
        self._ids = np.empty(self._cap, np.int32)
        self._recs = (Completion * 4096)()

    def add(self, index: "Index") -> int:
        c = ctypes.c_int32()
        _check(lib().rk_server_add_catalog(self._h, index._h, ctypes.byref(c)))
        self._indices.append(index)
        return c.value

    def submit(self, catalog: int, q: np.ndarray, k: int, tag: int):
        q = np.ascontiguousarray(q, np.float32)
        _check(lib().rk_server_submit(self._h, int(catalog), _ptr(q), int(k), int(tag)))

    def submit_many(self, catalogs, queries, ks, tags, arrival_ms=None):
        """Queue many requests in one call; queries is a list of float32 rows
        (kept alive by the caller until the call returns)."""
        n = len(ks)
        cat = np.ascontiguousarray(catalogs, np.int32)
        kk = np.ascontiguousarray(ks, np.int32)
        tg = np.ascontiguousarray(tags, np.int64)
        rows = [np.ascontiguousarray(q, np.float32) for q in queries]
        ptrs = (ctypes.c_void_p * max(n, 1))(*[r.ctypes.data for r in rows])
        arr = None if arrival_ms is None else np.ascontiguousarray(arrival_ms, np.float64)
        _check(lib().rk_server_submit_many(self._h, n, _ptr(cat), ptrs, _ptr(kk), _ptr(tg),
                                           _ptr(arr) if arr is not None else None))

    def now_ms(self) -> float:
        return lib().rk_server_now_ms(self._h)

    def poll(self, wait_us: int = 0) -> list:
        """Finished requests as (tag, catalog, status, ids, submit_ms, done_ms)."""
        while True:
            n = lib().rk_server_poll(self._h, self._recs, len(self._recs), _ptr(self._ids),
                                     self._cap, int(wait_us))
            if n >= 0:
                break
            msg = lib().rk_last_error().decode()
            if "ids" not in msg:
                raise RkError(RK_E_INVAL, msg)
            self._cap *= 4  # the next result is larger than the id buffer
            self._ids = np.empty(self._cap, np.int32)
        out = []
        for i in range(n):
            r = self._recs[i]
            ids = self._ids[r.ids_offset:r.ids_offset + r.count].copy()
            out.append((r.tag, r.catalog, r.status, ids, r.submit_ms, r.done_ms))
        return out

    def inflight(self) -> int:
        return lib().rk_server_inflight(self._h)

    def catalog_state(self, catalog: int) -> tuple[int, int]:
        """(queued requests, slots with a launch in flight) of a catalog."""
        q, r = ctypes.c_int64(), ctypes.c_int32()
        _check(lib().rk_server_catalog_state(self._h, int(catalog), ctypes.byref(q), ctypes.byref(r)))
        return q.value, r.value

    def used_bytes(self) -> int:
        return lib().rk_server_used_bytes(self._h)

    def close(self):
        if self._h:
            lib().rk_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
