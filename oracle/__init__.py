"""CPU oracle for round-synchronous contraction-hierarchy construction.

TEST INFRASTRUCTURE.  This package wraps ``spoch_oracle.c``, a plain,
sequential C implementation of the construction described by Wan et al.,
"Parallel Contraction Hierarchies Can Be Efficient and Scalable" (ICS 2025):
the main loop (Alg. 3), LocalSearch (Alg. 4), Score (Alg. 5), Select
(Alg. 6), Contract (Alg. 7), Postprocessing, and the bidirectional CH query.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import it.  It shares no code with the GPU library
``paper_2412_18008_amd`` and never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "spoch_oracle.c")

ORC_OK = 0
ORC_E_INVALID = -1
ORC_E_OOM = -2
ORC_E_OVERFLOW = -3
ORC_E_LIMIT = -4
ORC_E_STATE = -5

WPS_EXACT = 0
WPS_HOP = 1
WPS_SETTLED = 2

UINT64_MAX = np.uint64(0xFFFFFFFFFFFFFFFF)
NOMID = 0xFFFFFFFF


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(LIB_PATH) or (
        os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH)
    ):
        tmp = LIB_PATH + ".tmp"
        # -ffp-contract=off: the learned priority is evaluated without fused
        # multiply-add, so its single-precision result is reproducible
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-shared",
             "-fPIC", "-o", tmp, SRC_PATH, "-lm"]
        )
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Params(C.Structure):
    _fields_ = [("wps_mode", C.c_uint32), ("hop_limit", C.c_uint32),
                ("settle_limit", C.c_uint32), ("max_rounds", C.c_uint32),
                ("priority", C.c_uint32), ("record", C.c_uint32), ("mlp", C.c_void_p),
                ("k_ed", C.c_int32), ("k_cn", C.c_int32), ("k_depth", C.c_int32),
                ("tiebreak", C.c_uint32), ("mlp_qbits", C.c_uint32)]


TIE_HASHED_ID = 0
TIE_RAW_ID = 1

PRIO_PLAIN = 0
PRIO_LEARNED = 1
MLP_PARAMS = 4801


class RoundStats(C.Structure):
    _fields_ = [
        ("alive_before", C.c_uint32), ("n_sources", C.c_uint32),
        ("n_affected", C.c_uint32), ("n_searched", C.c_uint32),
        ("n_targets", C.c_uint64), ("n_pruned", C.c_uint64),
        ("n_selected", C.c_uint32), ("n_pairs_emitted", C.c_uint64),
        ("n_shortcuts", C.c_uint64), ("n_absent", C.c_uint64),
        ("n_settled", C.c_uint64), ("overlay_arcs", C.c_uint64),
    ]


_lib = None


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        vp, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
        L.orc_create.argtypes = [u32, u64, vp, vp, vp, vp, u64, C.POINTER(_Params),
                                 C.POINTER(vp)]
        L.orc_create.restype = i32
        L.orc_free.argtypes = [vp]
        for f in ("orc_round", "orc_run", "orc_finish"):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = i32
        for f in ("orc_n", "orc_rounds", "orc_alive_count"):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = u32
        for f in ("orc_overlay_count", "orc_memo_count", "orc_up_count", "orc_down_count"):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = u64
        L.orc_get_labels.argtypes = [vp, vp]
        L.orc_get_vertex_state.argtypes = [vp, vp, vp, vp, vp]
        L.orc_get_rank.argtypes = [vp, vp]
        L.orc_get_rank.restype = i32
        for f in ("orc_get_overlay", "orc_get_up", "orc_get_down"):
            getattr(L, f).argtypes = [vp, vp, vp, vp, vp]
        L.orc_get_memo.argtypes = [vp, vp, vp, vp]
        L.orc_get_round_stats.argtypes = [vp, vp]
        L.orc_query.argtypes = [vp, u32, u32, C.POINTER(u64)]
        L.orc_query.restype = u64
        L.orc_query_batch.argtypes = [vp, u64, vp, vp, vp, vp]
        L.orc_query_batch.restype = i32
        L.orc_dijkstra.argtypes = [u32, vp, vp, vp, u32, vp]
        L.orc_dijkstra.restype = i32
        L.orc_dijkstra_settle.argtypes = [u32, vp, vp, vp, u32, u64, vp, vp]
        L.orc_dijkstra_settle.restype = i32
        L.orc_overlay_dijkstra.argtypes = [vp, u32, vp]
        L.orc_overlay_dijkstra.restype = i32
        L.orc_default_label.argtypes = [u32, u64]
        L.orc_default_label.restype = u32
        L.orc_get_features.argtypes = [vp, vp]
        L.orc_get_features.restype = i32
        L.orc_mlp_priority.argtypes = [vp, vp, C.POINTER(C.c_float)]
        L.orc_mlp_priority.restype = C.c_int32
        L.orc_mlp_priority_q.argtypes = [vp, vp, C.c_uint32, C.POINTER(C.c_float)]
        L.orc_mlp_priority_q.restype = C.c_int32
        L.orc_gelu.argtypes = [C.c_float]
        L.orc_gelu.restype = C.c_float
        L.orc_load.argtypes = [u32, vp, u64, vp, vp, vp, u64, vp, vp, vp, C.POINTER(vp)]
        L.orc_load.restype = i32
        _lib = L
    return _lib


def _csr(off, dst, w):
    off = np.ascontiguousarray(off, dtype=np.uint64)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    return off, dst, w


class OracleCH:
    """One oracle construction.  Construct, then call ``round()`` repeatedly
    or ``run()`` once; inspection methods copy state into numpy arrays."""

    def __init__(self, off, dst, w, labels=None, seed=0, wps_mode=WPS_EXACT,
                 hop_limit=2, settle_limit=64, max_rounds=0, mlp=None, record=False,
                 k_ed=1, k_cn=0, k_depth=0, tiebreak=TIE_HASHED_ID, mlp_qbits=0):
        L = lib()
        off, dst, w = _csr(off, dst, w)
        n = len(off) - 1
        self._keep = (off, dst, w)
        lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.uint32)
        wts = None if mlp is None else np.ascontiguousarray(mlp, dtype=np.float32)
        if wts is not None and wts.size != MLP_PARAMS:
            raise ValueError("mlp must hold 4801 weights")
        p = _Params(wps_mode, hop_limit, settle_limit, max_rounds,
                    PRIO_LEARNED if wts is not None else PRIO_PLAIN, int(record), _p(wts),
                    k_ed, k_cn, k_depth, tiebreak, mlp_qbits)
        h = C.c_void_p()
        rc = L.orc_create(n, len(dst), _p(off), _p(dst), _p(w), _p(lab), seed,
                          C.byref(p), C.byref(h))
        if rc != ORC_OK:
            raise OracleError(rc, "orc_create")
        self.h = h
        self.n = n

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_free(self.h)
            self.h = None

    def features(self):
        x = np.empty((self.n, 8), np.float32)
        rc = lib().orc_get_features(self.h, _p(x))
        if rc:
            raise OracleError(rc, "orc_get_features")
        return x

    def round(self) -> int:
        rc = lib().orc_round(self.h)
        if rc < 0:
            raise OracleError(rc, "orc_round")
        return rc

    def run(self):
        rc = lib().orc_run(self.h)
        if rc < 0:
            raise OracleError(rc, "orc_run")
        return self

    def finish(self):
        rc = lib().orc_finish(self.h)
        if rc < 0:
            raise OracleError(rc, "orc_finish")
        return self

    @property
    def rounds(self) -> int:
        return lib().orc_rounds(self.h)

    @property
    def alive_count(self) -> int:
        return lib().orc_alive_count(self.h)

    def labels(self):
        a = np.empty(self.n, np.uint32)
        lib().orc_get_labels(self.h, _p(a))
        return a

    def vertex_state(self):
        n = self.n
        level = np.empty(n, np.uint32)
        pc = np.empty(n, np.int32)
        p = np.empty(n, np.int32)
        alive = np.empty(n, np.uint8)
        lib().orc_get_vertex_state(self.h, _p(level), _p(pc), _p(p), _p(alive))
        return dict(level=level, pc=pc, p=p, alive=alive.astype(bool))

    def rank(self):
        a = np.empty(self.n, np.uint32)
        rc = lib().orc_get_rank(self.h, _p(a))
        if rc:
            raise OracleError(rc, "orc_get_rank")
        return a

    def _arcs(self, count_fn, get_fn):
        k = count_fn(self.h)
        t, h_, w, mid = (np.empty(k, np.uint32) for _ in range(4))
        get_fn(self.h, _p(t), _p(h_), _p(w), _p(mid))
        return dict(tail=t, head=h_, w=w, mid=mid)

    def overlay(self):
        L = lib()
        return self._arcs(L.orc_overlay_count, L.orc_get_overlay)

    def up(self):
        L = lib()
        return self._arcs(L.orc_up_count, L.orc_get_up)

    def down(self):
        L = lib()
        return self._arcs(L.orc_down_count, L.orc_get_down)

    def memo(self):
        L = lib()
        k = L.orc_memo_count(self.h)
        s, t, d = (np.empty(k, np.uint32) for _ in range(3))
        L.orc_get_memo(self.h, _p(s), _p(t), _p(d))
        return dict(s=s, t=t, d=d)

    def round_stats(self):
        k = self.rounds
        arr = (RoundStats * max(k, 1))()
        lib().orc_get_round_stats(self.h, C.cast(arr, C.c_void_p))
        return [{f: getattr(arr[i], f) for f, _ in RoundStats._fields_} for i in range(k)]

    def query(self, s, t):
        c = C.c_uint64()
        d = lib().orc_query(self.h, int(s), int(t), C.byref(c))
        return d, c.value

    def query_batch(self, s, t):
        s = np.ascontiguousarray(s, np.uint32)
        t = np.ascontiguousarray(t, np.uint32)
        dist = np.empty(len(s), np.uint64)
        settled = np.empty(len(s), np.uint64)
        rc = lib().orc_query_batch(self.h, len(s), _p(s), _p(t), _p(dist), _p(settled))
        if rc:
            raise OracleError(rc, "orc_query_batch")
        return dist, settled

    def overlay_dijkstra(self, s):
        d = np.empty(self.n, np.uint64)
        rc = lib().orc_overlay_dijkstra(self.h, int(s), _p(d))
        if rc:
            raise OracleError(rc, "orc_overlay_dijkstra")
        return d


class LoadedCH(OracleCH):
    """A finished CH given by its rank order and arc lists (queries only)."""

    def __init__(self, rank, up_tail, up_head, up_w, down_tail, down_head, down_w):
        L = lib()
        arrs = [np.ascontiguousarray(a, np.uint32) for a in
                (rank, up_tail, up_head, up_w, down_tail, down_head, down_w)]
        self._keep = arrs
        r, ut, uh, uw, dt, dh, dw = arrs
        h = C.c_void_p()
        rc = L.orc_load(len(r), _p(r), len(ut), _p(ut), _p(uh), _p(uw), len(dt), _p(dt), _p(dh),
                        _p(dw), C.byref(h))
        if rc != ORC_OK:
            raise OracleError(rc, "orc_load")
        self.h = h
        self.n = len(r)


def dijkstra(off, dst, w, s):
    """Plain binary-heap Dijkstra on a CSR graph (uint64, max = unreachable)."""
    off, dst, w = _csr(off, dst, w)
    n = len(off) - 1
    d = np.empty(n, np.uint64)
    rc = lib().orc_dijkstra(n, _p(off), _p(dst), _p(w), int(s), _p(d))
    if rc:
        raise OracleError(rc, "orc_dijkstra")
    return d


def dijkstra_settle(off, dst, w, s, max_settled):
    """Dijkstra stopped after max_settled vertices: (dist, settled count);
    dist is UINT64_MAX for every vertex not settled."""
    off, dst, w = _csr(off, dst, w)
    n = len(off) - 1
    d = np.empty(n, np.uint64)
    c = C.c_uint64()
    rc = lib().orc_dijkstra_settle(n, _p(off), _p(dst), _p(w), int(s), int(max_settled), _p(d),
                                   C.byref(c))
    if rc:
        raise OracleError(rc, "orc_dijkstra_settle")
    return d, c.value


def mlp_priority(w, x, qbits=16):
    """(priority, output y) of the learned priority for one feature vector,
    the output quantised to qbits fractional bits."""
    w = np.ascontiguousarray(w, np.float32)
    x = np.ascontiguousarray(x, np.float32)
    y = C.c_float()
    p = lib().orc_mlp_priority_q(_p(w), _p(x), int(qbits), C.byref(y))
    return p, y.value


def gelu(x):
    return lib().orc_gelu(float(x))


def default_label(v, seed):
    return lib().orc_default_label(int(v), int(seed))
