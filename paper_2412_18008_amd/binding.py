"""ctypes binding of the C ABI in ``include/spoch.h``.

Argument marshalling only: every step of the construction and of the
queries runs in the HIP kernels of ``libspoch.so``.  Inputs may be numpy
arrays (host) or torch CUDA tensors (device; passed by pointer with the
device flag).  The library must be built (``paper_2412_18008_amd.build``);
loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspoch.so")

CH_OK = 0
CH_E_INVALID = -1
CH_E_OOM = -2
CH_E_OVERFLOW = -3
CH_E_DEVICE = -4
CH_E_LIMIT = -5
CH_E_UNSUPPORTED = -6

CH_WPS_EXACT = 0
CH_WPS_HOP = 1
CH_WPS_SETTLED = 2
CH_F_INPUT_ON_DEVICE = 0x1
CH_F_STATS = 0x2
CH_F_NO_QUERY_INDEX = 0x4
CH_Q_ON_DEVICE = 0x1
CH_Q_FULL_CLOSURE = 1 << 20
CH_Q_COUNT = 1 << 21
CH_Q_NO_CORE = 1 << 26

EXPORTED = ("ch_build", "ch_build_batch", "ch_query_batch", "ch_export", "ch_get_summary",
            "ch_get_round_stats", "ch_free", "ch_last_error", "ch_version", "ch_export_features",
            "ch_mlp_forward", "ch_mlp_grad", "ch_mlp_train", "ch_query_batch_stats",
            "ch_query_batch_noalloc", "ch_get_query_stats", "ch_one_to_all")


class ChError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Graph(C.Structure):
    _fields_ = [("n", C.c_uint32), ("m", C.c_uint64), ("offsets", C.c_void_p),
                ("dst", C.c_void_p), ("w", C.c_void_p), ("labels", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("wps_mode", C.c_uint32), ("max_rounds", C.c_uint32), ("seed", C.c_uint64),
                ("flags", C.c_uint32), ("group", C.c_uint32), ("stream", C.c_void_p),
                ("ls_sparse", C.c_uint32), ("ls_dense", C.c_uint32),
                ("dense_deg10", C.c_uint32), ("priority", C.c_uint32), ("mlp", C.c_void_p),
                ("hop_limit", C.c_uint32), ("dense_tail", C.c_uint32),
                ("k_ed", C.c_int32), ("k_cn", C.c_int32), ("k_depth", C.c_int32),
                ("tiebreak", C.c_uint32), ("settle_limit", C.c_uint32),
                ("ls_step", C.c_uint32), ("mlp_qbits", C.c_uint32)]


CH_PRIO_PLAIN, CH_PRIO_LEARNED = 0, 1
CH_MLP_PARAMS = 4801
CH_F_RECORD_FEATURES = 0x8
CH_F_TAIL_STEPWISE = 0x10
CH_F_KEEP_ORDER = 0x20
CH_F_SCORE_WEIGHTS = 0x40
CH_F_PROGRESS = 0x80
CH_F_NO_GRAPH = 0x100
CH_TIE_HASHED_ID, CH_TIE_RAW_ID = 0, 1
CH_MLP_ON_DEVICE, CH_MLP_BF16 = 0x1, 0x2


def CH_Q_FIRST_TIER(t):
    """Query flag: the tier a batch starts in (1, 2, 3; 0 = chosen by the library)."""
    return int(t) << 22


def CH_Q_WAVES(nw):
    """Query flag: waves that share one query (1, 2, 4, 8; 0 = default)."""
    if nw not in (0, 1, 2, 4, 8):
        raise ValueError("waves must be 0, 1, 2, 4 or 8")
    return nw << 8


def CH_Q_LEVEL_WINDOW(w):
    """Query flag: level window of a search step (1 .. 254; 0 = default,
    255 = none)."""
    if not 0 <= w <= 255:
        raise ValueError("window must be in 0 .. 255")
    return w << 12


class MlpTrainParams(C.Structure):
    _fields_ = [("batch", C.c_uint32), ("steps", C.c_uint32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("seed", C.c_uint64)]


CH_LS_AUTO, CH_LS_16x128, CH_LS_32x512, CH_LS_64x512, CH_LS_64x2048 = 0, 1, 2, 3, 4
CH_LS_TABLE, CH_LS_TAIL = 5, 6
LS_KERNELS = {1: "k_local_search<16, 128>", 2: "k_local_search<32, 512>",
              3: "k_local_search<64, 512>", 4: "k_local_search<64, 2048>",
              5: "k_ls_table", 6: "k_tail_search"}
CH_DENSE_TAIL_OFF = 1


class RoundStats(C.Structure):
    _fields_ = [
        ("alive_before", C.c_uint32), ("n_sources", C.c_uint32), ("n_affected", C.c_uint32),
        ("n_selected", C.c_uint32), ("n_targets", C.c_uint64), ("n_pruned", C.c_uint64),
        ("n_shortcuts", C.c_uint64), ("overlay_arcs", C.c_uint64),
        ("rows_expanded", C.c_uint64), ("arcs_scanned", C.c_uint64),
        ("memo_probes", C.c_uint64), ("memo_inserts", C.c_uint64),
        ("n_ls_fallback", C.c_uint32), ("ls_tier1", C.c_uint32), ("ms_local_search", C.c_float),
        ("ms_total", C.c_float), ("n_ls_global", C.c_uint32),
        ("ms_ls_blk", C.c_float), ("ms_ls_global", C.c_float),
        ("rows2", C.c_uint64), ("arcs2", C.c_uint64), ("probes2", C.c_uint64),
        ("inserts2", C.c_uint64), ("rows3", C.c_uint64), ("arcs3", C.c_uint64),
        ("probes3", C.c_uint64), ("inserts3", C.c_uint64),
    ]


class QueryStats(C.Structure):
    _fields_ = [("queries", C.c_uint64), ("first_tier", C.c_uint32), ("counted", C.c_uint32),
                ("tier_queries", C.c_uint64 * 4), ("tier_ms", C.c_float * 4),
                ("rows", C.c_uint64), ("arcs", C.c_uint64)]


class Summary(C.Structure):
    _fields_ = [("n", C.c_uint32), ("rounds", C.c_uint32), ("m_input", C.c_uint64),
                ("up_arcs", C.c_uint64), ("down_arcs", C.c_uint64), ("shortcuts", C.c_uint64),
                ("memo_entries", C.c_uint64), ("ms_build", C.c_double)]


_lib = None


def lib():
    """Load libspoch.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run python -m paper_2412_18008_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
        L.ch_build.argtypes = [C.POINTER(Graph), C.POINTER(Params), C.POINTER(vp)]
        L.ch_build.restype = i32
        L.ch_build_batch.argtypes = [C.POINTER(Graph), u32, C.POINTER(Params), C.POINTER(vp)]
        L.ch_build_batch.restype = i32
        L.ch_query_batch.argtypes = [vp, vp, vp, u64, vp, u32, vp]
        L.ch_query_batch.restype = i32
        L.ch_export.argtypes = [vp] + [vp] * 11
        L.ch_export.restype = i32
        L.ch_get_summary.argtypes = [vp, C.POINTER(Summary)]
        L.ch_get_summary.restype = i32
        L.ch_get_round_stats.argtypes = [vp, vp, u32]
        L.ch_get_round_stats.restype = i32
        L.ch_free.argtypes = [vp]
        L.ch_free.restype = None
        L.ch_last_error.argtypes = []
        L.ch_last_error.restype = C.c_char_p
        L.ch_version.argtypes = []
        L.ch_version.restype = C.c_char_p
        L.ch_query_batch_stats.argtypes = [vp, vp, vp, u64, vp, vp, u32, vp]
        L.ch_query_batch_stats.restype = i32
        L.ch_query_batch_noalloc.argtypes = [vp, vp, vp, u64, vp, vp, u32, vp]
        L.ch_query_batch_noalloc.restype = i32
        L.ch_get_query_stats.argtypes = [vp, C.POINTER(QueryStats)]
        L.ch_get_query_stats.restype = i32
        L.ch_one_to_all.argtypes = [vp, vp, u32, vp, u32, vp, u32, vp]
        L.ch_one_to_all.restype = i32
        L.ch_export_features.argtypes = [vp, vp]
        L.ch_export_features.restype = i32
        L.ch_mlp_forward.argtypes = [vp, u64, vp, vp, vp, u32, vp]
        L.ch_mlp_forward.restype = i32
        L.ch_mlp_grad.argtypes = [vp, vp, u32, vp, vp, vp, u32, vp]
        L.ch_mlp_grad.restype = i32
        L.ch_mlp_train.argtypes = [vp, vp, u64, vp, C.POINTER(MlpTrainParams), vp, u32, vp]
        L.ch_mlp_train.restype = i32
        _lib = L
    return _lib


def _check(rc, what):
    if rc != CH_OK:
        msg = lib().ch_last_error().decode()
        raise ChError(rc, f"{what}: {msg}")


def _is_torch_cuda(a):
    return hasattr(a, "is_cuda") and a.is_cuda


def _ptr(a, dtype):
    """Pointer of a numpy array (converted to dtype) or of a CUDA tensor."""
    if a is None:
        return None, None
    if _is_torch_cuda(a):
        return a.data_ptr(), a
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data, arr


class CH:
    """A contraction hierarchy built on the GPU (owns a ch_t)."""

    def __init__(self, handle):
        self.h = handle
        s = Summary()
        _check(lib().ch_get_summary(self.h, C.byref(s)), "ch_get_summary")
        self.summary = {f: getattr(s, f) for f, _ in Summary._fields_}
        self.n = self.summary["n"]

    def __del__(self):
        self.free()

    def free(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ch_free(self.h)
            self.h = None

    def query(self, s, t, stream=None, waves=0, window=0, full=False, count=False, tier=0,
              core=True):
        """dist[i] = shortest s[i] -> t[i] distance (uint64, max = unreachable).
        numpy inputs give a numpy result; torch CUDA inputs give a torch CUDA
        int64 tensor (holding the uint64 bit patterns).  waves: waves per
        query in the kernel (1, 2, 4, 8; 0 = default); window: level window of
        a search step (0 = default, 255 = none); full: expand both upward
        search spaces completely (no pruning by the best path met); count:
        count expansions and relaxed arcs (last_query_stats); tier: the tier
        the batch starts in (1, 2, 3; 0 = chosen by the library); core: the
        first and second tiers finish at their core tables (the same
        distances)."""
        if tier not in (0, 1, 2, 3):
            raise ValueError("tier must be 0, 1, 2 or 3")
        qf = CH_Q_WAVES(waves) | CH_Q_LEVEL_WINDOW(window) | (CH_Q_FULL_CLOSURE if full else 0) | (
            CH_Q_COUNT if count else 0) | CH_Q_FIRST_TIER(tier) | (0 if core else CH_Q_NO_CORE)
        if _is_torch_cuda(s):
            import torch

            q = s.numel()
            dist = torch.empty(q, dtype=torch.int64, device=s.device)
            st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
            _check(lib().ch_query_batch(self.h, s.data_ptr(), t.data_ptr(), q, dist.data_ptr(),
                                        CH_Q_ON_DEVICE | qf, st), "ch_query_batch")
            return dist
        s = np.ascontiguousarray(s, np.uint32)
        t = np.ascontiguousarray(t, np.uint32)
        dist = np.empty(len(s), np.uint64)
        _check(lib().ch_query_batch(self.h, s.ctypes.data, t.ctypes.data, len(s),
                                    dist.ctypes.data, qf, stream), "ch_query_batch")
        return dist

    def query_stats(self, s, t, waves=0, window=0):
        """(dist, visited): distances and vertices in the two upward search
        spaces of each query (numpy, host)."""
        s = np.ascontiguousarray(s, np.uint32)
        t = np.ascontiguousarray(t, np.uint32)
        dist = np.empty(len(s), np.uint64)
        vis = np.empty(len(s), np.uint32)
        _check(lib().ch_query_batch_stats(self.h, s.ctypes.data, t.ctypes.data, len(s),
                                          dist.ctypes.data, vis.ctypes.data,
                                          CH_Q_WAVES(waves) | CH_Q_LEVEL_WINDOW(window),
                                          None),
               "ch_query_batch_stats")
        return dist, vis

    def one_to_all(self, s, t=None, stream=None):
        """Distances from each source in s to every vertex (rows of n), or to
        the targets t (rows of len(t)): numpy uint64 (host arrays), or a CUDA
        int64 tensor of uint64 bit patterns for CUDA inputs."""
        if _is_torch_cuda(s):
            import torch

            ks = s.numel()
            kt = t.numel() if t is not None else 0
            out = torch.empty(ks * (kt if t is not None else self.n), dtype=torch.int64,
                              device=s.device)
            st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
            _check(lib().ch_one_to_all(self.h, s.data_ptr(), ks,
                                       t.data_ptr() if t is not None else None, kt,
                                       out.data_ptr(), CH_Q_ON_DEVICE, st), "ch_one_to_all")
            return out.view(ks, -1)
        s = np.ascontiguousarray(s, np.uint32)
        tt = None if t is None else np.ascontiguousarray(t, np.uint32)
        nt = self.n if tt is None else len(tt)
        out = np.empty((len(s), nt), np.uint64)
        _check(lib().ch_one_to_all(self.h, s.ctypes.data, len(s),
                                   None if tt is None else tt.ctypes.data,
                                   0 if tt is None else len(tt), out.ctypes.data, 0, stream),
               "ch_one_to_all")
        return out

    def last_query_stats(self):
        """Counters and per-tier device times of the last query batch."""
        qs = QueryStats()
        _check(lib().ch_get_query_stats(self.h, C.byref(qs)), "ch_get_query_stats")
        return {"queries": qs.queries, "first_tier": qs.first_tier, "counted": bool(qs.counted),
                "tier_queries": list(qs.tier_queries), "tier_ms": list(qs.tier_ms),
                "rows": qs.rows, "arcs": qs.arcs}

    def query_noalloc(self, s, t, visited=True, stream=None, waves=0, window=0):
        """ch_query_batch_noalloc on torch CUDA uint32 tensors s, t: (dist,
        visited or None) as CUDA int64 / int32 tensors, after the call has
        finished."""
        import torch

        q = s.numel()
        dist = torch.empty(q, dtype=torch.int64, device=s.device)
        vis = torch.empty(q, dtype=torch.int32, device=s.device) if visited else None
        st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        _check(lib().ch_query_batch_noalloc(
            self.h, s.data_ptr(), t.data_ptr(), q, dist.data_ptr(),
            vis.data_ptr() if vis is not None else None,
            CH_Q_ON_DEVICE | CH_Q_WAVES(waves) | CH_Q_LEVEL_WINDOW(window), st),
            "ch_query_batch_noalloc")
        return dist, vis

    def export(self):
        n, nu, nd = self.n, self.summary["up_arcs"], self.summary["down_arcs"]
        out = dict(level=np.empty(n, np.uint32), score=np.empty(n, np.int32),
                   rank=np.empty(n, np.uint32))
        for k in ("up_tail", "up_head", "up_w", "up_mid"):
            out[k] = np.empty(nu, np.uint32)
        for k in ("down_tail", "down_head", "down_w", "down_mid"):
            out[k] = np.empty(nd, np.uint32)
        order = ("level", "score", "rank", "up_tail", "up_head", "up_w", "up_mid",
                 "down_tail", "down_head", "down_w", "down_mid")
        _check(lib().ch_export(self.h, *[out[k].ctypes.data for k in order]), "ch_export")
        return out

    def features(self):
        """Features (n x 8 float32) each vertex had when it was contracted."""
        x = np.empty((self.n, 8), np.float32)
        _check(lib().ch_export_features(self.h, x.ctypes.data), "ch_export_features")
        return x

    def round_stats(self):
        k = self.summary["rounds"]
        arr = (RoundStats * max(k, 1))()
        _check(lib().ch_get_round_stats(self.h, C.cast(arr, C.c_void_p), k),
               "ch_get_round_stats")
        return [{f: getattr(arr[i], f) for f, _ in RoundStats._fields_} for i in range(k)]


def build(off, dst, w, labels=None, seed=0, stats=False, group=0, max_rounds=0,
          query_index=True, stream=None, ls_sparse=0, ls_dense=0, dense_deg10=0, mlp=None,
          record=False, hop=0, dense_tail=0, tail_stepwise=False, keep_order=False,
          score_weights=None, raw_id=False, settle=0, ls_step=0, mlp_qbits=0, progress=False,
          graph=True):
    """ch_build on a CSR graph; numpy arrays or torch CUDA tensors.  hop > 0
    selects the hop-bounded witness search with walks of at most `hop` arcs;
    tail_stepwise runs the table rounds one launch per step; keep_order
    builds on the input's numbering (no locality renumbering); score_weights
    = (k_ed, k_cn, k_depth) sets the integer score weights; raw_id labels
    every vertex by its id; settle > 0 selects the settled(theta) witness
    search with theta = settle; ls_step: distance-bucket width D_s >> ls_step
    of exact-mode search steps (0 = default, 32 = whole frontier); mlp_qbits:
    fractional bits of the learned priority (0 = 16)."""
    dev = _is_torch_cuda(off)
    po, ko = _ptr(off, np.uint64)
    pd, kd = _ptr(dst, np.uint32)
    pw, kw = _ptr(w, np.uint32)
    pl, kl = _ptr(labels, np.uint32)
    n = (off.numel() if dev else len(ko)) - 1
    m = dst.numel() if dev else len(kd)
    g = Graph(n, m, po, pd, pw, pl)
    flags = (CH_F_INPUT_ON_DEVICE if dev else 0) | (CH_F_STATS if stats else 0) | (
        0 if query_index else CH_F_NO_QUERY_INDEX) | (CH_F_RECORD_FEATURES if record else 0) | (
        CH_F_TAIL_STEPWISE if tail_stepwise else 0) | (CH_F_KEEP_ORDER if keep_order else 0) | (
        CH_F_SCORE_WEIGHTS if score_weights is not None else 0) | (
        CH_F_PROGRESS if progress else 0) | (0 if graph else CH_F_NO_GRAPH)
    k_ed, k_cn, k_depth = score_weights if score_weights is not None else (1, 0, 0)
    if stream is None and dev:
        import torch

        stream = torch.cuda.current_stream().cuda_stream
    wts = None if mlp is None else np.ascontiguousarray(mlp, np.float32)
    if wts is not None and wts.size != CH_MLP_PARAMS:
        raise ValueError("mlp must hold 4801 weights")
    mode = CH_WPS_SETTLED if settle else (CH_WPS_HOP if hop else CH_WPS_EXACT)
    p = Params(mode, max_rounds, seed, flags, group, stream,
               ls_sparse, ls_dense, dense_deg10,
               CH_PRIO_LEARNED if wts is not None else CH_PRIO_PLAIN,
               None if wts is None else wts.ctypes.data, hop, dense_tail, k_ed, k_cn, k_depth,
               CH_TIE_RAW_ID if raw_id else CH_TIE_HASHED_ID, settle, ls_step, mlp_qbits)
    h = C.c_void_p()
    _check(lib().ch_build(C.byref(g), C.byref(p), C.byref(h)), "ch_build")
    return CH(h)


def build_batch(graphs, labels=None, seed=0, group=0, max_rounds=0, query_index=True,
                stream=None, hop=0, dense_tail=0, score_weights=None, raw_id=False, settle=0):
    """ch_build_batch on a list of (off, dst, w) CSR graphs (numpy arrays or
    torch CUDA tensors); returns one CH per graph."""
    k = len(graphs)
    keep = []
    arr = (Graph * max(k, 1))()
    dev = k > 0 and _is_torch_cuda(graphs[0][0])
    for i, (off, dst, w) in enumerate(graphs):
        po, ko = _ptr(off, np.uint64)
        pd, kd = _ptr(dst, np.uint32)
        pw, kw = _ptr(w, np.uint32)
        pl, kl = _ptr(None if labels is None else labels[i], np.uint32)
        keep += [ko, kd, kw, kl]
        n = (off.numel() if dev else len(ko)) - 1
        m = dst.numel() if dev else len(kd)
        arr[i] = Graph(n, m, po, pd, pw, pl)
    flags = (CH_F_INPUT_ON_DEVICE if dev else 0) | (0 if query_index else CH_F_NO_QUERY_INDEX) | (
        CH_F_SCORE_WEIGHTS if score_weights is not None else 0)
    k_ed, k_cn, k_depth = score_weights if score_weights is not None else (1, 0, 0)
    mode = CH_WPS_SETTLED if settle else (CH_WPS_HOP if hop else CH_WPS_EXACT)
    p = Params(mode, max_rounds, seed, flags, group, stream,
               0, 0, 0, CH_PRIO_PLAIN, None, hop, dense_tail, k_ed, k_cn, k_depth,
               CH_TIE_RAW_ID if raw_id else CH_TIE_HASHED_ID, settle)
    outs = (C.c_void_p * max(k, 1))()
    _check(lib().ch_build_batch(arr, k, C.byref(p), outs), "ch_build_batch")
    return [CH(C.c_void_p(outs[i])) for i in range(k)]


def mlp_forward(x, w, bf16=False, stream=None):
    """(y, priority) of the learned priority's network on n x 8 features.
    x and w as numpy (host) or as float32 CUDA tensors (device; the results
    are then device tensors and the call is asynchronous on ``stream``)."""
    if _is_torch_cuda(x):
        import torch

        n = x.numel() // 8
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        y = torch.empty(n, dtype=torch.float32, device=x.device)
        p = torch.empty(n, dtype=torch.int32, device=x.device)
        flags = CH_MLP_ON_DEVICE | (CH_MLP_BF16 if bf16 else 0)
        _check(lib().ch_mlp_forward(x.data_ptr(), n, w.data_ptr(), y.data_ptr(), p.data_ptr(),
                                    flags, stream), "ch_mlp_forward")
        return y, p
    x = np.ascontiguousarray(x, np.float32).reshape(-1, 8)
    w = np.ascontiguousarray(w, np.float32)
    y = np.empty(len(x), np.float32)
    p = np.empty(len(x), np.int32)
    _check(lib().ch_mlp_forward(x.ctypes.data, len(x), w.ctypes.data, y.ctypes.data,
                                p.ctypes.data, CH_MLP_BF16 if bf16 else 0, None), "ch_mlp_forward")
    return y, p


def mlp_grad(x, t, w, bf16=False):
    """(gradient, loss) of the mean squared error over all samples (bf16:
    on the matrix cores with bf16 operands)."""
    x = np.ascontiguousarray(x, np.float32).reshape(-1, 8)
    t = np.ascontiguousarray(t, np.float32)
    w = np.ascontiguousarray(w, np.float32)
    g = np.empty(CH_MLP_PARAMS, np.float32)
    loss = C.c_float()
    _check(lib().ch_mlp_grad(x.ctypes.data, t.ctypes.data, len(x), w.ctypes.data, g.ctypes.data,
                             C.byref(loss), CH_MLP_BF16 if bf16 else 0, None), "ch_mlp_grad")
    return g, loss.value


def mlp_train(x, t, w, batch=1024, steps=500, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0,
              bf16=False):
    """Adam on the GPU; returns (trained weights, per-step batch losses);
    bf16: gradients on the matrix cores with bf16 operands."""
    x = np.ascontiguousarray(x, np.float32).reshape(-1, 8)
    t = np.ascontiguousarray(t, np.float32)
    w = np.array(w, np.float32, copy=True)
    losses = np.empty(steps, np.float32)
    p = MlpTrainParams(batch, steps, lr, beta1, beta2, eps, seed)
    _check(lib().ch_mlp_train(x.ctypes.data, t.ctypes.data, len(x), w.ctypes.data, C.byref(p),
                              losses.ctypes.data, CH_MLP_BF16 if bf16 else 0, None),
           "ch_mlp_train")
    return w, losses


def version():
    return lib().ch_version().decode()
