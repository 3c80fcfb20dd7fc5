"""PM-LSH query path on AMD Instinct MI355X: Python binding of the C ABI.

This module only marshals arguments: every step of index construction,
(c,k)-ANN (Algorithm 2) and (c,k)-ACP (Section 6.3) runs in the HIP library
``libpmlsh.so`` (declared in ``include/pmlsh.h``). PyTorch supplies device
memory and the current HIP stream. There is no CPU fallback: a missing
library or a tensor that is not on the GPU raises.
"""

from __future__ import annotations

import ctypes
import math
import os

import numpy as np

__all__ = ["Index", "Server", "PmlshError", "plan_params", "library_path", "load_library",
           "ann_timing_enable", "ann_timing_read", "tune", "TUNE_GROUP_LIST",
           "TUNE_GROUP_MINIMA_LDS", "TUNE_FP32_PATH"]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libpmlsh.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4
EXIT_NEAR, EXIT_BUDGET = 1, 2
MAX_K = 1024


class PmlshError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"pmlsh error {code}: {message}")
        self.code = code


class _BuildArgs(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("hash", ctypes.c_void_p), ("m", ctypes.c_int32),
                ("data_on_device", ctypes.c_int32), ("num_pivots", ctypes.c_int32),
                ("leaf_size", ctypes.c_int32), ("fanout", ctypes.c_int32),
                ("filter_gemm", ctypes.c_int32), ("sample_seed", ctypes.c_uint64),
                ("r_min_kappa", ctypes.c_double), ("stream", ctypes.c_void_p)]


class _Plan(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("alpha1", ctypes.c_double),
                ("alpha2", ctypes.c_double), ("beta", ctypes.c_double),
                ("budget", ctypes.c_int64), ("acp_budget", ctypes.c_int64)]


class _AcpStats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("ub", ctypes.c_double), ("budget", ctypes.c_int64),
                ("n_seed", ctypes.c_int64), ("n_cand_raw", ctypes.c_int64),
                ("n_cand", ctypes.c_int64), ("tiles_total", ctypes.c_int64),
                ("tiles_scanned", ctypes.c_int64)]


class _Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("m", ctypes.c_int32),
                ("leaf_size", ctypes.c_int32), ("fanout", ctypes.c_int32),
                ("num_pivots", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("n_leaves", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("sample_size", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("filter_gemm", ctypes.c_int32), ("eps_max", ctypes.c_float)]


class _QueryArgs(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("reserved", ctypes.c_int32), ("c", ctypes.c_double),
                ("confidence", ctypes.c_double), ("beta", ctypes.c_double),
                ("r_min", ctypes.c_double)]


class _ServerArgs(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("hbm_budget", ctypes.c_int64)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_int64), ("queries", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("latency_p50_ms", ctypes.c_double),
                ("latency_p99_ms", ctypes.c_double), ("latency_max_ms", ctypes.c_double)]


STAGES = ("project", "tau", "filter", "finish", "per_query", "dist",
          "acp_selfjoin", "acp_select", "acp_tiles", "acp_scan", "acp_verify", "acp_topk")


class _Timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(STAGES)),
                ("launches", ctypes.c_int64 * len(STAGES))]

_LIB = None

# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "pmlsh_build": (ctypes.c_int, [ctypes.POINTER(_BuildArgs), ctypes.POINTER(ctypes.c_void_p)]),
    "pmlsh_free": (None, [ctypes.c_void_p]),
    "pmlsh_plan_params": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.POINTER(_Plan)]),
    "pmlsh_default_r_min": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_double)]),
    "pmlsh_ann": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                 ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pmlsh_ann_mixed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.POINTER(_QueryArgs), ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "pmlsh_ann_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pmlsh_bc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p]),
    "pmlsh_acp": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.POINTER(_AcpStats), ctypes.c_void_p]),
    "pmlsh_acp_bb": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.POINTER(_AcpStats), ctypes.c_void_p]),
    "pmlsh_acp_lca": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.POINTER(_AcpStats),
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "pmlsh_index_export_nodes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p]),
    "pmlsh_index_filter_projection": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                      ctypes.c_void_p]),
    "pmlsh_get_index_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Info)]),
    "pmlsh_index_export_leaves": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p]),
    "pmlsh_tune": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64]),
    "pmlsh_ann_timing_enable": (ctypes.c_int, [ctypes.c_int]),
    "pmlsh_ann_timing_read": (ctypes.c_int, [ctypes.POINTER(_Timing), ctypes.c_int]),
    "pmlsh_last_error": (ctypes.c_char_p, []),
    "pmlsh_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_ServerArgs),
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "pmlsh_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.POINTER(ctypes.c_uint64)]),
    "pmlsh_server_test": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64,
                                         ctypes.POINTER(ctypes.c_int)]),
    "pmlsh_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "pmlsh_server_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_ServerStats)]),
    "pmlsh_server_destroy": (None, [ctypes.c_void_p]),
}


def load_library():
    """Loads libpmlsh.so (built in-tree); raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(library_path):
            raise RuntimeError(
                f"{library_path} is missing: build it with "
                "`python -m paper_2107_05537_amd.build_lib`")
        lib = ctypes.CDLL(library_path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def _check(code: int):
    if code != OK:
        msg = load_library().pmlsh_last_error()
        raise PmlshError(code, msg.decode() if msg else "")


def _torch():
    import torch
    return torch


def _stream_handle(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require_gpu_f32(name, t):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    return t.contiguous()


def plan_params(n: int, m: int, k: int, c: float, confidence: float, beta: float = -1.0):
    """Parameters of Algorithm 2 / Section 6.3 as computed by the library (host only)."""
    out = _Plan()
    _check(load_library().pmlsh_plan_params(n, m, k, c, confidence, beta, ctypes.byref(out)))
    return {f: getattr(out, f) for f, _ in _Plan._fields_}


FILTER_GEMM_FP16 = 1          # filter rows from an FP16-input matrix-core projection
FILTER_GEMM_BF16 = 2          # ... from a BF16-input one

TUNE_GROUP_LIST = 0          # most 64-chunk groups the ANN bound lists per query
TUNE_GROUP_MINIMA_LDS = 1    # group minima in LDS (1) or read from HBM (0)
TUNE_FP32_PATH = 2           # 1: whole launches on the plain FP32 per-query kernel
TUNE_ACP_FIRST_CAP = 3       # first capacity of ACP's candidate and band buffers (0: defaults)
TUNE_SCAN_SHAPE = 4          # range filter block: 0 by index size, 1: 512 queries, 2: 1,024


def tune(key: int, value: int = -1):
    """Process-wide switch of the ANN bound kernel's group filter (pmlsh_tune;
    -1 restores the default). Results do not depend on it."""
    _check(load_library().pmlsh_tune(int(key), int(value)))


def ann_timing_enable(enable: bool = True, stages=None):
    """Switch the per-stage HIP-event timing of pmlsh_ann on or off; `stages`
    (names from STAGES) limits it to those stages."""
    if not enable:
        mask = 0
    elif stages is None:
        mask = (1 << len(STAGES)) - 1
    else:
        mask = 0
        for name in stages:
            mask |= 1 << STAGES.index(name)
    _check(load_library().pmlsh_ann_timing_enable(mask))


def ann_timing_read(reset: bool = True) -> dict:
    """Per-stage GPU milliseconds and launch counts since the last reset."""
    out = _Timing()
    _check(load_library().pmlsh_ann_timing_read(ctypes.byref(out), 1 if reset else 0))
    return {name: {"ms": out.ms[i], "launches": out.launches[i]}
            for i, name in enumerate(STAGES)}


class Index:
    """A PM-tree index over FP32 data, resident in HBM.

    data: (n, d) float32 torch tensor on the GPU, or a NumPy array on the host.
    hash: (m, d) float32 projection vectors (N(0,1) entries), same residency.
    """

    def __init__(self, data, hash, num_pivots: int = 5, leaf_size: int = 64,
                 fanout: int = 16, sample_seed: int = 0x5EED, r_min_kappa: float = 0.9,
                 filter_gemm: int = 0):
        lib = load_library()
        self._h = ctypes.c_void_p()
        args = _BuildArgs()
        keep = []
        if isinstance(data, np.ndarray):
            if not isinstance(hash, np.ndarray):
                raise TypeError("data and hash must both be NumPy arrays or both GPU tensors")
            D = np.ascontiguousarray(data, dtype=np.float32)
            H = np.ascontiguousarray(hash, dtype=np.float32)
            keep += [D, H]
            args.data, args.hash = D.ctypes.data, H.ctypes.data
            args.data_on_device = 0
            self.device = None
            stream = None
        else:
            D = _require_gpu_f32("data", data)
            H = _require_gpu_f32("hash", hash)
            if H.device != D.device:
                raise ValueError("data and hash must be on the same device")
            keep += [D, H]
            args.data, args.hash = D.data_ptr(), H.data_ptr()
            args.data_on_device = 1
            self.device = D.device
            stream = _stream_handle(D.device)
        if D.ndim != 2 or H.ndim != 2 or H.shape[1] != D.shape[1]:
            raise ValueError("data must be (n, d) and hash (m, d)")
        args.n, args.d = D.shape[0], D.shape[1]
        args.m = H.shape[0]
        args.num_pivots, args.leaf_size, args.fanout = num_pivots, leaf_size, fanout
        args.sample_seed = sample_seed
        args.r_min_kappa = r_min_kappa
        args.filter_gemm = filter_gemm
        args.stream = stream
        _check(lib.pmlsh_build(ctypes.byref(args), ctypes.byref(self._h)))
        if self.device is None:
            self.device = _torch().device("cuda", _torch().cuda.current_device())
        info = self.info()
        self.n, self.d, self.m = info["n"], info["d"], info["m"]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.pmlsh_free(h)
            self._h = None

    def info(self) -> dict:
        out = _Info()
        _check(load_library().pmlsh_get_index_info(self._h, ctypes.byref(out)))
        return {f: getattr(out, f) for f, _ in _Info._fields_}

    def filter_projection(self):
        """Low-precision projection behind the filter rows of an index built
        with filter_gemm != 0, recomputed in id order: (proj (n, m), eps (n,))
        float32 NumPy arrays, eps bounding each row's distance to the exact
        projection."""
        proj = np.empty((self.n, self.m), dtype=np.float32)
        eps = np.empty(self.n, dtype=np.float32)
        _check(load_library().pmlsh_index_filter_projection(self._h, proj.ctypes.data,
                                                            eps.ctypes.data))
        return proj, eps

    def default_r_min(self, budget: int) -> float:
        v = ctypes.c_double()
        _check(load_library().pmlsh_default_r_min(self._h, budget, ctypes.byref(v)))
        return v.value

    def export_leaves(self):
        """Leaf partition: leaf b holds ids perm[offsets[b]:offsets[b+1]]."""
        info = self.info()
        perm = np.empty(info["n"], dtype=np.int32)
        offsets = np.empty(info["n_leaves"] + 1, dtype=np.int64)
        _check(load_library().pmlsh_index_export_leaves(self._h, perm.ctypes.data,
                                                        offsets.ctypes.data))
        return perm, offsets

    def ann(self, queries, k: int, c: float = 1.5, confidence: float = 1 - 1 / math.e,
            beta: float = -1.0, r_min: float = 0.0, stats: bool = False):
        """(c,k)-ANN for every row of `queries` ((nq, d) float32 on the GPU).

        Returns (ids int64 (nq,k), dist float32 (nq,k)) and, with stats=True,
        an int32 (nq, 4) tensor: rounds, |C|, exit kind, points scanned.
        Enqueued on the current stream (results valid after it completes).
        """
        torch = _torch()
        Q = _require_gpu_f32("queries", queries)
        if Q.ndim != 2 or Q.shape[1] != self.d:
            raise ValueError(f"queries must be (nq, {self.d})")
        nq = Q.shape[0]
        ids = torch.empty((nq, k), dtype=torch.int64, device=Q.device)
        dist = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
        st = torch.empty((nq, 4), dtype=torch.int32, device=Q.device) if stats else None
        _check(load_library().pmlsh_ann(
            self._h, Q.data_ptr(), nq, k, c, confidence, beta, r_min, ids.data_ptr(),
            dist.data_ptr(), st.data_ptr() if st is not None else None,
            _stream_handle(Q.device)))
        return (ids, dist, st) if stats else (ids, dist)

    def ann_into(self, queries, k, c, confidence, beta, r_min, ids, dist, stats=None):
        """Like ann() but writes into caller-provided GPU tensors (no allocation)."""
        _check(load_library().pmlsh_ann(
            self._h, queries.data_ptr(), queries.shape[0], k, c, confidence, beta, r_min,
            ids.data_ptr(), dist.data_ptr(), stats.data_ptr() if stats is not None else None,
            _stream_handle(queries.device)))

    def ann_mixed(self, queries, params, out_stride: int = 0, stats: bool = False):
        """(c,k)-ANN with per-query parameters: params is a list of dicts (one
        per row of `queries`) with keys k and optionally c (1.5), confidence
        (1 - 1/e), beta (-1) and r_min (0). Returns ids int64 and dist float32
        tensors of shape (nq, out_stride) (out_stride 0: the largest k); row i
        holds query i's answer in its first k entries. Enqueued on the current
        stream."""
        torch = _torch()
        Q = _require_gpu_f32("queries", queries)
        if Q.ndim != 2 or Q.shape[1] != self.d:
            raise ValueError(f"queries must be (nq, {self.d})")
        nq = Q.shape[0]
        if len(params) != nq:
            raise ValueError("one parameter set per query")
        arr = (_QueryArgs * max(1, nq))()
        for i, p in enumerate(params):
            arr[i] = _QueryArgs(int(p["k"]), 0, float(p.get("c", 1.5)),
                                float(p.get("confidence", 1 - 1 / math.e)),
                                float(p.get("beta", -1.0)), float(p.get("r_min", 0.0)))
        stride = out_stride if out_stride > 0 else max([int(p["k"]) for p in params] or [1])
        ids = torch.full((nq, stride), -1, dtype=torch.int64, device=Q.device)
        dist = torch.full((nq, stride), float("inf"), dtype=torch.float32, device=Q.device)
        st = torch.empty((nq, 4), dtype=torch.int32, device=Q.device) if stats else None
        _check(load_library().pmlsh_ann_mixed(
            self._h, Q.data_ptr(), nq, arr, stride, ids.data_ptr(), dist.data_ptr(),
            st.data_ptr() if st is not None else None, _stream_handle(Q.device)))
        return (ids, dist, st) if stats else (ids, dist)

    def ann_noalloc(self, queries, k, c, confidence, beta, r_min, ids, dist, stats=None):
        """pmlsh_ann_noalloc into caller-provided GPU tensors: the workspace is
        the library's fixed per-device array (calls overlapping on one device
        race). Enqueued on the current stream."""
        _check(load_library().pmlsh_ann_noalloc(
            self._h, queries.data_ptr(), queries.shape[0], k, c, confidence, beta, r_min,
            ids.data_ptr(), dist.data_ptr(), stats.data_ptr() if stats is not None else None,
            _stream_handle(queries.device)))

    def bc(self, queries, r: float, c: float = 1.5, confidence: float = 1 - 1 / math.e,
           beta: float = -1.0, stats: bool = False):
        """(r,c)-BC query (Algorithm 1) for every row of `queries`.

        Returns (ids int64 (nq,), dist float32 (nq,)): the point found, or -1
        and +inf for nothing; with stats=True also the int32 (nq, 4) stats.
        Enqueued on the current stream."""
        torch = _torch()
        Q = _require_gpu_f32("queries", queries)
        if Q.ndim != 2 or Q.shape[1] != self.d:
            raise ValueError(f"queries must be (nq, {self.d})")
        nq = Q.shape[0]
        ids = torch.empty((nq,), dtype=torch.int64, device=Q.device)
        dist = torch.empty((nq,), dtype=torch.float32, device=Q.device)
        st = torch.empty((nq, 4), dtype=torch.int32, device=Q.device) if stats else None
        _check(load_library().pmlsh_bc(
            self._h, Q.data_ptr(), nq, r, c, confidence, beta, ids.data_ptr(), dist.data_ptr(),
            st.data_ptr() if st is not None else None, _stream_handle(Q.device)))
        return (ids, dist, st) if stats else (ids, dist)

    def acp(self, k: int, c: float = 1.5, confidence: float = 1 - 1 / math.e,
            beta: float = -1.0):
        """(c,k)-ACP. Returns (pairs int64 (k,2) with i<j, dist float32 (k,), stats dict)."""
        torch = _torch()
        pairs = torch.empty((k, 2), dtype=torch.int64, device=self.device)
        dist = torch.empty((k,), dtype=torch.float32, device=self.device)
        st = _AcpStats()
        _check(load_library().pmlsh_acp(self._h, k, c, confidence, beta, pairs.data_ptr(),
                                        dist.data_ptr(), ctypes.byref(st),
                                        _stream_handle(self.device)))
        return pairs, dist, {f: getattr(st, f) for f, _ in _AcpStats._fields_}

    def acp_lca(self, k: int, c: float = 1.5, confidence: float = 1 - 1 / math.e,
                beta: float = -1.0, gamma: float = 0.0):
        """(c,k)-ACP by radius filtering with FindLCA (Algorithms 4-5); gamma <= 0
        estimates it (Pr(gamma) = 0.85). Returns (pairs, dist, stats dict with
        the gamma applied under "gamma")."""
        torch = _torch()
        pairs = torch.empty((k, 2), dtype=torch.int64, device=self.device)
        dist = torch.empty((k,), dtype=torch.float32, device=self.device)
        st = _AcpStats()
        g = ctypes.c_double(0.0)
        _check(load_library().pmlsh_acp_lca(self._h, k, c, confidence, beta, gamma,
                                            pairs.data_ptr(), dist.data_ptr(), ctypes.byref(st),
                                            ctypes.byref(g), _stream_handle(self.device)))
        out = {f: getattr(st, f) for f, _ in _AcpStats._fields_}
        out["gamma"] = g.value
        return pairs, dist, out

    def export_nodes(self):
        """Node structure (level, first_leaf, end_leaf, radius), NumPy arrays."""
        nn = self.info()["n_nodes"]
        level = np.empty(nn, dtype=np.int32)
        lf = np.empty(nn, dtype=np.int32)
        le = np.empty(nn, dtype=np.int32)
        rad = np.empty(nn, dtype=np.float32)
        _check(load_library().pmlsh_index_export_nodes(
            self._h, level.ctypes.data, lf.ctypes.data, le.ctypes.data, rad.ctypes.data))
        return {"level": level, "first_leaf": lf, "end_leaf": le, "radius": rad}

    def acp_bb(self, k: int, c: float = 1.5, confidence: float = 1 - 1 / math.e,
               beta: float = -1.0):
        """(c,k)-ACP by branch and bound (Algorithm 3): the T projected-nearest
        pairs are verified. Returns (pairs, dist, stats dict) like acp()."""
        torch = _torch()
        pairs = torch.empty((k, 2), dtype=torch.int64, device=self.device)
        dist = torch.empty((k,), dtype=torch.float32, device=self.device)
        st = _AcpStats()
        _check(load_library().pmlsh_acp_bb(self._h, k, c, confidence, beta, pairs.data_ptr(),
                                           dist.data_ptr(), ctypes.byref(st),
                                           _stream_handle(self.device)))
        return pairs, dist, {f: getattr(st, f) for f, _ in _AcpStats._fields_}


class Request:
    """One submitted request of a Server; holds its tensors until it completes."""

    def __init__(self, server, ticket, queries, ids, dist):
        self._server, self.ticket = server, ticket
        self._queries, self.ids, self.dist = queries, ids, dist
        self._done = False

    def done(self) -> bool:
        if self._done:
            return True
        flag = ctypes.c_int(0)
        _check(load_library().pmlsh_server_test(self._server._h, self.ticket,
                                                 ctypes.byref(flag)))
        return bool(flag.value)

    def wait(self):
        """Blocks until the answers are written; returns (ids, dist)."""
        if not self._done:
            # the GIL is released by ctypes during the call
            code = load_library().pmlsh_server_wait(self._server._h, self.ticket)
            self._done = True
            self._queries = None
            _check(code)
        return self.ids, self.dist


class Server:
    """Serving loop over a resident index (continuous batching, see
    pmlsh_server_create in include/pmlsh.h). submit() may be called from
    several threads; each request's answer equals Index.ann on its own."""

    def __init__(self, index: "Index", max_batch: int = 1024, max_inflight: int = 2,
                 hbm_budget: int = 0):
        self.index = index
        args = _ServerArgs(max_batch, max_inflight, hbm_budget)
        self._h = ctypes.c_void_p()
        _check(load_library().pmlsh_server_create(index._h, ctypes.byref(args),
                                                  ctypes.byref(self._h)))

    def submit(self, queries, k: int, c: float = 1.5, confidence: float = 1 - 1 / math.e,
               beta: float = -1.0, r_min: float = 0.0, out=None) -> Request:
        """Queues a request; `out` = (ids int64 (nq, k), dist float32 (nq, k)),
        contiguous on the queries' device, receives the answers (allocated
        here when None)."""
        torch = _torch()
        Q = _require_gpu_f32("queries", queries)
        if Q.ndim != 2 or Q.shape[1] != self.index.d:
            raise ValueError(f"queries must be (nq, {self.index.d})")
        nq = Q.shape[0]
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int64, device=Q.device)
            dist = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
        else:
            ids, dist = out
            for name, t, dt in (("ids", ids, torch.int64), ("dist", dist, torch.float32)):
                if (t.dtype != dt or t.device != Q.device or tuple(t.shape) != (nq, k)
                        or not t.is_contiguous()):
                    raise ValueError(f"out {name} must be a contiguous ({nq}, {k}) {dt} "
                                     f"tensor on {Q.device}")
        ticket = ctypes.c_uint64(0)
        _check(load_library().pmlsh_server_submit(
            self._h, Q.data_ptr(), nq, k, c, confidence, beta, r_min, ids.data_ptr(),
            dist.data_ptr(), _stream_handle(Q.device), ctypes.byref(ticket)))
        return Request(self, ticket.value, Q, ids, dist)

    def stats(self) -> dict:
        st = _ServerStats()
        _check(load_library().pmlsh_server_get_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_}

    def close(self):
        """Completes every submitted request and stops the server."""
        h = getattr(self, "_h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.pmlsh_server_destroy(h)
            self._h = None

    def __del__(self):
        self.close()
