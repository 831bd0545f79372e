"""MI355X robust-spanner (RS) scoring: Python binding of the C ABI in include/rs.h.

Argument marshalling only: every step of the scoring pass runs in the HIP
kernels of ``librs.so``.  The functions keep the C names.  Arrays may be numpy
(host) or torch tensors (host or HIP device; device tensors are passed as
device pointers).  If ``librs.so`` has not been built this package raises on
import -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

try:
    # torch ships its own HIP runtime.  Importing it first makes librs.so bind
    # to that same runtime instead of loading a second copy, so one process
    # has one HIP runtime and torch streams / device pointers are valid here.
    import torch  # noqa: F401
except ImportError:  # the library itself does not need torch
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librs.so")

RS_OK, RS_ERR_ARG, RS_ERR_GRAPH, RS_ERR_RANGE, RS_ERR_NOMEM, RS_ERR_HIP, RS_ERR_STATE = range(7)
RS_LOAD_WIDE_OFFSETS = 1  # 64-bit device edge offsets even when nnz fits 32 bits


class RSError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {_STATUS.get(status, status)} ({detail})")
        self.status = status
        self.detail = detail


_STATUS = {0: "RS_OK", 1: "RS_ERR_ARG", 2: "RS_ERR_GRAPH", 3: "RS_ERR_RANGE", 4: "RS_ERR_NOMEM",
           5: "RS_ERR_HIP", 6: "RS_ERR_STATE"}


class rs_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("offset_bytes", ctypes.c_int32),
                ("on_device", ctypes.c_int32), ("row_offsets", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("labels", ctypes.c_void_p)]


class rs_removals(ctypes.Structure):
    _fields_ = [("n_edges", ctypes.c_int64), ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
                ("n_vertices", ctypes.c_int64), ("vertices", ctypes.c_void_p)]


class rs_removal_result(ctypes.Structure):
    _fields_ = [("edges_removed", ctypes.c_int64), ("edges_ignored", ctypes.c_int64),
                ("vertices_removed", ctypes.c_int64), ("affected", ctypes.c_int64)]


class rs_counts(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("n_alive", ctypes.c_int64),
                ("n_communities", ctypes.c_int64), ("n_border", ctypes.c_int64),
                ("m_inter", ctypes.c_int64), ("sum_ell", ctypes.c_int64), ("sum_ell_x", ctypes.c_int64),
                ("sum_tI", ctypes.c_int64),
                ("sum_tII", ctypes.c_int64), ("sum_work_I", ctypes.c_int64), ("omega_max", ctypes.c_double)]


class rs_tiling(ctypes.Structure):
    _fields_ = [("row_entries", ctypes.c_int32), ("row_vertices", ctypes.c_int32), ("score_pairs", ctypes.c_int32),
                ("score_vertices", ctypes.c_int32), ("hub_list", ctypes.c_int32)]


TILING_FIELDS = ("row_entries", "row_vertices", "score_pairs", "score_vertices", "hub_list")


class rs_request_info(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_int64), ("t_start", ctypes.c_int64), ("t_done", ctypes.c_int64),
                ("affected", ctypes.c_int64), ("edges_removed", ctypes.c_int64), ("loaded", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class rs_server_stats_t(ctypes.Structure):
    _fields_ = [("requests_done", ctypes.c_int64), ("loads", ctypes.c_int64), ("evictions", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("peak_device_bytes", ctypes.c_int64)]


EXPORTS = [
    "rs_load_graph", "rs_score", "rs_topk", "rs_apply_removals", "rs_read_scores", "rs_read_counts",
    "rs_read_vertex_counts", "rs_read_rows", "rs_read_gprime", "rs_set_timing", "rs_read_timings",
    "rs_kernel_name", "rs_free_graph", "rs_status_string", "rs_last_error",
    "rs_server_create", "rs_server_add_graph", "rs_server_submit", "rs_server_wait", "rs_server_stats",
    "rs_server_free", "rs_load_batch", "rs_topk_batch", "rs_restrict_to_targets",
    "rs_reachable_communities", "rs_reachable_communities_static", "rs_get_tiling", "rs_set_tiling", "rs_autotune",
]


def _load_lib(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() (no fallback path exists)")
    lib = ctypes.CDLL(path)
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.rs_load_graph.argtypes = [ctypes.POINTER(rs_csr), P, ctypes.c_uint32, ctypes.POINTER(P)]
    lib.rs_score.argtypes = [P]
    lib.rs_topk.argtypes = [P, I64, P, P, ctypes.POINTER(I64)]
    lib.rs_apply_removals.argtypes = [P, ctypes.POINTER(rs_removals), ctypes.POINTER(rs_removal_result)]
    lib.rs_read_scores.argtypes = [P, P, I64, I32]
    lib.rs_read_counts.argtypes = [P, ctypes.POINTER(rs_counts)]
    lib.rs_read_vertex_counts.argtypes = [P, P, P, P, P, P, P]
    lib.rs_read_rows.argtypes = [P, P, P, P, P]
    lib.rs_read_gprime.argtypes = [P, P, P]
    lib.rs_set_timing.argtypes = [P, I32]
    lib.rs_read_timings.argtypes = [P, I32, P, P, ctypes.POINTER(I32)]
    lib.rs_kernel_name.argtypes = [I32]
    lib.rs_kernel_name.restype = ctypes.c_char_p
    lib.rs_free_graph.argtypes = [P]
    lib.rs_free_graph.restype = None
    lib.rs_status_string.argtypes = [ctypes.c_int]
    lib.rs_status_string.restype = ctypes.c_char_p
    lib.rs_last_error.argtypes = []
    lib.rs_last_error.restype = ctypes.c_char_p
    lib.rs_server_create.argtypes = [I32, I64, ctypes.POINTER(P)]
    lib.rs_server_add_graph.argtypes = [P, ctypes.POINTER(rs_csr), ctypes.POINTER(I32)]
    lib.rs_server_submit.argtypes = [P, I32, ctypes.POINTER(rs_removals), I64, ctypes.POINTER(I64)]
    lib.rs_server_wait.argtypes = [P, I64, P, P, ctypes.POINTER(I64), ctypes.POINTER(rs_request_info)]
    lib.rs_server_stats.argtypes = [P, ctypes.POINTER(rs_server_stats_t)]
    lib.rs_server_free.argtypes = [P]
    lib.rs_server_free.restype = None
    lib.rs_load_batch.argtypes = [I32, P, ctypes.POINTER(rs_csr), P, ctypes.c_uint32, ctypes.POINTER(P)]
    lib.rs_topk_batch.argtypes = [P, I64, P, P, P]
    lib.rs_restrict_to_targets.argtypes = [P, I32, ctypes.POINTER(rs_removal_result)]
    lib.rs_reachable_communities.argtypes = [P, I64, P, P]
    lib.rs_reachable_communities_static.argtypes = [P, I64, P, P]
    lib.rs_get_tiling.argtypes = [P, ctypes.POINTER(rs_tiling)]
    lib.rs_set_tiling.argtypes = [P, ctypes.POINTER(rs_tiling)]
    lib.rs_autotune.argtypes = [P, I32, P, I32, ctypes.POINTER(I32), P]
    for name in ("rs_load_graph", "rs_score", "rs_topk", "rs_apply_removals", "rs_read_scores",
                 "rs_read_counts", "rs_read_vertex_counts", "rs_read_rows", "rs_read_gprime",
                 "rs_set_timing", "rs_read_timings", "rs_server_create", "rs_server_add_graph",
                 "rs_server_submit", "rs_server_wait", "rs_server_stats", "rs_load_batch", "rs_topk_batch",
                 "rs_restrict_to_targets", "rs_reachable_communities", "rs_reachable_communities_static",
                 "rs_get_tiling", "rs_set_tiling", "rs_autotune"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = _load_lib()


def lib():
    return _lib


def _check(st: int, where: str):
    if st != RS_OK:
        raise RSError(st, where, _lib.rs_last_error().decode())


def _ptr(a):
    """(pointer, on_device, keepalive) for a numpy array or torch tensor."""
    if a is None:
        return None, 0, None
    if hasattr(a, "data_ptr"):  # torch tensor
        t = a.contiguous()
        return t.data_ptr(), int(t.is_cuda), t
    arr = np.ascontiguousarray(a)
    return arr.ctypes.data, 0, arr


class RSGraph:
    """Handle of one resident graph (wraps ``rs_graph*``)."""

    def __init__(self, handle, n, nnz):
        self.handle = handle
        self.n = int(n)
        self.nnz = int(nnz)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()

    def free(self):
        if self.handle:
            _lib.rs_free_graph(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def rs_load_graph(row_offsets, col, labels, stream=None, flags: int = 0) -> RSGraph:
    """Load a CSR graph + labels; ``stream`` is a hipStream_t handle (int) or a torch stream."""
    if hasattr(row_offsets, "element_size"):
        ob = row_offsets.element_size()
        n = row_offsets.numel() - 1
        nnz = col.numel()
    else:
        row_offsets = np.ascontiguousarray(row_offsets)
        if row_offsets.dtype not in (np.int32, np.int64):
            row_offsets = row_offsets.astype(np.int64)
        ob = row_offsets.dtype.itemsize
        n = row_offsets.size - 1
        col = np.ascontiguousarray(col, dtype=np.int32)
        labels = np.ascontiguousarray(labels, dtype=np.int32)
        nnz = col.size
    po, d0, k0 = _ptr(row_offsets)
    pc, d1, k1 = _ptr(col)
    pl, d2, k2 = _ptr(labels)
    on_dev = d0
    if n > 0 and not (d0 == d1 == d2):
        raise ValueError("row_offsets, col and labels must all be host or all be device arrays")
    csr = rs_csr(n, nnz, ob, on_dev, po, pc, pl)
    s = stream
    if s is not None and hasattr(s, "cuda_stream"):
        s = s.cuda_stream
    h = ctypes.c_void_p()
    _check(_lib.rs_load_graph(ctypes.byref(csr), s, flags, ctypes.byref(h)), "rs_load_graph")
    del k0, k1, k2
    return RSGraph(h, n, nnz)


def rs_score(g: RSGraph):
    _check(_lib.rs_score(g.handle), "rs_score")


def rs_topk(g: RSGraph, k: int):
    ids = np.zeros(max(k, 1), np.int32)
    sc = np.zeros(max(k, 1), np.float64)
    cnt = ctypes.c_int64(0)
    _check(_lib.rs_topk(g.handle, k, ids.ctypes.data, sc.ctypes.data, ctypes.byref(cnt)), "rs_topk")
    return ids[: cnt.value].copy(), sc[: cnt.value].copy()


def rs_apply_removals(g: RSGraph, edges=None, vertices=None) -> dict:
    e = np.zeros((0, 2), np.int32) if edges is None else np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    v = np.zeros(0, np.int32) if vertices is None else np.ascontiguousarray(vertices, dtype=np.int32).ravel()
    src = np.ascontiguousarray(e[:, 0])
    dst = np.ascontiguousarray(e[:, 1])
    b = rs_removals(e.shape[0], src.ctypes.data if e.shape[0] else None,
                    dst.ctypes.data if e.shape[0] else None, v.size, v.ctypes.data if v.size else None)
    r = rs_removal_result()
    _check(_lib.rs_apply_removals(g.handle, ctypes.byref(b), ctypes.byref(r)), "rs_apply_removals")
    return {k: getattr(r, k) for k, _ in rs_removal_result._fields_}


def rs_restrict_to_targets(g: RSGraph, k_c: int) -> dict:
    """Target-community mode: keep the k_c largest communities (removal result)."""
    r = rs_removal_result()
    _check(_lib.rs_restrict_to_targets(g.handle, int(k_c), ctypes.byref(r)), "rs_restrict_to_targets")
    return {k: getattr(r, k) for k, _ in rs_removal_result._fields_}


def rs_reachable_communities(g: RSGraph, sources) -> np.ndarray:
    """Distinct communities among the other members of each source's component."""
    src = np.ascontiguousarray(sources, dtype=np.int32).ravel()
    out = np.zeros(max(src.size, 1), np.int64)
    _check(_lib.rs_reachable_communities(g.handle, src.size, src.ctypes.data if src.size else None,
                                         out.ctypes.data), "rs_reachable_communities")
    return out[: src.size]


def rs_reachable_communities_static(g: RSGraph, sources) -> np.ndarray:
    """rs_reachable_communities without any allocation in the library (the
    device's static scratch array)."""
    src = np.ascontiguousarray(sources, dtype=np.int32).ravel()
    out = np.zeros(max(src.size, 1), np.int64)
    _check(_lib.rs_reachable_communities_static(g.handle, src.size, src.ctypes.data if src.size else None,
                                                out.ctypes.data), "rs_reachable_communities_static")
    return out[: src.size]


def rs_get_tiling(g: RSGraph) -> dict:
    """The graph's schedule cut-offs (see rs.h)."""
    t = rs_tiling()
    _check(_lib.rs_get_tiling(g.handle, ctypes.byref(t)), "rs_get_tiling")
    return {f: int(getattr(t, f)) for f in TILING_FIELDS}


def rs_set_tiling(g: RSGraph, tiling: dict):
    """Re-cut the graph's schedule; the graph must be scored again."""
    t = rs_tiling(*[int(tiling[f]) for f in TILING_FIELDS])
    _check(_lib.rs_set_tiling(g.handle, ctypes.byref(t)), "rs_set_tiling")


def rs_autotune(g: RSGraph, candidates, reps: int = 3):
    """(index of the fastest candidate, mean pass ms of each); the graph keeps
    the fastest cut-offs."""
    arr = (rs_tiling * len(candidates))(*[rs_tiling(*[int(c[f]) for f in TILING_FIELDS]) for c in candidates])
    ms = np.zeros(max(len(candidates), 1), np.float64)
    best = ctypes.c_int32(-1)
    _check(_lib.rs_autotune(g.handle, len(candidates), ctypes.cast(arr, ctypes.c_void_p), int(reps),
                            ctypes.byref(best), ms.ctypes.data), "rs_autotune")
    return int(best.value), ms[: len(candidates)]


def rs_read_scores(g: RSGraph, raw: bool = False):
    out = np.zeros(max(g.n, 1), np.float64)
    _check(_lib.rs_read_scores(g.handle, out.ctypes.data, g.n, int(raw)), "rs_read_scores")
    return out[: g.n]


def rs_read_counts(g: RSGraph) -> dict:
    c = rs_counts()
    _check(_lib.rs_read_counts(g.handle, ctypes.byref(c)), "rs_read_counts")
    return {k: getattr(c, k) for k, _ in rs_counts._fields_}


def rs_read_vertex_counts(g: RSGraph) -> dict:
    nn = max(g.n, 1)
    out = {"border": np.zeros(nn, np.int32), "ell": np.zeros(nn, np.int32), "dprime": np.zeros(nn, np.int32),
           "tI": np.zeros(nn, np.int64), "tII": np.zeros(nn, np.int64), "w_own": np.zeros(nn)}
    _check(_lib.rs_read_vertex_counts(g.handle, *(out[k].ctypes.data for k in
                                                  ("border", "ell", "dprime", "tI", "tII", "w_own"))),
           "rs_read_vertex_counts")
    return {k: v[: g.n] for k, v in out.items()}


def rs_read_rows(g: RSGraph):
    off = np.zeros(g.n + 1, np.int64)
    _check(_lib.rs_read_rows(g.handle, off.ctypes.data, None, None, None), "rs_read_rows")
    tot = max(int(off[-1]), 1)
    comm = np.zeros(tot, np.int32)
    cnt = np.zeros(tot, np.int32)
    w = np.zeros(tot)
    _check(_lib.rs_read_rows(g.handle, off.ctypes.data, comm.ctypes.data, cnt.ctypes.data, w.ctypes.data),
           "rs_read_rows")
    t = int(off[-1])
    return off, comm[:t], cnt[:t], w[:t]


def rs_read_gprime(g: RSGraph):
    off = np.zeros(g.n + 1, np.int64)
    _check(_lib.rs_read_gprime(g.handle, off.ctypes.data, None), "rs_read_gprime")
    col = np.zeros(max(int(off[-1]), 1), np.int32)
    _check(_lib.rs_read_gprime(g.handle, off.ctypes.data, col.ctypes.data), "rs_read_gprime")
    return off, col[: int(off[-1])]


def rs_set_timing(g: RSGraph, on: bool = True):
    _check(_lib.rs_set_timing(g.handle, int(on)), "rs_set_timing")


def rs_read_timings(g: RSGraph) -> dict:
    ms = np.zeros(64)
    ln = np.zeros(64, np.int64)
    nk = ctypes.c_int32(0)
    _check(_lib.rs_read_timings(g.handle, 64, ms.ctypes.data, ln.ctypes.data, ctypes.byref(nk)), "rs_read_timings")
    return {_lib.rs_kernel_name(i).decode(): (float(ms[i]), int(ln[i])) for i in range(nk.value)}


def rs_kernel_name(i: int):
    name = _lib.rs_kernel_name(i)
    return None if name is None else name.decode()


def rs_free_graph(g: RSGraph):
    g.free()


def rs_status_string(s: int) -> str:
    return _lib.rs_status_string(s).decode()


def rs_last_error() -> str:
    return _lib.rs_last_error().decode()


class RSServer:
    """The served form (wraps ``rs_server*``): register graphs, submit removal
    requests (each followed by a top-k), wait for their results."""

    def __init__(self, slots: int = 4, hbm_budget: int = 0):
        h = ctypes.c_void_p()
        _check(_lib.rs_server_create(int(slots), int(hbm_budget), ctypes.byref(h)), "rs_server_create")
        self.handle = h
        self.k = {}

    def add_graph(self, row_offsets, col, labels) -> int:
        off = np.ascontiguousarray(row_offsets, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        lab = np.ascontiguousarray(labels, dtype=np.int32)
        csr = rs_csr(off.size - 1, col.size, 8, 0, off.ctypes.data, col.ctypes.data, lab.ctypes.data)
        gid = ctypes.c_int32()
        _check(_lib.rs_server_add_graph(self.handle, ctypes.byref(csr), ctypes.byref(gid)), "rs_server_add_graph")
        return gid.value

    def submit(self, graph_id: int, k: int, edges=None, vertices=None) -> int:
        e = np.zeros((0, 2), np.int32) if edges is None else np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
        v = np.zeros(0, np.int32) if vertices is None else np.ascontiguousarray(vertices, dtype=np.int32).ravel()
        src = np.ascontiguousarray(e[:, 0])
        dst = np.ascontiguousarray(e[:, 1])
        b = rs_removals(e.shape[0], src.ctypes.data if e.shape[0] else None,
                        dst.ctypes.data if e.shape[0] else None, v.size, v.ctypes.data if v.size else None)
        rid = ctypes.c_int64()
        _check(_lib.rs_server_submit(self.handle, int(graph_id), ctypes.byref(b), int(k), ctypes.byref(rid)),
               "rs_server_submit")
        self.k[rid.value] = int(k)
        return rid.value

    def wait(self, request_id: int):
        """(ids, scores, info dict) of a finished request."""
        k = max(self.k.pop(request_id, 0), 1)
        ids = np.zeros(k, np.int32)
        sc = np.zeros(k, np.float64)
        cnt = ctypes.c_int64()
        info = rs_request_info()
        _check(_lib.rs_server_wait(self.handle, int(request_id), ids.ctypes.data, sc.ctypes.data, ctypes.byref(cnt),
                                   ctypes.byref(info)), "rs_server_wait")
        return ids[: cnt.value], sc[: cnt.value], {f: getattr(info, f) for f, _ in rs_request_info._fields_}

    def stats(self) -> dict:
        st = rs_server_stats_t()
        _check(_lib.rs_server_stats(self.handle, ctypes.byref(st)), "rs_server_stats")
        return {f: getattr(st, f) for f, _ in rs_server_stats_t._fields_}

    def free(self):
        if self.handle:
            _lib.rs_server_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def rs_server_create(slots: int = 4, hbm_budget: int = 0) -> RSServer:
    return RSServer(slots, hbm_budget)


def rs_server_add_graph(s: RSServer, row_offsets, col, labels) -> int:
    return s.add_graph(row_offsets, col, labels)


def rs_server_submit(s: RSServer, graph_id: int, k: int, edges=None, vertices=None) -> int:
    return s.submit(graph_id, k, edges=edges, vertices=vertices)


def rs_server_wait(s: RSServer, request_id: int):
    return s.wait(request_id)


def rs_server_stats(s: RSServer) -> dict:
    return s.stats()


def rs_server_free(s: RSServer):
    s.free()


def rs_load_batch(vertex_offsets, row_offsets, col, labels, stream=None, flags: int = 0) -> RSGraph:
    """Load a batch: the disjoint union of graphs (graph i = vertices
    [vertex_offsets[i], vertex_offsets[i+1]), global ids, per-graph labels)."""
    vo = np.ascontiguousarray(vertex_offsets, dtype=np.int64)
    off = np.ascontiguousarray(row_offsets, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    csr = rs_csr(off.size - 1, col.size, 8, 0, off.ctypes.data, col.ctypes.data, lab.ctypes.data)
    s = stream
    if s is not None and hasattr(s, "cuda_stream"):
        s = s.cuda_stream
    h = ctypes.c_void_p()
    _check(_lib.rs_load_batch(vo.size - 1, vo.ctypes.data, ctypes.byref(csr), s, flags, ctypes.byref(h)),
           "rs_load_batch")
    g = RSGraph(h, off.size - 1, col.size)
    g.n_graphs = vo.size - 1
    return g


def rs_topk_batch(g: RSGraph, k: int):
    """(ids [G, k] relative to each graph, scores [G, k], counts [G])."""
    G = g.n_graphs
    ids = np.zeros((G, k), np.int32)
    sc = np.zeros((G, k), np.float64)
    cnt = np.zeros(G, np.int64)
    _check(_lib.rs_topk_batch(g.handle, int(k), ids.ctypes.data, sc.ctypes.data, cnt.ctypes.data), "rs_topk_batch")
    return ids, sc, cnt
