"""Batches of independent graphs: concatenated CSR, color_graph_batched and
the launch-shape autotuner (C ABI in include/adg.h).

A batch is one CSR over all graphs: graph g owns the global vertex slots
vtx_off[g] .. vtx_off[g+1]-1; row_ptr holds absolute offsets into col_idx and
col_idx holds each graph's local vertex ids, so every graph is coloured as a
standalone color_graph call would colour it.  This module only packs arrays
and marshals calls; all colouring work runs in the library's kernels.
"""
import ctypes

import numpy as np

from . import _Stats, _check, _ptr, _stream, _torch, lib

__all__ = ["Batch", "BatchConfig", "batched_workspace_bytes", "color_graph_batched", "autotune", "batched_error",
           "batched_stats", "default_config"]

ADG_SCHED_LPT = 0
ADG_SCHED_NATURAL = 1


class _Batch(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_int32), ("total_n", ctypes.c_int64), ("total_nnz", ctypes.c_int64),
                ("vtx_off", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class BatchConfig(ctypes.Structure):
    """Launch shape of the persistent batched kernel (results do not depend on it)."""
    _fields_ = [("block_threads", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32), ("schedule", ctypes.c_int32)]

    def as_dict(self):
        return {"block_threads": self.block_threads, "blocks_per_cu": self.blocks_per_cu,
                "schedule": "natural" if self.schedule == ADG_SCHED_NATURAL else "lpt"}

    def __repr__(self):
        return "BatchConfig(%s)" % self.as_dict()


def _setup(L):
    if getattr(L, "_batched_ready", False):
        return L
    vp, i32, i64, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    P = ctypes.POINTER
    L.adg_batched_workspace_bytes.restype = sz
    L.adg_batched_workspace_bytes.argtypes = [i32, i64, i64]
    L.adg_batched_default_config.restype = BatchConfig
    L.adg_batched_default_config.argtypes = []
    L.color_graph_batched.restype = ctypes.c_int
    L.color_graph_batched.argtypes = [P(_Batch), i32, i32, u64, vp, vp, vp, vp, P(BatchConfig), vp, sz, vp]
    L.adg_batched_get_stats.restype = ctypes.c_int
    L.adg_batched_get_stats.argtypes = [vp, sz, P(_Stats), vp]
    L.adg_batched_autotune.restype = ctypes.c_int
    L.adg_batched_autotune.argtypes = [P(_Batch), i32, i32, u64, vp, vp, vp, sz, vp, i32, P(BatchConfig),
                                       P(ctypes.c_float)]
    L._batched_ready = True
    return L


def _lib():
    return _setup(lib())


class Batch:
    """Independent CSR graphs packed into one device-resident batch.

    ``graphs`` is a list of (row_ptr, col_idx) pairs (numpy, per-graph local
    ids).  Host copies of the offsets are kept for splitting results."""

    def __init__(self, graphs, device="cuda"):
        torch = _torch()
        ns = np.array([np.asarray(rp).size - 1 for rp, _ in graphs], dtype=np.int64)
        nnzs = np.array([np.asarray(ci).size for _, ci in graphs], dtype=np.int64)
        self.num_graphs = len(graphs)
        self.vtx_off = np.zeros(self.num_graphs + 1, dtype=np.int64)
        np.cumsum(ns, out=self.vtx_off[1:])
        nnz_off = np.zeros(self.num_graphs + 1, dtype=np.int64)
        np.cumsum(nnzs, out=nnz_off[1:])
        self.total_n = int(self.vtx_off[-1])
        self.total_nnz = int(nnz_off[-1])
        rp = np.empty(self.total_n + 1, dtype=np.int64)
        col = np.empty(self.total_nnz, dtype=np.int32)
        for g, (r, c) in enumerate(graphs):
            r = np.asarray(r, dtype=np.int64)
            v0, v1 = self.vtx_off[g], self.vtx_off[g + 1]
            rp[v0:v1] = r[:-1] + nnz_off[g]
            col[nnz_off[g]:nnz_off[g + 1]] = np.asarray(c, dtype=np.int32)
        rp[self.total_n] = self.total_nnz
        self.nnz_off = nnz_off
        self.device = torch.device(device)
        self.d_vtx_off = torch.from_numpy(self.vtx_off).to(self.device)
        self.d_row_ptr = torch.from_numpy(rp).to(self.device)
        self.d_col_idx = torch.from_numpy(col).to(self.device)

    def desc(self):
        return _Batch(self.num_graphs, self.total_n, self.total_nnz, _ptr(self.d_vtx_off).value,
                      _ptr(self.d_row_ptr).value, _ptr(self.d_col_idx).value)

    def split(self, arr):
        """Per-graph slices of a [total_n] array (host numpy)."""
        a = arr.cpu().numpy() if hasattr(arr, "cpu") else np.asarray(arr)
        return [a[self.vtx_off[g]:self.vtx_off[g + 1]] for g in range(self.num_graphs)]


def batched_workspace_bytes(num_graphs, total_n, total_nnz):
    b = _lib().adg_batched_workspace_bytes(int(num_graphs), int(total_n), int(total_nnz))
    if b == 0:
        raise ValueError("invalid batch size")
    return b


def default_config():
    return _lib().adg_batched_default_config()


def _workspace(batch, workspace):
    torch = _torch()
    need = batched_workspace_bytes(batch.num_graphs, batch.total_n, batch.total_nnz)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=batch.device)
    if workspace.numel() < need:
        raise ValueError("workspace too small: %d < %d bytes" % (workspace.numel(), need))
    return workspace


def color_graph_batched(batch, eps_num, eps_den, seed, workspace=None, stream=None, config=None, want_rounds=False,
                        out=None):
    """JP-ADG on every graph of ``batch`` in one persistent launch.
    Returns (color [total_n], num_colors [G], round [total_n] or None,
    num_rounds [G]) as GPU tensors; ``out`` may hold them preallocated."""
    torch = _torch()
    ws = _workspace(batch, workspace)
    dev = batch.device
    if out is None:
        color = torch.empty(max(batch.total_n, 1), dtype=torch.int32, device=dev)
        rnd = torch.empty(max(batch.total_n, 1), dtype=torch.int32, device=dev) if want_rounds else None
        nc = torch.zeros(max(batch.num_graphs, 1), dtype=torch.int32, device=dev)
        nr = torch.zeros(max(batch.num_graphs, 1), dtype=torch.int32, device=dev)
    else:
        color, rnd, nc, nr = out
    d = batch.desc()
    cfg = ctypes.byref(config) if config is not None else None
    rc = _lib().color_graph_batched(ctypes.byref(d), int(eps_num), int(eps_den), int(seed) & (2**64 - 1),
                                    _ptr(color), _ptr(rnd) if rnd is not None else ctypes.c_void_p(0), _ptr(nc),
                                    _ptr(nr), cfg, _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "color_graph_batched")
    return (color[:batch.total_n], nc[:batch.num_graphs], rnd[:batch.total_n] if rnd is not None else None,
            nr[:batch.num_graphs])


def batched_stats(workspace, stream=None):
    """Counters of the last batched call on ``workspace``, summed over the
    batch (num_rounds / num_colors: the largest of any graph)."""
    st = _Stats()
    _check(_lib().adg_batched_get_stats(_ptr(workspace), workspace.numel(), ctypes.byref(st), _stream(stream)),
           "adg_batched_get_stats")
    return {k: int(getattr(st, k)) for k, _ in _Stats._fields_}


def batched_error(workspace, stream=None):
    """Device-side error code of the last batched call on ``workspace`` (0 = none)."""
    return batched_stats(workspace, stream)["error"]


def autotune(batch, eps_num, eps_den, seed, workspace=None, stream=None, reuse=True, out=None):
    """Time every candidate launch shape on this batch and return
    (BatchConfig, milliseconds) of the fastest."""
    torch = _torch()
    ws = _workspace(batch, workspace)
    if out is None:
        color = torch.empty(max(batch.total_n, 1), dtype=torch.int32, device=batch.device)
        nc = torch.zeros(max(batch.num_graphs, 1), dtype=torch.int32, device=batch.device)
    else:
        color, nc = out
    best = BatchConfig()
    ms = ctypes.c_float(0.0)
    d = batch.desc()
    rc = _lib().adg_batched_autotune(ctypes.byref(d), int(eps_num), int(eps_den), int(seed) & (2**64 - 1),
                                     _ptr(color), _ptr(nc), _ptr(ws), ws.numel(), _stream(stream),
                                     1 if reuse else 0, ctypes.byref(best), ctypes.byref(ms))
    _check(rc, "adg_batched_autotune")
    return best, float(ms.value)
