"""Serving loop: colour graphs as requests arrive, with continuous batching
(adg_server_* in include/adg.h).

The native server admits requests by device-arena footprint, groups small
ones into batched launches and overlaps jobs on several streams; this module
only passes host arrays in and results out, and replays an arrival schedule.
"""
import ctypes

import numpy as np

from . import AdgError, _check, _torch, lib

__all__ = ["Server", "ServerConfig", "footprint", "replay", "latency_summary"]


class ServerConfig(ctypes.Structure):
    _fields_ = [("eps_num", ctypes.c_int32), ("eps_den", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("workers", ctypes.c_int32), ("small_nnz", ctypes.c_int64), ("max_group", ctypes.c_int32),
                ("max_bypass", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("num_colors", ctypes.c_int32),
                ("num_rounds", ctypes.c_int32), ("group_size", ctypes.c_int32), ("n", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]


class Counters(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("single_jobs", "grouped_jobs", "grouped_requests", "vertices",
                                              "entries", "sum_active", "cut_edges")]


def _lib():
    L = lib()
    if getattr(L, "_serving_ready", False):
        return L
    vp, i32, i64, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    P = ctypes.POINTER
    L.adg_server_default_config.restype = ServerConfig
    L.adg_server_default_config.argtypes = []
    L.adg_server_footprint.restype = sz
    L.adg_server_footprint.argtypes = [P(ServerConfig), i64, i64]
    L.adg_server_create.restype = ctypes.c_int
    L.adg_server_create.argtypes = [P(ServerConfig), vp, sz, P(vp)]
    L.adg_server_submit.restype = ctypes.c_int
    L.adg_server_submit.argtypes = [vp, i64, i64, vp, vp, vp, u64]
    L.adg_server_poll.restype = ctypes.c_int
    L.adg_server_poll.argtypes = [vp, P(_Result), i32, i32, P(i32)]
    L.adg_server_in_flight.restype = i64
    L.adg_server_in_flight.argtypes = [vp]
    L.adg_server_clock.restype = ctypes.c_double
    L.adg_server_clock.argtypes = []
    L.adg_server_get_counters.restype = ctypes.c_int
    L.adg_server_get_counters.argtypes = [vp, P(Counters)]
    L.adg_server_destroy.restype = ctypes.c_int
    L.adg_server_destroy.argtypes = [vp]
    L._serving_ready = True
    return L


def default_config():
    return _lib().adg_server_default_config()


def footprint(n, nnz, config=None):
    cfg = config if config is not None else default_config()
    return int(_lib().adg_server_footprint(ctypes.byref(cfg), int(n), int(nnz)))


class Server:
    """A running server on the current GPU with an arena of ``arena_bytes``."""

    def __init__(self, arena_bytes, eps=(1, 10), seed=5, workers=4, small_nnz=1 << 20, max_group=256,
                 max_bypass=64, device="cuda"):
        torch = _torch()
        self.config = ServerConfig(int(eps[0]), int(eps[1]), int(seed) & (2**64 - 1), int(workers), int(small_nnz),
                                   int(max_group), int(max_bypass))
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _check(_lib().adg_server_create(ctypes.byref(self.config), ctypes.c_void_p(self.arena.data_ptr()),
                                        self.arena.numel(), ctypes.byref(h)), "adg_server_create")
        self._h = h
        self._live = {}   # tag -> (row_ptr, col_idx, color) kept alive until polled

    def submit(self, row_ptr, col_idx, tag):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col_idx, dtype=np.int32)
        n = rp.size - 1
        color = np.empty(max(n, 1), dtype=np.int32)
        if tag in self._live:
            raise ValueError("tag %r already in flight" % (tag,))
        self._live[tag] = (rp, col, color)
        rc = _lib().adg_server_submit(self._h, n, col.size, rp.ctypes.data, col.ctypes.data if col.size else None,
                                      color.ctypes.data, int(tag))
        if rc != 0:
            del self._live[tag]
            raise AdgError(rc, "adg_server_submit")

    def poll(self, max_results=256, wait_ms=0):
        """Finished requests as dicts (times in server-clock seconds; 'color'
        is the host array of colours)."""
        buf = (_Result * max(int(max_results), 1))()
        cnt = ctypes.c_int32(0)
        _check(_lib().adg_server_poll(self._h, buf, int(max_results), int(wait_ms), ctypes.byref(cnt)),
               "adg_server_poll")
        out = []
        for i in range(cnt.value):
            r = buf[i]
            d = {k: getattr(r, k) for k, _ in _Result._fields_}
            rp, col, color = self._live.pop(int(r.tag))
            d["color"] = color[:rp.size - 1]
            out.append(d)
        return out

    def counters(self):
        c = Counters()
        _check(_lib().adg_server_get_counters(self._h, ctypes.byref(c)), "adg_server_get_counters")
        return {k: int(getattr(c, k)) for k, _ in Counters._fields_}

    def in_flight(self):
        return int(_lib().adg_server_in_flight(self._h))

    @staticmethod
    def clock():
        return float(_lib().adg_server_clock())

    def close(self):
        if self._h:
            _lib().adg_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def replay(server, graphs, arrivals=None, timeout_s=600.0):
    """Submit graph i at arrivals[i] seconds after the start (all at once if
    arrivals is None) and collect every result.  Returns the results sorted
    by tag (= index)."""
    done = {}
    t0 = server.clock()
    i = 0
    deadline = t0 + timeout_s
    while len(done) < len(graphs):
        now = server.clock()
        if now > deadline:
            raise TimeoutError("serving replay did not finish in %.0f s" % timeout_s)
        while i < len(graphs) and (arrivals is None or t0 + arrivals[i] <= now):
            server.submit(graphs[i][0], graphs[i][1], i)
            i += 1
        wait = 50
        if i < len(graphs) and arrivals is not None:
            wait = max(0, min(50, int((t0 + arrivals[i] - server.clock()) * 1000)))
        for r in server.poll(256, wait):
            done[int(r["tag"])] = r
    return [done[k] for k in range(len(graphs))]


def latency_summary(results):
    lat = np.array([r["t_done"] - r["t_submit"] for r in results])
    q = np.array([r["t_admit"] - r["t_submit"] for r in results])
    span = max(r["t_done"] for r in results) - min(r["t_submit"] for r in results)
    m = sum(r["nnz"] for r in results) // 2
    return {"requests": len(results), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "queue_p50_ms": float(np.percentile(q, 50) * 1e3), "span_s": span, "edges_per_s": m / span,
            "requests_per_s": len(results) / span,
            "mean_group": float(np.mean([r["group_size"] for r in results]))}
