"""Seeded synthetic graphs in simple undirected CSR form.

Inputs for both the GPU library and the CPU checker come from here.  The
module holds no step of the colouring method: it draws random graphs
(Erdos-Renyi, R-MAT, Chung-Lu) from counter-based SplitMix64 streams and
builds a symmetric CSR without self-loops or duplicate entries, rows sorted.

Every function returns ``(row_ptr, col_idx)`` as numpy arrays
(``int64[n+1]``, ``int32[nnz]``).
"""
import ctypes
import math
import os

import numpy as np

from . import _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        vp, i64, u64, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        lib.gg_n.restype = i64
        lib.gg_n.argtypes = [vp]
        lib.gg_nnz.restype = i64
        lib.gg_nnz.argtypes = [vp]
        lib.gg_copy.restype = None
        lib.gg_copy.argtypes = [vp, vp, vp]
        lib.gg_free.restype = None
        lib.gg_free.argtypes = [vp]
        lib.gg_from_edges.restype = vp
        lib.gg_from_edges.argtypes = [i64, i64, vp, vp]
        lib.gg_erdos_renyi.restype = vp
        lib.gg_erdos_renyi.argtypes = [i64, f64, u64]
        lib.gg_rmat.restype = vp
        lib.gg_rmat.argtypes = [ctypes.c_int, i64, f64, f64, f64, u64]
        lib.gg_chung_lu.restype = vp
        lib.gg_chung_lu.argtypes = [i64, f64, f64, u64]
        lib.gg_chung_lu_weights.restype = ctypes.c_int
        lib.gg_chung_lu_weights.argtypes = [i64, f64, f64, vp]
        lib.gg_splitmix64_draw.restype = u64
        lib.gg_splitmix64_draw.argtypes = [u64, u64]
        lib.gg_num_threads.restype = ctypes.c_int
        lib.gg_chung_lu_many.restype = None
        lib.gg_chung_lu_many.argtypes = [i64, vp, vp, f64, vp, vp]
        _lib = lib
    return _lib


def _take(h):
    if not h:
        raise ValueError("graph generation failed (bad arguments or out of memory)")
    lib = _load()
    try:
        n, nnz = lib.gg_n(h), lib.gg_nnz(h)
        rp = np.empty(n + 1, dtype=np.int64)
        col = np.empty(nnz, dtype=np.int32)
        lib.gg_copy(h, rp.ctypes.data, col.ctypes.data)
    finally:
        lib.gg_free(h)
    return rp, col


def from_edges(n, src, dst):
    """Simple undirected CSR spanned by the listed edges (either direction,
    repeats allowed, self-loops dropped)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    return _take(_load().gg_from_edges(int(n), int(src.size), src.ctypes.data, dst.ctypes.data))


def erdos_renyi(n, p, seed):
    """G(n, p): each unordered pair independently with probability p."""
    return _take(_load().gg_erdos_renyi(int(n), float(p), int(seed) & (2**64 - 1)))


def rmat(scale, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=0):
    """R-MAT on 2^scale vertices with edge_factor * 2^scale edge draws."""
    ne = int(edge_factor) << int(scale)
    return _take(_load().gg_rmat(int(scale), ne, float(a), float(b), float(c), int(seed) & (2**64 - 1)))


def chung_lu(n, mean_deg, gamma=2.3, seed=0):
    """Chung-Lu expected-degree graph with power-law weights (exponent gamma)."""
    return _take(_load().gg_chung_lu(int(n), float(mean_deg), float(gamma), int(seed) & (2**64 - 1)))


def chung_lu_many(specs, gamma=2.3):
    """[(row_ptr, col_idx)] for a list of (n, mean_deg, seed): the same graphs
    as chung_lu, generated one graph per thread."""
    G = len(specs)
    n = np.array([s[0] for s in specs], dtype=np.int64)
    k = np.array([s[1] for s in specs], dtype=np.float64)
    seeds = np.array([int(s[2]) & (2**64 - 1) for s in specs], dtype=np.uint64)
    handles = (ctypes.c_void_p * max(G, 1))()
    _load().gg_chung_lu_many(G, n.ctypes.data, k.ctypes.data, float(gamma), seeds.ctypes.data, handles)
    out = []
    try:
        for g in range(G):
            out.append(_take(handles[g]))
            handles[g] = None
    finally:
        for g in range(G):
            if handles[g]:
                _load().gg_free(handles[g])
    return out


def batched_graphs(num_graphs=4096, seed=4, size_scale=1.0):
    """The graphs of the batched workload (see batched_config)."""
    specs = batched_config(num_graphs=num_graphs, seed=seed, size_scale=size_scale)
    return chung_lu_many([(n, min(k, n - 1.0), s) for n, k, s in specs], 2.3)


def serving_specs(count, seed=5):
    """Request mix of the serving workload: 70% Erdos-Renyi (n log-uniform
    in [1e3, 1e5], mean degree 10), 25% Chung-Lu (n log-uniform in [1e4, 1e6],
    mean degree 16, exponent 2.3), 5% R-MAT (scale uniform in 20..23, edge
    factor 16).  Returns [(kind, size, gen_seed)], size = n or the R-MAT scale."""
    key = stream_seed(seed, 0x5E7E)
    out = []
    for i in range(count):
        u = uniform01(key, 4 * i)
        gs = stream_seed(seed, 0x6E, i)
        if u < 0.70:
            out.append(("er", log_uniform_int(uniform01(key, 4 * i + 1), 1_000, 100_000), gs))
        elif u < 0.95:
            out.append(("chung_lu", log_uniform_int(uniform01(key, 4 * i + 1), 10_000, 1_000_000), gs))
        else:
            out.append(("rmat", 20 + min(3, int(4 * uniform01(key, 4 * i + 1))), gs))
    return out


def serving_graph(spec, scale_down=False):
    """The graph of one serving request.  scale_down shrinks it (ER n / 5,
    at least 1000; Chung-Lu n / 10, at least 10^4; R-MAT scale - 6)."""
    kind, size, gs = spec
    if kind == "er":
        n = max(1000, size // 5) if scale_down else size
        return erdos_renyi(n, min(1.0, 10.0 / max(n - 1, 1)), gs)
    if kind == "chung_lu":
        n = max(10_000, size // 10) if scale_down else size
        return chung_lu(n, 16.0, 2.3, gs)
    return rmat(size - 6 if scale_down else size, 16, 0.57, 0.19, 0.19, gs)


def poisson_arrivals(count, qps, seed=5):
    """Arrival times (seconds from 0) of a Poisson stream at rate qps."""
    key = stream_seed(seed, 0xA771)
    t = 0.0
    out = []
    for i in range(count):
        t += -math.log1p(-uniform01(key, i)) / qps
        out.append(t)
    return out


def chung_lu_weights(n, mean_deg, gamma=2.3):
    w = np.empty(int(n), dtype=np.float64)
    if _load().gg_chung_lu_weights(int(n), float(mean_deg), float(gamma), w.ctypes.data) != 0:
        raise ValueError("bad Chung-Lu parameters")
    return w


def splitmix64_draw(key, i):
    """i-th output (0-based) of the SplitMix64 stream started at state key."""
    return int(_load().gg_splitmix64_draw(int(key) & (2**64 - 1), int(i)))


def stream_seed(seed, *path):
    """Derive a deterministic 64-bit seed for a sub-case (e.g. graph g of a
    batch) from a base seed, using SplitMix64 outputs."""
    k = int(seed) & (2**64 - 1)
    for p in path:
        k = splitmix64_draw(k ^ (int(p) & (2**64 - 1)), 0)
    return k


def log_uniform_int(rng_u01, lo, hi):
    """Map a uniform draw in [0,1) to an integer log-uniform in [lo, hi]."""
    x = math.exp(math.log(lo) + rng_u01 * (math.log(hi + 1) - math.log(lo)))
    return max(lo, min(hi, int(x)))


def uniform01(key, i):
    return (splitmix64_draw(key, i) >> 11) * (1.0 / 9007199254740992.0)


# ---------------------------------------------------------------------------
# Named workloads (shapes of the paper's inputs; see the design notes).

def er_config(n=10_000, mean_deg=10.0, seed=1):
    """G(n, p = mean_deg / n)."""
    return erdos_renyi(n, mean_deg / n, seed)


def rmat_config(scale, seed, edge_factor=16):
    return rmat(scale, edge_factor, 0.57, 0.19, 0.19, seed)


def batched_config(num_graphs=4096, seed=4, n_lo=100, n_hi=50_000, deg_lo=8.0, deg_hi=32.0,
                   gamma=2.3, size_scale=1.0):
    """Per-graph (n, mean degree, generator seed) of the batched workload:
    n log-uniform in [n_lo, n_hi], mean degree uniform in [deg_lo, deg_hi],
    Chung-Lu exponent gamma.  size_scale shrinks n for quick tests."""
    key = stream_seed(seed, 0xBA7C)
    specs = []
    for g in range(num_graphs):
        n = log_uniform_int(uniform01(key, 3 * g), n_lo, n_hi)
        n = max(2, int(n * size_scale))
        k = deg_lo + (deg_hi - deg_lo) * uniform01(key, 3 * g + 1)
        k = min(k, n - 1.0)
        specs.append((n, k, stream_seed(seed, 0xC1, g)))
    return specs
