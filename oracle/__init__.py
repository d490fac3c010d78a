"""CPU oracle for ADG and JP-ADG -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never imports, links or calls it, and
shares no code with it.  See ``oracle.c`` for what each function follows in
the paper.

Parity status: every function here is pinned by CPU tests against properties
the paper or the mathematics fix (definition-level checks of the ADG
selection rule, closed forms, exact degeneracy by brute force, the colour
bound, JP's smallest-free-colour rule, published hash test vectors).
"""
import ctypes
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
        vp, i64, u64, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32
        lib.or_adg.restype = i64
        lib.or_adg.argtypes = [i64, vp, vp, i64, i64, vp, vp]
        lib.or_jp.restype = i64
        lib.or_jp.argtypes = [i64, vp, vp, vp, u64, vp]
        lib.or_color_graph.restype = i64
        lib.or_color_graph.argtypes = [i64, vp, vp, i64, i64, u64, vp, vp, vp, vp]
        lib.or_pred_counts.restype = i64
        lib.or_pred_counts.argtypes = [i64, vp, vp, vp, u64, vp]
        lib.or_adg_ex.restype = i64
        lib.or_adg_ex.argtypes = [i64, vp, vp, i64, i64, u64, ctypes.c_uint32, vp, vp, vp]
        lib.or_dec_itr.restype = i64
        lib.or_dec_itr.argtypes = [i64, vp, vp, vp, u64, vp, vp, vp]
        lib.or_jp_total.restype = i64
        lib.or_jp_total.argtypes = [i64, vp, vp, vp, vp]
        lib.or_degeneracy.restype = i64
        lib.or_degeneracy.argtypes = [i64, vp, vp]
        lib.or_tiebreak.restype = u32
        lib.or_tiebreak.argtypes = [u64, u32]
        lib.or_fmix32.restype = u32
        lib.or_fmix32.argtypes = [u32]
        lib.or_splitmix64_first.restype = u64
        lib.or_splitmix64_first.argtypes = [u64]
        _lib = lib
    return _lib


def _csr(row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    if c.size == 0:
        c = np.zeros(1, dtype=np.int32)
    return rp, c, rp.size - 1


def adg(row_ptr, col, eps_num, eps_den):
    """ADG (Algorithm 1).  Returns (rho int32[n] in 1..L, L, stats) where
    stats = dict(sum_active, cut_edges)."""
    rp, c, n = _csr(row_ptr, col)
    rho = np.zeros(max(n, 1), dtype=np.int32)
    st = np.zeros(4, dtype=np.int64)
    L = _load().or_adg(n, rp.ctypes.data, c.ctypes.data, int(eps_num), int(eps_den), rho.ctypes.data,
                       st.ctypes.data)
    if L < 0:
        raise ValueError("oracle ADG: bad arguments")
    return rho[:n], int(L), {"sum_active": int(st[0]), "cut_edges": int(st[1])}


def jp(row_ptr, col, rho, seed):
    """JP under <rho_ADG, rho_R> (greedy definition).  Returns (color, num_colors)."""
    rp, c, n = _csr(row_ptr, col)
    r = np.ascontiguousarray(rho, dtype=np.int32)
    if r.size == 0:
        r = np.zeros(1, dtype=np.int32)
    color = np.zeros(max(n, 1), dtype=np.int32)
    k = _load().or_jp(n, rp.ctypes.data, c.ctypes.data, r.ctypes.data, int(seed) & (2**64 - 1),
                      color.ctypes.data)
    if k < 0:
        raise ValueError("oracle JP failed (%d)" % k)
    return color[:n], int(k)


def color_graph(row_ptr, col, eps_num, eps_den, seed):
    """JP-ADG: returns (color, num_colors, rho, L, stats)."""
    rho, L, st = adg(row_ptr, col, eps_num, eps_den)
    color, k = jp(row_ptr, col, rho, seed)
    return color, k, rho, L, st


def pred_counts(row_ptr, col, rho, seed):
    rp, c, n = _csr(row_ptr, col)
    r = np.ascontiguousarray(rho, dtype=np.int32)
    out = np.zeros(max(n, 1), dtype=np.int32)
    if n:
        _load().or_pred_counts(n, rp.ctypes.data, c.ctypes.data, r.ctypes.data, int(seed) & (2**64 - 1),
                               out.ctypes.data)
    return out[:n]


def degeneracy(row_ptr, col):
    rp, c, n = _csr(row_ptr, col)
    return int(_load().or_degeneracy(n, rp.ctypes.data, c.ctypes.data))


def tiebreak(seed, v):
    """rho_R(v) = fmix32(v XOR low32(splitmix64_first(seed)))."""
    return int(_load().or_tiebreak(int(seed) & (2**64 - 1), int(v) & 0xFFFFFFFF))


def tiebreak_array(seed, n):
    lib = _load()
    s = int(seed) & (2**64 - 1)
    return np.array([lib.or_tiebreak(s, v) for v in range(n)], dtype=np.uint32)


def fmix32(x):
    return int(_load().or_fmix32(int(x) & 0xFFFFFFFF))


def splitmix64_first(s):
    return int(_load().or_splitmix64_first(int(s) & (2**64 - 1)))



SORTED = 1   # ADG-O: R sorted by D at selection, ties by rho_R
MEDIAN = 2   # ADG-M: lower median of D times (1+eps), R capped at ceil(|U|/2)


def adg_ex(row_ptr, col, eps_num, eps_den, seed, flags):
    """ADG with variant flags (SORTED, MEDIAN; or_adg_ex).  Returns
    (round int32[n], pos int64[n], L, stats); pos is the total order JP
    colours by (larger = first)."""
    rp, c, n = _csr(row_ptr, col)
    rnd = np.zeros(max(n, 1), dtype=np.int32)
    pos = np.zeros(max(n, 1), dtype=np.int64)
    st = np.zeros(4, dtype=np.int64)
    L = _load().or_adg_ex(n, rp.ctypes.data, c.ctypes.data, int(eps_num), int(eps_den),
                          int(seed) & (2**64 - 1), int(flags), rnd.ctypes.data, pos.ctypes.data, st.ctypes.data)
    if L < 0:
        raise ValueError("or_adg_ex failed (%d)" % L)
    return rnd[:n], pos[:n], int(L), {"sum_active": int(st[0]), "cut_edges": int(st[1])}


def jp_total(row_ptr, col, pos):
    """JP under a total order pos (larger = coloured first) = greedy in that order."""
    rp, c, n = _csr(row_ptr, col)
    p = np.ascontiguousarray(pos, dtype=np.int64)
    color = np.zeros(max(n, 1), dtype=np.int32)
    k = _load().or_jp_total(n, rp.ctypes.data, c.ctypes.data, p.ctypes.data, color.ctypes.data)
    if k < 0:
        raise ValueError("or_jp_total failed")
    return color[:n], int(k)


def color_graph_ex(row_ptr, col, eps_num, eps_den, seed, flags):
    """JP-ADG with variant flags: adg_ex, then JP under its total order.
    Returns (color, num_colors, round, L, pos, stats)."""
    rnd, pos, L, st = adg_ex(row_ptr, col, eps_num, eps_den, seed, flags)
    color, k = jp_total(row_ptr, col, pos)
    return color, k, rnd, L, pos, st


def dec_itr(row_ptr, col, rho, seed):
    """DEC-ADG-ITR's colouring of the ADG partitions rho (or_dec_itr).
    Returns (color int32[n], num_colors, step int64[n], iterations)."""
    rp, c, n = _csr(row_ptr, col)
    r = np.ascontiguousarray(rho, dtype=np.int32)
    color = np.zeros(max(n, 1), dtype=np.int32)
    step = np.zeros(max(n, 1), dtype=np.int64)
    st = np.zeros(2, dtype=np.int64)
    k = _load().or_dec_itr(n, rp.ctypes.data, c.ctypes.data, r.ctypes.data, int(seed) & (2**64 - 1),
                           color.ctypes.data, step.ctypes.data, st.ctypes.data)
    if k < 0:
        raise ValueError("or_dec_itr failed")
    return color[:n], int(k), step[:n], int(st[0])


def color_graph_dec(row_ptr, col, eps_num, eps_den, seed, flags=0):
    """DEC-ADG-ITR end to end: ADG (Algorithm 1; ADG-M's partitions with
    flags = MEDIAN), then dec_itr.  Returns (color, num_colors, round, L,
    step, iterations)."""
    if flags:
        rho, _, L, _ = adg_ex(row_ptr, col, eps_num, eps_den, seed, flags)
    else:
        rho, L, _ = adg(row_ptr, col, eps_num, eps_den)
    color, k, step, it = dec_itr(row_ptr, col, rho, seed)
    return color, k, rho, L, step, it
