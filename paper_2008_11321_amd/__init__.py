"""ADG and JP-ADG graph colouring on AMD MI355X (gfx950).

Thin ctypes binding over ``libadg_hip.so`` (C ABI in ``include/adg.h``).
Every step of the method runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch provides device memory (``torch.empty``) and the
current HIP stream.  There is no CPU fallback: if the library is missing or no
GPU is visible, the calls raise.

Method: Besta et al., "High-Performance Parallel Graph Coloring with Strong
Guarantees on Work, Depth, and Quality" -- ADG (Algorithm 1) and JP
(Algorithm 3) under the priority <rho_ADG, rho_R>.
"""
import ctypes
import os

from . import _build

__all__ = [
    "AdgError", "lib", "workspace_bytes", "adg_order", "jp_color", "color_graph", "color_graph_batched",
    "batched_workspace_bytes", "get_stats", "validate_csr", "error_string", "Graph", "profile_enable",
    "profile_read",
]

ADG_OK = 0
_ERRS = {-1: "ADG_ERR_ARG", -2: "ADG_ERR_WORKSPACE", -3: "ADG_ERR_HIP", -4: "ADG_ERR_INTERNAL",
         -5: "ADG_ERR_UNSUPPORTED", -6: "ADG_ERR_SCRATCH"}


class AdgError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s failed: %s (%s)" % (where, _ERRS.get(code, code), error_string(code)))


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p)]


class _Stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("num_rounds", "num_colors", "sum_active", "cut_edges", "frontier", "jp_levels", "error")]


class _Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 32), ("launches", ctypes.c_int64 * 32)]


KERNEL_CLASSES = ["init", "stats", "count", "scan", "scatter", "update", "part1", "jp_prep", "jp", "finish",
                  "batched", "jp_narrow", "update_huge", "median_select", "order_sort", "dec_itr", "update_pull",
                  "jp_phase", "dec_phase", "adg_phase", "update_sub"]

# ADG variants (bit set): ADG-O's sorted rounds and ADG-M's median selection
SORTED = 1
MEDIAN = 2
DEC_ITR = 4   # colouring by DEC-ADG-ITR instead of JP (color_graph_ex only)
PULL = 8      # pull (CREW) UPDATE: same output, no atomics on D
MULTI_LAUNCH = 16   # keep a small graph on the per-round kernels (color_graph_ex only)
RELAX_ALL = 32      # JP relaxes every round from its start (color_graph_ex only; same output)
LEVELS_ONLY = 64    # JP colours every round level by level (color_graph_ex only; same output)

_lib = None


def lib():
    """Load libadg_hip.so (building it first only if no build exists)."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("ADG_HIP_LIB") or _build.LIB   # another build of the library (tuning runs)
    if path == _build.LIB and not os.path.exists(path):
        _build.build()
    L = ctypes.CDLL(path)
    vp, i32, i64, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    P = ctypes.POINTER
    L.adg_workspace_bytes.restype = sz
    L.adg_workspace_bytes.argtypes = [i64, i64]
    L.adg_order.restype = ctypes.c_int
    L.adg_order.argtypes = [P(_Csr), i32, i32, vp, vp, vp, sz, vp]
    L.jp_color.restype = ctypes.c_int
    L.jp_color.argtypes = [P(_Csr), vp, u64, vp, vp, vp, sz, vp]
    L.color_graph.restype = ctypes.c_int
    L.color_graph.argtypes = [P(_Csr), i32, i32, u64, vp, vp, vp, vp, vp, sz, vp]
    L.adg_order_workspace_bytes.restype = sz
    L.adg_order_workspace_bytes.argtypes = [i64, i64]
    L.adg_order_ex.restype = ctypes.c_int
    L.adg_order_ex.argtypes = [P(_Csr), i32, i32, u64, ctypes.c_uint32, vp, vp, vp, vp, sz, vp]
    L.color_graph_ex.restype = ctypes.c_int
    L.color_graph_ex.argtypes = [P(_Csr), i32, i32, u64, ctypes.c_uint32, vp, vp, vp, vp, vp, sz, vp]
    L.adg_get_stats.restype = ctypes.c_int
    L.adg_get_stats.argtypes = [vp, sz, P(_Stats), vp]
    L.adg_validate_csr.restype = ctypes.c_int
    L.adg_validate_csr.argtypes = [P(_Csr), vp, sz, vp]
    L.adg_error_string.restype = ctypes.c_char_p
    L.adg_error_string.argtypes = [ctypes.c_int]
    L.adg_profile_enable.restype = ctypes.c_int
    L.adg_profile_enable.argtypes = [ctypes.c_uint32]
    L.adg_profile_read.restype = ctypes.c_int
    L.adg_profile_read.argtypes = [P(_Profile)]
    L.adg_kernel_class_name.restype = ctypes.c_char_p
    L.adg_kernel_class_name.argtypes = [ctypes.c_int]
    L.color_graph_static.restype = ctypes.c_int
    L.color_graph_static.argtypes = [P(_Csr), i32, i32, u64, vp, vp, vp, vp, vp]
    L.adg_static_scratch_bytes.restype = sz
    L.adg_static_scratch_bytes.argtypes = []
    _lib = L
    return L


def error_string(code):
    try:
        return lib().adg_error_string(int(code)).decode()
    except OSError:
        return "library not loaded"


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2008_11321_amd needs a visible AMD GPU (no CPU fallback)")
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc, where):
    if rc != ADG_OK:
        raise AdgError(rc, where)


class Graph:
    """A CSR graph resident on the GPU: row_ptr int64[n+1], col_idx int32[nnz]."""

    def __init__(self, row_ptr, col_idx, device="cuda"):
        torch = _torch()
        rp = torch.as_tensor(row_ptr, dtype=torch.int64)
        ci = torch.as_tensor(col_idx, dtype=torch.int32)
        self.row_ptr = rp.to(device).contiguous()
        self.col_idx = ci.to(device).contiguous()
        self.n = self.row_ptr.numel() - 1
        self.nnz = self.col_idx.numel()
        self.device = self.row_ptr.device

    def csr(self):
        return _Csr(self.n, self.nnz, _ptr(self.row_ptr).value, _ptr(self.col_idx).value)


def workspace_bytes(n, nnz):
    b = lib().adg_workspace_bytes(int(n), int(nnz))
    if b == 0:
        raise ValueError("invalid graph size")
    return b


def _workspace(g, workspace):
    torch = _torch()
    need = workspace_bytes(g.n, g.nnz)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=g.device)
    if workspace.numel() < need:
        raise ValueError("workspace too small: %d < %d bytes" % (workspace.numel(), need))
    return workspace


def adg_order(g, eps_num, eps_den, workspace=None, stream=None):
    """ADG (Algorithm 1).  Returns (round int32[n] on the GPU, num_rounds int32[1])."""
    torch = _torch()
    ws = _workspace(g, workspace)
    rnd = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.device)
    nr = torch.zeros(1, dtype=torch.int32, device=g.device)
    csr = g.csr()
    rc = lib().adg_order(ctypes.byref(csr), int(eps_num), int(eps_den), _ptr(rnd), _ptr(nr), _ptr(ws),
                         ws.numel(), _stream(stream))
    _check(rc, "adg_order")
    return rnd[:g.n], nr


def jp_color(g, rounds, seed, workspace=None, stream=None):
    """JP (Algorithm 3) under <rounds, rho_R(seed)>.  Returns (color int32[n], num_colors int32[1])."""
    torch = _torch()
    ws = _workspace(g, workspace)
    r = rounds.to(device=g.device, dtype=torch.int32).contiguous()
    color = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.device)
    nc = torch.zeros(1, dtype=torch.int32, device=g.device)
    csr = g.csr()
    rc = lib().jp_color(ctypes.byref(csr), _ptr(r), int(seed) & (2**64 - 1), _ptr(color), _ptr(nc), _ptr(ws),
                        ws.numel(), _stream(stream))
    _check(rc, "jp_color")
    return color[:g.n], nc


def color_graph(g, eps_num, eps_den, seed, workspace=None, stream=None, want_rounds=True, out=None):
    """JP-ADG.  Returns (color, num_colors, round or None, num_rounds) as GPU tensors.
    ``out`` may hold preallocated (color, round, num_colors, num_rounds) tensors."""
    torch = _torch()
    ws = _workspace(g, workspace)
    if out is None:
        color = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.device)
        rnd = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.device) if want_rounds else None
        nc = torch.zeros(1, dtype=torch.int32, device=g.device)
        nr = torch.zeros(1, dtype=torch.int32, device=g.device)
    else:
        color, rnd, nc, nr = out
    csr = g.csr()
    rc = lib().color_graph(ctypes.byref(csr), int(eps_num), int(eps_den), int(seed) & (2**64 - 1), _ptr(color),
                           _ptr(rnd) if rnd is not None else ctypes.c_void_p(0), _ptr(nc), _ptr(nr), _ptr(ws),
                           ws.numel(), _stream(stream))
    _check(rc, "color_graph")
    return color[:g.n], nc, (rnd[:g.n] if rnd is not None else None), nr


def order_workspace_bytes(n, nnz):
    b = lib().adg_order_workspace_bytes(int(n), int(nnz))
    if b == 0:
        raise ValueError("invalid graph size")
    return b


def adg_order_ex(g, eps_num, eps_den, seed, variant, want_pos=True, workspace=None, stream=None):
    """ADG with a variant (SORTED, MEDIAN).  Returns (round int32[n], pos int32[n] or None,
    num_rounds int32[1]); pos ranks the vertices in the order JP colours by (larger first)."""
    torch = _torch()
    need = order_workspace_bytes(g.n, g.nnz) if want_pos else workspace_bytes(g.n, g.nnz)
    ws = workspace if workspace is not None else torch.empty(need, dtype=torch.uint8, device=g.device)
    if ws.numel() < need:
        raise ValueError("workspace too small: %d < %d bytes" % (ws.numel(), need))
    rnd = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.device)
    pos = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.device) if want_pos else None
    nr = torch.zeros(1, dtype=torch.int32, device=g.device)
    csr = g.csr()
    rc = lib().adg_order_ex(ctypes.byref(csr), int(eps_num), int(eps_den), int(seed) & (2**64 - 1), int(variant),
                            _ptr(rnd), _ptr(pos) if pos is not None else ctypes.c_void_p(0), _ptr(nr), _ptr(ws),
                            ws.numel(), _stream(stream))
    _check(rc, "adg_order_ex")
    return rnd[:g.n], (pos[:g.n] if pos is not None else None), nr


def color_graph_ex(g, eps_num, eps_den, seed, variant, workspace=None, stream=None, want_rounds=True, out=None):
    """JP-ADG with a variant (SORTED = JP-ADG-O, MEDIAN = JP-ADG-M; DEC_ITR =
    DEC-ADG-ITR's colouring instead of JP, alone or with MEDIAN).  Returns
    (color, num_colors, round or None, num_rounds) as GPU tensors.  ``out``
    may hold preallocated (color, round, num_colors, num_rounds) tensors."""
    torch = _torch()
    ws = _workspace(g, workspace)
    if out is None:
        color = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.device)
        rnd = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.device) if want_rounds else None
        nc = torch.zeros(1, dtype=torch.int32, device=g.device)
        nr = torch.zeros(1, dtype=torch.int32, device=g.device)
    else:
        color, rnd, nc, nr = out
    csr = g.csr()
    rc = lib().color_graph_ex(ctypes.byref(csr), int(eps_num), int(eps_den), int(seed) & (2**64 - 1), int(variant),
                              _ptr(color), _ptr(rnd) if rnd is not None else ctypes.c_void_p(0), _ptr(nc), _ptr(nr),
                              _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "color_graph_ex")
    return color[:g.n], nc, (rnd[:g.n] if rnd is not None else None), nr


def static_scratch_bytes():
    """Size of the static scratch color_graph_static works in."""
    return int(lib().adg_static_scratch_bytes())


def color_graph_static(g, eps_num, eps_den, seed, out, stream=None):
    """JP-ADG through the allocation-free entry point: the caller passes
    every output, preallocated, as ``out`` = (color, round or None,
    num_colors, num_rounds); the library works in its static scratch."""
    color, rnd, nc, nr = out
    csr = g.csr()
    rc = lib().color_graph_static(ctypes.byref(csr), int(eps_num), int(eps_den), int(seed) & (2**64 - 1),
                                  _ptr(color), _ptr(rnd) if rnd is not None else ctypes.c_void_p(0), _ptr(nc),
                                  _ptr(nr), _stream(stream))
    _check(rc, "color_graph_static")
    return color[:g.n], nc, (rnd[:g.n] if rnd is not None else None), nr


def get_stats(workspace, stream=None):
    st = _Stats()
    rc = lib().adg_get_stats(_ptr(workspace), workspace.numel(), ctypes.byref(st), _stream(stream))
    _check(rc, "adg_get_stats")
    return {k: int(getattr(st, k)) for k, _ in _Stats._fields_}


def validate_csr(g, workspace=None, stream=None):
    """True if g is a simple undirected graph with sorted rows (checked on the GPU)."""
    torch = _torch()
    ws = workspace if workspace is not None else torch.empty(256, dtype=torch.uint8, device=g.device)
    csr = g.csr()
    rc = lib().adg_validate_csr(ctypes.byref(csr), _ptr(ws), ws.numel(), _stream(stream))
    if rc == -1:
        return False
    _check(rc, "adg_validate_csr")
    return True


def batched_workspace_bytes(num_graphs, total_n, total_nnz):
    from .batched import batched_workspace_bytes as f
    return f(num_graphs, total_n, total_nnz)


def color_graph_batched(*args, **kwargs):
    """See batched.color_graph_batched."""
    from .batched import color_graph_batched as f
    return f(*args, **kwargs)


def profile_enable(classes):
    """Time every later launch of the named kernel classes with HIP events on
    their launch stream (see adg_profile_enable)."""
    mask = 0
    for c in classes:
        mask |= 1 << KERNEL_CLASSES.index(c)
    _check(lib().adg_profile_enable(mask), "adg_profile_enable")


def profile_read():
    """{class: (total_ms, launches)} for the launches recorded since the last read."""
    pr = _Profile()
    _check(lib().adg_profile_read(ctypes.byref(pr)), "adg_profile_read")
    return {KERNEL_CLASSES[i]: (pr.ms[i], int(pr.launches[i])) for i in range(len(KERNEL_CLASSES))
            if pr.launches[i]}
