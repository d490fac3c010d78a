"""C ABI checks that need no GPU: the library loads, exports every function
that include/adg.h declares, and rejects bad arguments before touching the
device."""
import ctypes
import os
import re

import pytest

import paper_2008_11321_amd as pkg

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "adg.h")


def declared_functions():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ["adg_workspace_bytes", "adg_order", "jp_color", "color_graph", "adg_get_stats", "adg_validate_csr",
              "adg_error_string"]:
        assert f in names


def test_library_exports_every_declared_symbol():
    L = pkg.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_workspace_size_and_errors_without_gpu():
    L = pkg.lib()
    assert L.adg_workspace_bytes(-1, 0) == 0
    small = L.adg_workspace_bytes(10, 20)
    big = L.adg_workspace_bytes(10_000, 100_000)
    assert 0 < small < big
    assert L.adg_error_string(0) == b"ok"
    assert L.adg_error_string(-1) == b"invalid argument"
    # null graph pointer and bad eps are rejected on the host
    assert L.adg_order(None, 1, 10, None, None, None, 0, None) == -1
    csr = pkg._Csr(5, 0, 0, 0)
    assert L.adg_order(ctypes.byref(csr), -1, 10, None, None, None, 0, None) == -1
    assert L.adg_order(ctypes.byref(csr), 1, 0, None, None, None, 0, None) == -1
    assert L.color_graph(ctypes.byref(csr), 1, 10, 0, None, None, None, None, None, 0, None) == -1


def test_no_cpu_fallback():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    g = None
    with pytest.raises(RuntimeError):
        pkg.Graph([0, 0], [])


def test_batched_entry_points_reject_bad_arguments_without_gpu():
    import paper_2008_11321_amd.batched as bt
    L = bt._lib()
    assert L.adg_batched_workspace_bytes(-1, 0, 0) == 0
    assert 0 < L.adg_batched_workspace_bytes(4, 100, 1000) < L.adg_batched_workspace_bytes(4, 10_000, 100_000)
    c = L.adg_batched_default_config()
    assert c.block_threads in (256, 512, 1024) and c.blocks_per_cu >= 1
    args = (1, 10, 0, None, None, None, None)
    assert L.color_graph_batched(None, *args, None, None, 0, None) == -1
    # sizes without arrays
    b = bt._Batch(2, 10, 20, None, None, None)
    assert L.color_graph_batched(ctypes.byref(b), *args, None, None, 0, None) == -1
    # an empty batch is a no-op that needs no device memory
    b0 = bt._Batch(0, 0, 0, None, None, None)
    assert L.color_graph_batched(ctypes.byref(b0), *args, None, None, 0, None) == 0
    # a batch of two graphs (fake, never dereferenced on the host)
    fake = 1 << 20
    b2 = bt._Batch(2, 10, 20, fake, fake, fake)
    out = (1, 10, 0, fake, None, fake, None)
    bad = bt.BatchConfig(300, 1, 0)
    assert L.color_graph_batched(ctypes.byref(b2), *out, ctypes.byref(bad), fake, 1 << 30, None) == -1
    bad = bt.BatchConfig(256, 0, 0)
    assert L.color_graph_batched(ctypes.byref(b2), *out, ctypes.byref(bad), fake, 1 << 30, None) == -1
    good = bt.BatchConfig(256, 2, 1)
    assert L.color_graph_batched(ctypes.byref(b2), *out, ctypes.byref(good), fake, 16, None) == -2
    assert L.color_graph_batched(ctypes.byref(b2), *out, ctypes.byref(good), fake + 8, 1 << 30, None) == -2
    assert L.color_graph_batched(ctypes.byref(b2), -1, 10, 0, fake, None, fake, None, None, fake, 1 << 30,
                                 None) == -1


def test_variant_entry_points_reject_bad_arguments_without_gpu():
    L = pkg.lib()
    assert L.adg_order_workspace_bytes(-1, 0) == 0
    assert L.adg_order_workspace_bytes(1000, 10_000) > L.adg_workspace_bytes(1000, 10_000)
    fake = 1 << 20
    csr = pkg._Csr(5, 8, fake, fake)
    ws = L.adg_workspace_bytes(5, 8)
    # unknown variant bits
    assert L.color_graph_ex(ctypes.byref(csr), 1, 10, 0, 128, fake, None, None, None, fake, ws, None) == -1
    # JP's schedule bits: not together, not with DEC-ADG-ITR, not for adg_order_ex
    both = pkg.RELAX_ALL | pkg.LEVELS_ONLY
    assert L.color_graph_ex(ctypes.byref(csr), 1, 10, 0, both, fake, None, None, None, fake, ws, None) == -1
    for bit in (pkg.RELAX_ALL, pkg.LEVELS_ONLY):
        assert L.color_graph_ex(ctypes.byref(csr), 1, 10, 0, bit | pkg.DEC_ITR, fake, None, None, None, fake, ws,
                                None) == -1
        assert L.adg_order_ex(ctypes.byref(csr), 1, 10, 0, bit, fake, None, None, fake, ws, None) == -1
    assert L.adg_order_ex(ctypes.byref(csr), 1, 10, 0, 16, fake, None, None, fake, ws, None) == -1
    # DEC-ADG-ITR colours only, and not with ADG-O's order
    assert L.color_graph_ex(ctypes.byref(csr), 1, 10, 0, 5, fake, None, None, None, fake, ws, None) == -1
    assert L.adg_order_ex(ctypes.byref(csr), 1, 10, 0, 4, fake, None, None, fake, ws, None) == -1
    # a pos output needs the larger workspace
    assert L.adg_order_ex(ctypes.byref(csr), 1, 10, 0, 1, fake, fake, None, fake, ws, None) == -2
    assert L.adg_order_ex(None, 1, 10, 0, 1, fake, fake, None, fake, ws, None) == -1


def test_profile_class_names_match_the_binding():
    """The Python class list and the library's class names agree index by
    index (adg_profile_enable takes bits by these indices)."""
    L = pkg.lib()
    L.adg_kernel_class_name.restype = ctypes.c_char_p
    L.adg_kernel_class_name.argtypes = [ctypes.c_int]
    for i, name in enumerate(pkg.KERNEL_CLASSES):
        assert L.adg_kernel_class_name(i).decode() == name, i
    assert L.adg_kernel_class_name(len(pkg.KERNEL_CLASSES)).decode() == ""
    assert len(pkg.KERNEL_CLASSES) <= 32


def test_threshold_product_is_exact_beyond_64_bits(tmp_path):
    """Algorithm 1's threshold floor((q+p) S / (q N)) as the kernels compute it
    (the header both paths include, built for the host) against Python's exact
    integers, also where (q+p) S passes 2^64: p, q up to 2^31 - 1 and S up to
    2^37 adjacency entries are accepted at the boundary."""
    import random
    import subprocess
    csrc = os.path.join(os.path.dirname(pkg.__file__), "csrc")
    src = tmp_path / "t.cpp"
    src.write_text('#include "adg_intmath.h"\n#include <cstdio>\n'
                   'int main() { unsigned long long a, b, d, c;\n'
                   '  while (scanf("%llu %llu %llu %llu", &a, &b, &d, &c) == 4)\n'
                   '    printf("%llu\\n", (unsigned long long)adg::mul_div_floor_sat(a, b, d, c));\n'
                   '  return 0; }\n')
    exe = tmp_path / "t"
    subprocess.run(["hipcc", "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17", "-I", csrc, str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    M = 2**64 - 1
    rng = random.Random(7)
    cases = [(3, 5, 2, 100), (2**32, 2**37, 1, M), (2**32, 2**37, 2**62, M), (2**32 - 2, 2**37 - 1, 3 * 2**30, M),
             (2**32, 2**36 + 12345, 2**31 - 1, 2**31 - 1), (1, M, 1, M), (M, M, M, M), (M, M, M - 1, M),
             (2**33, 2**33, 2**2, M), (2**31 + 5, 2**40 + 3, 2**31 * 7, M), (0, 5, 3, M), (5, 0, 3, M)]
    for _ in range(3000):
        q = rng.randrange(1, 2**31)
        p = rng.randrange(0, 2**31)
        S = rng.randrange(0, 2**38)
        N = rng.randrange(1, 2**31)
        cases.append((q + p, S, q * N, rng.choice([2**31 - 1, M])))
    for _ in range(1000):
        a, b, d = rng.randrange(0, 2**64), rng.randrange(0, 2**64), rng.randrange(1, 2**64)
        cases.append((a, b, d, M))
    inp = "".join("%d %d %d %d\n" % c for c in cases)
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split()
    assert len(out) == len(cases)
    for (a, b, d, cap), got in zip(cases, out):
        assert int(got) == min(a * b // d, cap), (a, b, d, cap)
