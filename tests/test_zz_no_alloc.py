"""The allocation-free entry point color_graph_static (callers that cannot
allocate): the same result as color_graph, element by element, on two calls
in a row (the second on a smaller graph, so that the static scratch still
holds the first call's state), and the size check that keeps a graph whose
workspace exceeds the scratch from running."""
import ctypes

import numpy as np
import pytest

import graphgen


def _run_pair(pkg, torch, rp, col, p, q, seed):
    g = pkg.Graph(rp, col)
    n = g.n
    ref = pkg.color_graph(g, p, q, seed)
    out = (torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda"),
           torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda"),
           torch.zeros(1, dtype=torch.int32, device="cuda"), torch.zeros(1, dtype=torch.int32, device="cuda"))
    got = pkg.color_graph_static(g, p, q, seed, out)
    torch.cuda.synchronize()
    return ref, got


@pytest.mark.gpu
def test_static_entry_equals_color_graph_on_two_calls():
    import torch

    import oracle
    import paper_2008_11321_amd as pkg
    assert torch.cuda.is_available()
    cases = [("rmat18", graphgen.rmat_config(18, seed=2), 1, 10, 2),      # about half the scratch
             ("er1e4", graphgen.er_config(10_000, 10.0, seed=1), 1, 100, 1)]   # smaller, after it
    for name, (rp, col), p, q, seed in cases:
        n, nnz = rp.size - 1, col.size
        assert pkg.workspace_bytes(n, nnz) <= pkg.static_scratch_bytes()
        print("case", name, "n", n, "nnz", nnz, flush=True)
        ref, got = _run_pair(pkg, torch, rp, col, p, q, seed)
        for a, b, what in [(ref[0], got[0], "colours"), (ref[2], got[2], "rounds")]:
            assert torch.equal(a, b), "%s: %s differ at %d vertices" % (name, what, int((a != b).sum()))
        assert int(ref[1].item()) == int(got[1].item()) and int(ref[3].item()) == int(got[3].item()), name
        oc, ok, orho, oL, _ = oracle.color_graph(rp, col, p, q, seed)
        assert np.array_equal(got[0].cpu().numpy(), oc) and np.array_equal(got[2].cpu().numpy(), orho), name
        assert int(got[1].item()) == ok and int(got[3].item()) == oL, name


def test_static_entry_rejects_a_graph_larger_than_its_scratch():
    """Checked on the host before any device work (runs without a GPU)."""
    import paper_2008_11321_amd as pkg
    L = pkg.lib()
    cap = pkg.static_scratch_bytes()
    assert cap == 128 << 20
    fake = 1 << 20
    n, nnz = 1 << 20, 1 << 26   # about 0.5 GB of workspace
    assert L.adg_workspace_bytes(n, nnz) > cap
    csr = pkg._Csr(n, nnz, fake, fake)
    rc = L.color_graph_static(ctypes.byref(csr), 1, 10, 0, fake, None, fake, fake, None)
    assert rc == -6
    assert b"static scratch" in L.adg_error_string(-6)
    assert L.color_graph_static(None, 1, 10, 0, fake, None, fake, fake, None) == -1
    small = pkg._Csr(5, 8, fake, fake)
    assert L.color_graph_static(ctypes.byref(small), 1, 0, 0, fake, None, fake, fake, None) == -1
