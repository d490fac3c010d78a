"""Parity of DEC-ADG-ITR on the GPU (color_graph_ex with ADG_VARIANT_DEC_ITR)
with the CPU oracle, bit-exact: colours, rounds, colour count and the number
of iterations.  GPU only."""
import itertools

import numpy as np
import pytest

import graphgen
import oracle
from checkers import check_dec_itr, edges_to_csr

pytestmark = pytest.mark.gpu

MEDIAN, DEC, PULL = 2, 4, 8


@pytest.fixture(scope="module")
def dev():
    import paper_2008_11321_amd as pkg
    import torch
    assert torch.cuda.is_available()
    assert pkg.DEC_ITR == DEC
    return pkg


def _compare(pkg, rp, col, p, q, seed, flags=0, label="", ws=None):
    import torch
    print("case", label, "n", rp.size - 1, "nnz", col.size, "eps", p, q, "seed", seed, "flags", flags, flush=True)
    color, k, rho, L, step, it = oracle.color_graph_dec(rp, col, p, q, seed, flags & MEDIAN)
    g = pkg.Graph(rp, col)
    if ws is None:
        ws = torch.empty(pkg.workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device="cuda")
    gc, gk, gr, gL = pkg.color_graph_ex(g, p, q, seed, DEC | flags, workspace=ws)
    torch.cuda.synchronize()
    st = pkg.get_stats(ws)
    assert int(gL.item()) == L, label
    assert np.array_equal(gr.cpu().numpy(), rho), label
    assert int(gk.item()) == k, (label, int(gk.item()), k)
    assert np.array_equal(gc.cpu().numpy(), color), label
    assert st["jp_levels"] == it, (label, st["jp_levels"], it)
    assert st["error"] == 0
    return st


SMALL_CASES = [
    ("K1", 1, []),
    ("K2", 2, [(0, 1)]),
    ("edgeless7", 7, []),
    ("K17", 17, list(itertools.combinations(range(17), 2))),
    ("star50", 51, [(0, i) for i in range(1, 51)]),
    ("K4_9", 13, [(i, 4 + j) for i in range(4) for j in range(9)]),
    ("path31", 31, [(i, i + 1) for i in range(30)]),
    ("cycle64", 64, [(i, (i + 1) % 64) for i in range(64)]),
    ("K80", 80, list(itertools.combinations(range(80), 2))),
]


@pytest.mark.parametrize("name,n,edges", SMALL_CASES)
def test_small_graphs(dev, name, n, edges):
    rp, col = edges_to_csr(n, edges)
    for p, q in [(0, 1), (1, 10), (10**6, 1)]:
        _compare(dev, rp, col, p, q, 3, 0, name)
        _compare(dev, rp, col, p, q, 3, MEDIAN, name)


def test_empty_graph(dev):
    import torch
    g = dev.Graph(np.zeros(1, np.int64), np.zeros(0, np.int32))
    c, k, r, L = dev.color_graph_ex(g, 1, 10, 0, DEC)
    torch.cuda.synchronize()
    assert int(k.item()) == 0 and int(L.item()) == 0


@pytest.mark.parametrize("seed", range(3))
def test_random_graphs(dev, seed):
    rng = np.random.default_rng(90 + seed)
    for trial in range(3):
        n = int(rng.integers(300, 20_000))
        if trial == 0:
            rp, col = graphgen.erdos_renyi(n, float(rng.uniform(2, 30)) / n, seed * 10 + trial)
        elif trial == 1:
            rp, col = graphgen.chung_lu(n, float(rng.uniform(4, 24)), 2.3, seed * 10 + trial)
        else:
            rp, col = graphgen.rmat(int(np.log2(n)) + 1, 8, 0.57, 0.19, 0.19, seed * 10 + trial)
        for p, q in [(1, 10), (0, 1), (10**6, 1)]:
            _compare(dev, rp, col, p, q, trial, 0, "random %d/%d" % (seed, trial))
    # the definition, iteration by iteration, on a small one
    rp, col = graphgen.chung_lu(400, 8, 2.3, seed)
    import torch
    g = dev.Graph(rp, col)
    c, k, r, L = dev.color_graph_ex(g, 1, 10, seed, DEC)
    torch.cuda.synchronize()
    _, _, _, _, step, _ = oracle.color_graph_dec(rp, col, 1, 10, seed)
    check_dec_itr(rp, col, r.cpu().numpy(), seed, c.cpu().numpy(), step)


@pytest.mark.parametrize("scale", [16, 18])
def test_rmat_mid(dev, scale):
    rp, col = graphgen.rmat_config(scale, seed=2)
    _compare(dev, rp, col, 1, 10, 2, 0, "rmat%d" % scale)
    _compare(dev, rp, col, 1, 10, 2, MEDIAN, "rmat%d median" % scale)
    _compare(dev, rp, col, 1, 10, 2, PULL, "rmat%d pull" % scale)


def test_chung_lu_hubs(dev):
    rp, col = graphgen.chung_lu(200_000, 32, 2.3, seed=9)
    _compare(dev, rp, col, 1, 10, 4, 0, "chung-lu 2e5")


def test_hub_rows_longer_than_the_chunk_threshold(dev):
    """Rows above 16384 entries (UPDATE's chunked hub kernels), and long
    same-round rows walked by whole wavefronts: 20 hubs forming a clique,
    each with 17000 private leaves."""
    rng = np.random.default_rng(11)
    hubs, leaves = 20, 17_000
    n = hubs * (leaves + 1)
    edges = [(a, b) for a in range(hubs) for b in range(a + 1, hubs)]
    src = np.repeat(np.arange(hubs), leaves)
    dst = hubs + np.arange(hubs * leaves)
    extra = rng.integers(hubs, n, size=(5000, 2))
    es = np.concatenate([np.array(edges).T, np.stack([src, dst]), extra.T], axis=1)
    rp, col = graphgen.from_edges(n, es[0], es[1])
    for p, q in [(1, 10), (10**6, 1)]:
        _compare(dev, rp, col, p, q, 7, 0, "hubs")


def test_workspace_reused_with_jp(dev):
    import torch
    rp, col = graphgen.rmat_config(15, seed=4)
    ws = torch.empty(dev.workspace_bytes(rp.size - 1, col.size), dtype=torch.uint8, device="cuda")
    g = dev.Graph(rp, col)
    for flags in [0, MEDIAN, 0]:
        _compare(dev, rp, col, 1, 10, 5, flags, "reuse", ws=ws)
        c, k, _, _ = dev.color_graph(g, 1, 10, 5, workspace=ws)
        torch.cuda.synchronize()
        oc, ok, _, _, _ = oracle.color_graph(rp, col, 1, 10, 5)
        assert np.array_equal(c.cpu().numpy(), oc) and int(k.item()) == ok


def test_rmat22_bit_exact(dev):
    """DEC-ADG-ITR at the RMAT-22 size (n = 4,194,304, edge factor 16)."""
    rp, col = graphgen.rmat_config(22, seed=2)
    st = _compare(dev, rp, col, 1, 10, 2, 0, "rmat22 dec")
    print("stats", st)
