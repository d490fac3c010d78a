"""Parity of the ADG variants on the GPU (color_graph_ex, adg_order_ex) with
the CPU oracle, bit-exact: rounds, the total order pos, colours, counts.
ADG-O = SORTED (R ordered by D at selection, then rho_R); ADG-M = MEDIAN
(R = the lower half of U by (D, rho_R)); PULL (UPDATE pulls into the
survivors' own D, no atomics) must not change any output.  GPU only."""
import itertools

import numpy as np
import pytest

import graphgen
import oracle
from checkers import check_adg_variant, check_jp_order, edges_to_csr

pytestmark = pytest.mark.gpu

SORTED, MEDIAN, PULL = 1, 2, 8
FLAGS = [SORTED, MEDIAN, SORTED | MEDIAN]
PULL_FLAGS = [PULL, PULL | SORTED, PULL | MEDIAN]


@pytest.fixture(scope="module")
def dev():
    import paper_2008_11321_amd as pkg
    import torch
    assert torch.cuda.is_available()
    assert pkg.SORTED == SORTED and pkg.MEDIAN == MEDIAN and pkg.PULL == PULL
    return pkg


def _compare(pkg, rp, col, p, q, seed, flags, label="", ws=None, order=True):
    import torch
    print("case", label, "n", rp.size - 1, "nnz", col.size, "eps", p, q, "seed", seed, "flags", flags, flush=True)
    # the oracle has no pull UPDATE: pulling must give the push output
    color, k, rnd, L, pos, st = oracle.color_graph_ex(rp, col, p, q, seed, flags & (SORTED | MEDIAN))
    g = pkg.Graph(rp, col)
    if ws is None:
        ws = torch.empty(pkg.order_workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device="cuda")
    gc, gk, gr, gL = pkg.color_graph_ex(g, p, q, seed, flags, workspace=ws)
    torch.cuda.synchronize()
    gst = pkg.get_stats(ws)
    assert int(gL.item()) == L, (label, int(gL.item()), L)
    assert np.array_equal(gr.cpu().numpy(), rnd), label
    assert int(gk.item()) == k, (label, int(gk.item()), k)
    assert np.array_equal(gc.cpu().numpy(), color), label
    assert gst["sum_active"] == st["sum_active"] and gst["cut_edges"] == st["cut_edges"]
    assert gst["error"] == 0
    if order:
        r2, gpos, L2 = pkg.adg_order_ex(g, p, q, seed, flags, workspace=ws)
        torch.cuda.synchronize()
        assert int(L2.item()) == L and np.array_equal(r2.cpu().numpy(), rnd), label
        assert np.array_equal(gpos.cpu().numpy().astype(np.int64), pos), label
    return gst


SMALL_CASES = [
    ("K1", 1, []),
    ("K2", 2, [(0, 1)]),
    ("edgeless7", 7, []),
    ("K17", 17, list(itertools.combinations(range(17), 2))),
    ("star50", 51, [(0, i) for i in range(1, 51)]),
    ("K4_9", 13, [(i, 4 + j) for i in range(4) for j in range(9)]),
    ("path31", 31, [(i, i + 1) for i in range(30)]),
    ("cycle64", 64, [(i, (i + 1) % 64) for i in range(64)]),
]


@pytest.mark.parametrize("flags", FLAGS + PULL_FLAGS)
@pytest.mark.parametrize("name,n,edges", SMALL_CASES)
def test_small_graphs(dev, name, n, edges, flags):
    rp, col = edges_to_csr(n, edges)
    for p, q in [(0, 1), (1, 10), (10**6, 1)]:
        _compare(dev, rp, col, p, q, 3, flags, name)


@pytest.mark.parametrize("flags", FLAGS)
def test_empty_graph(dev, flags):
    import torch
    g = dev.Graph(np.zeros(1, np.int64), np.zeros(0, np.int32))
    c, k, r, L = dev.color_graph_ex(g, 1, 10, 0, flags)
    torch.cuda.synchronize()
    assert int(k.item()) == 0 and int(L.item()) == 0
    r, pos, L = dev.adg_order_ex(g, 1, 10, 0, flags)
    torch.cuda.synchronize()
    assert int(L.item()) == 0


@pytest.mark.parametrize("flags", FLAGS + PULL_FLAGS)
@pytest.mark.parametrize("seed", range(3))
def test_random_graphs(dev, seed, flags):
    rng = np.random.default_rng(50 + seed)
    for trial in range(3):
        n = int(rng.integers(500, 30_000))
        if trial == 0:
            rp, col = graphgen.erdos_renyi(n, float(rng.uniform(2, 20)) / n, seed * 10 + trial)
        elif trial == 1:
            rp, col = graphgen.chung_lu(n, float(rng.uniform(4, 24)), 2.3, seed * 10 + trial)
        else:
            rp, col = graphgen.rmat(int(np.log2(n)) + 1, 8, 0.57, 0.19, 0.19, seed * 10 + trial)
        for p, q in [(1, 10), (0, 1)]:
            _compare(dev, rp, col, p, q, trial, flags, "random %d/%d" % (seed, trial))


@pytest.mark.parametrize("flags", FLAGS + PULL_FLAGS)
@pytest.mark.parametrize("scale", [16, 18])
def test_rmat_mid(dev, scale, flags):
    rp, col = graphgen.rmat_config(scale, seed=2)
    _compare(dev, rp, col, 1, 10, 2, flags, "rmat%d" % scale)


def test_median_many_equal_degrees(dev):
    """A 3-regular-like graph (cycle plus matching): nearly every D is equal,
    so the lower half is decided by rho_R through every radix pass."""
    n = 100_000
    a = np.arange(n)
    es = np.concatenate([np.stack([a, (a + 1) % n]), np.stack([a[: n // 2], a[: n // 2] + n // 2])], axis=1)
    rp, col = graphgen.from_edges(n, es[0], es[1])
    for flags in [MEDIAN, MEDIAN | SORTED]:
        _compare(dev, rp, col, 1, 10, 9, flags, "cycle+matching")


def test_chung_lu_hubs(dev):
    rp, col = graphgen.chung_lu(200_000, 32, 2.3, seed=9)
    for flags in FLAGS + PULL_FLAGS:
        _compare(dev, rp, col, 1, 10, 4, flags, "chung-lu 2e5")


def test_hub_rows_longer_than_the_chunk_threshold(dev):
    """Rows above 16384 entries go through the chunked hub kernels, whose
    same-round comparisons use the variant's key."""
    rng = np.random.default_rng(11)
    hubs, leaves = 20, 17_000
    n = hubs * (leaves + 1)
    edges = [(a, b) for a in range(hubs) for b in range(a + 1, hubs)]
    src = np.repeat(np.arange(hubs), leaves)
    dst = hubs + np.arange(hubs * leaves)
    extra = rng.integers(hubs, n, size=(5000, 2))
    es = np.concatenate([np.array(edges).T, np.stack([src, dst]), extra.T], axis=1)
    rp, col = graphgen.from_edges(n, es[0], es[1])
    for flags in FLAGS + PULL_FLAGS:
        _compare(dev, rp, col, 10**6, 1, 7, flags, "hubs, one round")
        _compare(dev, rp, col, 1, 10, 7, flags, "hubs")


def test_workspace_reused_across_variants(dev):
    import torch
    rp, col = graphgen.rmat_config(15, seed=4)
    ws = torch.empty(dev.order_workspace_bytes(rp.size - 1, col.size), dtype=torch.uint8, device="cuda")
    for flags in [MEDIAN, 0, SORTED, MEDIAN | SORTED, MEDIAN]:
        _compare(dev, rp, col, 1, 10, 5, flags, "reuse", ws=ws)


def test_rmat22_sorted_bit_exact(dev):
    """JP-ADG-O at the RMAT-22 size (n = 4,194,304, edge factor 16)."""
    rp, col = graphgen.rmat_config(22, seed=2)
    st = _compare(dev, rp, col, 1, 10, 2, SORTED, "rmat22 sorted", order=True)
    print("stats", st)


def test_rmat20_median_definition(dev):
    """ADG-M at RMAT-20, checked against the definition (every round's lower
    half recomputed from the graph) as well as the oracle."""
    import torch
    rp, col = graphgen.rmat_config(20, seed=3)
    _compare(dev, rp, col, 1, 10, 3, MEDIAN, "rmat20 median")
    g = dev.Graph(rp, col)
    r, pos, L = dev.adg_order_ex(g, 1, 10, 3, MEDIAN)
    c, k, _, _ = dev.color_graph_ex(g, 1, 10, 3, MEDIAN)
    torch.cuda.synchronize()
    r, pos, c = r.cpu().numpy(), pos.cpu().numpy().astype(np.int64), c.cpu().numpy()
    check_adg_variant(rp, col, 1, 10, 3, MEDIAN, r, pos, int(L.item()))
    check_jp_order(rp, col, pos, c)


def test_pull_alone_equals_algorithm_1(dev):
    """PULL with no other bit is JP-ADG exactly (colours, rounds, counters),
    also through adg_order_ex, on graphs with long rows and many rounds."""
    import torch
    for label, (rp, col), eps in [("rmat17", graphgen.rmat_config(17, seed=8), (1, 10)),
                                  ("chung-lu 1e5", graphgen.chung_lu(100_000, 24, 2.1, seed=5), (1, 100)),
                                  ("path 3000", edges_to_csr(3000, [(i, i + 1) for i in range(2999)]), (0, 1))]:
        p, q = eps
        _compare(dev, rp, col, p, q, 6, PULL, label)
        rho, L, st = oracle.adg(rp, col, p, q)
        g = dev.Graph(rp, col)
        r, pos, nr = dev.adg_order_ex(g, p, q, 6, PULL, want_pos=False)
        torch.cuda.synchronize()
        assert int(nr.item()) == L and np.array_equal(r.cpu().numpy(), rho), label


def test_rmat22_pull_bit_exact(dev):
    rp, col = graphgen.rmat_config(22, seed=2)
    _compare(dev, rp, col, 1, 10, 2, PULL, "rmat22 pull", order=False)
