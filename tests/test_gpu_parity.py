"""Parity of the HIP path with the CPU oracle (bit-exact: rounds, colours,
round count, colour count), through the C ABI.  GPU only."""
import itertools

import numpy as np
import pytest

import graphgen
import oracle
from checkers import check_jp, edges_to_csr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import paper_2008_11321_amd as pkg
    import torch
    assert torch.cuda.is_available()
    return pkg


def _gpu_color(pkg, rp, col, p, q, seed, variant=0):
    import torch
    g = pkg.Graph(rp, col)
    ws = torch.empty(pkg.workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device="cuda")
    if variant:
        color, nc, rnd, nr = pkg.color_graph_ex(g, p, q, seed, variant, workspace=ws)
    else:
        color, nc, rnd, nr = pkg.color_graph(g, p, q, seed, workspace=ws)
    torch.cuda.synchronize()
    st = pkg.get_stats(ws)
    return color.cpu().numpy(), int(nc.item()), rnd.cpu().numpy(), int(nr.item()), st


def _compare(pkg, rp, col, p, q, seed, label=""):
    """Every route of color_graph against the oracle: the default one (a
    graph of at most 2^17 entries goes to the one-launch engine), the
    per-round kernels (MULTI_LAUNCH), and those with JP relaxing every round
    (RELAX_ALL) or none (LEVELS_ONLY)."""
    print("case", label, "n", rp.size - 1, "nnz", col.size, "eps", p, q, "seed", seed, flush=True)
    color, k, rho, L, st = oracle.color_graph(rp, col, p, q, seed)
    for variant in (0, pkg.MULTI_LAUNCH, pkg.RELAX_ALL, pkg.LEVELS_ONLY):
        gc, gk, gr, gL, gst = _gpu_color(pkg, rp, col, p, q, seed, variant)
        lab = (label, "route", variant)
        assert gL == L, (lab, gL, L)
        assert np.array_equal(gr, rho), lab
        assert gk == k, (lab, gk, k)
        assert np.array_equal(gc, color), lab
        assert gst["sum_active"] == st["sum_active"], lab
        assert gst["cut_edges"] == st["cut_edges"], lab
        assert gst["num_rounds"] == L and gst["num_colors"] == k, lab
        assert gst["error"] == 0, lab
    return gst


SMALL_CASES = [
    ("K1", 1, []),
    ("K2", 2, [(0, 1)]),
    ("edgeless7", 7, []),
    ("K17", 17, list(itertools.combinations(range(17), 2))),
    ("star50", 51, [(0, i) for i in range(1, 51)]),
    ("K4_9", 13, [(i, 4 + j) for i in range(4) for j in range(9)]),
    ("path31", 31, [(i, i + 1) for i in range(30)]),
    ("path64", 64, [(i, i + 1) for i in range(63)]),
    ("two_triangles_isolated", 9, [(0, 1), (1, 2), (0, 2), (5, 6), (6, 7), (5, 7)]),
]


@pytest.mark.parametrize("name,n,edges", SMALL_CASES)
@pytest.mark.parametrize("eps", [(0, 1), (1, 100), (1, 10), (1, 2), (10**6, 1)])
def test_small_closed_form_graphs(dev, name, n, edges, eps):
    rp, col = edges_to_csr(n, edges)
    _compare(dev, rp, col, eps[0], eps[1], 3, name)


def test_path_many_rounds(dev):
    n = 257
    rp, col = edges_to_csr(n, [(i, i + 1) for i in range(n - 1)])
    _compare(dev, rp, col, 1, 10 * n, 4, "path257")  # 129 rounds


def test_empty_graph(dev):
    import torch
    g = dev.Graph(np.zeros(1, np.int64), np.zeros(0, np.int32))
    color, nc, rnd, nr = dev.color_graph(g, 1, 10, 1)
    torch.cuda.synchronize()
    assert int(nc.item()) == 0 and int(nr.item()) == 0 and color.numel() == 0


@pytest.mark.parametrize("seed", range(4))
def test_random_small_graphs(dev, seed):
    rng = np.random.default_rng(seed)
    for trial in range(5):
        n = int(rng.integers(50, 3000))
        kind = trial % 3
        if kind == 0:
            rp, col = graphgen.erdos_renyi(n, float(rng.uniform(0.002, 0.05)), seed * 10 + trial)
        elif kind == 1:
            rp, col = graphgen.chung_lu(n, float(rng.uniform(2, 30)), 2.3, seed * 10 + trial)
        else:
            rp, col = graphgen.rmat(int(np.log2(n)) + 1, 16, 0.57, 0.19, 0.19, seed * 10 + trial)
        for (p, q) in [(0, 1), (1, 100), (1, 10), (1, 2)]:
            _compare(dev, rp, col, p, q, trial, "rand%d/%d" % (seed, trial))


def test_er_config_bit_exact(dev):
    rp, col = graphgen.er_config(10_000, 10.0, seed=1)
    _compare(dev, rp, col, 1, 100, 1, "ER n=1e4 eps=0.01 seed=1")


@pytest.mark.parametrize("scale,eps", [(14, (1, 100)), (16, (1, 10)), (18, (1, 2))])
def test_rmat_mid(dev, scale, eps):
    rp, col = graphgen.rmat_config(scale, seed=2)
    _compare(dev, rp, col, eps[0], eps[1], 2, "rmat%d" % scale)


def test_chung_lu_hubs(dev):
    rp, col = graphgen.chung_lu(200_000, 32, 2.3, seed=9)
    _compare(dev, rp, col, 1, 10, 4, "chung-lu 2e5")


def test_rmat22_config_bit_exact(dev):
    rp, col = graphgen.rmat_config(22, seed=2)
    st = _compare(dev, rp, col, 1, 10, 2, "rmat22 eps=0.1 seed=2")
    print("stats", st)


def test_adg_order_and_jp_color_separately(dev):
    import torch
    rp, col = graphgen.rmat_config(15, seed=5)
    rho, L, _ = oracle.adg(rp, col, 1, 10)
    g = dev.Graph(rp, col)
    rnd, nr = dev.adg_order(g, 1, 10)
    torch.cuda.synchronize()
    assert int(nr.item()) == L and np.array_equal(rnd.cpu().numpy(), rho)
    color, k = oracle.jp(rp, col, rho, 11)
    gc, gk = dev.jp_color(g, rnd, 11)
    torch.cuda.synchronize()
    assert int(gk.item()) == k and np.array_equal(gc.cpu().numpy(), color)
    # JP on an arbitrary ranking (all equal = JP-R; and degree ranking = JP-LF)
    for ranking in [np.ones(rp.size - 1, np.int32), np.diff(rp).astype(np.int32) + 1]:
        color, k = oracle.jp(rp, col, ranking, 12)
        gc, gk = dev.jp_color(g, torch.from_numpy(ranking).cuda(), 12)
        torch.cuda.synchronize()
        assert int(gk.item()) == k and np.array_equal(gc.cpu().numpy(), color)
        check_jp(rp, col, ranking, 12, gc.cpu().numpy())


def test_jp_color_on_a_zeroed_workspace(dev):
    """jp_color colours every vertex as one pseudo-round in id order (its
    own ORD slot is never written): on a workspace of zeros, with the ADG
    ranking of an R-MAT graph deep enough for the relaxation of the
    pseudo-round, the colours still equal the oracle's JP (Algorithm 3)."""
    import torch
    rp, col = graphgen.rmat_config(16, seed=5)
    rho, L, _ = oracle.adg(rp, col, 1, 10)
    color, k = oracle.jp(rp, col, rho, 11)
    g = dev.Graph(rp, col)
    ws = torch.zeros(dev.workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device="cuda")
    for _ in range(2):   # and again on what the first call left
        gc, gk = dev.jp_color(g, torch.from_numpy(rho.astype(np.int32)).cuda(), 11, workspace=ws)
        torch.cuda.synchronize()
        assert dev.get_stats(ws)["error"] == 0
        assert int(gk.item()) == k and np.array_equal(gc.cpu().numpy(), color)


def test_repeatable(dev):
    import torch
    rp, col = graphgen.rmat_config(17, seed=7)
    outs = [_gpu_color(dev, rp, col, 1, 10, 7) for _ in range(3)]
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[2], outs[0][2])


def test_adjacency_order_does_not_matter(dev):
    rp, col = graphgen.chung_lu(20_000, 16, 2.3, seed=3)
    rng = np.random.default_rng(0)
    col2 = col.copy()
    for v in range(rp.size - 1):
        seg = col2[rp[v]:rp[v + 1]]
        rng.shuffle(seg)
    a = _gpu_color(dev, rp, col, 1, 10, 5)
    b = _gpu_color(dev, rp, col2, 1, 10, 5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


def test_validate_csr(dev):
    rp, col = graphgen.rmat_config(12, seed=1)
    assert dev.validate_csr(dev.Graph(rp, col))
    bad = col.copy()
    bad[0] = 0  # vertex 0 lists itself or breaks symmetry
    assert not dev.validate_csr(dev.Graph(rp, bad))


def test_hub_rows_longer_than_the_chunk_threshold(dev):
    """Rows above 16384 entries are split into chunks across wavefronts in
    UPDATE: 20 hubs forming a clique (same round, so same-round predecessors
    and successors among them), each with 17000 private leaves and a few
    random extra edges."""
    rng = np.random.default_rng(11)
    hubs, leaves = 20, 17_000
    n = hubs * (leaves + 1)
    edges = [(a, b) for a in range(hubs) for b in range(a + 1, hubs)]
    src = np.repeat(np.arange(hubs), leaves)
    dst = hubs + np.arange(hubs * leaves)
    extra = rng.integers(hubs, n, size=(5000, 2))
    es = np.concatenate([np.array(edges).T, np.stack([src, dst]), extra.T], axis=1)
    rp, col = graphgen.from_edges(n, es[0], es[1])
    assert np.diff(rp).max() > 16384
    for p, q in [(1, 10), (0, 1), (1, 2)]:
        _compare(dev, rp, col, p, q, 7, "hubs eps %d/%d" % (p, q))
    import torch
    rho, L, _ = oracle.adg(rp, col, 1, 10)
    rnd, nr = dev.adg_order(dev.Graph(rp, col), 1, 10)
    torch.cuda.synchronize()
    assert int(nr.item()) == L and np.array_equal(rnd.cpu().numpy(), rho)


def binned_limit_graph():
    """A graph for the binned decrements of D (taken at 2^22 entries and
    more): two hubs with adjacent ids, 65536 and 65537, so that their sums
    share one LDS word of the apply pass, each losing 60000 leaves in round 1
    -- a chunk of 65535 targets of their bin then holds over 47000 of one
    hub's decrements, past 2^15 in a 16-bit half.  n = 4 * 2^15 + 17 leaves
    the last bin ragged; random edges among the other vertices make up the
    entry count."""
    rng = np.random.default_rng(23)
    n = 4 * 2 ** 15 + 17
    a, b = 65536, 65537
    la = np.arange(0, 60_000)
    lb = np.concatenate([np.arange(30_000, 60_000), np.arange(66_000, 96_000)])
    rnd = rng.integers(96_000, n, size=(2, 2_300_000))
    src = np.concatenate([np.full(la.size, a), np.full(lb.size, b), rnd[0]])
    dst = np.concatenate([la, lb, rnd[1]])
    return graphgen.from_edges(n, src, dst)


def test_binned_decrements_at_the_sum_limit(dev):
    rp, col = binned_limit_graph()
    assert col.size >= 2 ** 22
    rho, _, _ = oracle.adg(rp, col, 1, 10)
    leaves = np.concatenate([np.arange(0, 60_000), np.arange(66_000, 96_000)])
    assert rho[65536] > 1 and rho[65537] > 1 and (rho[leaves] == 1).all()
    _compare(dev, rp, col, 1, 10, 3, "binned sum limit")
