"""The RMAT-26 configuration (n = 2^26, edge factor 16, eps = 1/10, seed 3:
the bench's rmat26 workload, in the launch configuration bench.py times),
compared element by element with the serial CPU oracle at eps = 1/100, 1/10
and 1/2 (the three oracle runs start on host threads when the graph is made
and finish while the other tests use the GPU), and checked on the GPU output
against properties that define the result at any size:

* ADG (Algorithm 1): for every round l, with U_l = {v : round(v) >= l} and
  deg_U recomputed from the graph, exactly the vertices of U_l with
  q |U_l| deg_U <= (q + p) sum(deg_U) get round l;
* JP (Algorithm 3): the colouring is proper and every vertex has the
  smallest colour >= 1 that none of its predecessors under
  <round, rho_R(seed)> has (GetColor);
* the counts the library reports (rounds, colours, sum |U_l|);
* ADG-O (sorted R): JP's total order pos ranks the vertices by (round, D at
  selection = deg_U, rho_R), and the colouring follows pos;
* ADG-M (median): every round removes exactly the ceil(|U_l|/2) vertices of
  U_l lowest by (deg_U, rho_R).

The checks are plain torch reductions on the GPU, chunked by adjacency
entries; the graph is generated on the host as for the bench.  GPU only."""
import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

CHUNK = 1 << 28   # adjacency entries per checking pass
VCHUNK = 1 << 23  # and vertices (the colour table of a pass is vertices x colours bytes)
MASK32 = 0xFFFFFFFF


def _tiebreak_torch(torch, seed, v):
    """rho_R(v) = fmix32(v ^ k), k = low 32 bits of the first SplitMix64
    output from state seed (the published definitions, in int64 arithmetic
    whose low 32 bits wrap as uint32 arithmetic does)."""
    z = (int(seed) + 0x9E3779B97F4A7C15) & (2**64 - 1)
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & (2**64 - 1)
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & (2**64 - 1)
    k = (z ^ (z >> 31)) & MASK32
    h = (v.to(torch.int64) ^ k) & MASK32
    h = h ^ (h >> 16)
    h = (h * 0x85EBCA6B) & MASK32
    h = h ^ (h >> 13)
    h = (h * 0xC2B2AE35) & MASK32
    return h ^ (h >> 16)


def _chunks(rp_host, n):
    """Vertex ranges [v0, v1) of at most VCHUNK vertices whose rows hold at
    most about CHUNK entries (a longer row forms a range of its own)."""
    bounds = [0]
    while bounds[-1] < n:
        v0 = bounds[-1]
        v1 = int(np.searchsorted(rp_host, rp_host[v0] + CHUNK, side="right")) - 1
        bounds.append(min(n, v0 + VCHUNK, max(v1, v0 + 1)))
    return list(zip(bounds[:-1], bounds[1:]))


def check_definition(torch, rp, col_d, rnd, color, p, q, seed, device, median=False, pos=None):
    """Raise AssertionError unless (rnd, color) is ADG's rounds (ADG-M's with
    median) and JP's colouring on the graph (host row_ptr rp, col_d on
    `device`); with pos, JP's order is pos and pos must be ADG-O's order.
    Returns sum |U_l|."""
    n = rp.size - 1
    L, K = int(rnd.max()), int(color.max())
    rnd = rnd.to(torch.int64)
    color = color.to(torch.int64)
    assert int(rnd.min()) >= 1 and int(color.min()) >= 1
    rpd = torch.as_tensor(rp, device=device)
    deg = rpd[1:] - rpd[:-1]
    chunks = _chunks(rp, n)
    h = _tiebreak_torch(torch, seed, torch.arange(n, device=device))
    key = (rnd << 32) | h if pos is None else pos.to(torch.int64)
    dsel = torch.zeros(n, dtype=torch.int64, device=device)

    def rows(v0, v1):
        e0, e1 = int(rp[v0]), int(rp[v1])
        src = torch.repeat_interleave(torch.arange(v0, v1, device=device), deg[v0:v1])
        return src, col_d[e0:e1].to(torch.int64)

    # ADG: the selection rule of every round
    sum_active = 0
    for l in range(1, L + 1):
        inU = rnd >= l
        degU = torch.zeros(n, dtype=torch.int64, device=device)
        for v0, v1 in chunks:
            src, c = rows(v0, v1)
            both = inU[src] & inU[c]
            degU.index_add_(0, src[both], torch.ones(int(both.sum()), dtype=torch.int64, device=device))
            del src, c, both
        size_u = int(inU.sum())
        if median:
            mk = (degU << 32) | h
            kth = torch.sort(mk[inU]).values[(size_u + 1) // 2 - 1]
            sel = mk <= kth
        else:
            cnt = int(degU[inU].sum())
            sel = (q * size_u) * degU <= (q + p) * cnt
        assert torch.equal(sel[inU], (rnd == l)[inU]), "round %d" % l
        dsel = torch.where(rnd == l, degU, dsel)
        sum_active += size_u
        print("round", l, "|U|", size_u, "removed", int((rnd == l).sum()), flush=True)

    if pos is not None:
        # ADG-O: ranks by (round, D at selection, rho_R), stable sorts from the last key
        order = torch.argsort(h, stable=True)
        order = order[torch.argsort(dsel[order], stable=True)]
        order = order[torch.argsort(rnd[order], stable=True)]
        expect = torch.empty_like(order)
        expect[order] = torch.arange(n, device=device)
        assert torch.equal(expect, pos.to(torch.int64)), "ADG-O order"

    # JP: proper, and the colour is the first one missing among the predecessors
    width = K + 2
    for v0, v1 in chunks:
        src, c = rows(v0, v1)
        assert not bool((color[src] == color[c]).any()), "improper in [%d, %d)" % (v0, v1)
        pred = key[c] > key[src]
        used = torch.zeros((v1 - v0, width), dtype=torch.bool, device=device)
        used[src[pred] - v0, color[c[pred]]] = True
        first_missing = (~used[:, 1:]).to(torch.uint8).argmax(dim=1) + 1
        assert torch.equal(first_missing, color[v0:v1]), "GetColor in [%d, %d)" % (v0, v1)
        del src, c, pred, used
    return sum_active


def check_adg_by_removal(torch, rp, col_d, rnd, p, q, device):
    """Algorithm 1's selection rule for every round, with deg_U kept by
    definition as it shrinks: it starts as the degree, and once round l is
    checked every edge from a vertex of R_l to a vertex still in U takes one
    off that vertex's count.  Each row is read once in all, so this suits
    runs with many rounds (small eps).  Returns sum |U_l|."""
    n = rp.size - 1
    L = int(rnd.max())
    rnd = rnd.to(torch.int64)
    rpd = torch.as_tensor(rp, device=device)
    deg = rpd[1:] - rpd[:-1]
    degU = deg.clone()
    order = torch.argsort(rnd, stable=True)
    starts = [0] + torch.cumsum(torch.bincount(rnd, minlength=L + 1)[1:], 0).tolist()
    sum_active = 0
    for l in range(1, L + 1):
        inU = rnd >= l
        size_u = n - starts[l - 1]
        assert size_u == int(inU.sum())
        cnt = int(degU[inU].sum())
        sel = (q * size_u) * degU <= (q + p) * cnt
        assert torch.equal(sel[inU], (rnd == l)[inU]), "round %d" % l
        sum_active += size_u
        # remove R_l: its edges to U_{l+1}
        verts = order[starts[l - 1]:starts[l]]
        dv = deg[verts]
        csum = torch.cumsum(dv, 0)
        b0 = 0
        while b0 < verts.numel():
            base = int(csum[b0 - 1]) if b0 else 0
            b1 = int(torch.searchsorted(csum, base + CHUNK, right=True))
            b1 = max(b1, b0 + 1)
            vv, dd = verts[b0:b1], dv[b0:b1]
            tot = int(dd.sum())
            if tot:
                first = torch.repeat_interleave(rpd[vv], dd)
                within = torch.arange(tot, device=device) - torch.repeat_interleave(torch.cumsum(dd, 0) - dd, dd)
                c = col_d[first + within].to(torch.int64)
                keep = rnd[c] > l
                degU.index_add_(0, c[keep], torch.full((int(keep.sum()),), -1, dtype=torch.int64, device=device))
                del first, within, c, keep
            b0 = b1
        if l % 16 == 0 or l == L:
            print("round", l, "|U|", size_u, "removed", starts[l] - starts[l - 1], flush=True)
    return sum_active


def check_jp(torch, rp, col_d, rnd, color, seed, device):
    """JP (Algorithm 3) under <round, rho_R(seed)>: proper, GetColor at every
    vertex."""
    n = rp.size - 1
    K = int(color.max())
    assert int(color.min()) >= 1
    rnd = rnd.to(torch.int64)
    color = color.to(torch.int64)
    rpd = torch.as_tensor(rp, device=device)
    deg = rpd[1:] - rpd[:-1]
    key = (rnd << 32) | _tiebreak_torch(torch, seed, torch.arange(n, device=device))
    width = K + 2
    for v0, v1 in _chunks(rp, n):
        e0, e1 = int(rp[v0]), int(rp[v1])
        src = torch.repeat_interleave(torch.arange(v0, v1, device=device), deg[v0:v1])
        c = col_d[e0:e1].to(torch.int64)
        assert not bool((color[src] == color[c]).any()), "improper in [%d, %d)" % (v0, v1)
        pred = key[c] > key[src]
        used = torch.zeros((v1 - v0, width), dtype=torch.bool, device=device)
        used[src[pred] - v0, color[c[pred]]] = True
        first_missing = (~used[:, 1:]).to(torch.uint8).argmax(dim=1) + 1
        assert torch.equal(first_missing, color[v0:v1]), "GetColor in [%d, %d)" % (v0, v1)
        del src, c, pred, used


EPS_ALL = [(1, 100), (1, 10), (1, 2)]


@pytest.fixture(scope="module")
def rmat26():
    """The graph on the GPU, and the serial oracle's JP-ADG at the three eps
    of the configuration started on host threads (the C oracle runs outside
    the interpreter lock), so that they run while the GPU tests do."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    import oracle
    import paper_2008_11321_amd as pkg
    assert torch.cuda.is_available()
    print("case rmat26 full size: generating", flush=True)
    rp, col = graphgen.rmat_config(26, seed=3)
    g = pkg.Graph(rp, col)
    print("n", g.n, "nnz", g.nnz, flush=True)
    pool = ThreadPoolExecutor(max_workers=len(EPS_ALL))
    runs = {pq: pool.submit(oracle.color_graph, rp, col, pq[0], pq[1], 3) for pq in EPS_ALL}
    yield pkg, rp, g, runs
    pool.shutdown(wait=True, cancel_futures=True)


def test_rmat26_at_full_size(rmat26):
    import torch
    pkg, rp, g, _ = rmat26
    seed, p, q = 3, 1, 10
    ws = torch.empty(pkg.workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device="cuda")
    color, nc, rnd, nr = pkg.color_graph(g, p, q, seed, workspace=ws)
    torch.cuda.synchronize()
    st = pkg.get_stats(ws)
    print("coloured: rounds", int(nr.item()), "colours", int(nc.item()), st, flush=True)
    assert st["error"] == 0
    assert int(rnd.max()) == int(nr.item()) and int(color.max()) == int(nc.item())
    del ws
    sum_active = check_definition(torch, rp, g.col_idx, rnd, color, p, q, seed, "cuda")
    assert sum_active == st["sum_active"]
    print("rmat26 checked", flush=True)


def test_rmat26_sorted_and_median_at_full_size(rmat26):
    """JP-ADG-O (colours and the total order) and ADG-M with JP-ADG-M."""
    import torch
    pkg, rp, g, _ = rmat26
    seed, p, q = 3, 1, 10
    ws = torch.empty(pkg.order_workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device="cuda")
    color, nc, rnd, nr = pkg.color_graph_ex(g, p, q, seed, pkg.SORTED, workspace=ws)
    r2, pos, _ = pkg.adg_order_ex(g, p, q, seed, pkg.SORTED, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(r2, rnd)
    print("sorted: rounds", int(nr.item()), "colours", int(nc.item()), flush=True)
    check_definition(torch, rp, g.col_idx, rnd, color, p, q, seed, "cuda", pos=pos)
    del r2, pos, color, rnd
    color, nc, rnd, nr = pkg.color_graph_ex(g, p, q, seed, pkg.MEDIAN, workspace=ws)
    torch.cuda.synchronize()
    print("median: rounds", int(nr.item()), "colours", int(nc.item()), flush=True)
    assert int(nr.item()) == g.n.bit_length()
    check_definition(torch, rp, g.col_idx, rnd, color, p, q, seed, "cuda", median=True)
    print("rmat26 variants checked", flush=True)


@pytest.mark.parametrize("p,q", [(1, 100), (1, 2)])
def test_rmat26_other_eps_at_full_size(rmat26, p, q):
    """The other eps of the RMAT-26 configuration (the bench's rmat26_e001 and
    rmat26_e05 workloads): eps = 1/100 takes many rounds."""
    import torch
    pkg, rp, g, _ = rmat26
    seed = 3
    print("case rmat26 eps %d/%d" % (p, q), flush=True)
    ws = torch.empty(pkg.workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device="cuda")
    color, nc, rnd, nr = pkg.color_graph(g, p, q, seed, workspace=ws)
    torch.cuda.synchronize()
    st = pkg.get_stats(ws)
    print("coloured: rounds", int(nr.item()), "colours", int(nc.item()), st, flush=True)
    assert st["error"] == 0
    assert int(rnd.max()) == int(nr.item()) and int(color.max()) == int(nc.item())
    del ws
    assert check_adg_by_removal(torch, rp, g.col_idx, rnd, p, q, "cuda") == st["sum_active"]
    check_jp(torch, rp, g.col_idx, rnd, color, seed, "cuda")
    print("rmat26 eps %d/%d checked" % (p, q), flush=True)


@pytest.mark.parametrize("p,q", EPS_ALL)
def test_rmat26_equals_the_oracle(rmat26, p, q):
    """Element by element against the serial CPU oracle (Algorithm 1 step by
    step, then greedy colouring in decreasing <round, rho_R> order) at every
    eps of the configuration: rounds, colours, L, the colour count and the
    counters sum |U_l| and cut edges.  JP runs with each of its schedules:
    the default (levels, deep rounds relaxed), every round relaxed, and
    levels only."""
    import torch
    pkg, rp, g, runs = rmat26
    seed = 3
    oc, ok, orho, oL, ost = None, None, None, None, None
    ws = torch.empty(pkg.workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device="cuda")
    for variant in (0, pkg.RELAX_ALL, pkg.LEVELS_ONLY):
        print("case rmat26 eps %d/%d variant %d vs the oracle" % (p, q, variant), flush=True)
        color, nc, rnd, nr = pkg.color_graph_ex(g, p, q, seed, variant, workspace=ws)
        torch.cuda.synchronize()
        st = pkg.get_stats(ws)
        colour_h, rnd_h = color.cpu().numpy(), rnd.cpu().numpy()
        del color, rnd
        if oc is None:
            oc, ok, orho, oL, ost = runs[(p, q)].result(timeout=600)
        print("gpu: rounds", int(nr.item()), "colours", int(nc.item()), "oracle: rounds", oL, "colours", ok, flush=True)
        assert st["error"] == 0
        assert int(nr.item()) == oL and st["num_rounds"] == oL
        assert int(nc.item()) == ok and st["num_colors"] == ok
        assert st["sum_active"] == ost["sum_active"] and st["cut_edges"] == ost["cut_edges"]
        bad_r = int((rnd_h != orho).sum())
        bad_c = int((colour_h != oc).sum())
        assert bad_r == 0, "variant %d: %d rounds differ" % (variant, bad_r)
        assert bad_c == 0, "variant %d: %d colours differ" % (variant, bad_c)
    del ws
