"""Batched JP-ADG (color_graph_batched): every graph of a batch must come out
exactly as the CPU oracle colours it alone (rounds, colours, round and colour
counts), whatever the launch shape, and the call must replay correctly from a
captured HIP graph.  GPU only."""
import itertools

import numpy as np
import pytest

import graphgen
import oracle
from checkers import edges_to_csr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bt():
    import torch
    import paper_2008_11321_amd.batched as b
    assert torch.cuda.is_available()
    return b


def _mixed_graphs(seed, count, n_hi=3000):
    rng = np.random.default_rng(seed)
    out = [edges_to_csr(1, []), edges_to_csr(0, []), edges_to_csr(7, []),
           edges_to_csr(17, list(itertools.combinations(range(17), 2))),
           edges_to_csr(51, [(0, i) for i in range(1, 51)]),
           edges_to_csr(65, [(i, i + 1) for i in range(64)])]
    for t in range(count):
        n = int(rng.integers(2, n_hi))
        kind = t % 3
        if kind == 0:
            out.append(graphgen.erdos_renyi(n, float(rng.uniform(0.002, 0.05)), seed * 100 + t))
        elif kind == 1:
            out.append(graphgen.chung_lu(n, float(min(rng.uniform(2, 40), n - 1)), 2.3, seed * 100 + t))
        else:
            out.append(graphgen.rmat(max(1, int(np.log2(n))), 16, 0.57, 0.19, 0.19, seed * 100 + t))
    return out


def _run(bt, batch, p, q, seed, config=None):
    import torch
    color, nc, rnd, nr = bt.color_graph_batched(batch, p, q, seed, config=config, want_rounds=True)
    torch.cuda.synchronize()
    return color.cpu().numpy(), nc.cpu().numpy(), rnd.cpu().numpy(), nr.cpu().numpy()


def _check_all(batch, graphs, res, p, q, seed, label, which=None):
    color, nc, rnd, nr = res
    cs, rs = batch.split(color), batch.split(rnd)
    for g in (range(len(graphs)) if which is None else which):
        rp, col = graphs[g]
        oc, ok, orho, oL, _ = oracle.color_graph(rp, col, p, q, seed)
        assert nr[g] == oL, (label, g, nr[g], oL)
        assert np.array_equal(rs[g], orho), (label, g)
        assert nc[g] == ok, (label, g, nc[g], ok)
        assert np.array_equal(cs[g], oc), (label, g)


@pytest.mark.parametrize("eps", [(0, 1), (1, 100), (1, 10), (1, 2), (10**6, 1)])
def test_mixed_batch_matches_oracle(bt, eps):
    graphs = _mixed_graphs(1, 40)
    batch = bt.Batch(graphs)
    print("case mixed40 eps", eps, flush=True)
    res = _run(bt, batch, eps[0], eps[1], 5)
    _check_all(batch, graphs, res, eps[0], eps[1], 5, "mixed eps=%s" % (eps,))


def test_every_launch_shape_gives_the_same_result(bt):
    graphs = _mixed_graphs(2, 60, n_hi=6000)
    batch = bt.Batch(graphs)
    ref = None
    for threads, bpc, sched in [(256, 1, 0), (256, 8, 0), (512, 2, 1), (512, 4, 0), (1024, 1, 0), (1024, 2, 1)]:
        print("case shape", threads, bpc, sched, flush=True)
        res = _run(bt, batch, 1, 10, 9, config=bt.BatchConfig(threads, bpc, sched))
        if ref is None:
            ref = res
            _check_all(batch, graphs, res, 1, 10, 9, "shape")
        else:
            for a, b in zip(res, ref):
                assert np.array_equal(a, b)


def test_many_colours_use_extension_words(bt):
    # K_60 needs colours above 40; two of them plus a small graph in one batch
    k60 = edges_to_csr(60, list(itertools.combinations(range(60), 2)))
    k45 = edges_to_csr(45, list(itertools.combinations(range(45), 2)))
    graphs = [k60, graphgen.erdos_renyi(300, 0.05, 3), k45, graphgen.chung_lu(5000, 60, 2.1, 4)]
    batch = bt.Batch(graphs)
    res = _run(bt, batch, 1, 10, 2)
    _check_all(batch, graphs, res, 1, 10, 2, "ext")
    assert res[1][0] == 60 and res[1][2] == 45


def test_batched_equals_standalone_gpu_calls(bt):
    import torch
    import paper_2008_11321_amd as pkg
    graphs = _mixed_graphs(3, 12)
    batch = bt.Batch(graphs)
    color, nc, rnd, nr = _run(bt, batch, 1, 10, 4)
    cs = batch.split(color)
    for g, (rp, col) in enumerate(graphs):
        c1, k1, _, L1 = pkg.color_graph(pkg.Graph(rp, col), 1, 10, 4)
        torch.cuda.synchronize()
        assert np.array_equal(c1.cpu().numpy(), cs[g]) and int(k1.item()) == nc[g] and int(L1.item()) == nr[g]


def test_batched_config_scaled_down(bt):
    # the batched workload's recipe (Chung-Lu, exponent 2.3, mean degree
    # 8..32, log-uniform n) at 1/20 of the sizes, every graph checked
    specs = graphgen.batched_config(num_graphs=256, seed=4, size_scale=0.05)
    graphs = [graphgen.chung_lu(n, min(k, n - 1), 2.3, s) for n, k, s in specs]
    batch = bt.Batch(graphs)
    print("case batched256 total_n", batch.total_n, "nnz", batch.total_nnz, flush=True)
    res = _run(bt, batch, 1, 10, 4)
    _check_all(batch, graphs, res, 1, 10, 4, "batched256")
    import torch
    ws = torch.empty(bt.batched_workspace_bytes(batch.num_graphs, batch.total_n, batch.total_nnz),
                     dtype=torch.uint8, device="cuda")
    bt.color_graph_batched(batch, 1, 10, 4, workspace=ws)
    st = bt.batched_stats(ws)
    assert st["error"] == 0
    # batch-wide counters against the oracle's per-graph counters
    ost = [oracle.color_graph(rp, col, 1, 10, 4) for rp, col in graphs]
    assert st["sum_active"] == sum(o[4]["sum_active"] for o in ost)
    assert st["cut_edges"] == sum(o[4]["cut_edges"] for o in ost)
    assert st["num_rounds"] == max(o[3] for o in ost) and st["num_colors"] == max(o[1] for o in ost)


def test_graph_capture_replays(bt):
    """The batched call records into a HIP graph (no host sync, no memset);
    every replay, with eager work in between, gives the eager result."""
    import torch
    graphs = _mixed_graphs(4, 30)
    batch = bt.Batch(graphs)
    ws = torch.empty(bt.batched_workspace_bytes(batch.num_graphs, batch.total_n, batch.total_nnz),
                     dtype=torch.uint8, device="cuda")
    out = (torch.empty(batch.total_n, dtype=torch.int32, device="cuda"),
           torch.empty(batch.total_n, dtype=torch.int32, device="cuda"),
           torch.zeros(batch.num_graphs, dtype=torch.int32, device="cuda"),
           torch.zeros(batch.num_graphs, dtype=torch.int32, device="cuda"))
    color, rnd, nc, nr = out
    bt.color_graph_batched(batch, 1, 10, 6, workspace=ws, out=(color, rnd, nc, nr))
    torch.cuda.synchronize()
    eager = [t.clone() for t in (color, rnd, nc, nr)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            bt.color_graph_batched(batch, 1, 10, 6, workspace=ws, out=(color, rnd, nc, nr), stream=s)
    torch.cuda.synchronize()
    for rep in range(4):
        for t in (color, rnd, nc, nr):
            t.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((color, rnd, nc, nr), eager):
            assert torch.equal(a, b), rep
        # unrelated eager work between replays
        x = torch.arange(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert int(x.item()) == (1 << 20) * ((1 << 20) - 1) // 2
    assert bt.batched_error(ws) == 0


def test_autotune_returns_a_valid_shape(bt):
    import torch
    graphs = _mixed_graphs(5, 80, n_hi=8000)
    batch = bt.Batch(graphs)
    cfg, ms = bt.autotune(batch, 1, 10, 3, reuse=False)
    assert cfg.block_threads in (256, 512, 1024) and 1 <= cfg.blocks_per_cu <= 32 and ms > 0
    cfg2, ms2 = bt.autotune(batch, 1, 10, 3, reuse=True)   # cached
    assert cfg2.as_dict() == cfg.as_dict() and ms2 == ms
    res = _run(bt, batch, 1, 10, 3, config=cfg)
    _check_all(batch, graphs, res, 1, 10, 3, "tuned")


def test_empty_batch_and_empty_graphs(bt):
    import torch
    batch = bt.Batch([edges_to_csr(0, []), edges_to_csr(0, [])])
    color, nc, rnd, nr = bt.color_graph_batched(batch, 1, 10, 1)
    torch.cuda.synchronize()
    assert nc.cpu().tolist() == [0, 0] and nr.cpu().tolist() == [0, 0]


def test_full_batched_workload_in_the_tuned_launch_shape(bt):
    """The batched workload at full size (4096 Chung-Lu graphs, n log-uniform
    in [100, 50000], mean degree 8..32, exponent 2.3, eps = 1/10, seed 4) in
    the launch shape the autotuner picks (the one the benchmark times):
    every graph against the oracle."""
    graphs = graphgen.batched_graphs(4096, seed=4)
    batch = bt.Batch(graphs)
    print("case batched4096 total_n", batch.total_n, "nnz", batch.total_nnz, flush=True)
    cfg, ms = bt.autotune(batch, 1, 10, 4, reuse=False)
    print("tuned", cfg, ms, flush=True)
    res = _run(bt, batch, 1, 10, 4, config=cfg)
    _check_all(batch, graphs, res, 1, 10, 4, "batched4096")
