"""Serving loop (adg_server_*): requests arriving while others run are
admitted by arena footprint, grouped and overlapped, and every result is the
same as when the request is served alone -- and equal to the CPU oracle.
GPU only, except the argument checks at the end."""
import ctypes

import numpy as np
import pytest

import graphgen
import oracle


def _mix(count, seed):
    """A scaled-down serving mix: ER n 1e3..2e4 (mean degree 10), Chung-Lu n
    1e4..1e5 (mean degree 16), R-MAT scale 14..17."""
    return [graphgen.serving_graph(sp, scale_down=True) for sp in graphgen.serving_specs(count, seed=seed)]


@pytest.fixture(scope="module")
def sv():
    import torch
    import paper_2008_11321_amd.serving as s
    assert torch.cuda.is_available()
    return s


@pytest.mark.gpu
def test_alone_and_in_the_mix_give_the_same_result(sv):
    graphs = _mix(48, seed=5)
    # alone: one worker, each request submitted after the previous finished
    alone = []
    with sv.Server(2 << 30, eps=(1, 10), seed=5, workers=1, small_nnz=1 << 18) as s:
        for i, (rp, col) in enumerate(graphs):
            alone.append(sv.replay(s, [(rp, col)])[0])
    # the mix: Poisson arrivals faster than service, four workers, grouping
    arrivals = graphgen.poisson_arrivals(len(graphs), qps=2000.0, seed=5)
    with sv.Server(2 << 30, eps=(1, 10), seed=5, workers=4, small_nnz=1 << 18, max_group=16) as s:
        mix = sv.replay(s, graphs, arrivals)
    grouped = sum(1 for r in mix if r["group_size"] > 1)
    print("grouped", grouped, "of", len(mix), flush=True)
    assert grouped > 0
    # jobs overlapped in time
    iv = sorted((r["t_start"], r["t_done"]) for r in mix)
    assert any(iv[k + 1][0] < iv[k][1] for k in range(len(iv) - 1))
    bad = []
    for i, (rp, col) in enumerate(graphs):
        a, m = alone[i], mix[i]
        oc, ok, _, oL, _ = oracle.color_graph(rp, col, 1, 10, 5)
        da, dm = int((a["color"] != oc).sum()), int((m["color"] != oc).sum())
        if (a["status"] or m["status"] or da or dm or a["num_rounds"] != oL or m["num_rounds"] != oL
                or a["num_colors"] != ok or m["num_colors"] != ok):
            bad.append(dict(request=i, n=rp.size - 1, nnz=col.size, status=(a["status"], m["status"]),
                            wrong_alone=da, wrong_mix=dm, group=m["group_size"],
                            colours=(a["num_colors"], m["num_colors"], ok),
                            rounds=(a["num_rounds"], m["num_rounds"], oL)))
    print("requests that differ from the oracle:", bad, flush=True)
    assert not bad


@pytest.mark.gpu
def test_small_arena_admits_by_footprint(sv):
    """An arena that holds about two of the larger jobs at a time: everything
    still completes, correctly, and large requests are not starved."""
    graphs = _mix(24, seed=6)
    cfg = sv.default_config()
    cfg.small_nnz = 1 << 18
    fp = [sv.footprint(rp.size - 1, col.size, cfg) for rp, col in graphs]
    arena = int(2.2 * max(fp))
    with sv.Server(arena, eps=(1, 10), seed=6, workers=4, small_nnz=1 << 18, max_group=8, max_bypass=4) as s:
        res = sv.replay(s, graphs, None)
    for i, (rp, col) in enumerate(graphs):
        oc, ok, _, oL, _ = oracle.color_graph(rp, col, 1, 10, 6)
        assert res[i]["status"] == 0 and np.array_equal(res[i]["color"], oc), i
        assert res[i]["num_colors"] == ok and res[i]["num_rounds"] == oL, (i, res[i]["num_colors"], ok)


@pytest.mark.gpu
def test_submit_rejects_what_cannot_run(sv):
    from paper_2008_11321_amd import AdgError
    rp, col = graphgen.erdos_renyi(5000, 0.002, 1)
    need = sv.footprint(rp.size - 1, col.size)
    with sv.Server(need // 2, workers=1) as s:   # too small for this graph
        with pytest.raises(AdgError) as e:
            s.submit(rp, col, 1)
        assert e.value.code == -5
        bad = rp.copy()
        bad[-1] += 1   # row_ptr does not end at nnz
        with pytest.raises(AdgError) as e:
            s.submit(bad, col, 2)
        assert e.value.code == -1


def test_server_arguments_without_gpu():
    import paper_2008_11321_amd.serving as s
    L = s._lib()
    cfg = L.adg_server_default_config()
    assert cfg.workers >= 1 and cfg.eps_den >= 1
    small = L.adg_server_footprint(ctypes.byref(cfg), 1000, 10_000)
    big = L.adg_server_footprint(ctypes.byref(cfg), 10_000_000, 200_000_000)
    assert 0 < small < big
    assert L.adg_server_footprint(ctypes.byref(cfg), -1, 0) == 0
    h = ctypes.c_void_p()
    assert L.adg_server_create(ctypes.byref(cfg), None, 1 << 20, ctypes.byref(h)) == -1
    bad = s.ServerConfig(1, 10, 0, 0, 1 << 20, 16, 4)     # no workers
    assert L.adg_server_create(ctypes.byref(bad), ctypes.c_void_p(1 << 20), 1 << 20, ctypes.byref(h)) == -1
    cnt = ctypes.c_int32()
    assert L.adg_server_submit(None, 1, 0, None, None, None, 0) == -1
    assert L.adg_server_poll(None, None, 0, 0, ctypes.byref(cnt)) == -1
    assert L.adg_server_in_flight(None) == -1
    assert L.adg_server_destroy(None) == -1
