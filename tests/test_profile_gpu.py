"""Kernel-class timing (adg_profile_*): recording events changes no result,
and the JP loop's single event pair stands for exactly the launches that
the per-launch classes count.  GPU only."""
import numpy as np
import pytest

import graphgen
import oracle


@pytest.mark.gpu
def test_jp_phase_counts_the_loops_launches():
    import torch
    import paper_2008_11321_amd as pkg
    assert torch.cuda.is_available()
    rp, col = graphgen.rmat_config(14, seed=4)
    print("case rmat14 seed 4 n", rp.size - 1, "nnz", col.size, flush=True)
    g = pkg.Graph(rp, col)
    ws = torch.empty(pkg.workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device="cuda")
    ref = oracle.color_graph(rp, col, 1, 10, 4)[0]
    pkg.profile_read()
    try:
        pkg.profile_enable(["jp", "jp_narrow", "jp_phase", "update"])
        color = pkg.color_graph(g, 1, 10, 4, workspace=ws)[0]
        torch.cuda.synchronize()
    finally:
        pkg.profile_enable([])
    prof = pkg.profile_read()
    assert np.array_equal(color.cpu().numpy(), ref)
    ms, launches = prof["jp_phase"]
    assert launches == prof["jp"][1] + prof["jp_narrow"][1] > 0
    assert ms > 0 and prof["update"][1] >= pkg.get_stats(ws)["num_rounds"] > 0
    # nothing stays recorded once read
    assert pkg.profile_read() == {}
