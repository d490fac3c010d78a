"""The full-size checkers (test_zfull_size_gpu) run on the CPU at small
sizes: they accept the oracle's rounds and colours, and reject a round or a
colour changed at one vertex."""
import numpy as np
import pytest

import graphgen
import oracle
import test_zfull_size_gpu as fz


@pytest.mark.parametrize("p,q", [(1, 100), (1, 2), (1, 10)])
def test_checkers_accept_the_oracle_and_catch_one_change(p, q):
    import torch
    rp, col = graphgen.rmat_config(11, seed=3)
    seed = 3
    color, k, rho, L, st = oracle.color_graph(rp, col, p, q, seed)
    col_t = torch.as_tensor(col)
    rnd = torch.as_tensor(rho.astype(np.int32))
    clr = torch.as_tensor(color.astype(np.int32))
    assert fz.check_adg_by_removal(torch, rp, col_t, rnd, p, q, "cpu") == st["sum_active"]
    fz.check_jp(torch, rp, col_t, rnd, clr, seed, "cpu")
    # one vertex of the last round moved one round down
    v = int(np.flatnonzero(rho == L)[0])
    bad = rnd.clone()
    bad[v] = L - 1
    with pytest.raises(AssertionError):
        fz.check_adg_by_removal(torch, rp, col_t, bad, p, q, "cpu")
    # one vertex with a non-minimal colour
    w = int(np.argmax(np.diff(rp)))
    badc = clr.clone()
    badc[w] = k + 1
    with pytest.raises(AssertionError):
        fz.check_jp(torch, rp, col_t, rnd, badc, seed, "cpu")
