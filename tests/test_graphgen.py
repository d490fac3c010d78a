"""Generator tests: simple undirected CSR, determinism, expected statistics."""
import math

import numpy as np
import pytest

import graphgen
import oracle
from checkers import check_csr


def test_from_edges_cleans_input():
    rp, col = graphgen.from_edges(5, [0, 1, 1, 2, 3, 3], [1, 0, 1, 3, 2, 4])
    check_csr(rp, col)
    assert rp.tolist() == [0, 1, 2, 3, 5, 6]
    assert col.tolist() == [1, 0, 3, 2, 4, 3]


def test_er_shape_and_stats():
    n, p = 10_000, 10 / 10_000
    rp, col = graphgen.er_config(n, 10.0, seed=1)
    check_csr(rp, col)
    m = col.size // 2
    mean = p * n * (n - 1) / 2
    sd = math.sqrt(mean * (1 - p))
    assert abs(m - mean) < 6 * sd
    assert np.all(np.diff(col[rp[0]:rp[1]]) > 0)


def test_determinism_and_seed_sensitivity():
    a = graphgen.rmat(12, 16, 0.57, 0.19, 0.19, 2)
    b = graphgen.rmat(12, 16, 0.57, 0.19, 0.19, 2)
    c = graphgen.rmat(12, 16, 0.57, 0.19, 0.19, 3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[1][: min(a[1].size, c[1].size)], c[1][: min(a[1].size, c[1].size)])


def test_rmat_shape():
    rp, col = graphgen.rmat_config(14, seed=2)
    check_csr(rp, col)
    n = 1 << 14
    assert rp.size == n + 1
    assert col.size <= 2 * 16 * n
    deg = np.diff(rp)
    # R-MAT with a = 0.57 concentrates degree at low ids
    assert deg[:64].mean() > 10 * deg.mean()


def test_chung_lu_stats():
    n, k = 20_000, 16.0
    w = graphgen.chung_lu_weights(n, k, 2.3)
    assert abs(w.sum() - n * k) < 1e-6 * n * k
    assert abs(w[0] - math.sqrt(n * k)) < 1e-6 * w[0]
    assert np.all(np.diff(w) <= 0)
    rp, col = graphgen.chung_lu(n, k, 2.3, seed=4)
    check_csr(rp, col)
    assert abs(col.size / n - k) < 0.08 * k


def test_degeneracy_bound_sqrt_m():
    # d <= 2 sqrt(m) (lemma on degeneracy and edge count)
    for seed in range(3):
        rp, col = graphgen.rmat(11, 16, 0.57, 0.19, 0.19, seed)
        d = oracle.degeneracy(rp, col)
        assert d <= 2 * math.sqrt(col.size // 2)


def test_batched_specs():
    specs = graphgen.batched_config(4096, seed=4)
    ns = np.array([s[0] for s in specs])
    ks = np.array([s[1] for s in specs])
    assert ns.min() >= 100 and ns.max() <= 50_000
    assert 6000 < ns.mean() < 10000
    assert ks.min() >= 8 and ks.max() <= 32
    assert len({s[2] for s in specs}) == 4096
