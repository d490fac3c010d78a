"""Pins for the CPU oracle: it is checked against what the paper and the
mathematics fix, never against itself or the GPU path.

* definition-level checks of ADG's selection rule (Algorithm 1) and JP's
  smallest-free-colour rule (Algorithm 3, GetColor) on every labelled graph
  with up to 6 vertices at every eps, a seeded sample of the graphs with 7,
  and seeded random graphs;
* the ADG counters against closed forms in rho: sum over rounds of |U_l| is
  the sum of rho, and UPDATE's decrements of vertices staying in U are the
  edges whose ends leave in different rounds;
* closed forms worked out by hand from Algorithm 1 and 3 (edgeless graph,
  K_n, star, complete bipartite, path, very large eps = JP-R);
* exact degeneracy by brute force over vertex subsets (definition in
  "Degeneracy, Coreness, and Related Concepts");
* the paper's bounds: round count (proof of the ADG depth lemma), the
  per-round shrink factor, the partial 2(1+eps)-approximate degeneracy order
  (ADG approximation lemma) and the colour bound 2(1+eps)d + 1 (JP-ADG colour
  corollary);
* published test vectors of the hash building blocks (SplitMix64,
  MurmurHash3's fmix32) and the bijectivity of the tie-break hash;
* the variants ADG-O (sorted R, the ADG-O listing) and ADG-M (median, the
  section on the degree median): definition checks per round, ADG-M's round
  count (halving), ADG-O's full 2(1+eps)-approximate order, ADG-M's partial
  4-approximate order and 4d + 1 colours, hand-worked small cases;
* DEC-ADG-ITR (section "Enhancing Existing Coloring Algorithms"): its
  iterations characterised vertex by vertex (check_dec_itr), the colour
  bound 2(1+eps)d + 1, hand-worked K_2, K_n, edgeless and K_{a,b}.
"""
import itertools
import math

import numpy as np
import pytest

import graphgen
import oracle
from checkers import (MEDIAN, SORTED, brute_degeneracy, check_adg, check_adg_variant, check_dec_itr, check_jp,
                      check_jp_order, edges_to_csr, fmix32_np, pred_count, priority_keys, splitmix64_first,
                      tiebreak_np)

EPS = [(0, 1), (1, 100), (1, 10), (1, 2), (1, 1), (10**6, 1)]


# ---------------------------------------------------------------- hash pins

def test_splitmix64_published_sequence():
    # First three outputs of SplitMix64 from state 0 (reference sequence of
    # Steele, Lea and Flood's generator).
    expect = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert oracle.splitmix64_first(0) == expect[0]
    assert [graphgen.splitmix64_draw(0, i) for i in range(3)] == expect
    assert splitmix64_first(0) == expect[0]


def test_fmix32_murmur3_vectors():
    # MurmurHash3_x86_32 of the empty key reduces to fmix32(seed); its
    # published verification values for seeds 1 and 0xffffffff:
    assert oracle.fmix32(1) == 0x514E28B7
    assert oracle.fmix32(0xFFFFFFFF) == 0x81F16F39
    assert oracle.fmix32(0) == 0
    assert int(fmix32_np([1])[0]) == 0x514E28B7


def _fmix32_inverse(h):
    # Each step of fmix32 is invertible mod 2^32: xorshift by s is undone by
    # repeated xorshift, multiplication by an odd constant by its inverse.
    def unxorshift(x, s):
        y = x
        for _ in range(32 // s + 1):
            y = x ^ (y >> s)
        return y & 0xFFFFFFFF
    inv1 = pow(0x85EBCA6B, -1, 1 << 32)
    inv2 = pow(0xC2B2AE35, -1, 1 << 32)
    h = unxorshift(h, 16)
    h = (h * inv2) & 0xFFFFFFFF
    h = unxorshift(h, 13)
    h = (h * inv1) & 0xFFFFFFFF
    return unxorshift(h, 16)


def test_tiebreak_is_bijection():
    rng = np.random.default_rng(7)
    xs = [0, 1, 2, 0xFFFFFFFF, 0x80000000] + [int(x) for x in rng.integers(0, 2**32, 2000)]
    for x in xs:
        assert _fmix32_inverse(oracle.fmix32(x)) == x
    for seed in [0, 1, 2, 12345678901234567]:
        n = 5000
        h = oracle.tiebreak_array(seed, n)
        assert np.unique(h).size == n
        assert np.array_equal(h, tiebreak_np(seed, n))


# ---------------------------------------------------------------- degeneracy

def test_degeneracy_matches_brute_force():
    rng = np.random.default_rng(3)
    for trial in range(120):
        n = int(rng.integers(1, 11))
        p = float(rng.uniform(0.1, 0.9))
        edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
        rp, col = edges_to_csr(n, edges)
        assert oracle.degeneracy(rp, col) == brute_degeneracy(n, edges), (n, edges)


def test_degeneracy_closed_forms():
    for n in range(1, 9):
        rp, col = edges_to_csr(n, [(u, v) for u in range(n) for v in range(u + 1, n)])
        assert oracle.degeneracy(rp, col) == n - 1  # K_n
    rp, col = edges_to_csr(10, [(i, i + 1) for i in range(9)])
    assert oracle.degeneracy(rp, col) == 1  # path (a tree)
    rp, col = edges_to_csr(6, [(i, (i + 1) % 6) for i in range(6)])
    assert oracle.degeneracy(rp, col) == 2  # cycle


# ---------------------------------------------------------------- helpers

def _bounds_hold(rp, col, p, q, rho, L, color, k, seed):
    n = rp.size - 1
    d = oracle.degeneracy(rp, col)
    rounds = check_adg(rp, col, p, q, rho, L)
    # per-round shrink: |U_{l+1}| (1+eps) < |U_l| unless U_{l+1} is empty
    sizes = [r[0] for r in rounds] + [0]
    for a, b in zip(sizes, sizes[1:]):
        assert b == 0 or b * (q + p) < a * q
    if n >= 2 and p > 0:
        assert L <= math.ceil(math.log(n) / math.log1p(p / q) + 1)
    # partial 2(1+eps)-approximate degeneracy order: neighbours with equal or
    # higher round, at most 2(1+eps)d
    src = np.repeat(np.arange(n), np.diff(rp))
    ge = np.bincount(src[rho[col] >= rho[src]], minlength=n) if n else np.zeros(0)
    assert np.all(q * ge <= (q + p) * 2 * d)
    check_jp(rp, col, rho, seed, color)
    npred = pred_count(rp, col, rho, seed)
    assert k == (color.max() if n else 0)
    assert k <= (npred.max() + 1 if n else 0)
    # JP-ADG colour bound, integer form: k <= floor(2(1+eps)d) + 1
    assert k <= (q + p) * 2 * d // q + 1
    deg = np.diff(rp)
    assert k <= (deg.max() + 1 if n else 0)


def _counters_hold(rp, col, rho, st):
    """The oracle's ADG counters against their closed forms.  A vertex of
    round r belongs to U_1 .. U_r, so sum over rounds of |U_l| = sum of rho.
    UPDATE decrements D[u] for every edge between R_l and U_l \\ R_l: each
    undirected edge whose endpoints leave in different rounds is counted
    once (when its lower-round end is removed), an edge inside one round
    never (both ends leave together)."""
    n = rp.size - 1
    rho = np.asarray(rho, dtype=np.int64)
    assert st["sum_active"] == int(rho.sum())
    src = np.repeat(np.arange(n), np.diff(rp))
    cut = int(np.count_nonzero(rho[src] != rho[col])) // 2 if n else 0
    assert st["cut_edges"] == cut


# ---------------------------------------------------------------- exhaustive small graphs

@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5])
def test_all_graphs_up_to_5_vertices(n):
    pairs = [(u, v) for u in range(n) for v in range(u + 1, n)]
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        rp, col = edges_to_csr(n, edges)
        for (p, q) in EPS:
            color, k, rho, L, st = oracle.color_graph(rp, col, p, q, seed=mask)
            _bounds_hold(rp, col, p, q, rho, L, color, k, mask)
            _counters_hold(rp, col, rho, st)


@pytest.mark.parametrize("eps", EPS)
def test_all_graphs_with_6_vertices(eps):
    n = 6
    p, q = eps
    pairs = [(u, v) for u in range(n) for v in range(u + 1, n)]
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        rp, col = edges_to_csr(n, edges)
        rho, L, st = oracle.adg(rp, col, p, q)
        check_adg(rp, col, p, q, rho, L)
        _counters_hold(rp, col, rho, st)
        color, k = oracle.jp(rp, col, rho, mask)
        check_jp(rp, col, rho, mask, color)


def test_sampled_graphs_with_7_vertices():
    # 2^21 labelled graphs on 7 vertices: a seeded sample of 3000 masks, at
    # every eps
    n = 7
    pairs = [(u, v) for u in range(n) for v in range(u + 1, n)]
    rng = np.random.default_rng(12)
    for mask in rng.integers(0, 1 << len(pairs), 3000):
        mask = int(mask)
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        rp, col = edges_to_csr(n, edges)
        for (p, q) in EPS:
            rho, L, st = oracle.adg(rp, col, p, q)
            check_adg(rp, col, p, q, rho, L)
            _counters_hold(rp, col, rho, st)
            color, k = oracle.jp(rp, col, rho, mask)
            check_jp(rp, col, rho, mask, color)


@pytest.mark.parametrize("seed", range(6))
def test_random_graphs_medium(seed):
    rng = np.random.default_rng(100 + seed)
    for trial in range(6):
        n = int(rng.integers(20, 400))
        kind = trial % 3
        if kind == 0:
            rp, col = graphgen.erdos_renyi(n, float(rng.uniform(0.01, 0.2)), seed * 10 + trial)
        elif kind == 1:
            rp, col = graphgen.chung_lu(n, float(rng.uniform(2, 12)), 2.3, seed * 10 + trial)
        else:
            rp, col = graphgen.rmat(int(np.log2(n)) + 1, 8, 0.57, 0.19, 0.19, seed * 10 + trial)
        for (p, q) in [(0, 1), (1, 100), (1, 10), (1, 2)]:
            color, k, rho, L, st = oracle.color_graph(rp, col, p, q, seed=trial)
            _bounds_hold(rp, col, p, q, rho, L, color, k, trial)
            _counters_hold(rp, col, rho, st)


# ---------------------------------------------------------------- closed forms

def test_edgeless():
    for n in [1, 2, 7, 100]:
        rp, col = edges_to_csr(n, [])
        for (p, q) in EPS:
            color, k, rho, L, _ = oracle.color_graph(rp, col, p, q, 5)
            assert L == 1 and np.all(rho == 1) and np.all(color == 1) and k == 1


def test_empty_graph():
    rp = np.zeros(1, dtype=np.int64)
    col = np.zeros(0, dtype=np.int32)
    color, k, rho, L, _ = oracle.color_graph(rp, col, 1, 10, 1)
    assert L == 0 and k == 0 and color.size == 0


def test_complete_graph_colours_by_hash_rank():
    for n in [2, 3, 5, 17, 64]:
        rp, col = edges_to_csr(n, list(itertools.combinations(range(n), 2)))
        for (p, q) in EPS:
            for seed in [0, 9]:
                color, k, rho, L, _ = oracle.color_graph(rp, col, p, q, seed)
                assert L == 1 and np.all(rho == 1)
                h = tiebreak_np(seed, n).astype(np.int64)
                rank = np.array([int((h > h[v]).sum()) for v in range(n)])
                assert np.array_equal(color, rank + 1) and k == n


def test_star():
    for k in [2, 3, 10, 50]:
        n = k + 1
        rp, col = edges_to_csr(n, [(0, i) for i in range(1, n)])
        for (p, q) in EPS:
            color, nc, rho, L, _ = oracle.color_graph(rp, col, p, q, 3)
            if q * k > q + 2 * p:  # k > 1 + 2 eps: leaves first, centre in round 2
                assert L == 2 and rho[0] == 2 and np.all(rho[1:] == 1)
                assert color[0] == 1 and np.all(color[1:] == 2)
            else:
                assert L == 1 and np.all(rho == 1)
            assert nc == 2


def test_complete_bipartite():
    for a, b in [(1, 3), (2, 5), (3, 4), (4, 9), (5, 5)]:
        n = a + b
        rp, col = edges_to_csr(n, [(i, a + j) for i in range(a) for j in range(b)])
        for (p, q) in EPS:
            color, nc, rho, L, _ = oracle.color_graph(rp, col, p, q, 8)
            if q * b > a * (q + 2 * p):  # b > a(1+2eps): side B peeled first
                assert L == 2 and np.all(rho[:a] == 2) and np.all(rho[a:] == 1)
                assert np.all(color[:a] == 1) and np.all(color[a:] == 2)
            else:
                assert L == 1
                # JP-R on K_{a,b}: the side holding the top-priority vertex gets 1
                top = int(np.argmax(tiebreak_np(8, n)))
                side = slice(0, a) if top < a else slice(a, n)
                assert np.all(color[side] == 1)
            assert nc == 2


def test_path_many_rounds():
    for n in [2, 3, 4, 9, 10, 31, 64]:
        rp, col = edges_to_csr(n, [(i, i + 1) for i in range(n - 1)])
        p, q = 1, 10 * n  # eps < 1/(n-1): only the two ends go each round
        color, nc, rho, L, _ = oracle.color_graph(rp, col, p, q, 4)
        v = np.arange(n)
        assert np.array_equal(rho, np.minimum(v + 1, n - v))
        assert L == (n + 1) // 2
        assert nc == (2 if n >= 2 else 1)
        if n % 2 == 1:
            c = (n - 1) // 2
            assert np.array_equal(color, 1 + (np.abs(v - c) % 2))


def test_huge_eps_is_jp_random():
    # eps >= n * Delta forces a single round, so JP-ADG = JP-R: greedy by
    # decreasing hash (the eps -> infinity limit of the trade-off discussion).
    rng = np.random.default_rng(5)
    for trial in range(20):
        n = int(rng.integers(2, 60))
        rp, col = graphgen.erdos_renyi(n, 0.3, trial)
        if col.size == 0:
            continue
        delta = int(np.diff(rp).max())
        color, nc, rho, L, _ = oracle.color_graph(rp, col, n * delta, 1, trial)
        assert L == 1
        h = tiebreak_np(trial, n)
        order = np.argsort(-h.astype(np.int64), kind="stable")
        want = np.zeros(n, dtype=np.int64)
        for v in order:
            used = {int(want[u]) for u in col[rp[v]:rp[v + 1]] if want[u] > 0}
            c = 1
            while c in used:
                c += 1
            want[v] = c
        assert np.array_equal(color, want)


def test_adjacency_order_invariance():
    rng = np.random.default_rng(9)
    rp, col = graphgen.chung_lu(3000, 12, 2.3, 77)
    col2 = col.copy()
    for v in range(rp.size - 1):
        seg = col2[rp[v]:rp[v + 1]]
        rng.shuffle(seg)
    a = oracle.color_graph(rp, col, 1, 10, 3)
    b = oracle.color_graph(rp, col2, 1, 10, 3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2]) and a[1] == b[1] and a[3] == b[3]


def test_pred_counts_match_definition():
    rp, col = graphgen.rmat(10, 8, 0.57, 0.19, 0.19, 1)
    rho, L, _ = oracle.adg(rp, col, 1, 10)
    assert np.array_equal(oracle.pred_counts(rp, col, rho, 6), pred_count(rp, col, rho, 6))


def test_priority_key_orientation():
    # higher round => higher priority regardless of hash
    k = priority_keys(np.array([1, 2]), 0)
    assert k[1] > k[0]


# ---------------------------------------------------------------- ADG-O and ADG-M

def _variant_bounds(rp, col, p, q, seed, flags, color, k, rnd, L, pos):
    n = rp.size - 1
    check_adg_variant(rp, col, p, q, seed, flags, rnd, pos, L)
    check_jp_order(rp, col, pos, color)
    assert k == (color.max() if n else 0)
    if n == 0:
        return
    d = oracle.degeneracy(rp, col)
    src = np.repeat(np.arange(n), np.diff(rp))
    later = np.bincount(src[pos[col] > pos[src]], minlength=n)   # neighbours coloured earlier
    same_or_later = np.bincount(src[rnd[col] >= rnd[src]], minlength=n)
    if flags & MEDIAN:
        # ADG-M halves U: |U_{l+1}| = floor(|U_l| / 2), so L = bit length of n
        assert L == n.bit_length()
        # partial 4-approximate order and JP-ADG-M's colour bound 4d + 1
        assert np.all(same_or_later <= 4 * d)
        assert k <= 4 * d + 1
    else:
        # ADG-O's order is total: at most 2(1+eps)d neighbours come later
        if flags & SORTED:
            assert np.all(q * later <= (q + p) * 2 * d)
        assert k <= (q + p) * 2 * d // q + 1


@pytest.mark.parametrize("flags", [SORTED, MEDIAN, SORTED | MEDIAN])
@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5])
def test_variants_all_graphs_up_to_5_vertices(n, flags):
    pairs = [(u, v) for u in range(n) for v in range(u + 1, n)]
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        rp, col = edges_to_csr(n, edges)
        for (p, q) in [(0, 1), (1, 10), (10**6, 1)]:
            color, k, rnd, L, pos, _ = oracle.color_graph_ex(rp, col, p, q, mask, flags)
            _variant_bounds(rp, col, p, q, mask, flags, color, k, rnd, L, pos)


@pytest.mark.parametrize("flags", [0, SORTED, MEDIAN, SORTED | MEDIAN])
@pytest.mark.parametrize("seed", range(3))
def test_variants_random_graphs(seed, flags):
    rng = np.random.default_rng(300 + seed)
    for trial in range(4):
        n = int(rng.integers(20, 300))
        if trial % 2:
            rp, col = graphgen.chung_lu(n, float(rng.uniform(2, 12)), 2.3, seed * 10 + trial)
        else:
            rp, col = graphgen.erdos_renyi(n, float(rng.uniform(0.01, 0.2)), seed * 10 + trial)
        for (p, q) in [(0, 1), (1, 10), (1, 2)]:
            color, k, rnd, L, pos, st = oracle.color_graph_ex(rp, col, p, q, trial, flags)
            _variant_bounds(rp, col, p, q, trial, flags, color, k, rnd, L, pos)
            if flags & MEDIAN:
                # sum of |U_l| over the halving sequence n, floor(n/2), ...
                sizes, m = [], n
                while m:
                    sizes.append(m)
                    m //= 2
                assert st["sum_active"] == sum(sizes)
            else:
                # Algorithm 1's rounds; with no flag, also its JP colouring
                c0, k0, r0, L0, st0 = oracle.color_graph(rp, col, p, q, trial)
                assert np.array_equal(rnd, r0) and L == L0 and st == st0
                if not flags:
                    assert np.array_equal(color, c0) and k == k0


def test_sorted_star_colours_the_centre_first():
    """One round (huge eps): ADG-O puts the centre (largest D) last in R, so
    it has the highest rho and takes colour 1; the leaves take colour 2, in
    increasing order of rho_R among themselves."""
    s = 9
    rp, col = edges_to_csr(s + 1, [(0, i) for i in range(1, s + 1)])
    for seed in range(5):
        color, k, rnd, L, pos, _ = oracle.color_graph_ex(rp, col, 10**6, 1, seed, SORTED)
        assert L == 1 and k == 2 and color[0] == 1 and np.all(color[1:] == 2)
        assert pos[0] == s
        h = tiebreak_np(seed, s + 1)
        assert np.array_equal(np.argsort(pos[1:]), np.argsort(h[1:]))


def test_sorted_path_order_by_hand():
    """P_5 in one round: ends (D = 1) at positions 0 and 1, inner vertices
    (D = 2) at 2, 3, 4; each pair ordered by rho_R."""
    rp, col = edges_to_csr(5, [(0, 1), (1, 2), (2, 3), (3, 4)])
    seed = 7
    h = tiebreak_np(seed, 5)
    _, pos, L, _ = oracle.adg_ex(rp, col, 10**6, 1, seed, SORTED)
    ends = sorted([0, 4], key=lambda v: h[v])
    inner = sorted([1, 2, 3], key=lambda v: h[v])
    expect = np.zeros(5, dtype=np.int64)
    for i, v in enumerate(ends + inner):
        expect[v] = i
    assert L == 1 and np.array_equal(pos, expect)


def test_median_path_by_hand():
    """P_4 under ADG-M: round 1 removes the two ends (D = 1), round 2 the
    inner vertex with the smaller rho_R (both have D = 1 then), round 3 the
    other, for every eps."""
    rp, col = edges_to_csr(4, [(0, 1), (1, 2), (2, 3)])
    for seed in range(4):
        h = tiebreak_np(seed, 4)
        first, second = (1, 2) if h[1] < h[2] else (2, 1)
        for (p, q) in [(0, 1), (1, 10), (10**6, 1)]:
            rnd, pos, L, _ = oracle.adg_ex(rp, col, p, q, seed, MEDIAN)
            assert L == 3 and rnd[0] == 1 and rnd[3] == 1 and rnd[first] == 2 and rnd[second] == 3


def test_median_complete_graph():
    """K_n: every D equal, so ADG-M removes the lower half by rho_R each round."""
    n = 11
    rp, col = edges_to_csr(n, [(u, v) for u in range(n) for v in range(u + 1, n)])
    seed = 3
    h = tiebreak_np(seed, n)
    rnd, pos, L, _ = oracle.adg_ex(rp, col, 1, 10, seed, MEDIAN)
    order = np.argsort(h)          # increasing rho_R
    sizes = [11, 5, 2, 1]          # |U| per round; ceil(|U|/2) removed
    start = 0
    for l, m in enumerate(sizes, 1):
        take = (m + 1) // 2
        assert np.all(rnd[order[start:start + take]] == l)
        start += take
    assert L == 4
    color, k = oracle.jp_total(rp, col, pos)
    assert k == n and np.array_equal(np.argsort(-pos), np.argsort(color))


# ---------------------------------------------------------------- DEC-ADG-ITR

def _dec_bounds(rp, col, p, q, seed):
    color, k, rho, L, step, it = oracle.color_graph_dec(rp, col, p, q, seed)
    n = rp.size - 1
    check_dec_itr(rp, col, rho, seed, color, step)
    assert k == (color.max() if n else 0)
    assert it == (step.max() if n else 0)
    if n:
        d = oracle.degeneracy(rp, col)
        # each vertex has at most 2(1+eps)d neighbours coloured before it
        assert k <= (q + p) * 2 * d // q + 1
    return color, k, rho, L, step, it


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5])
def test_dec_itr_all_graphs_up_to_5_vertices(n):
    pairs = [(u, v) for u in range(n) for v in range(u + 1, n)]
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        rp, col = edges_to_csr(n, edges)
        for (p, q) in [(0, 1), (1, 10), (10**6, 1)]:
            _dec_bounds(rp, col, p, q, mask)


@pytest.mark.parametrize("seed", range(3))
def test_dec_itr_random_graphs(seed):
    rng = np.random.default_rng(700 + seed)
    for trial in range(4):
        n = int(rng.integers(20, 200))
        if trial % 2:
            rp, col = graphgen.chung_lu(n, float(rng.uniform(2, 12)), 2.3, seed * 10 + trial)
        else:
            rp, col = graphgen.erdos_renyi(n, float(rng.uniform(0.02, 0.3)), seed * 10 + trial)
        for (p, q) in [(0, 1), (1, 10), (1, 2)]:
            _dec_bounds(rp, col, p, q, trial)


def test_dec_itr_k2_by_hand():
    """One partition {0, 1}: both try colour 1, the larger rho_R keeps it;
    the other takes colour 2 in the second iteration."""
    rp, col = edges_to_csr(2, [(0, 1)])
    for seed in range(6):
        h = tiebreak_np(seed, 2)
        win = 0 if h[0] > h[1] else 1
        color, k, step, it = oracle.dec_itr(rp, col, np.ones(2, np.int32), seed)
        assert it == 2 and k == 2
        assert color[win] == 1 and step[win] == 1 and color[1 - win] == 2 and step[1 - win] == 2


def test_dec_itr_complete_graph_by_hash_rank():
    """K_n in one partition: iteration i colours the vertex of i-th largest
    rho_R with colour i."""
    n = 9
    rp, col = edges_to_csr(n, [(u, v) for u in range(n) for v in range(u + 1, n)])
    seed = 4
    color, k, step, it = oracle.dec_itr(rp, col, np.ones(n, np.int32), seed)
    rank = np.argsort(np.argsort(-tiebreak_np(seed, n).astype(np.int64))) + 1
    assert k == n and it == n and np.array_equal(color, rank) and np.array_equal(step, rank)


def test_dec_itr_edgeless_and_bipartite():
    rp, col = edges_to_csr(7, [])
    color, k, rho, L, step, it = oracle.color_graph_dec(rp, col, 1, 10, 1)
    assert k == 1 and it == 1 and np.all(color == 1)
    # K_{3,8}: ADG removes the larger side first, so the smaller side (a
    # higher partition) is coloured first, with colour 1, in one iteration;
    # the larger side then takes colour 2 in one iteration
    a, b = 3, 8
    rp, col = edges_to_csr(a + b, [(i, a + j) for i in range(a) for j in range(b)])
    color, k, rho, L, step, it = oracle.color_graph_dec(rp, col, 0, 1, 2)
    assert L == 2 and k == 2 and it == 2
    assert np.all(color[:a] == 1) and np.all(color[a:] == 2)


def test_dec_itr_colours_beyond_small_bitmaps():
    """K_70 coloured first (colours 1..70), then pendant vertices of degree
    1 and 2 hanging off it: a pendant's bitmap holds a few colours only, and
    its neighbours' large colours must neither count nor spill into other
    vertices' bitmaps."""
    k = 70
    edges = [(u, v) for u in range(k) for v in range(u + 1, k)]
    n = k
    for i in range(k):
        edges.append((i, n))            # a pendant of degree 1
        edges.append((i, n + 1))        # and one of degree 2
        edges.append(((i + 1) % k, n + 1))
        n += 2
    rp, col = edges_to_csr(n, edges)
    color, kk, rho, L, step, it = oracle.color_graph_dec(rp, col, 0, 1, 5)
    check_dec_itr(rp, col, rho, 5, color, step)
    assert kk == k
    assert np.all(color[k:] <= 3)
