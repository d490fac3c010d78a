"""Definition-level verifiers, written from the paper independently of the
oracle (numpy, non-incremental).  They pin the oracle, and check GPU output at
sizes the oracle's own run would make slow.

* check_adg: the output of ADG (Algorithm 1) is fixed round by round by its
  selection rule: with U_l = {v : rho(v) >= l}, deg_U the degree inside
  G[U_l], |U_l| and cnt = sum of deg_U over U_l, a vertex of U_l is removed in
  round l exactly when deg_U(v) <= (1 + p/q) * cnt / |U_l| (evaluated as
  q |U| deg <= (q + p) cnt).  Every degree is recomputed from the graph, so
  incremental bookkeeping errors (wrong vertices decremented, missed
  decrements, wrong counts) show up.
* check_jp: a JP colouring for the total order <rho_ADG, rho_R> is proper and
  gives every vertex the smallest colour >= 1 not used by its higher-priority
  neighbours (GetColor in Algorithm 3).
"""
import numpy as np

MASK64 = (1 << 64) - 1


def splitmix64_first(s):
    """SplitMix64 (Steele, Lea, Flood 2014), first output from state s."""
    z = (s + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def fmix32_np(x):
    """MurmurHash3 32-bit finaliser on a uint32 array."""
    x = np.asarray(x, dtype=np.uint64) & 0xFFFFFFFF
    x ^= x >> 16
    x = (x * 0x85EBCA6B) & 0xFFFFFFFF
    x ^= x >> 13
    x = (x * 0xC2B2AE35) & 0xFFFFFFFF
    x ^= x >> 16
    return x.astype(np.uint32)


def tiebreak_np(seed, n):
    k = splitmix64_first(int(seed) & MASK64) & 0xFFFFFFFF
    return fmix32_np(np.arange(n, dtype=np.uint64) ^ np.uint64(k))


def priority_keys(rho, seed):
    rho = np.asarray(rho, dtype=np.uint64)
    return (rho << np.uint64(32)) | tiebreak_np(seed, rho.size).astype(np.uint64)


def _src(row_ptr):
    n = row_ptr.size - 1
    return np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))


def check_csr(row_ptr, col):
    """Simple undirected graph in CSR: symmetric, no loops, no duplicates."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = row_ptr.size - 1
    assert row_ptr[0] == 0 and row_ptr[-1] == col.size
    assert np.all(np.diff(row_ptr) >= 0)
    if col.size == 0:
        return
    assert col.min() >= 0 and col.max() < n
    src = _src(row_ptr)
    assert not np.any(src == col), "self-loop"
    fwd = src * n + col
    assert np.unique(fwd).size == fwd.size, "duplicate entry"
    assert np.array_equal(np.sort(fwd), np.sort(col * n + src)), "not symmetric"


def check_adg(row_ptr, col, p, q, rho, L):
    """Raise AssertionError unless rho is exactly ADG's output (see module doc).
    Returns the per-round thresholds' data for further checks."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    rho = np.asarray(rho, dtype=np.int64)
    n = row_ptr.size - 1
    if n == 0:
        assert L == 0
        return []
    assert rho.min() >= 1 and rho.max() == L
    src = _src(row_ptr)
    rounds = []
    for l in range(1, L + 1):
        inU = rho >= l
        sizeU = int(inU.sum())
        assert sizeU > 0
        edge_in = inU[src] & inU[col]
        degU = np.bincount(src[edge_in], minlength=n)
        cnt = int(degU[inU].sum())
        # exact: q*|U|*deg <= (q+p)*cnt ; python ints avoid overflow
        lhs_scale = q * sizeU
        rhs = (q + p) * cnt
        sel = np.array([lhs_scale * int(d) <= rhs for d in degU[inU]]) if sizeU < 4096 else (
            (degU[inU].astype(object) * lhs_scale) <= rhs)
        removed = rho[inU] == l
        assert np.array_equal(sel.astype(bool), removed), "round %d selection mismatch" % l
        assert removed.any(), "empty round %d" % l
        rounds.append((sizeU, cnt, degU))
    return rounds


def check_jp(row_ptr, col, rho, seed, color):
    """Proper, and colour(v) = smallest colour >= 1 not used by pred(v)."""
    check_jp_order(row_ptr, col, priority_keys(rho, seed), color)


def check_jp_order(row_ptr, col, key, color):
    """JP's output for the total order `key` (distinct; larger = coloured
    first): proper, and colour(v) = smallest colour >= 1 not used by the
    neighbours with a larger key."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    color = np.asarray(color, dtype=np.int64)
    key = np.asarray(key)
    n = row_ptr.size - 1
    if n == 0:
        return
    assert np.unique(key).size == n, "not a total order"
    assert color.min() >= 1
    src = _src(row_ptr)
    assert not np.any(color[src] == color[col]), "improper colouring"
    pred = key[col] > key[src]  # col is a predecessor of src
    # pred colours below colour(v), distinct per v: must be exactly colour(v)-1 of them
    s, c = src[pred], color[col[pred]]
    low = c < color[s]
    pairs = np.unique(s[low] * (int(color.max()) + 2) + c[low])
    have = np.bincount(pairs // (int(color.max()) + 2), minlength=n)
    assert np.array_equal(have, color - 1), "colour is not the smallest free colour over pred(v)"


def pred_count(row_ptr, col, rho, seed):
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = row_ptr.size - 1
    key = priority_keys(rho, seed)
    src = _src(row_ptr)
    return np.bincount(src[key[col] > key[src]], minlength=n)


def edges_to_csr(n, edges):
    """Tiny helper: symmetric CSR from an undirected edge list (no generator)."""
    adj = [set() for _ in range(n)]
    for u, v in edges:
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    rp = np.zeros(n + 1, dtype=np.int64)
    cols = []
    for v in range(n):
        nb = sorted(adj[v])
        cols.extend(nb)
        rp[v + 1] = rp[v] + len(nb)
    return rp, np.array(cols, dtype=np.int32)


def brute_degeneracy(n, edges):
    """max over non-empty vertex subsets S of the minimum degree in G[S]."""
    nb = [0] * n
    for u, v in edges:
        nb[u] |= 1 << v
        nb[v] |= 1 << u
    best = 0
    for S in range(1, 1 << n):
        mn = None
        for v in range(n):
            if S >> v & 1:
                d = bin(nb[v] & S).count("1")
                mn = d if mn is None or d < mn else mn
        best = max(best, mn)
    return best


SORTED, MEDIAN = 1, 2


def check_adg_variant(row_ptr, col, p, q, seed, flags, rnd, pos, L):
    """The ADG variants from their definitions, every degree recomputed from
    the graph (deg_U over U_l = {v : round(v) >= l}):
    * MEDIAN (ADG-M): R_l is the ceil(|U_l|/2) vertices of U_l lowest by
      (deg_U, rho_R) -- the cap of half of U always binds, because at least
      ceil(|U|/2) vertices have deg_U <= the lower median <= (1+eps) times
      it, and this is checked too;
    * otherwise R_l follows Algorithm 1's selection rule (check_adg);
    * pos is the total order JP colours by: rounds in increasing order, and
      inside a round increasing (deg_U at selection, rho_R) with SORTED
      (ADG-O), increasing rho_R without.
    Returns D at selection per vertex."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    rnd = np.asarray(rnd, dtype=np.int64)
    pos = np.asarray(pos, dtype=np.int64)
    n = row_ptr.size - 1
    if n == 0:
        assert L == 0
        return np.zeros(0, dtype=np.int64)
    assert rnd.min() >= 1 and rnd.max() == L
    assert np.array_equal(np.sort(pos), np.arange(n)), "pos is not a permutation"
    h = tiebreak_np(seed, n).astype(np.int64)
    src = _src(row_ptr)
    dsel = np.zeros(n, dtype=np.int64)
    if not flags & MEDIAN:
        check_adg(row_ptr, col, p, q, rnd, L)
    for l in range(1, L + 1):
        inU = rnd >= l
        sizeU = int(inU.sum())
        edge_in = inU[src] & inU[col]
        degU = np.bincount(src[edge_in], minlength=n)
        removed = rnd == l
        dsel[removed] = degU[removed]
        if flags & MEDIAN:
            ids = np.flatnonzero(inU)
            k = (sizeU + 1) // 2
            dm = int(np.sort(degU[ids])[k - 1])
            assert int(np.sum(q * degU[ids] <= (q + p) * dm)) >= k
            low = ids[np.lexsort((h[ids], degU[ids]))[:k]]
            expect = np.zeros(n, dtype=bool)
            expect[low] = True
            assert np.array_equal(expect, removed), "round %d: not the lowest half" % l
    inner = dsel * (1 << 32) + h if flags & SORTED else h
    order = np.lexsort((inner, rnd))
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n)
    assert np.array_equal(rank, pos), "order inside the rounds"
    return dsel


def _mex(colors):
    s = set(int(c) for c in colors)
    c = 1
    while c in s:
        c += 1
    return c


def check_dec_itr(row_ptr, col, rho, seed, color, step):
    """DEC-ADG-ITR's output characterised iteration by iteration (not
    simulated): with step(v) the iteration that coloured v,
    * the colouring is proper and partitions are coloured from the highest
      rho down, each over a contiguous range of iterations;
    * at iteration s every uncoloured v of the running partition tries
      t_s(v) = the smallest colour missing among its neighbours coloured
      before s (B_v), and color(v) = t_{step(v)}(v);
    * v is not coloured at s < step(v) exactly when some neighbour u of the
      same partition, still uncoloured at s, tried the same colour and has a
      larger rho_R (and at step(v) no such neighbour exists).
    Small graphs only (Python loops)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    rho = np.asarray(rho, dtype=np.int64)
    color = np.asarray(color, dtype=np.int64)
    step = np.asarray(step, dtype=np.int64)
    n = row_ptr.size - 1
    if n == 0:
        return
    assert color.min() >= 1 and step.min() >= 1
    src = _src(row_ptr)
    assert not np.any(color[src] == color[col]), "improper colouring"
    h = tiebreak_np(seed, n).astype(np.int64)
    nb = [col[row_ptr[v]:row_ptr[v + 1]] for v in range(n)]
    # partitions in decreasing rho, over contiguous iteration ranges
    L = int(rho.max())
    prev_last = 0
    first = {}
    for l in range(L, 0, -1):
        vs = np.flatnonzero(rho == l)
        if vs.size == 0:
            continue
        lo, hi = int(step[vs].min()), int(step[vs].max())
        assert lo == prev_last + 1, "partition %d does not start right after the previous one" % l
        first[l] = lo
        prev_last = hi
        for s in range(lo, hi + 1):
            assert np.any(step[vs] == s), "iteration %d colours nothing" % s

    def tried(v, s):
        return _mex(color[u] for u in nb[v] if step[u] < s)

    for v in range(n):
        l = int(rho[v])
        assert tried(v, step[v]) == color[v], "vertex %d: not the smallest free colour" % v
        for s in range(first[l], int(step[v]) + 1):
            tv = tried(v, s)
            beaten = any(rho[u] == l and step[u] >= s and h[u] > h[v] and tried(u, s) == tv for u in nb[v])
            assert beaten == (s < step[v]), "vertex %d at iteration %d" % (v, s)
