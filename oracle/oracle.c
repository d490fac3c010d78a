/*
 * CPU oracle for ADG and JP-ADG -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the reference the GPU library is checked against.  Only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it; the GPU library neither links nor calls it, and the two share no
 * source, header, table or helper.  It is plain, serial and slow on purpose.
 *
 * What it computes (Besta et al., "High-Performance Parallel Graph Coloring
 * with Strong Guarantees on Work, Depth, and Quality"):
 *
 *   or_adg  -- ADG, Algorithm 1 (Section "Parallel Approximate Degeneracy
 *              Ordering"), step by step: D holds degrees, U the active set;
 *              every iteration l takes |U| = Count(U) and cnt = Reduce(U) over
 *              D, selects R = {u in U : D[u] <= (1 + eps) * cnt / |U|},
 *              runs UPDATE (DecrementAndFetch of D[u] for u in N_U(v), v in R,
 *              with U taken before R is removed), removes R from U and gives
 *              every v in R the priority rho_ADG(v) = l.
 *   or_jp   -- JP (Algorithm 3) under rho = <rho_ADG, rho_R> (Section
 *              "Graph Coloring by Color Scheduling (JP-ADG)").  JP with a
 *              total priority order gives the same colours as the sequential
 *              greedy colouring that visits vertices by decreasing priority
 *              and gives each the smallest colour >= 1 unused by its
 *              already-coloured neighbours: GetColor only looks at pred(v),
 *              and pred(v) are exactly the neighbours coloured before v in
 *              that order.  The oracle is that greedy definition.
 *   or_degeneracy -- exact degeneracy d by repeatedly removing a vertex of
 *              minimum degree (Matula and Beck), the definition used in
 *              Section "Degeneracy, Coreness, and Related Concepts".
 *
 * Readings of the paper that this file fixes (each is listed in the design
 * notes):
 *   - eps is the rational p/q (p >= 0, q >= 1); the selection test
 *     D[u] <= (1 + p/q) * cnt / |U| is evaluated exactly as
 *     q * |U| * D[u] <= (q + p) * cnt in 128-bit integers.
 *   - Selection uses "<=" as in the listing and the proof of the round bound.
 *   - Rounds are numbered from 1; a larger rho_ADG means a higher priority
 *     (coloured earlier), so vertices peeled last are coloured first.
 *   - rho_R is a seeded bijective hash h(v) = fmix32(v XOR k) with
 *     k = low 32 bits of the first SplitMix64 output from state `seed`
 *     (fmix32 is the MurmurHash3 finaliser; SplitMix64 is Steele, Lea and
 *     Flood, OOPSLA 2014).  Larger h wins.  Being a bijection on 32-bit
 *     words, it never ties.
 *   - Colours are numbered from 1; num_colors = max colour (0 if n = 0).
 *
 * Vertices are 0..n-1.  CSR: row_ptr[n+1] (int64), col[nnz] (int32), simple
 * undirected graph (symmetric, no self-loops, no duplicates).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ---- rho_R: seeded tie-break hash ---------------------------------------- */

static uint64_t splitmix64_first(uint64_t state) {
  uint64_t z = state + 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

static uint32_t murmur3_fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bU;
  h ^= h >> 13;
  h *= 0xc2b2ae35U;
  h ^= h >> 16;
  return h;
}

uint32_t or_fmix32(uint32_t x) { return murmur3_fmix32(x); }
uint64_t or_splitmix64_first(uint64_t s) { return splitmix64_first(s); }

uint32_t or_tiebreak(uint64_t seed, uint32_t v) {
  uint32_t k = (uint32_t)splitmix64_first(seed);
  return murmur3_fmix32(v ^ k);
}

/* ---- ADG (Algorithm 1) --------------------------------------------------- */

/* Returns the number of iterations L (>= 0), -1 on bad arguments / no
 * memory, -3 if an iteration selected nothing (cannot happen for Alg. 1).  rho_out[v] in 1..L.  Optional stats_out[4]:
 *   [0] sum over iterations of |U|, [1] number of decrements that hit a vertex
 *   staying in U (edges between R and U \ R, summed over iterations),
 *   [2] sum over iterations of |R| (= n), [3] L. */
int64_t or_adg(int64_t n, const int64_t* row_ptr, const int32_t* col, int64_t p, int64_t q,
               int32_t* rho_out, int64_t* stats_out) {
  if (n < 0 || p < 0 || q < 1) return -1;
  int64_t* D = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  unsigned char* inU = (unsigned char*)malloc((size_t)(n ? n : 1));
  unsigned char* inR = (unsigned char*)malloc((size_t)(n ? n : 1));
  int64_t* U = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  int64_t* R = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  if (!D || !inU || !inR || !U || !R) {
    free(D); free(inU); free(inR); free(U); free(R);
    return -1;
  }
  int64_t sum_U = 0, cut = 0;
  /* D = [deg(v_1) ... deg(v_n)]; l = 1; U = V. */
  for (int64_t v = 0; v < n; ++v) {
    D[v] = row_ptr[v + 1] - row_ptr[v];
    inU[v] = 1;
    inR[v] = 0;
    U[v] = v;
  }
  int64_t sizeU = n;
  int64_t l = 1;
  while (sizeU > 0) {
    /* |U| = Count(U); cnt = Reduce(U) with f(v) = D[v]. */
    int64_t count = 0;
    int64_t cntD = 0;
    for (int64_t i = 0; i < sizeU; ++i) {
      count += 1;
      cntD += D[U[i]];
    }
    sum_U += count;
    /* R = {u in U | D[u] <= (1 + p/q) * cnt / |U|}. */
    int64_t sizeR = 0;
    for (int64_t i = 0; i < sizeU; ++i) {
      int64_t u = U[i];
      u128 lhs = (u128)(uint64_t)q * (u128)(uint64_t)count * (u128)(uint64_t)D[u];
      u128 rhs = (u128)(uint64_t)(q + p) * (u128)(uint64_t)cntD;
      if (lhs <= rhs) {
        R[sizeR++] = u;
        inR[u] = 1;
      }
    }
    /* min D over U is at most the average, so R is never empty; an empty R
     * would mean a broken selection rule, reported instead of looping. */
    if (sizeR == 0) {
      free(D); free(inU); free(inR); free(U); free(R);
      return -3;
    }
    /* UPDATE(U, R, D): for v in R, for u in N_U(v): DecrementAndFetch(D[u]).
     * U is still the set before removing R, so members of R are decremented
     * too; those values are never read again. */
    for (int64_t i = 0; i < sizeR; ++i) {
      int64_t v = R[i];
      for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        int64_t u = col[e];
        if (inU[u]) {
          D[u] -= 1;
          if (!inR[u]) cut += 1;
        }
      }
    }
    /* U = U \ R; rho_ADG(v) = l for v in R; l = l + 1. */
    int64_t k = 0;
    for (int64_t i = 0; i < sizeU; ++i) {
      int64_t u = U[i];
      if (inR[u]) {
        inU[u] = 0;
        inR[u] = 0;
        rho_out[u] = (int32_t)l;
      } else {
        U[k++] = u;
      }
    }
    sizeU = k;
    l += 1;
  }
  if (stats_out) {
    stats_out[0] = sum_U;
    stats_out[1] = cut;
    stats_out[2] = n;
    stats_out[3] = l - 1;
  }
  free(D); free(inU); free(inR); free(U); free(R);
  return l - 1;
}

/* ---- ADG variants: ADG-O (sorted R) and ADG-M (median threshold) --------- */

#define OR_SORTED 1u  /* ADG-O: rho_ADG(r_i) = l + i over R sorted by D (listing ADG-O) */
#define OR_MEDIAN 2u  /* ADG-M: median instead of average (section on the degree median) */

typedef struct {
  int64_t d;   /* D[u] at selection */
  uint32_t h;  /* rho_R(u) */
  int64_t u;
} okey_t;

static int cmp_okey_asc(const void* a, const void* b) {
  const okey_t* x = (const okey_t*)a;
  const okey_t* y = (const okey_t*)b;
  if (x->d != y->d) return x->d < y->d ? -1 : 1;
  if (x->h != y->h) return x->h < y->h ? -1 : 1;
  return x->u < y->u ? -1 : (x->u > y->u);
}

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return x < y ? -1 : (x > y);
}

/* ADG with optional variant flags, in the paper's steps:
 *  - every round takes N = |U| and D over U (D[u] = deg_U(u), kept by the
 *    decrements of UPDATE);
 *  - default (Algorithm 1): R = {u : D[u] <= (1+p/q) * sum(D) / N};
 *  - OR_MEDIAN (ADG-M): delta_m = the lower median of D over U (the value at
 *    rank ceil(N/2) in increasing order; a reading, the paper does not say
 *    which median), R = {u : D[u] <= (1+p/q) delta_m}, and when R holds more
 *    than ceil(N/2) vertices (half of U, +1 if N is odd) it keeps the
 *    ceil(N/2) lowest by D, ties by increasing rho_R (a reading: the paper
 *    removes the lowest-degree vertices and leaves ties open);
 *  - OR_SORTED (ADG-O): R is sorted by increasing D, ties by increasing rho_R
 *    (a reading: the paper leaves ties to its sort), and rho_ADG(r_i) = l + i
 *    with l the number of vertices removed before; UPDATE decrements D[w] for
 *    neighbours w with a larger rho_ADG (w still in U has rho_ADG = n).
 *    Without OR_SORTED the order inside a round is JP's tie-break: pos ranks
 *    R by increasing rho_R.
 * Writes the round (1..L) of each vertex to round_out and the total order
 * JP colours by to pos_out: a permutation of 0..n-1, larger = coloured
 * first (with OR_SORTED it is rho_ADG-O itself).  Returns L, or -1 (bad
 * arguments / out of memory), -3 (an empty R). */
int64_t or_adg_ex(int64_t n, const int64_t* row_ptr, const int32_t* col, int64_t p, int64_t q, uint64_t seed,
                  uint32_t flags, int32_t* round_out, int64_t* pos_out, int64_t* stats_out) {
  if (n < 0 || p < 0 || q < 1 || (flags & ~(OR_SORTED | OR_MEDIAN))) return -1;
  size_t nn = (size_t)(n ? n : 1);
  int64_t* D = (int64_t*)malloc(sizeof(int64_t) * nn);
  int64_t* rho = (int64_t*)malloc(sizeof(int64_t) * nn);
  int64_t* U = (int64_t*)malloc(sizeof(int64_t) * nn);
  int64_t* Dsorted = (int64_t*)malloc(sizeof(int64_t) * nn);
  okey_t* R = (okey_t*)malloc(sizeof(okey_t) * nn);
  if (!D || !rho || !U || !Dsorted || !R) {
    free(D); free(rho); free(U); free(Dsorted); free(R);
    return -1;
  }
  int64_t sum_U = 0, cut = 0;
  for (int64_t v = 0; v < n; ++v) {
    D[v] = row_ptr[v + 1] - row_ptr[v];
    rho[v] = n; /* not removed yet */
    U[v] = v;
  }
  int64_t sizeU = n, removed = 0, l = 1;
  int64_t rc = 0;
  while (sizeU > 0) {
    sum_U += sizeU;
    /* the threshold and R */
    int64_t sizeR = 0, k = 0;
    u128 lhs_scale, rhs;
    if (flags & OR_MEDIAN) {
      for (int64_t i = 0; i < sizeU; ++i) Dsorted[i] = D[U[i]];
      qsort(Dsorted, (size_t)sizeU, sizeof(int64_t), cmp_i64);
      const int64_t dm = Dsorted[(sizeU + 1) / 2 - 1];
      lhs_scale = (u128)(uint64_t)q;                    /* q D <= (q+p) dm */
      rhs = (u128)(uint64_t)(q + p) * (u128)(uint64_t)dm;
    } else {
      int64_t cntD = 0;
      for (int64_t i = 0; i < sizeU; ++i) cntD += D[U[i]];
      lhs_scale = (u128)(uint64_t)q * (u128)(uint64_t)sizeU; /* q N D <= (q+p) cnt */
      rhs = (u128)(uint64_t)(q + p) * (u128)(uint64_t)cntD;
    }
    for (int64_t i = 0; i < sizeU; ++i) {
      int64_t u = U[i];
      if (lhs_scale * (u128)(uint64_t)D[u] <= rhs) {
        R[sizeR].d = D[u];
        R[sizeR].h = or_tiebreak(seed, (uint32_t)u);
        R[sizeR].u = u;
        ++sizeR;
      } else {
        U[k++] = u;
      }
    }
    if (sizeR == 0) {
      rc = -3;
      break;
    }
    qsort(R, (size_t)sizeR, sizeof(okey_t), cmp_okey_asc);
    if ((flags & OR_MEDIAN) && sizeR > (sizeU + 1) / 2) {
      /* keep the lowest half; the rest stays in U */
      for (int64_t i = (sizeU + 1) / 2; i < sizeR; ++i) U[k++] = R[i].u;
      sizeR = (sizeU + 1) / 2;
    }
    /* order inside the round: by (D, rho_R) for ADG-O, else by rho_R */
    if (!(flags & OR_SORTED))
      for (int64_t i = 0; i < sizeR; ++i) R[i].d = 0;
    qsort(R, (size_t)sizeR, sizeof(okey_t), cmp_okey_asc);
    for (int64_t i = 0; i < sizeR; ++i) {
      rho[R[i].u] = removed + i;
      round_out[R[i].u] = (int32_t)l;
    }
    /* UPDATE: decrement D[w] of the neighbours w with a larger rho_ADG */
    for (int64_t i = 0; i < sizeR; ++i) {
      int64_t v = R[i].u;
      for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        int64_t w = col[e];
        if (rho[w] > rho[v]) {
          D[w] -= 1;
          if (rho[w] == n) cut += 1;
        }
      }
    }
    sizeU = k;
    removed += sizeR;
    l += 1;
  }
  if (rc == 0) {
    for (int64_t v = 0; v < n; ++v) pos_out[v] = rho[v];
    if (stats_out) {
      stats_out[0] = sum_U;
      stats_out[1] = cut;
      stats_out[2] = n;
      stats_out[3] = l - 1;
    }
    rc = l - 1;
  }
  free(D); free(rho); free(U); free(Dsorted); free(R);
  return rc;
}

/* Greedy colouring in decreasing order of a total order pos (a permutation
 * of 0..n-1): JP's result under rho = pos.  Returns num_colors, or -1. */
int64_t or_jp_total(int64_t n, const int64_t* row_ptr, const int32_t* col, const int64_t* pos,
                    int32_t* color_out) {
  if (n < 0) return -1;
  if (n == 0) return 0;
  int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* stamp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 2));
  if (!order || !stamp) {
    free(order); free(stamp);
    return -1;
  }
  for (int64_t v = 0; v < n; ++v) order[v] = -1;
  for (int64_t v = 0; v < n; ++v) {
    if (pos[v] < 0 || pos[v] >= n || order[n - 1 - pos[v]] != -1) {
      free(order); free(stamp);
      return -1;
    }
    order[n - 1 - pos[v]] = v;
    color_out[v] = 0;
  }
  for (int64_t c = 0; c < n + 2; ++c) stamp[c] = -1;
  int64_t num_colors = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t v = order[i];
    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      int32_t c = color_out[col[e]];
      if (c > 0 && c <= n + 1) stamp[c] = v;
    }
    int64_t c = 1;
    while (stamp[c] == v) ++c;
    color_out[v] = (int32_t)c;
    if (c > num_colors) num_colors = c;
  }
  free(order); free(stamp);
  return num_colors;
}

/* ---- JP under rho = <rho_ADG, rho_R> (greedy definition) ------------------ */

typedef struct {
  uint64_t key; /* (rho_ADG << 32) | h(v): larger = higher priority */
  int64_t v;
} prio_t;

static int cmp_prio_desc(const void* a, const void* b) {
  const prio_t* x = (const prio_t*)a;
  const prio_t* y = (const prio_t*)b;
  if (x->key != y->key) return x->key > y->key ? -1 : 1;
  return x->v < y->v ? -1 : (x->v > y->v);
}

/* Colours color_out[v] >= 1; returns num_colors (max colour), or -1 on bad
 * arguments, -2 on a priority tie (impossible for a bijective hash). */
int64_t or_jp(int64_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* rho,
              uint64_t seed, int32_t* color_out) {
  if (n < 0) return -1;
  if (n == 0) return 0;
  prio_t* order = (prio_t*)malloc(sizeof(prio_t) * (size_t)n);
  int64_t* stamp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 2));
  if (!order || !stamp) {
    free(order); free(stamp);
    return -1;
  }
  for (int64_t v = 0; v < n; ++v) {
    if (rho[v] < 0) {
      free(order); free(stamp);
      return -1;
    }
    order[v].key = ((uint64_t)(uint32_t)rho[v] << 32) | (uint64_t)or_tiebreak(seed, (uint32_t)v);
    order[v].v = v;
    color_out[v] = 0; /* 0 = not yet coloured */
  }
  qsort(order, (size_t)n, sizeof(prio_t), cmp_prio_desc);
  for (int64_t i = 1; i < n; ++i)
    if (order[i].key == order[i - 1].key) {
      free(order); free(stamp);
      return -2;
    }
  for (int64_t c = 0; c < n + 2; ++c) stamp[c] = -1;
  int64_t num_colors = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t v = order[i].v;
    /* Colours of already-coloured neighbours (= pred(v)) are forbidden. */
    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      int32_t c = color_out[col[e]];
      if (c > 0 && c <= n + 1) stamp[c] = v;
    }
    int64_t c = 1;
    while (stamp[c] == v) ++c;
    color_out[v] = (int32_t)c;
    if (c > num_colors) num_colors = c;
  }
  free(order); free(stamp);
  return num_colors;
}

/* JP-ADG end to end: ADG, then JP.  Returns num_colors; *num_rounds = L. */
int64_t or_color_graph(int64_t n, const int64_t* row_ptr, const int32_t* col, int64_t p, int64_t q,
                       uint64_t seed, int32_t* color_out, int32_t* rho_out, int64_t* num_rounds,
                       int64_t* stats_out) {
  int64_t L = or_adg(n, row_ptr, col, p, q, rho_out, stats_out);
  if (L < 0) return -1;
  if (num_rounds) *num_rounds = L;
  return or_jp(n, row_ptr, col, rho_out, seed, color_out);
}

/* Number of neighbours with a higher JP priority, |pred(v)|. */
int64_t or_pred_counts(int64_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* rho,
                       uint64_t seed, int32_t* npred_out) {
  for (int64_t v = 0; v < n; ++v) {
    uint64_t kv = ((uint64_t)(uint32_t)rho[v] << 32) | or_tiebreak(seed, (uint32_t)v);
    int32_t c = 0;
    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      int32_t u = col[e];
      uint64_t ku = ((uint64_t)(uint32_t)rho[u] << 32) | or_tiebreak(seed, (uint32_t)u);
      if (ku > kv) ++c;
    }
    npred_out[v] = c;
  }
  return 0;
}

/* ---- exact degeneracy (min-degree peeling) ------------------------------- */

int64_t or_degeneracy(int64_t n, const int64_t* row_ptr, const int32_t* col) {
  if (n <= 0) return 0;
  int64_t maxdeg = 0;
  int64_t* deg = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  for (int64_t v = 0; v < n; ++v) {
    deg[v] = row_ptr[v + 1] - row_ptr[v];
    if (deg[v] > maxdeg) maxdeg = deg[v];
  }
  /* Bucket queue: bucket[d] holds vertices of current degree d, as a doubly
   * linked list. */
  int64_t* head = (int64_t*)malloc(sizeof(int64_t) * (size_t)(maxdeg + 1));
  int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* prev = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  unsigned char* gone = (unsigned char*)calloc((size_t)n, 1);
  for (int64_t d = 0; d <= maxdeg; ++d) head[d] = -1;
  for (int64_t v = 0; v < n; ++v) {
    prev[v] = -1;
    next[v] = head[deg[v]];
    if (head[deg[v]] >= 0) prev[head[deg[v]]] = v;
    head[deg[v]] = v;
  }
  int64_t d_out = 0, cur = 0;
  for (int64_t it = 0; it < n; ++it) {
    if (cur > 0) cur -= 1; /* a removal lowers the minimum by at most one */
    while (head[cur] < 0) ++cur;
    int64_t v = head[cur];
    head[cur] = next[v];
    if (next[v] >= 0) prev[next[v]] = -1;
    gone[v] = 1;
    if (cur > d_out) d_out = cur;
    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      int64_t u = col[e];
      if (gone[u]) continue;
      int64_t du = deg[u];
      /* unlink u from bucket du */
      if (prev[u] >= 0) next[prev[u]] = next[u]; else head[du] = next[u];
      if (next[u] >= 0) prev[next[u]] = prev[u];
      deg[u] = du - 1;
      prev[u] = -1;
      next[u] = head[du - 1];
      if (head[du - 1] >= 0) prev[head[du - 1]] = u;
      head[du - 1] = u;
    }
  }
  free(deg); free(head); free(next); free(prev); free(gone);
  return d_out;
}

/* ---- DEC-ADG-ITR (section "Enhancing Existing Coloring Algorithms") -------
 *
 * DEC-ADG's outer loop (the DEC-ADG listing): the ADG partitions
 * R(l) = {v : rho_ADG(v) = l} are coloured from the highest l down to 1.
 * Before partition l, B_v (the colours v may not take) receives the colours
 * of v's neighbours in the partitions already coloured.  The partition is
 * then coloured by SIM-COL (the SIM-COL listing) with ITR's choice: in every
 * iteration each uncoloured v of the partition takes the smallest colour not
 * in B_v (Part 1); v gives it up when a neighbour still uncoloured in the
 * partition took the same colour (Part 2) -- reading: only the endpoint with
 * the smaller rho_R gives it up, since with a deterministic choice both
 * giving up could repeat forever (two adjacent vertices with equal B_v); the
 * vertices that keep a colour are coloured and their colours enter the B_u
 * of their still-uncoloured neighbours in the partition (Part 3).
 * Iterations are synchronous: every Part reads the state the previous Part
 * left.  B_v has bits for colours 1 .. deg(v) + 1 (v never has more than
 * deg(v) coloured neighbours, so its smallest free colour is at most
 * deg(v) + 1 and larger colours of its neighbours cannot matter; they are
 * not recorded).
 * Writes colours (>= 1), the global iteration at which each vertex was
 * coloured (1-based, increasing over the partitions) and returns the number
 * of colours; stats_out[0] = iterations.  Returns -1 on bad input. */
int64_t or_dec_itr(int64_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* rho, uint64_t seed,
                   int32_t* color_out, int64_t* step_out, int64_t* stats_out) {
  if (n < 0) return -1;
  if (n == 0) {
    if (stats_out) stats_out[0] = 0;
    return 0;
  }
  int64_t L = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (rho[v] < 1) return -1;
    if (rho[v] > L) L = rho[v];
  }
  int64_t* boff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t* start = (int64_t*)calloc((size_t)(L + 2), sizeof(int64_t));
  int64_t* part = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* U = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int32_t* T = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  char* inU = (char*)calloc((size_t)n, 1);
  char* lose = (char*)calloc((size_t)n, 1);
  if (!boff || !start || !part || !U || !T || !inU || !lose) {
    free(boff); free(start); free(part); free(U); free(T); free(inU); free(lose);
    return -1;
  }
  boff[0] = 0;
  for (int64_t v = 0; v < n; ++v) boff[v + 1] = boff[v] + (row_ptr[v + 1] - row_ptr[v] + 1 + 63) / 64;
  uint64_t* B = (uint64_t*)calloc((size_t)(boff[n] ? boff[n] : 1), sizeof(uint64_t));
  if (!B) {
    free(boff); free(start); free(part); free(U); free(T); free(inU); free(lose);
    return -1;
  }
  /* the partitions, as lists (counting sort by rho) */
  for (int64_t v = 0; v < n; ++v) start[rho[v] + 1] += 1;
  for (int64_t l = 1; l <= L + 1; ++l) start[l] += start[l - 1];
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(L + 1));
    if (!fill) {
      free(B); free(boff); free(start); free(part); free(U); free(T); free(inU); free(lose);
      return -1;
    }
    for (int64_t l = 0; l <= L; ++l) fill[l] = start[l];
    for (int64_t v = 0; v < n; ++v) part[fill[rho[v]]++] = v;
    free(fill);
  }
  for (int64_t v = 0; v < n; ++v) color_out[v] = 0;
  int64_t step = 0, num_colors = 0;
  for (int64_t l = L; l >= 1; --l) {
    int64_t sizeU = 0;
    for (int64_t i = start[l]; i < start[l + 1]; ++i) U[sizeU++] = part[i];
    /* B_v gets the colours of v's neighbours in the partitions coloured so far */
    for (int64_t i = 0; i < sizeU; ++i) {
      int64_t v = U[i];
      for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        int64_t u = col[e];
        if (rho[u] > l) {
          int64_t c = color_out[u];
          if (c <= row_ptr[v + 1] - row_ptr[v] + 1) B[boff[v] + (c - 1) / 64] |= 1ull << ((c - 1) % 64);
        }
      }
    }
    while (sizeU > 0) {
      step += 1;
      for (int64_t i = 0; i < sizeU; ++i) inU[U[i]] = 1;
      /* Part 1: the smallest colour not in B_v */
      for (int64_t i = 0; i < sizeU; ++i) {
        int64_t v = U[i];
        int64_t c = 1;
        while (B[boff[v] + (c - 1) / 64] >> ((c - 1) % 64) & 1) ++c;
        T[v] = (int32_t)c;
      }
      /* Part 2: conflicts with neighbours in U (the smaller rho_R gives up) */
      for (int64_t i = 0; i < sizeU; ++i) {
        int64_t v = U[i];
        uint32_t hv = or_tiebreak(seed, (uint32_t)v);
        lose[v] = 0;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
          int64_t u = col[e];
          if (inU[u] && T[u] == T[v] && or_tiebreak(seed, (uint32_t)u) > hv) lose[v] = 1;
        }
        int64_t c = T[v];
        if (B[boff[v] + (c - 1) / 64] >> ((c - 1) % 64) & 1) lose[v] = 1;
      }
      for (int64_t i = 0; i < sizeU; ++i) {
        int64_t v = U[i];
        if (!lose[v]) {
          color_out[v] = T[v];
          step_out[v] = step;
          if (T[v] > num_colors) num_colors = T[v];
        }
      }
      /* Part 3: colours fixed in this iteration enter the B of the others in U */
      for (int64_t i = 0; i < sizeU; ++i) {
        int64_t v = U[i];
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
          int64_t u = col[e];
          if (inU[u] && color_out[u] > 0) {
            int64_t c = color_out[u];
            if (c <= row_ptr[v + 1] - row_ptr[v] + 1) B[boff[v] + (c - 1) / 64] |= 1ull << ((c - 1) % 64);
          }
        }
      }
      /* U = U \ {coloured} */
      int64_t k = 0;
      for (int64_t i = 0; i < sizeU; ++i) {
        inU[U[i]] = 0;
        if (color_out[U[i]] == 0) U[k++] = U[i];
      }
      sizeU = k;
    }
  }
  if (stats_out) stats_out[0] = step;
  free(B); free(boff); free(start); free(part); free(U); free(T); free(inU); free(lose);
  return num_colors;
}
