// Seeded synthetic graph generators and a CSR builder.
//
// This module produces the inputs that both the GPU library and the CPU
// checker consume.  It contains no step of the colouring method itself: it
// only draws random graphs and turns edge lists into a simple undirected CSR
// (symmetric adjacency, no self-loops, no duplicate entries, rows sorted by
// neighbour id), which is the representation the paper assumes for its input
// graphs (Section "Graph Model and Representation").
//
// Randomness: every draw is a pure function of (key, counter), taken from the
// SplitMix64 generator of Steele, Lea and Flood ("Fast splittable
// pseudorandom number generators", OOPSLA 2014): the i-th output of the stream
// started at state `key` is mix64(key + (i+1) * GAMMA).  Results therefore do
// not depend on the number of OpenMP threads.
//
// Generators:
//   * Erdos-Renyi G(n, p) with geometric skipping per row
//     (Batagelj and Brandes, "Efficient generation of large random networks",
//     Phys. Rev. E 71, 2005).
//   * R-MAT / Kronecker edge draws with quadrant probabilities a, b, c, d
//     (Chakrabarti, Zhan and Faloutsos, SDM 2004), without noise.
//   * Chung-Lu expected-degree graphs with power-law weights, generated in
//     O(n + m) with the skipping method of Miller and Hagberg ("Efficient
//     generation of networks with given expected degrees", WAW 2011).
//
// C ABI: every generator returns an opaque handle owning (row_ptr, col_idx);
// the caller copies the arrays out and frees the handle.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t GAMMA = 0x9e3779b97f4a7c15ULL;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// i-th output (0-based) of the SplitMix64 stream whose state starts at key.
inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GAMMA); }

// Key of an independent sub-stream: first output of the stream at (key ^ tag).
inline uint64_t subkey(uint64_t key, uint64_t tag) { return draw(key ^ (tag * 0xd1b54a32d192ed03ULL), 0); }

// Uniform double in [0, 1) with 53 random bits.
inline double unit(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

// Stream tags, so that the same user seed gives unrelated streams per use.
constexpr uint64_t TAG_ER = 0x4552ULL, TAG_RMAT = 0x524d4154ULL, TAG_CL = 0x434cULL;

struct Graph {
  int64_t n = 0;
  int64_t nnz = 0;
  int64_t* row_ptr = nullptr;  // [n+1]
  int32_t* col = nullptr;      // [nnz]
  ~Graph() {
    std::free(row_ptr);
    std::free(col);
  }
};

// Build a simple symmetric CSR from an undirected edge list (each edge may be
// listed in either or both directions, any number of times; self-loops are
// dropped).  Rows come out sorted and duplicate-free.
Graph* build_csr(int64_t n, int64_t m, const int32_t* src, const int32_t* dst) {
  Graph* g = new (std::nothrow) Graph();
  if (!g) return nullptr;
  g->n = n;
  std::vector<std::atomic<int64_t>> cnt(n + 1);
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v <= n; ++v) cnt[v].store(0, std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u == v) continue;
    cnt[u].fetch_add(1, std::memory_order_relaxed);
    cnt[v].fetch_add(1, std::memory_order_relaxed);
  }
  // Exclusive prefix over raw (pre-dedup) counts.
  std::vector<int64_t> off(n + 1);
  int64_t run = 0;
  for (int64_t v = 0; v < n; ++v) {
    off[v] = run;
    run += cnt[v].load(std::memory_order_relaxed);
  }
  off[n] = run;
  const int64_t raw = run;
  int32_t* col = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(raw, 1));
  if (!col) {
    delete g;
    return nullptr;
  }
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) cnt[v].store(off[v], std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u == v) continue;
    col[cnt[u].fetch_add(1, std::memory_order_relaxed)] = v;
    col[cnt[v].fetch_add(1, std::memory_order_relaxed)] = u;
  }
  // Sort and dedup every row in place; remember the unique length.
  std::vector<int64_t> ulen(n);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t v = 0; v < n; ++v) {
    int32_t* b = col + off[v];
    int32_t* e = col + off[v + 1];
    std::sort(b, e);
    ulen[v] = std::unique(b, e) - b;
  }
  int64_t* rp = (int64_t*)std::malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!rp) {
    std::free(col);
    delete g;
    return nullptr;
  }
  run = 0;
  for (int64_t v = 0; v < n; ++v) {
    rp[v] = run;
    run += ulen[v];
  }
  rp[n] = run;
  // Compact rows to the left.  Row v moves from off[v] to rp[v] <= off[v];
  // doing it serially in increasing v never overwrites unread data.
  for (int64_t v = 0; v < n; ++v)
    if (rp[v] != off[v]) std::memmove(col + rp[v], col + off[v], sizeof(int32_t) * (size_t)ulen[v]);
  g->nnz = run;
  g->row_ptr = rp;
  g->col = (int32_t*)std::realloc(col, sizeof(int32_t) * (size_t)std::max<int64_t>(run, 1));
  if (!g->col) g->col = col;
  return g;
}

// Geometric skip: number of failures before the next success of a Bernoulli(p)
// sequence, using one uniform draw.
inline int64_t geo_skip(double r, double log1mp) {
  double k = std::floor(std::log1p(-r) / log1mp);
  if (!(k < 9.0e18)) return INT64_MAX / 4;
  return (int64_t)k;
}

}  // namespace

extern "C" {

// Number of OpenMP threads the generators use.
int gg_num_threads(void) { return omp_get_max_threads(); }

int64_t gg_n(const void* h) { return static_cast<const Graph*>(h)->n; }
int64_t gg_nnz(const void* h) { return static_cast<const Graph*>(h)->nnz; }
const int64_t* gg_row_ptr(const void* h) { return static_cast<const Graph*>(h)->row_ptr; }
const int32_t* gg_col_idx(const void* h) { return static_cast<const Graph*>(h)->col; }
void gg_copy(const void* h, int64_t* row_ptr_out, int32_t* col_out) {
  const Graph* g = static_cast<const Graph*>(h);
  std::memcpy(row_ptr_out, g->row_ptr, sizeof(int64_t) * (size_t)(g->n + 1));
  if (g->nnz) std::memcpy(col_out, g->col, sizeof(int32_t) * (size_t)g->nnz);
}
void gg_free(void* h) { delete static_cast<Graph*>(h); }

// CSR of the simple undirected graph spanned by m listed edges (src[e], dst[e]).
void* gg_from_edges(int64_t n, int64_t m, const int32_t* src, const int32_t* dst) {
  if (n < 0 || m < 0 || n > INT32_MAX) return nullptr;
  for (int64_t e = 0; e < m; ++e)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return nullptr;
  return build_csr(n, m, src, dst);
}

// G(n, p): every unordered pair {u, v} is an edge independently with
// probability p.  Row u draws its partners v > u by geometric skipping from
// the sub-stream (seed, u).
void* gg_erdos_renyi(int64_t n, double p, uint64_t seed) {
  if (n < 0 || n > INT32_MAX || !(p >= 0.0) || p > 1.0) return nullptr;
  const uint64_t key = subkey(seed, TAG_ER);
  std::vector<std::vector<int32_t>> rows(n);
  if (p > 0.0) {
    const double log1mp = std::log1p(-p);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t u = 0; u < n; ++u) {
      const uint64_t ku = subkey(key, (uint64_t)u);
      uint64_t ctr = 0;
      int64_t v = u;
      std::vector<int32_t>& row = rows[u];
      while (true) {
        int64_t skip = (p >= 1.0) ? 0 : geo_skip(unit(draw(ku, ctr++)), log1mp);
        v += 1 + skip;
        if (v >= n) break;
        row.push_back((int32_t)v);
      }
    }
  }
  std::vector<int64_t> start(n + 1, 0);
  for (int64_t u = 0; u < n; ++u) start[u + 1] = start[u] + (int64_t)rows[u].size();
  const int64_t m = start[n];
  std::vector<int32_t> src(m), dst(m);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t u = 0; u < n; ++u)
    for (size_t k = 0; k < rows[u].size(); ++k) {
      src[start[u] + k] = (int32_t)u;
      dst[start[u] + k] = rows[u][k];
    }
  rows.clear();
  rows.shrink_to_fit();
  return build_csr(n, m, src.data(), dst.data());
}

// R-MAT: num_edges draws on 2^scale vertices.  Draw e picks one quadrant per
// level, most significant bit first, with probabilities a, b, c and
// 1 - a - b - c; two levels share one 64-bit draw (32 bits each).  The
// resulting edge list is symmetrised and deduplicated; self-loops are dropped.
void* gg_rmat(int scale, int64_t num_edges, double a, double b, double c, uint64_t seed) {
  if (scale < 1 || scale > 30 || num_edges < 0) return nullptr;
  if (!(a >= 0 && b >= 0 && c >= 0 && a + b + c <= 1.0)) return nullptr;
  const int64_t n = int64_t(1) << scale;
  const uint64_t key = subkey(seed, TAG_RMAT);
  const double two32 = 4294967296.0;
  auto thr = [&](double x) -> uint64_t {
    double t = std::floor(x * two32);
    return t >= two32 ? (uint64_t(1) << 32) : (uint64_t)t;
  };
  const uint64_t ta = thr(a), tab = thr(a + b), tabc = thr(a + b + c);
  const int words = (scale + 1) / 2;
  int32_t* src = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(num_edges, 1));
  int32_t* dst = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(num_edges, 1));
  if (!src || !dst) {
    std::free(src);
    std::free(dst);
    return nullptr;
  }
#pragma omp parallel for schedule(static, 65536)
  for (int64_t e = 0; e < num_edges; ++e) {
    uint32_t u = 0, v = 0;
    int level = 0;
    for (int w = 0; w < words; ++w) {
      const uint64_t x = draw(key, (uint64_t)e * (uint64_t)words + (uint64_t)w);
      for (int half = 0; half < 2 && level < scale; ++half, ++level) {
        const uint64_t r = half == 0 ? (x >> 32) : (x & 0xffffffffULL);
        uint32_t bu, bv;
        if (r < ta) {
          bu = 0; bv = 0;
        } else if (r < tab) {
          bu = 0; bv = 1;
        } else if (r < tabc) {
          bu = 1; bv = 0;
        } else {
          bu = 1; bv = 1;
        }
        u = (u << 1) | bu;
        v = (v << 1) | bv;
      }
    }
    src[e] = (int32_t)u;
    dst[e] = (int32_t)v;
  }
  Graph* g = build_csr(n, num_edges, src, dst);
  std::free(src);
  std::free(dst);
  return g;
}

// Power-law expected-degree weights w_i = C * (i + i0)^(-1/(gamma-1)),
// i = 0..n-1 (non-increasing in i), scaled so that sum(w) = n * mean_deg, and
// with i0 > 0 chosen so that w_0 = sqrt(sum(w)) (then w_0 * w_0 / sum(w) = 1,
// so every pair probability min(w_u w_v / sum(w), 1) stays at most 1 without
// clipping the head).  Written to w_out[n]; returns 0 on success.
int gg_chung_lu_weights(int64_t n, double mean_deg, double gamma, double* w_out) {
  if (n < 1 || !(gamma > 1.0) || !(mean_deg >= 0.0)) return -1;
  const double beta = 1.0 / (gamma - 1.0);
  const double target = std::sqrt((double)n * mean_deg);
  auto w0_for = [&](double i0, double* csum) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += std::pow((double)i + i0, -beta);
    const double C = (double)n * mean_deg / s;
    if (csum) *csum = C;
    return C * std::pow(i0, -beta);
  };
  double lo = 1e-9, hi = 1e12, C = 0.0;
  if (mean_deg == 0.0) {
    for (int64_t i = 0; i < n; ++i) w_out[i] = 0.0;
    return 0;
  }
  // w_0(i0) decreases from +inf (i0 -> 0) to mean_deg (i0 -> inf) < target
  // whenever mean_deg < n; bisect in log space.
  if (w0_for(hi, nullptr) > target) lo = hi;
  for (int it = 0; it < 200 && lo != hi; ++it) {
    const double mid = std::sqrt(lo * hi);
    if (w0_for(mid, nullptr) > target) lo = mid; else hi = mid;
    if (hi / lo < 1.0 + 1e-12) break;
  }
  const double i0 = hi;
  w0_for(i0, &C);
  for (int64_t i = 0; i < n; ++i) w_out[i] = C * std::pow((double)i + i0, -beta);
  return 0;
}

// Chung-Lu graph: pair {u, v} is an edge with probability
// min(w_u w_v / sum(w), 1), with the weights above.  Row u uses the
// sub-stream (seed, u) and visits partners v > u by Miller-Hagberg skipping.
void* gg_chung_lu(int64_t n, double mean_deg, double gamma, uint64_t seed) {
  if (n < 0 || n > INT32_MAX) return nullptr;
  if (n == 0) return build_csr(0, 0, nullptr, nullptr);
  std::vector<double> w(n);
  if (gg_chung_lu_weights(n, mean_deg, gamma, w.data()) != 0) return nullptr;
  double S = 0.0;
  for (int64_t i = 0; i < n; ++i) S += w[i];
  const uint64_t key = subkey(seed, TAG_CL);
  std::vector<std::vector<int32_t>> rows(n);
  if (S > 0.0) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t u = 0; u < n - 1; ++u) {
      const uint64_t ku = subkey(key, (uint64_t)u);
      uint64_t ctr = 0;
      int64_t v = u + 1;
      double p = std::min(w[u] * w[v] / S, 1.0);
      std::vector<int32_t>& row = rows[u];
      while (v < n && p > 0.0) {
        if (p != 1.0) {
          const double r = unit(draw(ku, ctr++));
          const double k = std::floor(std::log1p(-r) / std::log1p(-p));
          if (!(k < (double)n)) break;
          v += (int64_t)k;
        }
        if (v < n) {
          const double q = std::min(w[u] * w[v] / S, 1.0);
          const double r = unit(draw(ku, ctr++));
          if (r < q / p) row.push_back((int32_t)v);
          p = q;
          v += 1;
        }
      }
    }
  }
  std::vector<int64_t> start(n + 1, 0);
  for (int64_t u = 0; u < n; ++u) start[u + 1] = start[u] + (int64_t)rows[u].size();
  const int64_t m = start[n];
  std::vector<int32_t> src(m), dst(m);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t u = 0; u < n; ++u)
    for (size_t k = 0; k < rows[u].size(); ++k) {
      src[start[u] + k] = (int32_t)u;
      dst[start[u] + k] = rows[u][k];
    }
  rows.clear();
  rows.shrink_to_fit();
  return build_csr(n, m, src.data(), dst.data());
}

// Many Chung-Lu graphs at once (graph g: n[g] vertices, mean degree k[g],
// seed seeds[g]), one graph per thread; out[g] receives its handle (null on
// failure).  Each graph is exactly gg_chung_lu's: rows use their own
// sub-streams and the weights are computed serially either way.
void gg_chung_lu_many(int64_t G, const int64_t* n, const double* k, double gamma, const uint64_t* seeds,
                      void** out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t g = 0; g < G; ++g) out[g] = gg_chung_lu(n[g], k[g], gamma, seeds[g]);
}

// Raw stream access, so that tests can pin the generator to SplitMix64's
// published output sequence.
uint64_t gg_splitmix64_draw(uint64_t key, uint64_t i) { return draw(key, i); }

}  // extern "C"
