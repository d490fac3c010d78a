// ADG and JP-ADG on one graph: kernels and the C ABI (include/adg.h).
//
// Paper: Besta et al., "High-Performance Parallel Graph Coloring with Strong
// Guarantees on Work, Depth, and Quality".
//
// ADG (Algorithm 1) runs as a short sequence of kernels per round, issued
// back to back on the caller's stream; loop control lives in a device-side
// control block, so the host only reads the termination flag between chunks
// of rounds.  Per round l:
//   k_stats    |U_l| and the degree sum S_l (Count and Reduce).  S_l is a
//              cached sum -- the sum over U_l of D at selection time minus the
//              previous UPDATE's decrements ("Caching Sums of Degrees") -- and
//              the threshold is the integer T_l = floor((q+p) S_l / (q |U_l|)),
//              so that D[u] <= (1 + p/q) S_l / |U_l|  <=>  D[u] <= T_l.
//   k_count    per-block counts of R (split by degree) and of U \ R.
//   k_scan     one block: exclusive scan of the per-block counts.
//   k_scatter  stable compaction of U_l into R_l and U_{l+1}; R_l is written
//              to its slot of the order array ORD = [R_1 | R_2 | ... | R_L]
//              (the contiguous [R(1) ... R(i) | U] array of "Representation of
//              U and R"); rho_ADG(v) = l for v in R_l.
//   k_update   UPDATE: for v in R_l and w in N(v) still in U, decrement D[w].
//              With fusion on, the same sweep also builds JP's DAG G_rho (JP
//              Part 1 inside UPDATE, "Combining JP and ADG"): v's row is
//              rewritten as [pred | same-round succ | earlier-round succ] and
//              |pred(v)|, the number of same-round successors and v's JP word
//              are stored.
// JP (Algorithm 3, Part 2) colours the rounds from L down to 1.  Every edge of
// G_rho between different rounds points from the higher round to the lower,
// so once rounds > l are coloured and have pushed their colours to round l,
// round l only waits on itself.  Per round: its vertices whose predecessors
// are all coloured form level 0; levels are processed one after the other
// over same-round successors only; then one bulk kernel pushes the round's
// colours to its earlier-round successors.  Narrow levels (and whole small
// rounds) run in a single block with block barriers; wide ones over the grid.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/adg.h"
#include "adg_device.h"
#include "adg_host.h"

namespace adg {

constexpr int BS = 256;                 // threads per block
constexpr int WPB = BS / WAVE;          // wavefronts per block
constexpr int SEL_BLOCKS = 2048;        // fixed grid of the selection kernels
constexpr int SMALL_DEG = 32;           // lane-per-vertex rows up to this length
constexpr int FB_CAP = 2048;            // per-block staging of level lists (LDS)
constexpr int JP_SMALL = 32;            // lane-per-vertex successor loops
constexpr int JP_UNROLL = 4;
constexpr int JP_CHUNK = WAVE * JP_UNROLL;   // successors per wavefront step / fan-out chunk
constexpr int FAN_LDS = 2048;                // fan-out list entries a grid block stages in LDS
constexpr int NARROW_BS = 1024;              // threads of the single-block JP kernel
constexpr int JP_NARROW_MAX = 2048;          // level size the single block takes
constexpr int JP_NARROW_EDGES = 1 << 14;     // level edges the single block takes
constexpr int NARROW_SCAN = 1 << 16;         // round size whose level-0 scan the block takes
constexpr int NARROW_PUSH_WORK = 1 << 16;    // push work (edges) the block takes

enum { JP_MODE_NARROW = 0, JP_MODE_WIDE = 1 };
enum { PH_FRONTIER = 0, PH_LEVEL = 1, PH_PUSH = 2 };
enum { OP_NONE = 0, OP_FRONTIER = 1, OP_LEVEL = 2, OP_PUSH = 3 };

// JP progress.  Lives in the control block between kernels; the single-block
// kernel keeps its own copy in LDS while it runs.
struct JpState {
  int round;                   // round being coloured (L .. 1)
  int phase;                   // PH_* of that round
  int level;                   // level inside the round
  int mode;                    // JP_MODE_* of that level
  int done;                    // JP finished
  int levels;                  // levels processed (all rounds)
  unsigned int F;              // vertices that started a level 0
  unsigned int fcnt[3];        // plain vertices per level (by level mod 3)
  unsigned long long hctr[3];  // fan-out vertices (low 32 bits) and chunks (high 32 bits)
  unsigned long long ecnt[3];  // same-round successor edges of each level's vertices
  unsigned long long phctr;    // push fan-out vertices and chunks of the current round
};

// Device-resident control block (one per workspace).
struct Ctrl {
  // ADG round state
  unsigned long long N;        // |U_l|
  unsigned long long S;        // sum of D over U_l
  unsigned long long Nnext;    // |U_{l+1}|
  unsigned long long SUnext;   // sum over U_{l+1} of D at selection time
  unsigned long long sum_active;
  unsigned long long cut_edges;
  unsigned int T;              // threshold of round l
  int round;                   // l
  unsigned int nRs, nRb;       // |R_l| split: lane-per-vertex / wave-per-vertex rows
  int done;                    // ADG finished
  int num_rounds;
  int error;                   // ADG_ERR_* raised on the device
  int stats_round;             // last round k_stats has computed
  // JP state
  int grid_op;                 // OP_* the grid kernel has to run next
  int grid_ran;                // the grid kernel has run grid_op
  int num_colors;
  int pad_jp;
  JpState js;
};

struct Params {
  int n;
  long long nnz;
  const long long* rp;
  const int* col;
  unsigned long long p, q;     // eps = p / q
  uint32_t hkey;               // tie-break hash key
  int fused;                   // JP Part 1 fused into UPDATE
  int max_rounds;
  int ord_identity;            // ORD is the identity (one pseudo-round: jp_color)
  Ctrl* ctrl;
  int* round;                  // rho_ADG (user output or workspace)
  int* D;
  unsigned char* status;       // 0 = active, else 1 + ((round - 1) mod 255)
  int* UL[2];                  // active lists (double-buffered)
  int* ORD;                    // [R_1 | R_2 | ... | R_L]
  unsigned* roundN;            // |U_l| per round, roundN[L+1] = 0
  unsigned long long* bcount;  // [SEL_BLOCKS][3] per-block counts
  unsigned long long* boff;    // [SEL_BLOCKS][3] their exclusive scan
  unsigned long long* bsum;    // [SEL_BLOCKS]
  unsigned long long* xpart;   // [upd_blocks] decrement counts
  int upd_blocks;
  int* dag;                    // [nnz] rows as [pred | same-round succ | earlier succ]
  int* npred;                  // |pred(v)|
  int* nsr;                    // same-round successors of v (JP levels walk these)
  unsigned long long* word;    // JP word (adg_device.h)
  unsigned* F[2];              // level lists, plain vertices (by level parity)
  unsigned long long* H[2];    // level lists, fan-out vertices: (first chunk << 32) | vertex
  unsigned long long* PH;      // push fan-out list of the current round
  unsigned hub_cap;
  int* eoff;                   // [n+1] extension-word offsets
  unsigned long long* ext;     // extension words (colours above 40)
  unsigned long long ext_cap;
  int* color;
};

// Status byte of a vertex removed in round l.  Codes repeat every 255 rounds,
// so a matching code is confirmed against the full round number.
__device__ __forceinline__ unsigned char round_code(int l) { return (unsigned char)(1 + ((l - 1) % 255)); }

// Scoped accesses for JP data.  The grid-wide kernels exchange data between
// workgroups and use agent scope; the single-block kernel is one workgroup
// and uses workgroup scope, which lets its accesses stay in the L2 instead of
// going to the device coherence point.
constexpr int SC_AGENT = __HIP_MEMORY_SCOPE_AGENT;
constexpr int SC_WG = __HIP_MEMORY_SCOPE_WORKGROUP;
template <int S>
__device__ __forceinline__ unsigned long long ld64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, S);
}
template <int S>
__device__ __forceinline__ unsigned ld32(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, S);
}
template <int S>
__device__ __forceinline__ int ldi(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, S);
}
template <int S>
__device__ __forceinline__ void st64(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, S);
}
template <int S>
__device__ __forceinline__ void sti(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, S);
}
template <int S>
__device__ __forceinline__ void or64(unsigned long long* p, unsigned long long v) {
  __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, S);
}
template <int S>
__device__ __forceinline__ unsigned long long add64(unsigned long long* p, unsigned long long v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, S);
}
template <int S>
__device__ __forceinline__ unsigned add32(unsigned* p, unsigned v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, S);
}

// ================================================================ ADG

__global__ void k_init(Params P) {
  Ctrl* c = P.ctrl;
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  c->N = c->S = c->Nnext = c->SUnext = 0;
  c->sum_active = c->cut_edges = 0;
  c->T = 0;
  c->round = 0;
  c->nRs = c->nRb = 0;
  c->done = 0;
  c->num_rounds = 0;
  c->error = 0;
  c->stats_round = 0;
  c->grid_op = OP_NONE;
  c->grid_ran = 0;
  c->num_colors = 0;
  JpState& j = c->js;
  j.round = 0;
  j.phase = PH_FRONTIER;
  j.level = 0;
  j.mode = JP_MODE_NARROW;
  j.done = 0;
  j.levels = 0;
  j.F = 0;
  for (int k = 0; k < 3; ++k) {
    j.fcnt[k] = 0;
    j.hctr[k] = 0;
    j.ecnt[k] = 0;
  }
  j.phctr = 0;
}

// One block.  Computes N_l, S_l and T_l for round l, or ends the loop.
// Idempotent per round (the host may issue it twice for one l).
__global__ void k_stats(Params P, int l) {
  Ctrl* c = P.ctrl;
  if (c->done || c->stats_round == l) return;
  __shared__ unsigned long long red[BS];
  unsigned long long x = 0;
  if (l > 1)
    for (int i = threadIdx.x; i < P.upd_blocks; i += BS) x += P.xpart[i];
  red[threadIdx.x] = x;
  __syncthreads();
  for (int s = BS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  c->stats_round = l;
  unsigned long long N, S;
  if (l == 1) {
    N = (unsigned long long)P.n;
    S = (unsigned long long)P.nnz;
  } else {
    N = c->Nnext;
    S = c->SUnext - red[0];
    c->cut_edges += red[0];
  }
  if (l <= P.max_rounds + 1) P.roundN[l] = (unsigned)N;
  if (N == 0) {
    c->done = 1;
    c->num_rounds = l - 1;
    return;
  }
  if (l > P.max_rounds) {
    c->error = ADG_ERR_INTERNAL;
    c->done = 1;
    c->num_rounds = l - 1;
    return;
  }
  unsigned long long T = ((P.q + P.p) * S) / (P.q * N);
  c->N = N;
  c->S = S;
  c->T = (unsigned)(T > 0x7fffffffull ? 0x7fffffffull : T);
  c->round = l;
  c->sum_active += N;
}

struct Chunk {
  long long beg, end;
};
// Contiguous slice of [0, N) for this block (a multiple of BS long).
__device__ __forceinline__ Chunk sel_chunk(unsigned long long N) {
  unsigned long long per = (N + gridDim.x - 1) / gridDim.x;
  per = (per + BS - 1) / BS * BS;
  long long b = (long long)(per * blockIdx.x);
  long long e = b + (long long)per;
  if (b > (long long)N) b = (long long)N;
  if (e > (long long)N) e = (long long)N;
  return {b, e};
}

// Category of element i of U_l: 0 = in R (lane-per-vertex row),
// 1 = in R (wave-per-vertex row), 2 = stays in U.
struct Sel {
  int u;
  int d;
  int cat;
};
__device__ __forceinline__ Sel classify(const Params& P, int l, long long i, unsigned T, const int* Uin) {
  Sel s;
  if (l == 1) {
    s.u = (int)i;
    s.d = (int)(P.rp[i + 1] - P.rp[i]);
    if ((unsigned)s.d <= T) s.cat = s.d <= SMALL_DEG ? 0 : 1;
    else s.cat = 2;
  } else {
    s.u = Uin[i];
    s.d = P.D[s.u];
    if ((unsigned)s.d <= T) {
      int deg = (int)(P.rp[s.u + 1] - P.rp[s.u]);
      s.cat = deg <= SMALL_DEG ? 0 : 1;
    } else {
      s.cat = 2;
    }
  }
  return s;
}

__global__ __launch_bounds__(BS) void k_count(Params P, int l) {
  Ctrl* c = P.ctrl;
  if (c->done) return;
  const unsigned long long N = c->N;
  const unsigned T = c->T;
  const int* Uin = P.UL[(l + 1) & 1];
  Chunk ch = sel_chunk(N);
  unsigned c0 = 0, c1 = 0, c2 = 0;
  unsigned long long s2 = 0;
  for (long long i = ch.beg + threadIdx.x; i < ch.end; i += BS) {
    Sel s = classify(P, l, i, T, Uin);
    c0 += s.cat == 0;
    c1 += s.cat == 1;
    if (s.cat == 2) {
      c2 += 1;
      s2 += (unsigned long long)s.d;
    }
  }
  c0 = wave_sum(c0);
  c1 = wave_sum(c1);
  c2 = wave_sum(c2);
  s2 = wave_sum(s2);
  __shared__ unsigned long long red[WPB][4];
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    red[w][0] = c0;
    red[w][1] = c1;
    red[w][2] = c2;
    red[w][3] = s2;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    unsigned long long t = 0;
    for (int k = 0; k < WPB; ++k) t += red[k][threadIdx.x];
    if (threadIdx.x < 3) P.bcount[blockIdx.x * 3 + threadIdx.x] = t;
    else P.bsum[blockIdx.x] = t;
  }
}

// One block: exclusive scan of SEL_BLOCKS x 3 counts.
__global__ __launch_bounds__(BS) void k_scan(Params P, int l) {
  Ctrl* c = P.ctrl;
  if (c->done) return;
  constexpr int PER = SEL_BLOCKS / BS;
  __shared__ unsigned long long part[3][BS];
  __shared__ unsigned long long sums[BS];
  unsigned long long loc[3] = {0, 0, 0};
  unsigned long long ssum = 0;
  const int b0 = threadIdx.x * PER;
  for (int k = 0; k < PER; ++k) {
    for (int j = 0; j < 3; ++j) loc[j] += P.bcount[(b0 + k) * 3 + j];
    ssum += P.bsum[b0 + k];
  }
  for (int j = 0; j < 3; ++j) part[j][threadIdx.x] = loc[j];
  sums[threadIdx.x] = ssum;
  __syncthreads();
  for (int off = 1; off < BS; off <<= 1) {
    unsigned long long v[3];
    unsigned long long sv = 0;
    for (int j = 0; j < 3; ++j) v[j] = threadIdx.x >= off ? part[j][threadIdx.x - off] : 0;
    if (threadIdx.x >= off) sv = sums[threadIdx.x - off];
    __syncthreads();
    for (int j = 0; j < 3; ++j) part[j][threadIdx.x] += v[j];
    sums[threadIdx.x] += sv;
    __syncthreads();
  }
  unsigned long long run[3];
  for (int j = 0; j < 3; ++j) run[j] = part[j][threadIdx.x] - loc[j];
  for (int k = 0; k < PER; ++k)
    for (int j = 0; j < 3; ++j) {
      unsigned long long v = P.bcount[(b0 + k) * 3 + j];
      P.boff[(b0 + k) * 3 + j] = run[j];
      run[j] += v;
    }
  if (threadIdx.x == BS - 1) {
    c->nRs = (unsigned)part[0][BS - 1];
    c->nRb = (unsigned)part[1][BS - 1];
    c->Nnext = part[2][BS - 1];
    c->SUnext = sums[BS - 1];
  }
}

// R_l's slot in ORD: vertices removed before round l take the first n - |U_l|.
__device__ __forceinline__ int* round_slot(const Params& P, unsigned long long N) { return P.ORD + (P.n - N); }

// Stable compaction of U_l into R_l (small rows, then big rows) and U_{l+1}.
__global__ __launch_bounds__(BS) void k_scatter(Params P, int l) {
  Ctrl* c = P.ctrl;
  if (c->done) return;
  const unsigned long long N = c->N;
  const unsigned T = c->T;
  const unsigned nRs = c->nRs;
  const int* Uin = P.UL[(l + 1) & 1];
  int* Uout = P.UL[l & 1];
  int* RL = round_slot(P, N);
  Chunk ch = sel_chunk(N);
  unsigned long long base0 = P.boff[blockIdx.x * 3 + 0];
  unsigned long long base1 = P.boff[blockIdx.x * 3 + 1];
  unsigned long long base2 = P.boff[blockIdx.x * 3 + 2];
  __shared__ unsigned wcnt[WPB][3];
  const int w = threadIdx.x / WAVE;
  const unsigned char code = round_code(l);
  for (long long t = ch.beg; t < ch.end; t += BS) {
    long long i = t + threadIdx.x;
    bool valid = i < ch.end;
    Sel s = {0, 0, 3};
    if (valid) s = classify(P, l, i, T, Uin);
    uint64_t m0 = ballot(s.cat == 0), m1 = ballot(s.cat == 1), m2 = ballot(s.cat == 2);
    if (lane_id() == 0) {
      wcnt[w][0] = __popcll(m0);
      wcnt[w][1] = __popcll(m1);
      wcnt[w][2] = __popcll(m2);
    }
    __syncthreads();
    unsigned pre[3] = {0, 0, 0}, tot[3] = {0, 0, 0};
    for (int k = 0; k < WPB; ++k)
      for (int j = 0; j < 3; ++j) {
        if (k < w) pre[j] += wcnt[k][j];
        tot[j] += wcnt[k][j];
      }
    if (s.cat == 0) RL[base0 + pre[0] + lanes_below(m0)] = s.u;
    else if (s.cat == 1) RL[nRs + base1 + pre[1] + lanes_below(m1)] = s.u;
    else if (s.cat == 2) Uout[base2 + pre[2] + lanes_below(m2)] = s.u;
    if (valid) {
      if (s.cat != 2) {
        P.round[s.u] = l;
        P.status[s.u] = code;
      } else if (l == 1) {
        P.round[s.u] = 0;
        P.status[s.u] = 0;
        P.D[s.u] = s.d;
      }
    }
    base0 += tot[0];
    base1 += tot[1];
    base2 += tot[2];
    __syncthreads();
  }
}

// Neighbour classes of v in round l: 0 = JP predecessor (w still in U, or
// removed in round l with a larger hash), 1 = same-round successor,
// 2 = successor from an earlier round.  Decrements D[w] for w still in U.
template <bool FUSED>
__device__ __forceinline__ int visit3(const Params& P, int w, int l, unsigned char code, uint32_t hv, unsigned& x,
                                      bool decrement) {
  unsigned char st = P.status[w];
  if (st == 0) {
    if (decrement) {
      atomicSub(&P.D[w], 1);
      x += 1;
    }
    return 0;
  }
  if (FUSED && st == code && P.round[w] == l) return tiebreak(P.hkey, (uint32_t)w) > hv ? 0 : 1;
  return 2;
}

__device__ __forceinline__ void store_row_meta(const Params& P, int v, long long np, long long ns) {
  P.npred[v] = (int)np;
  P.nsr[v] = (int)ns;
  P.word[v] = (unsigned long long)np << JP_MASK_BITS;
  if (np > JP_MAX_PRED) atomicExch(&P.ctrl->error, ADG_ERR_UNSUPPORTED);
}

// Lane-per-vertex UPDATE for rows of at most SMALL_DEG entries: one pass to
// count (and decrement), one pass to place the partitioned row.
template <bool FUSED>
__device__ void update_small(const Params& P, int v, bool valid, int l, unsigned char code, unsigned& x) {
  long long b = 0, e = 0;
  if (valid) {
    b = P.rp[v];
    e = P.rp[v + 1];
  }
  const uint32_t hv = tiebreak(P.hkey, (uint32_t)v);
  long long np = 0, ns = 0;
  for (long long j = b; j < e; ++j) {
    int cl = visit3<FUSED>(P, P.col[j], l, code, hv, x, true);
    np += cl == 0;
    ns += cl == 1;
  }
  if (!FUSED || !valid) return;
  long long f = b, s = b + np, r = e;
  for (long long j = b; j < e; ++j) {
    int w = P.col[j];
    int cl = visit3<FUSED>(P, w, l, code, hv, x, false);
    if (cl == 0) P.dag[f++] = w;
    else if (cl == 1) P.dag[s++] = w;
    else P.dag[--r] = w;
  }
  store_row_meta(P, v, np, ns);
}

// Wave-per-vertex UPDATE for longer rows: count pass (with the decrements),
// then a placing pass.
template <bool FUSED>
__device__ void update_big(const Params& P, int v, int l, unsigned char code, unsigned& x) {
  const long long b = P.rp[v], e = P.rp[v + 1];
  const uint32_t hv = tiebreak(P.hkey, (uint32_t)v);
  const unsigned lane = lane_id();
  long long np = 0, ns = 0;
  for (long long base = b; base < e; base += WAVE) {
    long long j = base + lane;
    bool valid = j < e;
    int w = valid ? P.col[j] : 0;
    int cl = valid ? visit3<FUSED>(P, w, l, code, hv, x, true) : 3;
    if (FUSED) {
      np += __popcll(ballot(cl == 0));
      ns += __popcll(ballot(cl == 1));
    }
  }
  if (!FUSED) return;
  long long fc = 0, sc = 0, lc = 0;
  for (long long base = b; base < e; base += WAVE) {
    long long j = base + lane;
    bool valid = j < e;
    int w = valid ? P.col[j] : 0;
    int cl = valid ? visit3<FUSED>(P, w, l, code, hv, x, false) : 3;
    uint64_t pm = ballot(cl == 0), sm = ballot(cl == 1), lm = ballot(cl == 2);
    if (cl == 0) P.dag[b + fc + lanes_below(pm)] = w;
    else if (cl == 1) P.dag[b + np + sc + lanes_below(sm)] = w;
    else if (cl == 2) P.dag[e - 1 - lc - lanes_below(lm)] = w;
    fc += __popcll(pm);
    sc += __popcll(sm);
    lc += __popcll(lm);
  }
  if (lane == 0) store_row_meta(P, v, np, ns);
}

template <bool FUSED>
__global__ __launch_bounds__(BS) void k_update(Params P, int l) {
  Ctrl* c = P.ctrl;
  if (c->done) return;
  const unsigned nRs = c->nRs, nRb = c->nRb;
  const int* RL = round_slot(P, c->N);
  const unsigned char code = round_code(l);
  __shared__ unsigned long long xred[WPB];
  const long long nsg = (nRs + WAVE - 1) / WAVE;
  const long long items = nsg + nRb;
  const long long gw = (long long)blockIdx.x * WPB + threadIdx.x / WAVE;
  const long long gstride = (long long)gridDim.x * WPB;
  unsigned x = 0;
  for (long long it = gw; it < items; it += gstride) {
    if (it < nsg) {
      long long idx = it * WAVE + lane_id();
      bool valid = idx < nRs;
      int v = valid ? RL[idx] : 0;
      update_small<FUSED>(P, v, valid, l, code, x);
    } else {
      update_big<FUSED>(P, RL[nRs + (it - nsg)], l, code, x);
    }
  }
  unsigned long long xs = wave_sum((unsigned long long)x);
  if (lane_id() == 0) xred[threadIdx.x / WAVE] = xs;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int k = 0; k < WPB; ++k) t += xred[k];
    P.xpart[blockIdx.x] = t;
  }
}

// ================================================================ JP Part 1 (stand-alone)

__device__ __forceinline__ uint64_t prio(const Params& P, int w) {
  return ((uint64_t)(uint32_t)P.round[w] << 32) | tiebreak(P.hkey, (uint32_t)w);
}

// For jp_color on a given ranking: classify every neighbour by the priority
// <round, hash> and write rows [pred | succ].  All vertices form one
// pseudo-round (ORD is the identity), so every successor is walked by the
// levels: nsr(v) = |succ(v)|.
__global__ __launch_bounds__(BS) void k_part1(Params P) {
  const long long gw = (long long)blockIdx.x * WPB + threadIdx.x / WAVE;
  const long long gstride = (long long)gridDim.x * WPB;
  const unsigned lane = lane_id();
  const long long groups = ((long long)P.n + WAVE - 1) / WAVE;
  for (long long g = gw; g < groups; g += gstride) {
    long long idx = g * WAVE + lane;
    bool valid = idx < P.n;
    int v = valid ? (int)idx : 0;
    long long b = valid ? P.rp[v] : 0, e = valid ? P.rp[v + 1] : 0;
    const uint64_t kv = prio(P, v);
    const bool small = valid && (e - b) <= SMALL_DEG;
    if (small) {
      long long f = b, s = e;
      for (long long j = b; j < e; ++j) {
        int w = P.col[j];
        if (prio(P, w) > kv) P.dag[f++] = w;
        else P.dag[--s] = w;
      }
      store_row_meta(P, v, f - b, e - f);
    }
    uint64_t big = ballot(valid && !small);
    while (big) {
      int L = __ffsll((long long)big) - 1;
      big &= big - 1;
      int u = readlane_i(v, L);
      long long ub = P.rp[u], ue = P.rp[u + 1];
      const uint64_t ku = prio(P, u);
      long long fc = 0, sc = 0;
      for (long long base = ub; base < ue; base += WAVE) {
        long long j = base + lane;
        bool ok = j < ue;
        int w = ok ? P.col[j] : 0;
        bool pr = ok && prio(P, w) > ku;
        uint64_t pm = ballot(pr), sm = ballot(ok && !pr);
        if (pr) P.dag[ub + fc + lanes_below(pm)] = w;
        else if (ok) P.dag[ue - 1 - sc - lanes_below(sm)] = w;
        fc += __popcll(pm);
        sc += __popcll(sm);
      }
      if (lane == 0) store_row_meta(P, u, fc, sc);
    }
  }
}

// ================================================================ JP Part 2

// Colours above 40 do not fit the JP word.  A vertex that may need them
// (|pred| + 1 > 40) owns E(v) = ceil((|pred| + 1 - 40) / 64) extension words
// ext[eoff[v] .. eoff[v+1]) with bits for colours 41, 42, ...; the smallest
// free colour never exceeds |pred| + 1, so they always suffice.  eoff is an
// exclusive scan of E over vertices.
__device__ __forceinline__ int ext_words(int np) {
  int over = np + 1 - JP_MASK_BITS;
  return over > 0 ? (over + 63) / 64 : 0;
}

__global__ __launch_bounds__(BS) void k_ext_count(Params P) {
  Chunk ch = sel_chunk((unsigned long long)P.n);
  unsigned long long s = 0;
  for (long long v = ch.beg + threadIdx.x; v < ch.end; v += BS) s += (unsigned long long)ext_words(P.npred[v]);
  s = wave_sum(s);
  __shared__ unsigned long long red[WPB];
  if (lane_id() == 0) red[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int k = 0; k < WPB; ++k) t += red[k];
    P.bsum[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(BS) void k_ext_scan(Params P) {
  constexpr int PER = SEL_BLOCKS / BS;
  __shared__ unsigned long long part[BS];
  unsigned long long loc = 0;
  const int b0 = threadIdx.x * PER;
  for (int k = 0; k < PER; ++k) loc += P.bsum[b0 + k];
  part[threadIdx.x] = loc;
  __syncthreads();
  for (int off = 1; off < BS; off <<= 1) {
    unsigned long long v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  unsigned long long run = part[threadIdx.x] - loc;
  for (int k = 0; k < PER; ++k) {
    P.boff[(b0 + k) * 3] = run;
    run += P.bsum[b0 + k];
  }
  if (threadIdx.x == BS - 1) {
    P.eoff[P.n] = (int)part[BS - 1];
    if (part[BS - 1] > P.ext_cap) atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
  }
}

// Writes eoff for the block's slice of vertices and clears their extension words.
__global__ __launch_bounds__(BS) void k_ext_fill(Params P) {
  Chunk ch = sel_chunk((unsigned long long)P.n);
  unsigned long long base = P.boff[blockIdx.x * 3];
  __shared__ unsigned wsum[WPB];
  const int w = threadIdx.x / WAVE;
  for (long long t = ch.beg; t < ch.end; t += BS) {
    long long v = t + threadIdx.x;
    int E = v < ch.end ? ext_words(P.npred[v]) : 0;
    int incl = E;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
      int o = __shfl_up(incl, off, WAVE);
      if ((int)lane_id() >= off) incl += o;
    }
    if (lane_id() == WAVE - 1) wsum[w] = incl;
    __syncthreads();
    unsigned pre = 0, tot = 0;
    for (int k = 0; k < WPB; ++k) {
      if (k < w) pre += wsum[k];
      tot += wsum[k];
    }
    unsigned long long off = base + pre + (incl - E);
    if (v < ch.end) {
      P.eoff[v] = (int)off;
      for (int k = 0; k < E && off + k < P.ext_cap; ++k) P.ext[off + k] = 0;
    }
    base += tot;
    __syncthreads();
  }
}

// Colour of v when colours 1..40 are all taken by its predecessors: the first
// clear bit of its extension words.  Whole wavefront.  Only called once every
// predecessor has finished (earlier level, round or push), so all bits are final.
template <int S>
__device__ int jp_ext_color(const Params& P, int v) {
  const unsigned lane = lane_id();
  const int e0 = P.eoff[v], e1 = P.eoff[v + 1];
  for (int base = e0; base < e1; base += WAVE) {
    int k = base + (int)lane;
    int found = 0x7fffffff;
    if (k < e1) {
      unsigned long long wd = ld64<S>(&P.ext[k]);
      if (~wd) found = (k - e0) * 64 + __ffsll((long long)~wd) - 1;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      int o = __shfl_xor(found, off, WAVE);
      found = o < found ? o : found;
    }
    if (found != 0x7fffffff) return JP_MASK_BITS + 1 + found;
  }
  // unreachable for a consistent DAG: E(v) words cover colours up to |pred|+1
  if (lane == 0) atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
  return JP_MASK_BITS + 1 + (e1 - e0) * 64;
}

// Record colour c (> 40) of a predecessor in successor u's extension words, if
// u has a word for it (colours beyond |pred(u)| + 1 cannot matter to u).
template <int S>
__device__ __forceinline__ void jp_ext_mark(const Params& P, int u, int c) {
  const int e0 = P.eoff[u], e1 = P.eoff[u + 1];
  const int k = (c - JP_MASK_BITS - 1) >> 6;
  if (k < e1 - e0) or64<S>(&P.ext[e0 + k], 1ull << ((c - JP_MASK_BITS - 1) & 63));
}

// Same-round successor update: record colour c, take one count unit off u's
// word; true if that was u's last uncoloured predecessor.
template <int S>
__device__ __forceinline__ bool jp_touch(const Params& P, int u, int c) {
  if (c > JP_MASK_BITS) jp_ext_mark<S>(P, u, c);
  else or64<S>(&P.word[u], 1ull << (c - 1));
  unsigned long long old = add64<S>(&P.word[u], (unsigned long long)(-(long long)JP_ONE));
  return (old >> JP_MASK_BITS) == 1;
}

// Earlier-round successor update (bulk push): the same, without a result --
// u becomes ready in its own round's level-0 scan.
template <int S>
__device__ __forceinline__ void jp_push_one(const Params& P, int u, int c) {
  if (c > JP_MASK_BITS) jp_ext_mark<S>(P, u, c);
  else or64<S>(&P.word[u], 1ull << (c - 1));
  add64<S>(&P.word[u], (unsigned long long)(-(long long)JP_ONE));
}

// GetColor for a ready vertex: the first clear bit of its word, or of its
// extension words when colours 1..40 are all taken.  Whole wavefront.
template <int S>
__device__ __forceinline__ int jp_colour(const Params& P, bool act, int v) {
  int col = 0;
  unsigned long long M = 0;
  if (act) M = ld64<S>(&P.word[v]) & JP_MASK;
  const bool full = act && M == JP_MASK;
  if (act && !full) col = __ffsll((long long)~M);  // first clear bit i -> colour i + 1
  uint64_t wide = ballot(full);
  while (wide) {
    int L = __ffsll((long long)wide) - 1;
    wide &= wide - 1;
    int cc = jp_ext_color<S>(P, readlane_i(v, L));
    if (lane_id() == (unsigned)L) col = cc;
  }
  return col;
}

// ---- level lists
// Level l's vertices with at most JP_SMALL same-round successors are in
// F[l & 1] (count fcnt[l % 3]); the others ("fan-out" vertices) are in
// H[l & 1] as (first chunk, vertex), their same-round successors cut into
// chunks of JP_CHUNK that different wavefronts process (hctr[l % 3]: entries
// in the low 32 bits, chunks in the high 32 bits, so one atomic gives both and
// the entries come out sorted by first chunk).

struct JpStage {
  unsigned* buf;                // LDS staging of plain vertices
  unsigned* cnt;                // its fill level (LDS)
  unsigned* fcnt;               // level counters (control block, or LDS in the single block)
  unsigned long long* hctr;
  unsigned long long* ecnt;
  unsigned long long* phctr;
};

// Append u (ready) to level l + 1.
template <int S>
__device__ __forceinline__ void jp_append(const Params& P, JpStage& st, int l, bool rdy, int u) {
  long long ns = 0;
  if (rdy) ns = P.nsr[u];
  if (ballot(rdy)) {
    unsigned long long es = wave_sum((unsigned long long)ns);
    if (lane_id() == 0 && es) add64<S>(&st.ecnt[(l + 1) % 3], es);
  }
  const bool fan = rdy && ns > JP_SMALL;
  if (fan) {
    unsigned long long nch = (unsigned long long)((ns + JP_CHUNK - 1) / JP_CHUNK);
    unsigned long long old = add64<S>(&st.hctr[(l + 1) % 3], (nch << 32) | 1ull);
    unsigned pos = (unsigned)old;
    if (pos < P.hub_cap) st64<S>(&P.H[(l + 1) & 1][pos], (old & 0xffffffff00000000ull) | (unsigned)u);
    else atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
  }
  const bool plain = rdy && !fan;
  uint64_t m = ballot(plain);
  if (!m) return;
  unsigned k = __popcll(m);
  unsigned base = 0;
  if (lane_id() == 0) base = atomicAdd(st.cnt, k);
  base = readlane_u(base, 0);
  const unsigned pos = base + lanes_below(m);
  if (plain && pos < (unsigned)FB_CAP) st.buf[pos] = (unsigned)u;
  if (base + k > (unsigned)FB_CAP) {
    uint64_t om = ballot(plain && pos >= (unsigned)FB_CAP);
    unsigned g = 0;
    if (lane_id() == 0) g = add32<S>(&st.fcnt[(l + 1) % 3], (unsigned)__popcll(om));
    g = readlane_u(g, 0);
    if (plain && pos >= (unsigned)FB_CAP) sti<S>((int*)&P.F[(l + 1) & 1][g + lanes_below(om)], u);
  }
}

// Block-wide: move the staged vertices to level l + 1's list.
template <int S>
__device__ __forceinline__ void jp_stage_flush(const Params& P, JpStage& st, int l) {
  __syncthreads();
  __shared__ unsigned gbase;
  unsigned k = *st.cnt;
  if (k > (unsigned)FB_CAP) k = FB_CAP;
  if (threadIdx.x == 0) gbase = k ? add32<S>(&st.fcnt[(l + 1) % 3], k) : 0;
  __syncthreads();
  for (unsigned i = threadIdx.x; i < k; i += blockDim.x)
    sti<S>((int*)&P.F[(l + 1) & 1][gbase + i], (int)st.buf[i]);
  __syncthreads();
  if (threadIdx.x == 0) *st.cnt = 0;
  __syncthreads();
}

// Whole wavefront: same-round successors dag[s0 .. s1) of a vertex of colour cc.
template <int S>
__device__ __forceinline__ void jp_succ_range(const Params& P, JpStage& st, int l, int cc, long long s0,
                                              long long s1) {
  const unsigned lane = lane_id();
  for (long long base = s0; base < s1; base += JP_CHUNK) {
    int u[JP_UNROLL];
    bool ok[JP_UNROLL];
#pragma unroll
    for (int t = 0; t < JP_UNROLL; ++t) {
      long long j = base + t * WAVE + lane;
      ok[t] = j < s1;
      u[t] = ok[t] ? P.dag[j] : 0;
    }
    bool rdy[JP_UNROLL];
#pragma unroll
    for (int t = 0; t < JP_UNROLL; ++t) rdy[t] = ok[t] && jp_touch<S>(P, u[t], cc);
#pragma unroll
    for (int t = 0; t < JP_UNROLL; ++t) jp_append<S>(P, st, l, rdy[t], u[t]);
  }
}

// Fan-out chunk k of a list sorted by first chunk: its entry (binary search,
// in the block's LDS copy `lds` when the list was staged there).
template <int S>
__device__ __forceinline__ unsigned long long fan_entry(const unsigned long long* Hl, unsigned nh, unsigned k,
                                                        const unsigned long long* lds) {
  unsigned lo = 0, hi = nh;
  if (lds) {
    while (hi - lo > 1) {
      unsigned mid = (lo + hi) >> 1;
      if ((unsigned)(lds[mid] >> 32) <= k) lo = mid;
      else hi = mid;
    }
    return lds[lo];
  }
  while (hi - lo > 1) {
    unsigned mid = (lo + hi) >> 1;
    if ((unsigned)(ld64<S>(&Hl[mid]) >> 32) <= k) lo = mid;
    else hi = mid;
  }
  return ld64<S>(&Hl[lo]);
}

// Block-wide: stage a fan-out list in LDS if it fits (returns the copy or null).
template <int S>
__device__ __forceinline__ const unsigned long long* fan_stage(const unsigned long long* Hl, unsigned nh,
                                                               unsigned long long* lds) {
  if (nh > (unsigned)FAN_LDS) return nullptr;
  for (unsigned i = threadIdx.x; i < nh; i += blockDim.x) lds[i] = ld64<S>(&Hl[i]);
  __syncthreads();
  return lds;
}

__device__ __forceinline__ long long succ_begin(const Params& P, int v) { return P.rp[v] + P.npred[v]; }

// The work items of level l for wavefronts gw, gw + gstride, ...: items
// [0, groups) are groups of 64 plain vertices (a lane each; the whole wave for
// more than JP_SMALL successors), then the fan-out chunks.
template <int S>
__device__ void jp_level_items(const Params& P, JpStage& st, int l, unsigned nf, unsigned long long hc, long long gw,
                               long long gstride, const unsigned long long* hlds) {
  const unsigned lane = lane_id();
  const unsigned nh = (unsigned)hc;
  const unsigned nch = (unsigned)(hc >> 32);
  const unsigned* Fl = P.F[l & 1];
  const unsigned long long* Hl = P.H[l & 1];
  const long long groups = ((long long)nf + WAVE - 1) / WAVE;
  for (long long it = gw; it < groups + (long long)nch; it += gstride) {
    if (it < groups) {
      // plain vertices: at most JP_SMALL same-round successors, a lane each
      const long long idx = it * WAVE + lane;
      const bool act = idx < nf;
      const int v = act ? (int)ld32<S>(&Fl[idx]) : 0;
      const int col = jp_colour<S>(P, act, v);
      if (act) sti<S>(&P.color[v], col);
      long long b = 0, e = 0;
      if (act) {
        b = succ_begin(P, v);
        e = b + P.nsr[v];
      }
      for (long long j = b; ballot(act && j < e); j += JP_UNROLL) {
        int u[JP_UNROLL];
        bool ok[JP_UNROLL];
#pragma unroll
        for (int t = 0; t < JP_UNROLL; ++t) {
          ok[t] = act && j + t < e;
          u[t] = ok[t] ? P.dag[j + t] : 0;
        }
        bool rdy[JP_UNROLL];
#pragma unroll
        for (int t = 0; t < JP_UNROLL; ++t) rdy[t] = ok[t] && jp_touch<S>(P, u[t], col);
#pragma unroll
        for (int t = 0; t < JP_UNROLL; ++t) jp_append<S>(P, st, l, rdy[t], u[t]);
      }
    } else {
      const unsigned k = (unsigned)(it - groups);
      const unsigned long long ent = fan_entry<S>(Hl, nh, k, hlds);
      const int v = (int)(unsigned)ent;
      const unsigned first = (unsigned)(ent >> 32);
      const int col = jp_colour<S>(P, true, v);
      if (k == first && lane == 0) sti<S>(&P.color[v], col);
      const long long b = succ_begin(P, v), e = b + P.nsr[v];
      const long long s0 = b + (long long)(k - first) * JP_CHUNK;
      const long long s1 = s0 + JP_CHUNK < e ? s0 + JP_CHUNK : e;
      jp_succ_range<S>(P, st, l, col, s0, s1);
    }
  }
}

// ---- per-round operations

__device__ __forceinline__ long long seg_begin(const Params& P, int r) { return (long long)P.n - P.roundN[r]; }
__device__ __forceinline__ long long seg_size(const Params& P, int r) {
  return (long long)P.roundN[r] - (long long)P.roundN[r + 1];
}
__device__ __forceinline__ int seg_vertex(const Params& P, long long i) { return P.ord_identity ? (int)i : P.ORD[i]; }

// Level 0 of round r: its vertices whose count is already zero.  Also lists
// the round's vertices with more than JP_SMALL earlier-round successors for
// the push (chunked across wavefronts), in PH with its counter phctr.
template <int S>
__device__ void jp_frontier_items(const Params& P, JpStage& st, int r, long long gw, long long gstride) {
  const long long b = seg_begin(P, r), sz = seg_size(P, r);
  const unsigned lane = lane_id();
  for (long long g = gw; g * WAVE < sz; g += gstride) {
    long long i = g * WAVE + lane;
    bool ok = i < sz;
    int v = ok ? seg_vertex(P, b + i) : 0;
    bool rdy = ok && (ld64<S>(&P.word[v]) >> JP_MASK_BITS) == 0;
    jp_append<S>(P, st, -1, rdy, v);
    if (ok && !P.ord_identity) {
      long long sb = succ_begin(P, v) + P.nsr[v], se = P.rp[v + 1];
      if (se - sb > JP_SMALL) {
        unsigned long long nch = (unsigned long long)((se - sb + JP_CHUNK - 1) / JP_CHUNK);
        unsigned long long old = add64<S>(st.phctr, (nch << 32) | 1ull);
        unsigned pos = (unsigned)old;
        if (pos < P.hub_cap) st64<S>(&P.PH[pos], (old & 0xffffffff00000000ull) | (unsigned)v);
        else atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
      }
    }
  }
}

// Bulk push of round r's colours to earlier-round successors.  Items: groups
// of 64 vertices of the round (a lane each, for at most JP_SMALL successors),
// then the JP_CHUNK-sized chunks of the longer ranges listed in PH.
template <int S>
__device__ void jp_push_items(const Params& P, int r, unsigned long long phc, long long gw, long long gstride,
                              const unsigned long long* plds) {
  const long long b = seg_begin(P, r), sz = seg_size(P, r);
  const unsigned lane = lane_id();
  const long long groups = (sz + WAVE - 1) / WAVE;
  const unsigned nh = (unsigned)phc, nch = (unsigned)(phc >> 32);
  for (long long it = gw; it < groups + (long long)nch; it += gstride) {
    if (it < groups) {
      long long i = it * WAVE + lane;
      bool act = i < sz;
      int v = act ? seg_vertex(P, b + i) : 0;
      long long s0 = 0, s1 = 0;
      int col = 0;
      if (act) {
        s0 = succ_begin(P, v) + P.nsr[v];
        s1 = P.rp[v + 1];
        act = s1 - s0 <= JP_SMALL;  // longer ranges are chunks
        if (act) col = ldi<S>(&P.color[v]);
      }
      for (long long j = s0; ballot(act && j < s1); j += JP_UNROLL) {
#pragma unroll
        for (int t = 0; t < JP_UNROLL; ++t)
          if (act && j + t < s1) jp_push_one<S>(P, P.dag[j + t], col);
      }
    } else {
      const unsigned k = (unsigned)(it - groups);
      const unsigned long long ent = fan_entry<S>(P.PH, nh, k, plds);
      const int v = (int)(unsigned)ent;
      const unsigned first = (unsigned)(ent >> 32);
      const long long sb = succ_begin(P, v) + P.nsr[v], se = P.rp[v + 1];
      const long long s0 = sb + (long long)(k - first) * JP_CHUNK;
      const long long s1 = s0 + JP_CHUNK < se ? s0 + JP_CHUNK : se;
      const int cc = ldi<S>(&P.color[v]);
#pragma unroll
      for (int t = 0; t < JP_UNROLL; ++t) {
        long long j = s0 + t * WAVE + lane;
        if (j < s1) jp_push_one<S>(P, P.dag[j], cc);
      }
    }
  }
}

// ---- a narrow level in one block, balanced over edges

struct NarrowLds {
  int v[JP_NARROW_MAX];            // the level's vertices
  int col[JP_NARROW_MAX];          // their colours
  long long b[JP_NARROW_MAX];      // first same-round successor in dag
  unsigned off[JP_NARROW_MAX + 1]; // exclusive scan of same-round successor counts
  unsigned wsum[NARROW_BS / WAVE];
};

// Colour of v computed by one thread (its word is final: v is ready).
template <int S>
__device__ __forceinline__ int jp_colour_thread(const Params& P, int v) {
  unsigned long long M = ld64<S>(&P.word[v]) & JP_MASK;
  if (M != JP_MASK) return __ffsll((long long)~M);
  const int e0 = P.eoff[v], e1 = P.eoff[v + 1];
  for (int k = e0; k < e1; ++k) {
    unsigned long long wd = ld64<S>(&P.ext[k]);
    if (~wd) return JP_MASK_BITS + 1 + (k - e0) * 64 + __ffsll((long long)~wd) - 1;
  }
  atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
  return JP_MASK_BITS + 1 + (e1 - e0) * 64;
}

// Level l with nf plain and nh fan-out vertices (nf + nh <= JP_NARROW_MAX):
// colour every vertex (a thread each), scan the same-round successor counts,
// then let every thread update single successors.
template <int S>
__device__ void jp_level_narrow(const Params& P, JpStage& st, NarrowLds& Z, int l, unsigned nf, unsigned nh) {
  const unsigned nv = nf + nh;
  const unsigned* Fl = P.F[l & 1];
  const unsigned long long* Hl = P.H[l & 1];
  const int tid = threadIdx.x;
  // 1. colours
  for (unsigned i = tid; i < nv; i += NARROW_BS) {
    int v = i < nf ? (int)ld32<S>(&Fl[i]) : (int)(unsigned)ld64<S>(&Hl[i - nf]);
    int c = jp_colour_thread<S>(P, v);
    sti<S>(&P.color[v], c);
    Z.v[i] = v;
    Z.col[i] = c;
    Z.b[i] = succ_begin(P, v);
    Z.off[i] = (unsigned)P.nsr[v];
  }
  __syncthreads();
  // 2. exclusive scan of Z.off[0 .. nv) (two entries per thread)
  const unsigned lane = lane_id();
  const int w = tid / WAVE;
  const unsigned a0 = 2u * tid < nv ? Z.off[2 * tid] : 0;
  const unsigned a1 = 2u * tid + 1 < nv ? Z.off[2 * tid + 1] : 0;
  unsigned incl = a0 + a1;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    unsigned t = __shfl_up(incl, o, WAVE);
    if ((int)lane >= o) incl += t;
  }
  if (lane == WAVE - 1) Z.wsum[w] = incl;
  __syncthreads();
  unsigned pre = 0, total = 0;
  for (int k = 0; k < NARROW_BS / WAVE; ++k) {
    if (k < w) pre += Z.wsum[k];
    total += Z.wsum[k];
  }
  __syncthreads();
  const unsigned ex = pre + incl - (a0 + a1);
  if (2u * tid < nv) Z.off[2 * tid] = ex;
  if (2u * tid + 1 < nv) Z.off[2 * tid + 1] = ex + a0;
  if (tid == 0) Z.off[nv] = total;
  __syncthreads();
  // 3. one successor per thread and step
  for (unsigned e0 = 0; e0 < total; e0 += NARROW_BS * JP_UNROLL) {
    int u[JP_UNROLL], cc[JP_UNROLL];
    bool ok[JP_UNROLL];
#pragma unroll
    for (int t = 0; t < JP_UNROLL; ++t) {
      const unsigned e = e0 + t * NARROW_BS + tid;
      ok[t] = e < total;
      u[t] = 0;
      cc[t] = 0;
      if (ok[t]) {
        unsigned lo = 0, hi = nv;  // last i with off[i] <= e
        while (hi - lo > 1) {
          unsigned mid = (lo + hi) >> 1;
          if (Z.off[mid] <= e) lo = mid;
          else hi = mid;
        }
        u[t] = P.dag[Z.b[lo] + (e - Z.off[lo])];
        cc[t] = Z.col[lo];
      }
    }
    bool rdy[JP_UNROLL];
#pragma unroll
    for (int t = 0; t < JP_UNROLL; ++t) rdy[t] = ok[t] && jp_touch<S>(P, u[t], cc[t]);
#pragma unroll
    for (int t = 0; t < JP_UNROLL; ++t) jp_append<S>(P, st, l, rdy[t], u[t]);
  }
}

// ---- JP state machine (plain accesses: the state is in LDS while the
// single-block kernel runs, in the control block between kernels)

__device__ __forceinline__ void jp_decide_level(JpState& j, int l) {
  const unsigned nf = j.fcnt[l % 3];
  const unsigned nh = (unsigned)j.hctr[l % 3];
  if (nf == 0 && nh == 0) {
    j.phase = PH_PUSH;
    return;
  }
  j.mode = (nf + nh > (unsigned)JP_NARROW_MAX || j.ecnt[l % 3] > (unsigned long long)JP_NARROW_EDGES)
               ? JP_MODE_WIDE
               : JP_MODE_NARROW;
}

// Start round r: level lists empty, level 0 to be scanned.
__device__ __forceinline__ void jp_begin_round(JpState& j, int r) {
  j.round = r;
  if (r <= 0) {
    j.done = 1;
    return;
  }
  j.phase = PH_FRONTIER;
  j.level = -1;
  for (int k = 0; k < 3; ++k) {
    j.fcnt[k] = 0;
    j.hctr[k] = 0;
    j.ecnt[k] = 0;
  }
  j.phctr = 0;
}

// After level l's items have been processed (or level 0 was scanned, l = -1).
__device__ __forceinline__ void jp_next_level(JpState& j, int l) {
  const int nl = l + 1;
  j.level = nl;
  j.fcnt[(nl + 1) % 3] = 0;
  j.hctr[(nl + 1) % 3] = 0;
  j.ecnt[(nl + 1) % 3] = 0;
  if (nl == 0) j.F += j.fcnt[0] + (unsigned)j.hctr[0];
  else j.levels += 1;
  j.phase = PH_LEVEL;
  jp_decide_level(j, nl);
}

// Work of round r's push, in successor entries, capped at limit + 1.
__device__ long long jp_push_work(const Params& P, int r, long long limit) {
  __shared__ unsigned long long acc;
  if (threadIdx.x == 0) acc = 0;
  __syncthreads();
  const long long b = seg_begin(P, r), sz = seg_size(P, r);
  unsigned long long mine = 0;
  for (long long i = threadIdx.x; i < sz; i += blockDim.x) {
    int v = seg_vertex(P, b + i);
    mine += (unsigned long long)(P.rp[v + 1] - succ_begin(P, v) - P.nsr[v]);
  }
  mine = wave_sum(mine);
  if (lane_id() == 0) atomicAdd(&acc, mine);
  __syncthreads();
  long long w = (long long)acc;
  __syncthreads();
  return w > limit ? limit + 1 : w;
}

// One block.  Finishes what the grid kernel has just done, then runs every
// step one block can take (scans of small rounds, narrow levels, small
// pushes) with its state in LDS, until JP ends or a step needs the grid.
__global__ __launch_bounds__(NARROW_BS) void k_jp_narrow(Params P, int max_steps) {
  Ctrl* c = P.ctrl;
  __shared__ unsigned fbuf[FB_CAP];
  __shared__ unsigned fcnt;
  __shared__ JpState S;
  __shared__ NarrowLds Z;
  if (threadIdx.x == 0) {
    fcnt = 0;
    S = c->js;
    if (!S.done && c->grid_ran) {
      const int op = c->grid_op;
      c->grid_ran = 0;
      c->grid_op = OP_NONE;
      if (op == OP_FRONTIER) jp_next_level(S, -1);
      else if (op == OP_LEVEL) jp_next_level(S, S.level);
      else if (op == OP_PUSH) jp_begin_round(S, S.round - 1);
    }
  }
  __syncthreads();
  JpStage st{fbuf, &fcnt, S.fcnt, S.hctr, S.ecnt, &S.phctr};
  const long long gw = threadIdx.x / WAVE;
  const long long gstride = NARROW_BS / WAVE;
  int handed = OP_NONE;
  for (int step = 0; step < max_steps && !S.done; ++step) {
    const int r = S.round;
    if (S.phase == PH_FRONTIER) {
      if (seg_size(P, r) > NARROW_SCAN) {
        handed = OP_FRONTIER;
      } else {
        jp_frontier_items<SC_WG>(P, st, r, gw, gstride);
        order_point();
        jp_stage_flush<SC_WG>(P, st, -1);
        order_point();
        __syncthreads();
        if (threadIdx.x == 0) jp_next_level(S, -1);
      }
    } else if (S.phase == PH_LEVEL) {
      if (S.mode == JP_MODE_WIDE) {
        handed = OP_LEVEL;
      } else {
        const int l = S.level;
        jp_level_narrow<SC_WG>(P, st, Z, l, S.fcnt[l % 3], (unsigned)S.hctr[l % 3]);
        order_point();
        jp_stage_flush<SC_WG>(P, st, l);
        order_point();
        __syncthreads();
        if (threadIdx.x == 0) jp_next_level(S, l);
      }
    } else {  // PH_PUSH
      const long long work = P.ord_identity ? 0 : jp_push_work(P, r, NARROW_PUSH_WORK);
      if (work > NARROW_PUSH_WORK) {
        handed = OP_PUSH;
      } else {
        if (work > 0) jp_push_items<SC_WG>(P, r, S.phctr, gw, gstride, nullptr);
        order_point();
        __syncthreads();
        if (threadIdx.x == 0) jp_begin_round(S, r - 1);
      }
    }
    __syncthreads();
    if (handed != OP_NONE) break;
  }
  if (threadIdx.x == 0) {
    c->js = S;
    c->grid_op = handed;
    order_point();
  }
}

// Grid-wide: the step the single-block kernel handed over.
__global__ __launch_bounds__(BS) void k_jp_grid(Params P) {
  Ctrl* c = P.ctrl;
  const int op = c->grid_op;
  if (c->js.done || op == OP_NONE || c->grid_ran) return;
  __shared__ unsigned fbuf[FB_CAP];
  __shared__ unsigned fcnt;
  __shared__ unsigned long long flds[FAN_LDS];
  if (threadIdx.x == 0) fcnt = 0;
  __syncthreads();
  JpStage st{fbuf, &fcnt, c->js.fcnt, c->js.hctr, c->js.ecnt, &c->js.phctr};
  const int r = c->js.round;
  const long long gw = (long long)blockIdx.x * WPB + threadIdx.x / WAVE;
  const long long gstride = (long long)gridDim.x * WPB;
  if (op == OP_FRONTIER) {
    jp_frontier_items<SC_AGENT>(P, st, r, gw, gstride);
    jp_stage_flush<SC_AGENT>(P, st, -1);
  } else if (op == OP_LEVEL) {
    const int l = c->js.level;
    const unsigned long long hc = c->js.hctr[l % 3];
    const unsigned long long* hl = fan_stage<SC_AGENT>(P.H[l & 1], (unsigned)hc, flds);
    jp_level_items<SC_AGENT>(P, st, l, c->js.fcnt[l % 3], hc, gw, gstride, hl);
    jp_stage_flush<SC_AGENT>(P, st, l);
  } else {
    const unsigned long long phc = c->js.phctr;
    const unsigned long long* pl = fan_stage<SC_AGENT>(P.PH, (unsigned)phc, flds);
    jp_push_items<SC_AGENT>(P, r, phc, gw, gstride, pl);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) c->grid_ran = 1;
}

__global__ void k_jp_start(Params P, int rounds) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  Ctrl* c = P.ctrl;
  c->grid_op = OP_NONE;
  c->grid_ran = 0;
  JpState& j = c->js;
  j.done = 0;
  j.levels = 0;
  j.F = 0;
  if (P.ord_identity) {
    P.roundN[1] = (unsigned)P.n;
    P.roundN[2] = 0;
  } else {
    P.roundN[rounds + 1] = 0;
  }
  jp_begin_round(j, rounds);
}

// Largest colour: per-block maxima, one atomic per block.
__global__ __launch_bounds__(BS) void k_max_color(Params P) {
  int m = 0;
  for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < P.n; i += (long long)gridDim.x * BS)
    m = P.color[i] > m ? P.color[i] : m;
  m = wave_max(m);
  __shared__ int red[WPB];
  if (lane_id() == 0) red[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < WPB; ++k) m = red[k] > m ? red[k] : m;
    atomicMax(&P.ctrl->num_colors, m);
  }
}

__global__ void k_finish(Params P, int* num_colors_out, int* num_rounds_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (num_colors_out) *num_colors_out = P.ctrl->num_colors;
  if (num_rounds_out) *num_rounds_out = P.ctrl->num_rounds;
}

// ================================================================ CSR validation

__global__ void k_validate(int n, long long nnz, const long long* rp, const int* col, int* bad) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; v < n; v += stride) {
    long long b = rp[v], e = rp[v + 1];
    if (v == 0 && b != 0) atomicOr(bad, 1);
    if (v == n - 1 && e != nnz) atomicOr(bad, 1);
    if (b > e || b < 0 || e > nnz) {
      atomicOr(bad, 1);
      continue;
    }
    int prev = -1;
    for (long long j = b; j < e; ++j) {
      int w = col[j];
      if (w < 0 || w >= n || w == v || w <= prev) {
        atomicOr(bad, 2);
        break;
      }
      prev = w;
      // symmetric: v must appear in row w
      long long lo = rp[w], hi = rp[w + 1];
      if (lo < 0 || hi > nnz || lo > hi) {
        atomicOr(bad, 1);
        break;
      }
      bool found = false;
      while (lo < hi) {
        long long mid = (lo + hi) >> 1;
        int x = col[mid];
        if (x == (int)v) {
          found = true;
          break;
        }
        if (x < (int)v) lo = mid + 1;
        else hi = mid;
      }
      if (!found) {
        atomicOr(bad, 4);
        break;
      }
    }
  }
}

}  // namespace adg

// ================================================================ host side

using namespace adg;

namespace adg {

// ---- optional per-kernel timing with HIP events on the launch stream
namespace {
const char* kclass_names[KC_NUM] = {"init", "stats", "count", "scan", "scatter", "update", "part1",
                                    "jp_prep", "jp", "finish", "batched", "jp_narrow"};
struct ProfRec {
  int cls;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
unsigned g_prof_mask = 0;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_pool;

hipEvent_t prof_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

hipEvent_t prof_begin(int cls, hipStream_t s) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (!(g_prof_mask & (1u << cls))) return nullptr;
  hipEvent_t a = prof_event();
  if (a && hipEventRecord(a, s) != hipSuccess) {
    g_pool.push_back(a);
    return nullptr;
  }
  return a;
}

void prof_end(int cls, hipStream_t s, hipEvent_t a) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  hipEvent_t b = prof_event();
  if (!b || hipEventRecord(b, s) != hipSuccess) {
    g_pool.push_back(a);
    if (b) g_pool.push_back(b);
    return;
  }
  g_prof.push_back({cls, a, b});
}

}  // namespace adg

namespace {

struct Layout {
  size_t ctrl, bcount, boff, bsum, xpart, D, status, UL0, UL1, ORD, roundN, round, dag, npred, nsr, word, F0, F1, H0,
      H1, PH, hub_cap, eoff, ext, ext_words, total;
};

constexpr int UPD_BLOCKS = 2048;

Layout make_layout(int64_t n, int64_t nnz) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + (bytes ? bytes : 1), 256);
    return o;
  };
  size_t nn = (size_t)n;
  L.ctrl = take(sizeof(Ctrl));
  L.bcount = take(sizeof(unsigned long long) * SEL_BLOCKS * 3);
  L.boff = take(sizeof(unsigned long long) * SEL_BLOCKS * 3);
  L.bsum = take(sizeof(unsigned long long) * SEL_BLOCKS);
  L.xpart = take(sizeof(unsigned long long) * UPD_BLOCKS);
  L.D = take(4 * nn);
  L.status = take(nn);
  L.UL0 = take(4 * nn);
  L.UL1 = take(4 * nn);
  L.ORD = take(4 * nn);
  L.roundN = take(4 * (nn + 4));
  L.round = take(4 * nn);
  L.dag = take(4 * (size_t)nnz);
  L.npred = take(4 * nn);
  L.nsr = take(4 * nn);
  L.word = take(8 * nn);
  L.F0 = take(4 * nn);
  L.F1 = take(4 * nn);
  // fan-out entries: vertices with more than JP_SMALL successors in the
  // range concerned (level lists, push list), at most m / JP_SMALL of them
  L.hub_cap = (size_t)nnz / (2 * JP_SMALL) + 64;
  L.H0 = take(8 * L.hub_cap);
  L.H1 = take(8 * L.hub_cap);
  L.PH = take(8 * L.hub_cap);
  L.eoff = take(4 * (nn + 1));
  // sum over v of ceil((|pred|+1-40)/64) <= m/64 + m/40 < nnz/48, plus slack
  L.ext_words = (size_t)nnz / 48 + 64;
  L.ext = take(8 * L.ext_words);
  L.total = off;
  return L;
}

int check_graph(const adg_csr_t* g) {
  if (!g) return ADG_ERR_ARG;
  if (g->n < 0 || g->n > 0x7ffffffeLL || g->nnz < 0) return ADG_ERR_ARG;
  if (g->n > 0 && (!g->row_ptr)) return ADG_ERR_ARG;
  if (g->nnz > 0 && !g->col_idx) return ADG_ERR_ARG;
  return ADG_OK;
}

int check_ws(void* ws, size_t ws_bytes, int64_t n, int64_t nnz) {
  if (!ws) return ADG_ERR_WORKSPACE;
  if (((uintptr_t)ws & 255) != 0) return ADG_ERR_WORKSPACE;
  if (ws_bytes < make_layout(n, nnz).total) return ADG_ERR_WORKSPACE;
  return ADG_OK;
}

Params make_params(const adg_csr_t* g, void* ws, uint64_t p, uint64_t q, uint64_t seed, int fused, int* round_buf,
                   int* color) {
  Layout L = make_layout(g->n, g->nnz);
  char* base = (char*)ws;
  Params P{};
  P.n = (int)g->n;
  P.nnz = g->nnz;
  P.rp = (const long long*)g->row_ptr;
  P.col = g->col_idx;
  P.p = p;
  P.q = q;
  P.hkey = hash_key_from_seed(seed);
  P.fused = fused;
  P.ord_identity = 0;
  P.ctrl = (Ctrl*)(base + L.ctrl);
  P.round = round_buf ? round_buf : (int*)(base + L.round);
  P.D = (int*)(base + L.D);
  P.status = (unsigned char*)(base + L.status);
  P.UL[0] = (int*)(base + L.UL0);
  P.UL[1] = (int*)(base + L.UL1);
  P.ORD = (int*)(base + L.ORD);
  P.roundN = (unsigned*)(base + L.roundN);
  P.bcount = (unsigned long long*)(base + L.bcount);
  P.boff = (unsigned long long*)(base + L.boff);
  P.bsum = (unsigned long long*)(base + L.bsum);
  P.xpart = (unsigned long long*)(base + L.xpart);
  P.upd_blocks = UPD_BLOCKS;
  P.dag = (int*)(base + L.dag);
  P.npred = (int*)(base + L.npred);
  P.nsr = (int*)(base + L.nsr);
  P.word = (unsigned long long*)(base + L.word);
  P.F[0] = (unsigned*)(base + L.F0);
  P.F[1] = (unsigned*)(base + L.F1);
  P.H[0] = (unsigned long long*)(base + L.H0);
  P.H[1] = (unsigned long long*)(base + L.H1);
  P.PH = (unsigned long long*)(base + L.PH);
  P.hub_cap = (unsigned)L.hub_cap;
  P.eoff = (int*)(base + L.eoff);
  P.ext = (unsigned long long*)(base + L.ext);
  P.ext_cap = L.ext_words;
  P.color = color;
  // Round-count bound from the ADG depth lemma: |U| shrinks by a factor
  // 1/(1+eps) per round, so L <= ceil(log n / log(1+eps)) + 1; +1 margin.
  long long bound = (long long)g->n + 1;
  if (p > 0 && g->n > 1) {
    double b = std::ceil(std::log((double)g->n) / std::log1p((double)p / (double)q)) + 2.0;
    if (b < (double)bound) bound = (long long)b;
  }
  if (bound < 1) bound = 1;
  P.max_rounds = (int)std::min<long long>(bound, 0x7fffffff);
  return P;
}

int* pinned_flags() {
  static int* h = nullptr;
  if (!h && hipHostMalloc((void**)&h, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess) h = nullptr;
  return h;
}

// ADG's round loop.  Synchronises the stream between chunks of rounds.
int run_adg(Params& P, hipStream_t s, bool fused, int* num_rounds_host) {
  {
    TIMED(KC_INIT, s);
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, s, P);
  }
  HIPCHK(hipGetLastError());
  *num_rounds_host = 0;
  if (P.n == 0) return ADG_OK;
  int* h = pinned_flags();
  if (!h) return ADG_ERR_HIP;
  int l = 1;
  int chunk = 8;
  while (true) {
    for (int k = 0; k < chunk; ++k, ++l) {
      {
        TIMED(KC_STATS, s);
        hipLaunchKernelGGL(k_stats, dim3(1), dim3(BS), 0, s, P, l);
      }
      {
        TIMED(KC_COUNT, s);
        hipLaunchKernelGGL(k_count, dim3(SEL_BLOCKS), dim3(BS), 0, s, P, l);
      }
      {
        TIMED(KC_SCAN, s);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(BS), 0, s, P, l);
      }
      {
        TIMED(KC_SCATTER, s);
        hipLaunchKernelGGL(k_scatter, dim3(SEL_BLOCKS), dim3(BS), 0, s, P, l);
      }
      {
        TIMED(KC_UPDATE, s);
        if (fused)
          hipLaunchKernelGGL(k_update<true>, dim3(P.upd_blocks), dim3(BS), 0, s, P, l);
        else
          hipLaunchKernelGGL(k_update<false>, dim3(P.upd_blocks), dim3(BS), 0, s, P, l);
      }
    }
    // one more stats call ends the loop on the device when U is empty
    {
      TIMED(KC_STATS, s);
      hipLaunchKernelGGL(k_stats, dim3(1), dim3(BS), 0, s, P, l);
    }
    HIPCHK(hipGetLastError());
    // done, num_rounds, error are adjacent in the control block
    HIPCHK(hipMemcpyAsync(h, &P.ctrl->done, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h[2]) return h[2];
    if (h[0]) {
      *num_rounds_host = h[1];
      return ADG_OK;
    }
    if (l > P.max_rounds + 1) return ADG_ERR_INTERNAL;
    chunk = std::min(chunk * 2, 64);
  }
}

// JP over the rounds (or one pseudo-round), issued in growing chunks of
// (single-block, grid) kernel pairs; the host reads the finish flag between
// chunks.  Every pair makes progress (each level colours at least one vertex,
// each push ends a round), so the loop ends; a watchdog guards a broken state.
int run_jp(Params& P, hipStream_t s, int rounds) {
  if (P.n == 0) return ADG_OK;
  {
    TIMED(KC_JP_PREP, s);
    hipLaunchKernelGGL(k_ext_count, dim3(SEL_BLOCKS), dim3(BS), 0, s, P);
    hipLaunchKernelGGL(k_ext_scan, dim3(1), dim3(BS), 0, s, P);
    hipLaunchKernelGGL(k_ext_fill, dim3(SEL_BLOCKS), dim3(BS), 0, s, P);
    hipLaunchKernelGGL(k_jp_start, dim3(1), dim3(64), 0, s, P, rounds);
  }
  HIPCHK(hipGetLastError());
  int* h = pinned_flags();
  if (!h) return ADG_ERR_HIP;
  int chunk = 2;
  long long pairs = 0;
  const long long max_pairs = 4LL * ((long long)P.n + rounds + 4);
  while (true) {
    for (int k = 0; k < chunk; ++k) {
      {
        TIMED(KC_JP_NARROW, s);
        hipLaunchKernelGGL(k_jp_narrow, dim3(1), dim3(NARROW_BS), 0, s, P, 1 << 30);
      }
      {
        TIMED(KC_JP, s);
        hipLaunchKernelGGL(k_jp_grid, dim3(P.upd_blocks), dim3(BS), 0, s, P);
      }
    }
    pairs += chunk;
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h, &P.ctrl->js.done, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h[0]) break;
    if (pairs > max_pairs) return ADG_ERR_INTERNAL;
    chunk = std::min(chunk * 2, 256);
  }
  {
    TIMED(KC_FINISH, s);
    hipLaunchKernelGGL(k_max_color, dim3(1024), dim3(BS), 0, s, P);
  }
  HIPCHK(hipGetLastError());
  return ADG_OK;
}

}  // namespace

extern "C" {

size_t adg_workspace_bytes(int64_t n, int64_t nnz) {
  if (n < 0 || nnz < 0 || n > 0x7ffffffeLL) return 0;
  return make_layout(n, nnz).total;
}

int adg_order(const adg_csr_t* g, int32_t eps_num, int32_t eps_den, int32_t* round_out, int32_t* num_rounds_out,
              void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (eps_num < 0 || eps_den < 1 || (g->n > 0 && !round_out)) return ADG_ERR_ARG;
  if ((rc = check_ws(workspace, ws_bytes, g->n, g->nnz))) return rc;
  hipStream_t s = (hipStream_t)stream;
  Params P = make_params(g, workspace, (uint64_t)eps_num, (uint64_t)eps_den, 0, 0, round_out, nullptr);
  int L = 0;
  if ((rc = run_adg(P, s, false, &L))) return rc;
  {
    TIMED(KC_FINISH, s);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, P, (int*)nullptr, num_rounds_out);
  }
  HIPCHK(hipGetLastError());
  return ADG_OK;
}

int jp_color(const adg_csr_t* g, const int32_t* round, uint64_t seed, int32_t* color_out, int32_t* num_colors_out,
             void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (g->n > 0 && (!round || !color_out)) return ADG_ERR_ARG;
  if ((rc = check_ws(workspace, ws_bytes, g->n, g->nnz))) return rc;
  hipStream_t s = (hipStream_t)stream;
  Params P = make_params(g, workspace, 0, 1, seed, 1, const_cast<int*>(round), color_out);
  P.ord_identity = 1;
  {
    TIMED(KC_INIT, s);
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, s, P);
  }
  if (P.n > 0) {
    {
      TIMED(KC_PART1, s);
      hipLaunchKernelGGL(k_part1, dim3(P.upd_blocks), dim3(BS), 0, s, P);
    }
    int* h = pinned_flags();
    if (!h) return ADG_ERR_HIP;
    HIPCHK(hipMemcpyAsync(h, &P.ctrl->error, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h[0]) return h[0];
    if ((rc = run_jp(P, s, 1))) return rc;
  }
  {
    TIMED(KC_FINISH, s);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, P, num_colors_out, (int*)nullptr);
  }
  HIPCHK(hipGetLastError());
  return ADG_OK;
}

int color_graph(const adg_csr_t* g, int32_t eps_num, int32_t eps_den, uint64_t seed, int32_t* color_out,
                int32_t* round_out, int32_t* num_colors_out, int32_t* num_rounds_out, void* workspace,
                size_t ws_bytes, void* stream) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (eps_num < 0 || eps_den < 1 || (g->n > 0 && !color_out)) return ADG_ERR_ARG;
  if ((rc = check_ws(workspace, ws_bytes, g->n, g->nnz))) return rc;
  hipStream_t s = (hipStream_t)stream;
  Params P = make_params(g, workspace, (uint64_t)eps_num, (uint64_t)eps_den, seed, 1, round_out, color_out);
  int L = 0;
  if ((rc = run_adg(P, s, true, &L))) return rc;
  if ((rc = run_jp(P, s, L))) return rc;
  {
    TIMED(KC_FINISH, s);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, P, num_colors_out, num_rounds_out);
  }
  HIPCHK(hipGetLastError());
  return ADG_OK;
}

int adg_get_stats(const void* workspace, size_t ws_bytes, adg_stats_t* out, void* stream) {
  if (!workspace || !out || ws_bytes < sizeof(Ctrl)) return ADG_ERR_ARG;
  Ctrl h;
  hipStream_t s = (hipStream_t)stream;
  const Ctrl* c = (const Ctrl*)workspace;
  HIPCHK(hipMemcpyAsync(&h, c, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  out->num_rounds = h.num_rounds;
  out->num_colors = h.num_colors;
  out->sum_active = (int64_t)h.sum_active;
  out->cut_edges = (int64_t)h.cut_edges;
  out->frontier = h.js.F;
  out->jp_levels = h.js.levels;
  out->error = h.error;
  return ADG_OK;
}

int adg_validate_csr(const adg_csr_t* g, void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (!workspace || ws_bytes < 256 || ((uintptr_t)workspace & 255)) return ADG_ERR_WORKSPACE;
  if (g->n == 0) return g->nnz == 0 ? ADG_OK : ADG_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  int* bad = (int*)workspace;
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), s));
  long long blocks = std::min<long long>((g->n + BS - 1) / BS, 4096);
  hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(BS), 0, s, (int)g->n, (long long)g->nnz,
                     (const long long*)g->row_ptr, g->col_idx, bad);
  HIPCHK(hipGetLastError());
  int hbad = 0;
  HIPCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return hbad ? ADG_ERR_ARG : ADG_OK;
}

int adg_profile_enable(uint32_t class_mask) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_mask = class_mask;
  return ADG_OK;
}

int adg_profile_read(adg_profile_t* out) {
  if (!out) return ADG_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  std::lock_guard<std::mutex> g(g_prof_mu);
  int rc = ADG_OK;
  for (const ProfRec& r : g_prof) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) rc = ADG_ERR_HIP;
    if (r.cls >= 0 && r.cls < ADG_PROFILE_CLASSES) {
      out->ms[r.cls] += ms;
      out->launches[r.cls] += 1;
    }
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_prof.clear();
  return rc;
}

const char* adg_kernel_class_name(int cls) {
  if (cls < 0 || cls >= KC_NUM) return "";
  return kclass_names[cls];
}

const char* adg_error_string(int code) {
  switch (code) {
    case ADG_OK: return "ok";
    case ADG_ERR_ARG: return "invalid argument";
    case ADG_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case ADG_ERR_HIP: return "HIP runtime error";
    case ADG_ERR_INTERNAL: return "internal error (watchdog or device-side check)";
    case ADG_ERR_UNSUPPORTED: return "input outside the supported range";
    default: return "unknown error";
  }
}

}  // extern "C"
