// ADG and JP-ADG on one graph: kernels and the C ABI (include/adg.h).
//
// Paper: Besta et al., "High-Performance Parallel Graph Coloring with Strong
// Guarantees on Work, Depth, and Quality".
//
// ADG (Algorithm 1) runs as one short sequence of kernels per round, issued
// back to back on the caller's stream; all loop control lives in device
// memory (a control block written by one-block kernels), so the host only
// looks at the termination flag once per chunk of rounds.  Per round l:
//   k_stats    |U_l| and the degree sum S_l (Count and Reduce): S_l is kept
//              as a cached sum -- the previous sum over U_l at selection time
//              minus the decrements of the previous UPDATE -- which is the
//              "Caching Sums of Degrees" optimisation; then the integer
//              threshold T_l = floor((q+p) S_l / (q |U_l|)), so that
//              D[u] <= (1 + p/q) S_l / |U_l|  <=>  D[u] <= T_l exactly.
//   k_count    per-block counts of R (split by degree) and U \ R.
//   k_scan     one block: exclusive scan of the per-block counts.
//   k_scatter  stable compaction of U into R and U \ R (the partitioned
//              [R | U \ R] array of "Representation of U and R"), writes
//              rho_ADG(v) = l for v in R.
//   k_update   UPDATE: for v in R, for w in N(v) still active, decrement
//              D[w].  With fusion on, the same sweep classifies every
//              neighbour as a JP predecessor or successor of v (JP Part 1,
//              "Combining JP and ADG"), writes v's adjacency partitioned as
//              [pred | succ], |pred(v)| and the JP word, and queues v if it
//              has no predecessor.
// JP (Algorithm 3, Part 2) is one persistent kernel (k_jp): each wavefront
// takes up to 64 ready vertices, colours them, and updates their
// successors' words; a successor whose count reaches zero is coloured next by
// the same wavefront (the recursive JPColor call), spilling to a global queue
// when the wavefront holds more than it can process at once.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/adg.h"
#include "adg_device.h"

namespace adg {

constexpr int BS = 256;                 // threads per block
constexpr int WPB = BS / WAVE;          // wavefronts per block
constexpr int SEL_BLOCKS = 2048;        // fixed grid of the selection kernels
constexpr int SMALL_DEG = 32;           // lane-per-vertex up to this degree
constexpr int FB_CAP = 2048;            // per-block frontier staging (LDS)
constexpr int JP_SMALL = 32;            // lane-per-vertex successor loops
constexpr int JP_LOCAL = 64;            // ready vertices a wave keeps locally
constexpr int JP_OVF_BITS = 4096;       // colour window of the wide path
constexpr unsigned Q_EMPTY = 0xffffffffu;

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
  unsigned int nRs, nRb;       // |R| split: lane-per-vertex / wave-per-vertex
  int done;                    // ADG finished
  int num_rounds;
  int error;                   // ADG_ERR_* raised on the device
  int stats_round;              // last round k_stats has computed
  // JP state
  unsigned int q_tail;         // entries pushed into Q
  unsigned int F;              // initial frontier size (pushed before JP)
  unsigned int q_head;         // entries claimed from Q
  unsigned int overflow;       // vertices coloured through the wide path
  unsigned int to_color;       // vertices JP has to colour
  int num_colors;
  unsigned int pad1[2];
  unsigned int colored[8 * 16];  // per-XCD counters, one 64-byte line each
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
  Ctrl* ctrl;
  int* round;                  // rho_ADG (user output or workspace)
  int* D;
  unsigned char* status;       // 0 = active, 1 + (round mod 3) = removed in round
  int* UL[2];                  // active lists (double-buffered)
  int* RL;                     // R: small part then big part
  unsigned long long* bcount;  // [SEL_BLOCKS][3] counts, then offsets
  unsigned long long* boff;
  unsigned long long* bsum;    // [SEL_BLOCKS]
  unsigned long long* xpart;   // [upd_blocks] decrement counts
  int upd_blocks;
  int* dag;                    // [nnz] adjacency partitioned [pred | succ]
  int* npred;                  // |pred(v)|
  unsigned long long* word;    // JP word
  unsigned* Q;                 // JP queue
  unsigned long long* QM;      // masks of spilled queue entries
  int* color;
};

__device__ __forceinline__ unsigned char round_code(int l) { return (unsigned char)(1 + (l % 3)); }

// ---------------------------------------------------------------- ADG: init / stats

__global__ void k_init(Params P) {
  Ctrl* c = P.ctrl;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c->N = c->S = c->Nnext = c->SUnext = 0;
    c->sum_active = c->cut_edges = 0;
    c->T = 0;
    c->round = 0;
    c->nRs = c->nRb = 0;
    c->done = 0;
    c->num_rounds = 0;
    c->error = 0;
    c->stats_round = 0;
    c->q_tail = c->F = c->q_head = 0;
    c->overflow = 0;
    c->to_color = 0;
    c->num_colors = 0;
  }
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < 8 * 16; i += blockDim.x) c->colored[i] = 0;
}

// One block.  Computes N_l, S_l and T_l for round l, or ends the loop.
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

// ---------------------------------------------------------------- ADG: selection

struct Chunk {
  long long beg, end;
};
__device__ __forceinline__ Chunk sel_chunk(unsigned long long N) {
  unsigned long long per = (N + gridDim.x - 1) / gridDim.x;
  per = (per + BS - 1) / BS * BS;
  long long b = (long long)(per * blockIdx.x);
  long long e = b + (long long)per;
  if (b > (long long)N) b = (long long)N;
  if (e > (long long)N) e = (long long)N;
  return {b, e};
}

// Category of element u in round l: 0 = R (lane-wise), 1 = R (wave-wise), 2 = stays.
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

// One block of BS threads: exclusive scan of SEL_BLOCKS x 3 counts.
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
  // Hillis-Steele inclusive scan over the BS partials (3 arrays), plus a sum.
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

// Stable compaction of U_l into R (small, big) and U_{l+1}; sets rho and status.
__global__ __launch_bounds__(BS) void k_scatter(Params P, int l) {
  Ctrl* c = P.ctrl;
  if (c->done) return;
  const unsigned long long N = c->N;
  const unsigned T = c->T;
  const unsigned nRs = c->nRs;
  const int* Uin = P.UL[(l + 1) & 1];
  int* Uout = P.UL[l & 1];
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
    if (s.cat == 0) {
      P.RL[base0 + pre[0] + lanes_below(m0)] = s.u;
    } else if (s.cat == 1) {
      P.RL[nRs + base1 + pre[1] + lanes_below(m1)] = s.u;
    } else if (s.cat == 2) {
      Uout[base2 + pre[2] + lanes_below(m2)] = s.u;
    }
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

// ---------------------------------------------------------------- ADG: UPDATE (+ JP Part 1)

// Frontier staging: vertices without predecessors, collected per block in LDS
// and appended to Q with one global atomic per flush.
struct Frontier {
  unsigned* buf;
  unsigned* cnt;
};

__device__ __forceinline__ void frontier_push(const Params& P, Frontier& F, bool pred, unsigned v) {
  uint64_t m = ballot(pred);
  if (m == 0) return;
  unsigned k = __popcll(m);
  unsigned base = 0;
  if (lane_id() == 0) base = atomicAdd(F.cnt, k);
  base = readlane_u(base, 0);
  const unsigned pos = base + lanes_below(m);
  if (pred && pos < (unsigned)FB_CAP) F.buf[pos] = v;
  if (base + k > (unsigned)FB_CAP) {
    // LDS stage full: the entries past its end go straight to Q.
    uint64_t om = ballot(pred && pos >= (unsigned)FB_CAP);
    unsigned g = 0;
    if (lane_id() == 0) g = atomicAdd(&P.ctrl->q_tail, (unsigned)__popcll(om));
    g = readlane_u(g, 0);
    if (pred && pos >= (unsigned)FB_CAP) P.Q[g + lanes_below(om)] = v;
  }
}

__device__ __forceinline__ void frontier_flush(const Params& P, Frontier& F) {
  __syncthreads();
  __shared__ unsigned gbase;
  unsigned k = *F.cnt;
  if (k > (unsigned)FB_CAP) k = FB_CAP;
  if (threadIdx.x == 0) gbase = k ? atomicAdd(&P.ctrl->q_tail, k) : 0;
  __syncthreads();
  for (unsigned i = threadIdx.x; i < k; i += BS) P.Q[gbase + i] = F.buf[i];
}

// Classify neighbour w of v (round l).  Returns 1 if w is a JP predecessor.
// Decrements D[w] when w is still active (it is in U \ R).
template <bool FUSED>
__device__ __forceinline__ bool visit(const Params& P, int w, unsigned char code, uint32_t hv, unsigned& x) {
  unsigned char st = P.status[w];
  if (st == 0) {
    atomicSub(&P.D[w], 1);
    x += 1;
    return true;
  }
  if (FUSED && st == code) return tiebreak(P.hkey, (uint32_t)w) > hv;
  return false;
}

template <bool FUSED>
__device__ void update_small(const Params& P, Frontier& F, int v, bool valid, unsigned char code, unsigned& x) {
  long long b = 0, e = 0;
  if (valid) {
    b = P.rp[v];
    e = P.rp[v + 1];
  }
  const uint32_t hv = tiebreak(P.hkey, (uint32_t)v);
  long long f = b, s = e;
  for (long long j = b; j < e; ++j) {
    int w = P.col[j];
    bool pr = visit<FUSED>(P, w, code, hv, x);
    if (FUSED) {
      if (pr) P.dag[f++] = w;
      else P.dag[--s] = w;
    }
  }
  if (FUSED) {
    int np = (int)(f - b);
    if (valid) {
      P.npred[v] = np;
      P.word[v] = (unsigned long long)np << JP_MASK_BITS;
    }
    frontier_push(P, F, valid && np == 0, (unsigned)v);
  }
}

template <bool FUSED>
__device__ void update_big(const Params& P, Frontier& F, int v, unsigned char code, unsigned& x) {
  const long long b = P.rp[v], e = P.rp[v + 1];
  const uint32_t hv = tiebreak(P.hkey, (uint32_t)v);
  long long fc = 0, sc = 0;
  const unsigned lane = lane_id();
  for (long long base = b; base < e; base += WAVE) {
    long long j = base + lane;
    bool valid = j < e;
    int w = valid ? P.col[j] : 0;
    bool pr = valid && visit<FUSED>(P, w, code, hv, x);
    if (FUSED) {
      uint64_t pm = ballot(pr), sm = ballot(valid && !pr);
      if (pr) P.dag[b + fc + lanes_below(pm)] = w;
      else if (valid) P.dag[e - 1 - sc - lanes_below(sm)] = w;
      fc += __popcll(pm);
      sc += __popcll(sm);
    }
  }
  if (FUSED) {
    if (lane == 0) {
      P.npred[v] = (int)fc;
      P.word[v] = (unsigned long long)fc << JP_MASK_BITS;
      if (fc > JP_MAX_PRED) atomicExch(&P.ctrl->error, ADG_ERR_UNSUPPORTED);
    }
    frontier_push(P, F, lane == 0 && fc == 0, (unsigned)v);
  }
}

template <bool FUSED>
__global__ __launch_bounds__(BS) void k_update(Params P, int l) {
  Ctrl* c = P.ctrl;
  if (c->done) return;
  const unsigned nRs = c->nRs, nRb = c->nRb;
  const unsigned char code = round_code(l);
  __shared__ unsigned fbuf[FUSED ? FB_CAP : 1];
  __shared__ unsigned fcnt;
  __shared__ unsigned long long xred[WPB];
  if (threadIdx.x == 0) fcnt = 0;
  __syncthreads();
  Frontier F{fbuf, &fcnt};
  const long long nsg = (nRs + WAVE - 1) / WAVE;
  const long long items = nsg + nRb;
  const long long gw = (long long)blockIdx.x * WPB + threadIdx.x / WAVE;
  const long long gstride = (long long)gridDim.x * WPB;
  unsigned x = 0;
  for (long long it = gw; it < items; it += gstride) {
    if (it < nsg) {
      long long idx = it * WAVE + lane_id();
      bool valid = idx < nRs;
      int v = valid ? P.RL[idx] : 0;
      update_small<FUSED>(P, F, v, valid, code, x);
    } else {
      int v = P.RL[nRs + (it - nsg)];
      update_big<FUSED>(P, F, v, code, x);
    }
  }
  unsigned long long xs = wave_sum((unsigned long long)x);
  if (lane_id() == 0) xred[threadIdx.x / WAVE] = xs;
  if (FUSED) frontier_flush(P, F);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int k = 0; k < WPB; ++k) t += xred[k];
    P.xpart[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------- JP Part 1 (stand-alone)

// For jp_color on a given ranking: classify every neighbour by the priority
// <round, hash>, write the [pred | succ] partition, |pred|, the JP word, and
// queue the vertices without predecessors.
__global__ __launch_bounds__(BS) void k_part1(Params P) {
  __shared__ unsigned fbuf[FB_CAP];
  __shared__ unsigned fcnt;
  if (threadIdx.x == 0) fcnt = 0;
  __syncthreads();
  Frontier F{fbuf, &fcnt};
  const long long gw = (long long)blockIdx.x * WPB + threadIdx.x / WAVE;
  const long long gstride = (long long)gridDim.x * WPB;
  const unsigned lane = lane_id();
  const long long groups = ((long long)P.n + WAVE - 1) / WAVE;
  for (long long g = gw; g < groups; g += gstride) {
    long long idx = g * WAVE + lane;
    bool valid = idx < P.n;
    int v = valid ? (int)idx : 0;
    long long b = valid ? P.rp[v] : 0, e = valid ? P.rp[v + 1] : 0;
    const uint64_t kv = ((uint64_t)(uint32_t)P.round[v] << 32) | tiebreak(P.hkey, (uint32_t)v);
    bool small = valid && (e - b) <= SMALL_DEG;
    if (small) {
      long long f = b, s = e;
      for (long long j = b; j < e; ++j) {
        int w = P.col[j];
        uint64_t kw = ((uint64_t)(uint32_t)P.round[w] << 32) | tiebreak(P.hkey, (uint32_t)w);
        if (kw > kv) P.dag[f++] = w;
        else P.dag[--s] = w;
      }
      int np = (int)(f - b);
      P.npred[v] = np;
      P.word[v] = (unsigned long long)np << JP_MASK_BITS;
    }
    frontier_push(P, F, small && P.npred[v] == 0, (unsigned)v);
    uint64_t big = ballot(valid && !small);
    while (big) {
      int L = __ffsll((long long)big) - 1;
      big &= big - 1;
      int u = readlane_i(v, L);
      long long ub = P.rp[u], ue = P.rp[u + 1];
      uint64_t ku = ((uint64_t)(uint32_t)P.round[u] << 32) | tiebreak(P.hkey, (uint32_t)u);
      long long fc = 0, sc = 0;
      for (long long base = ub; base < ue; base += WAVE) {
        long long j = base + lane;
        bool ok = j < ue;
        int w = ok ? P.col[j] : 0;
        bool pr = false;
        if (ok) {
          uint64_t kw = ((uint64_t)(uint32_t)P.round[w] << 32) | tiebreak(P.hkey, (uint32_t)w);
          pr = kw > ku;
        }
        uint64_t pm = ballot(pr), sm = ballot(ok && !pr);
        if (pr) P.dag[ub + fc + lanes_below(pm)] = w;
        else if (ok) P.dag[ue - 1 - sc - lanes_below(sm)] = w;
        fc += __popcll(pm);
        sc += __popcll(sm);
      }
      if (lane == 0) {
        P.npred[u] = (int)fc;
        P.word[u] = (unsigned long long)fc << JP_MASK_BITS;
        if (fc > JP_MAX_PRED) atomicExch(&P.ctrl->error, ADG_ERR_UNSUPPORTED);
      }
      frontier_push(P, F, lane == 0 && fc == 0, (unsigned)u);
    }
  }
  frontier_flush(P, F);
}

// ---------------------------------------------------------------- JP Part 2

__global__ void k_jp_prep(Params P) {
  Ctrl* c = P.ctrl;
  const unsigned F = c->q_tail;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)F + gid; i < P.n; i += stride) P.Q[i] = Q_EMPTY;
  for (long long i = gid; i < P.n; i += stride) P.color[i] = 0;
  if (gid == 0) {
    c->F = F;
    c->q_head = 0;
    c->to_color = (unsigned)P.n;
    c->overflow = 0;
  }
}

struct JpLds {
  unsigned lv[WPB][JP_LOCAL];
  unsigned long long lm[WPB][JP_LOCAL];
  unsigned bits[WPB][JP_OVF_BITS / 32];
  int bmax[WPB];
};

// Colour vertex v whose mask of colours 1..40 is full: gather the colours of
// all predecessors (those above 40 were published with a release fence before
// their decrement; smaller or stale ones are already in the mask) and take the
// smallest free colour above 40.  Whole wavefront; returns the colour.
__device__ int jp_wide_color(const Params& P, JpLds& S, int w, int v) {
  const unsigned lane = lane_id();
  const long long b = P.rp[v];
  const int np = P.npred[v];
  fence_acquire();
  for (int lo = JP_MASK_BITS + 1;; lo += JP_OVF_BITS) {
    for (int k = lane; k < JP_OVF_BITS / 32; k += WAVE) S.bits[w][k] = 0;
    __builtin_amdgcn_wave_barrier();
    for (int j = lane; j < np; j += WAVE) {
      int cu = agent_load_i32(&P.color[P.dag[b + j]]);
      int off = cu - lo;
      if (off >= 0 && off < JP_OVF_BITS) atomicOr(&S.bits[w][off >> 5], 1u << (off & 31));
    }
    __builtin_amdgcn_wave_barrier();
    int found = 0x7fffffff;
    for (int k = lane; k < JP_OVF_BITS / 32; k += WAVE) {
      unsigned m = ~S.bits[w][k];
      if (m && found == 0x7fffffff) found = k * 32 + __ffs(m) - 1;
    }
    // smallest across lanes
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      int o = __shfl_xor(found, off, WAVE);
      found = o < found ? o : found;
    }
    if (found != 0x7fffffff) return lo + found;
  }
}

// Successor update for one coloured vertex: OR the colour bit (colours up to
// 40), subtract one count unit, and report successors that became ready.
__device__ __forceinline__ bool jp_touch(const Params& P, int u, int c, unsigned long long& fin) {
  if (c <= JP_MASK_BITS) atomicOr(&P.word[u], 1ull << (c - 1));
  unsigned long long old = atomicAdd(&P.word[u], (unsigned long long)(-(long long)JP_ONE));
  fin = (old - JP_ONE) & JP_MASK;
  return (old >> JP_MASK_BITS) == 1;
}

// Push ready vertices (lanes with `rdy`) onto the wavefront's local stack;
// what does not fit goes to the global queue.
__device__ __forceinline__ void jp_ready(const Params& P, JpLds& S, int w, unsigned& lcount, bool rdy, unsigned u,
                                         unsigned long long fin) {
  uint64_t m = ballot(rdy);
  if (!m) return;
  unsigned k = __popcll(m);
  unsigned pos = lcount + lanes_below(m);
  unsigned room = JP_LOCAL - lcount;
  if (rdy && pos < JP_LOCAL) {
    S.lv[w][pos] = u;
    S.lm[w][pos] = fin;
  }
  if (k > room) {
    // spill the rest: data first, release, then publish the vertex id
    uint64_t sm = ballot(rdy && pos >= JP_LOCAL);
    unsigned ks = __popcll(sm);
    unsigned g = 0;
    if (lane_id() == 0) g = atomicAdd(&P.ctrl->q_tail, ks);
    g = readlane_u(g, 0);
    unsigned r = lanes_below(sm);
    const bool fits = g + r < (unsigned)P.n;  // every vertex is queued at most once
    if (rdy && pos >= JP_LOCAL && !fits) atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
    if (rdy && pos >= JP_LOCAL && fits) P.QM[g + r] = fin;
    // acquire: whatever this wave learnt through its decrements (colours
    // above 40 of the successor's predecessors) must reach the consumer too
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
    if (rdy && pos >= JP_LOCAL && fits) agent_store_i32((int*)&P.Q[g + r], (int)u);
    lcount = JP_LOCAL;
  } else {
    lcount += k;
  }
  __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(BS) void k_jp(Params P, long long spin_limit) {
  __shared__ JpLds S;
  Ctrl* c = P.ctrl;
  const int w = threadIdx.x / WAVE;
  const unsigned lane = lane_id();
  const unsigned F = c->F;
  const unsigned n = (unsigned)P.n;
  const unsigned xcd = blockIdx.x & 7;
  unsigned lcount = 0;          // local ready stack size (uniform)
  bool have_slot = false;       // lane holds a claimed queue slot
  unsigned slot = 0;
  int cmax = 0;
  long long idle = 0;
  while (true) {
    bool act = false;
    unsigned v = 0;
    unsigned long long M = 0;
    if (lcount > 0) {
      unsigned k = lcount < (unsigned)WAVE ? lcount : (unsigned)WAVE;
      if (lane < k) {
        act = true;
        v = S.lv[w][lcount - k + lane];
        M = S.lm[w][lcount - k + lane];
      }
      lcount -= k;
      __builtin_amdgcn_wave_barrier();
    } else {
      if (!ballot(have_slot)) {
        unsigned base = n;
        if (lane == 0 && agent_load_u32(&c->q_head) < n) base = atomicAdd(&c->q_head, (unsigned)WAVE);
        base = readlane_u(base, 0);
        slot = base + lane;
        have_slot = base < n && slot < n;
      }
      if (have_slot) {
        if (slot < F) {
          v = P.Q[F - 1 - slot];
          M = 0;
          act = true;
        } else {
          unsigned q = agent_load_u32(&P.Q[slot]);
          if (q != Q_EMPTY) {
            act = true;
            v = q;
          }
        }
      }
      uint64_t got = ballot(act && slot >= F);
      if (got) {
        fence_acquire();
        if (act && slot >= F) M = P.QM[slot];
      }
      if (act) have_slot = false;
    }
    const uint64_t am = ballot(act);
    if (!am) {
      // nothing to do: finished?
      unsigned done = 0;
      if (lane < 8) done = agent_load_u32(&c->colored[lane * 16]);
      done = wave_sum(done);
      if (done >= c->to_color) break;
      __builtin_amdgcn_s_sleep(2);
      if (++idle > spin_limit) {
        if (lane == 0) atomicExch(&c->error, ADG_ERR_INTERNAL);
        break;
      }
      continue;
    }
    idle = 0;
    // colour
    int col = 0;
    if (act && (M & JP_MASK) != JP_MASK) col = __ffsll((long long)~M) ;  // bit i free -> colour i+1
    uint64_t wide = ballot(act && (M & JP_MASK) == JP_MASK);
    while (wide) {
      int L = __ffsll((long long)wide) - 1;
      wide &= wide - 1;
      int u = readlane_i((int)v, L);
      int cc = jp_wide_color(P, S, w, u);
      if (lane == (unsigned)L) col = cc;
      if (lane == 0) atomicAdd(&c->overflow, 1u);
    }
    if (act) P.color[v] = col;
    cmax = act && col > cmax ? col : cmax;
    if (ballot(act && col > JP_MASK_BITS)) fence_release();
    // successors
    long long b = 0, e = 0;
    if (act) {
      b = P.rp[v] + P.npred[v];
      e = P.rp[v + 1];
    }
    bool small = act && (e - b) <= JP_SMALL;
    {
      long long j = b;
      while (ballot(small && j < e)) {
        bool go = small && j < e;
        bool rdy = false;
        unsigned long long fin = 0;
        int u = 0;
        if (go) {
          u = P.dag[j];
          rdy = jp_touch(P, u, col, fin);
          ++j;
        }
        jp_ready(P, S, w, lcount, rdy, (unsigned)u, fin);
      }
    }
    uint64_t big = ballot(act && !small);
    while (big) {
      int L = __ffsll((long long)big) - 1;
      big &= big - 1;
      long long bb = readlane_i64(b, L), ee = readlane_i64(e, L);
      int cc = readlane_i(col, L);
      for (long long base = bb; base < ee; base += WAVE) {
        long long j = base + lane;
        bool go = j < ee;
        bool rdy = false;
        unsigned long long fin = 0;
        int u = 0;
        if (go) {
          u = P.dag[j];
          rdy = jp_touch(P, u, cc, fin);
        }
        jp_ready(P, S, w, lcount, rdy, (unsigned)u, fin);
      }
    }
    if (lane == 0) atomicAdd(&c->colored[xcd * 16], (unsigned)__popcll(am));
  }
  cmax = wave_max(cmax);
  if (lane == 0) S.bmax[w] = cmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    int m = 0;
    for (int k = 0; k < WPB; ++k) m = S.bmax[k] > m ? S.bmax[k] : m;
    atomicMax(&c->num_colors, m);
  }
}

__global__ void k_finish(Params P, int* num_colors_out, int* num_rounds_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (num_colors_out) *num_colors_out = P.ctrl->num_colors;
  if (num_rounds_out) *num_rounds_out = P.ctrl->num_rounds;
}

__global__ void k_copy_rounds(Params P, int* num_rounds_out) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && num_rounds_out) *num_rounds_out = P.ctrl->num_rounds;
}

// ---------------------------------------------------------------- CSR validation

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

// =============================================================== host side

using namespace adg;

namespace {

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Layout {
  size_t ctrl, bcount, boff, bsum, xpart, D, status, UL0, UL1, RL, round, dag, npred, word, Q, QM, total;
};

int upd_blocks_for_device() { return 2048; }

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
  L.xpart = take(sizeof(unsigned long long) * upd_blocks_for_device());
  L.D = take(4 * nn);
  L.status = take(nn);
  L.UL0 = take(4 * nn);
  L.UL1 = take(4 * nn);
  L.RL = take(4 * nn);
  L.round = take(4 * nn);
  L.dag = take(4 * (size_t)nnz);
  L.npred = take(4 * nn);
  L.word = take(8 * nn);
  L.Q = take(4 * nn);
  L.QM = take(8 * nn);
  L.total = off;
  return L;
}

uint32_t hash_key_from_seed(uint64_t seed) {
  // low 32 bits of the first SplitMix64 output from state `seed`
  uint64_t z = seed + 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  z ^= z >> 31;
  return (uint32_t)z;
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
  P.ctrl = (Ctrl*)(base + L.ctrl);
  P.round = round_buf ? round_buf : (int*)(base + L.round);
  P.D = (int*)(base + L.D);
  P.status = (unsigned char*)(base + L.status);
  P.UL[0] = (int*)(base + L.UL0);
  P.UL[1] = (int*)(base + L.UL1);
  P.RL = (int*)(base + L.RL);
  P.bcount = (unsigned long long*)(base + L.bcount);
  P.boff = (unsigned long long*)(base + L.boff);
  P.bsum = (unsigned long long*)(base + L.bsum);
  P.xpart = (unsigned long long*)(base + L.xpart);
  P.upd_blocks = upd_blocks_for_device();
  P.dag = (int*)(base + L.dag);
  P.npred = (int*)(base + L.npred);
  P.word = (unsigned long long*)(base + L.word);
  P.Q = (unsigned*)(base + L.Q);
  P.QM = (unsigned long long*)(base + L.QM);
  P.color = color;
  // Round-count bound from the ADG depth lemma: |U| shrinks by a factor
  // 1/(1+eps) each round, so L <= ceil(log n / log(1+eps)) + 1; +1 margin.
  long long bound = (long long)g->n + 1;
  if (p > 0 && g->n > 1) {
    double b = std::ceil(std::log((double)g->n) / std::log1p((double)p / (double)q)) + 2.0;
    if (b < (double)bound) bound = (long long)b;
  }
  if (bound < 1) bound = 1;
  P.max_rounds = (int)std::min<long long>(bound, 0x7fffffff);
  return P;
}

#define HIPCHK(x)                          \
  do {                                     \
    if ((x) != hipSuccess) return ADG_ERR_HIP; \
  } while (0)

// Run ADG's round loop.  Returns an ADG_* code; synchronises the stream
// between chunks of rounds.
int run_adg(Params& P, hipStream_t s, bool fused) {
  hipLaunchKernelGGL(k_init, dim3(1), dim3(BS), 0, s, P);
  HIPCHK(hipGetLastError());
  if (P.n == 0) return ADG_OK;
  static int* done_h = nullptr;
  if (!done_h) HIPCHK(hipHostMalloc((void**)&done_h, 2 * sizeof(int), hipHostMallocDefault));
  int l = 1;
  int chunk = 8;
  int rc = ADG_OK;
  while (true) {
    for (int k = 0; k < chunk; ++k, ++l) {
      hipLaunchKernelGGL(k_stats, dim3(1), dim3(BS), 0, s, P, l);
      hipLaunchKernelGGL(k_count, dim3(SEL_BLOCKS), dim3(BS), 0, s, P, l);
      hipLaunchKernelGGL(k_scan, dim3(1), dim3(BS), 0, s, P, l);
      hipLaunchKernelGGL(k_scatter, dim3(SEL_BLOCKS), dim3(BS), 0, s, P, l);
      if (fused)
        hipLaunchKernelGGL(k_update<true>, dim3(P.upd_blocks), dim3(BS), 0, s, P, l);
      else
        hipLaunchKernelGGL(k_update<false>, dim3(P.upd_blocks), dim3(BS), 0, s, P, l);
    }
    // one more stats call ends the loop on the device when U is empty
    hipLaunchKernelGGL(k_stats, dim3(1), dim3(BS), 0, s, P, l);
    if (hipGetLastError() != hipSuccess) {
      rc = ADG_ERR_HIP;
      break;
    }
    if (hipMemcpyAsync(done_h, &P.ctrl->done, 2 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = ADG_ERR_HIP;
      break;
    }
    if (done_h[0]) break;
    if (l > P.max_rounds + 1) {
      rc = ADG_ERR_INTERNAL;
      break;
    }
    chunk = std::min(chunk * 2, 64);
  }
  if (rc == ADG_OK) {
    int err = 0;
    if (hipMemcpyAsync(&err, &P.ctrl->error, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = ADG_ERR_HIP;
    else if (err)
      rc = err;
  }
  return rc;
}

int jp_blocks(const void* fn) {
  static int cached = 0;
  if (cached) return cached;
  int dev = 0, cus = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, BS, 0) != hipSuccess || occ < 1) occ = 1;
  cached = cus * std::min(occ, 8);
  return cached;
}

int run_jp(Params& P, hipStream_t s) {
  if (P.n == 0) return ADG_OK;
  hipLaunchKernelGGL(k_jp_prep, dim3(1024), dim3(BS), 0, s, P);
  int blocks = jp_blocks((const void*)k_jp);
  // idle iterations (each one polls the finish counters) before the kernel
  // gives up and reports ADG_ERR_INTERNAL: a few seconds
  long long spin_limit = 1LL << 22;
  hipLaunchKernelGGL(k_jp, dim3(blocks), dim3(BS), 0, s, P, spin_limit);
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
  rc = run_adg(P, s, false);
  if (rc) return rc;
  if (num_rounds_out) hipLaunchKernelGGL(k_copy_rounds, dim3(1), dim3(64), 0, s, P, num_rounds_out);
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
  hipLaunchKernelGGL(k_init, dim3(1), dim3(BS), 0, s, P);
  if (P.n > 0) {
    hipLaunchKernelGGL(k_part1, dim3(P.upd_blocks), dim3(BS), 0, s, P);
    int err = 0;
    if (hipMemcpyAsync(&err, &P.ctrl->error, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return ADG_ERR_HIP;
    if (err) return err;
    if ((rc = run_jp(P, s))) return rc;
  }
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, P, num_colors_out, (int*)nullptr);
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
  if ((rc = run_adg(P, s, true))) return rc;
  if ((rc = run_jp(P, s))) return rc;
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, P, num_colors_out, num_rounds_out);
  HIPCHK(hipGetLastError());
  return ADG_OK;
}

int adg_get_stats(const void* workspace, size_t ws_bytes, adg_stats_t* out, void* stream) {
  if (!workspace || !out || ws_bytes < sizeof(Ctrl)) return ADG_ERR_ARG;
  Ctrl h;
  hipStream_t s = (hipStream_t)stream;
  const Ctrl* c = (const Ctrl*)workspace;
  if (hipMemcpyAsync(&h, c, sizeof(Ctrl), hipMemcpyDeviceToHost, s) != hipSuccess) return ADG_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return ADG_ERR_HIP;
  out->num_rounds = h.num_rounds;
  out->num_colors = h.num_colors;
  out->sum_active = (int64_t)h.sum_active;
  out->cut_edges = (int64_t)h.cut_edges;
  out->frontier = h.F;
  out->overflow = h.overflow;
  out->error = h.error;
  return ADG_OK;
}

int adg_validate_csr(const adg_csr_t* g, void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (!workspace || ws_bytes < 256 || ((uintptr_t)workspace & 255)) return ADG_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  int* bad = (int*)workspace;
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), s));
  if (g->n > 0) {
    long long blocks = std::min<long long>((g->n + BS - 1) / BS, 4096);
    hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(BS), 0, s, (int)g->n, (long long)g->nnz,
                       (const long long*)g->row_ptr, g->col_idx, bad);
    HIPCHK(hipGetLastError());
  } else if (g->nnz != 0) {
    return ADG_ERR_ARG;
  }
  int h = 0;
  HIPCHK(hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return h ? ADG_ERR_ARG : ADG_OK;
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
