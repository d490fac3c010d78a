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
//              rewritten as [preds from later rounds | same-round preds |
//              same-round succs], and |pred(v)|, the number of same-round
//              successors and v's JP record are stored.  The rest of the row's
//              slot (successors from earlier rounds) is left unwritten: no
//              step reads it.
// JP (Algorithm 3, Part 2) colours the rounds from L down to 1.  Every edge of
// G_rho between different rounds points from the higher round to the lower,
// so once rounds > l are coloured and have pushed their colours to round l,
// round l only waits on itself.  Per round: one bulk step ORs the colours of
// every predecessor from a later round (all final) into the round's bitmaps;
// its vertices with no same-round predecessor form level 0; levels follow
// one after the other over same-round successors only.  Narrow levels (and
// whole small rounds) run in a single block with block barriers; wide ones
// over the grid.
//
// Variants (flags of the _ex entry points):
//   ADG-O (the ADG-O listing): R is ordered by D at selection, so JP's order
//     inside a round is (D, rho_R) instead of rho_R.  D of a vertex removed in
//     round l stays at its selection value (UPDATE only touches vertices still
//     in U), so the key is available to UPDATE when it partitions the rows.
//   ADG-M (degree median): R is the ceil(|U|/2) vertices lowest by (D, rho_R).
//     Its threshold (1+eps) times the median always admits at least that
//     many, so the cap of half of U decides R; k_msel finds the
//     ceil(|U|/2)-th smallest 64-bit key (D << 32 | rho_R) by radix selection
//     and the selection kernels compare against it.
//   DEC-ADG-ITR ("Enhancing Existing Coloring Algorithms"): instead of JP, the
//     ADG partitions are coloured from the highest round down; inside a
//     partition, synchronous iterations let every uncoloured vertex try the
//     smallest colour free in its bitmap, keep it unless a same-round
//     predecessor (larger hash) tried the same colour, and push kept colours
//     to its same-round neighbours' bitmaps (k_dec_*).
//   Pull UPDATE (the CREW UPDATE of "Using Only Concurrent Reads", the pull
//     side of "Push vs. Pull"): k_update only partitions the rows of R, and
//     k_update_pull lets every vertex that stays in U count its neighbours
//     removed in the round and lower its own D -- no atomics on D, more reads.

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
#include "radix_sort.h"

namespace adg {

constexpr int BS = 256;                 // threads per block
constexpr int WPB = BS / WAVE;          // wavefronts per block
constexpr int SEL_BLOCKS = 2048;        // fixed grid of the selection kernels
#ifndef ADG_JP_RELAX
#define ADG_JP_RELAX 1   // deep rounds finished by relaxation
#endif
constexpr bool JP_RELAX = ADG_JP_RELAX;
#ifndef ADG_RELAX_COMPACT_MIN
#define ADG_RELAX_COMPACT_MIN 65536
#endif
#ifndef ADG_RELAX_COMPACT_N
#define ADG_RELAX_COMPACT_N 16777216
#endif
constexpr long long RELAX_COMPACT_MIN = ADG_RELAX_COMPACT_MIN;   // rounds of at least this many vertices relax by position,
constexpr long long RELAX_COMPACT_N = ADG_RELAX_COMPACT_N;       // in graphs of at least this many vertices
#ifndef ADG_JP_CORE
#define ADG_JP_CORE 1   // small rounds whose levels colour a vertex or two: one block, in JP's order
#endif
constexpr bool JP_CORE = ADG_JP_CORE;
constexpr int CORE_MAX = 4096;                  // rounds of at most this many vertices can take the core mode
#ifndef ADG_UPD_UNROLL
#define ADG_UPD_UNROLL 4
#endif
constexpr int UPD_UNROLL = ADG_UPD_UNROLL;   // 64-entry chunks of rows UPDATE reads at a time
#ifndef ADG_SUB_BINNED
#define ADG_SUB_BINNED 1
#endif
#ifndef ADG_SUB_SHIFT
#define ADG_SUB_SHIFT 15
#endif
constexpr int SUB_SHIFT = ADG_SUB_SHIFT;        // D decrements by bins of 2^SUB_SHIFT target vertices
constexpr int SUB_SPAN = 1 << SUB_SHIFT;
constexpr int SUB_MAX_BINS = 8192;              // (graphs up to 2^28 vertices; larger ones decrement at once)
#ifndef ADG_SUB_BLOCKS
#define ADG_SUB_BLOCKS 1024
#endif
constexpr int SUB_BLOCKS = ADG_SUB_BLOCKS;      // blocks of the count and scatter passes
#ifndef ADG_SUB_BS
#define ADG_SUB_BS 1024
#endif
constexpr int SUB_BS = ADG_SUB_BS;              // their threads
#ifndef ADG_SUB_CHUNK
#define ADG_SUB_CHUNK 65535
#endif
constexpr int SUB_CHUNK = ADG_SUB_CHUNK;        // targets an apply block takes at a time
constexpr int SUB_APPLY_BLOCKS = 1024;
constexpr int64_t SUB_MIN_NNZ = 1 << 22;        // smaller graphs decrement at once (the passes cost more than they save)
#ifndef ADG_SMALL_DEG
#define ADG_SMALL_DEG 32
#endif
constexpr int SMALL_DEG = ADG_SMALL_DEG;  // lane-per-vertex rows up to this length
constexpr int HUGE_DEG = 16384;         // rows longer than this are cut into chunks in UPDATE
constexpr int HUGE_CHUNK = 4096;        // entries of such a chunk
constexpr int FB_CAP = 2048;            // per-block staging of level lists (LDS)
#ifndef ADG_JP_SMALL
#define ADG_JP_SMALL 4
#endif
#ifndef ADG_JP_UNROLL
#define ADG_JP_UNROLL 1
#endif
constexpr int JP_SMALL = ADG_JP_SMALL;    // lane-per-vertex successor loops (more: fan-out chunks)
constexpr int JP_UNROLL = ADG_JP_UNROLL;  // successors in flight per lane
#ifndef ADG_JP_CHUNK_UNROLL
#define ADG_JP_CHUNK_UNROLL ADG_JP_UNROLL
#endif
constexpr int JP_CU = ADG_JP_CHUNK_UNROLL;   // successors per lane of a fan-out chunk
constexpr int JP_CHUNK = WAVE * JP_CU;       // successors per fan-out chunk (one wavefront step)
constexpr int FAN_LDS = 1024;                // fan-out list entries a grid block stages in LDS
constexpr int NARROW_BS = 1024;              // threads of the single-block JP kernel
constexpr int NARROW_MAX = 1024;             // level size the single block takes
// Work of a level the single block takes (it walks larger ones in passes of
// NARROW_BS * NARROW_UNROLL entries; beyond these sizes the grid is faster).
#ifndef ADG_NARROW_WORDS
#define ADG_NARROW_WORDS 3072
#endif
#ifndef ADG_NARROW_SUCC
#define ADG_NARROW_SUCC 3072
#endif
constexpr int NARROW_WORDS = ADG_NARROW_WORDS;  // colour bitmap words of a level
constexpr int NARROW_SUCC = ADG_NARROW_SUCC;    // same-round successor entries of a level
constexpr int NARROW_XPULL = 512;            // round size whose later-round colours it pulls in
#ifndef ADG_NARROW_UNROLL
#define ADG_NARROW_UNROLL 4
#endif
constexpr int NARROW_UNROLL = ADG_NARROW_UNROLL;  // edges per thread in flight in a narrow level
constexpr int MSEL_BINS = 2048;              // radix selection: 11-bit digits
constexpr int MSEL_PASSES = 6;               // 11 x 5 + 9 bits cover a 64-bit key
constexpr int MSEL_BLOCKS = 512;
#ifndef ADG_RELAX_AFTER
#define ADG_RELAX_AFTER 8
#endif
constexpr int RELAX_AFTER = ADG_RELAX_AFTER;   // levels of a round before its other vertices are relaxed
#ifndef ADG_RELAX_MIN_V
#define ADG_RELAX_MIN_V 2048
#endif
constexpr unsigned RELAX_MIN_V = ADG_RELAX_MIN_V;   // smaller rounds keep their levels to the end
#ifndef ADG_RELAX_DENSE
#define ADG_RELAX_DENSE 3
#endif
constexpr unsigned RELAX_DENSE = ADG_RELAX_DENSE;   // vertices per level below which a round keeps its levels
#ifndef ADG_RELAX_MID
#define ADG_RELAX_MID 8192
#endif
constexpr unsigned RELAX_MID = ADG_RELAX_MID;   // relaxation lists the steps launch takes (larger: the grid)
constexpr int RELAX_UNROLL = 4;                 // predecessor colours per lane in flight
constexpr int RELAX_LK = 32;                    // vertices a lane solves alone: same-round predecessors and successors
constexpr int RELAX_LW = 8;                     // and bitmap words

enum { OP_NONE = 0, OP_SPLIT = 1, OP_LEVEL = 2, OP_XPULL = 3, OP_RELAX = 4 };
// which rounds JP relaxes: by relax_pays (default), all from their start, none
enum { RELAX_MODE_RULE = 0, RELAX_MODE_ALL = 1, RELAX_MODE_NONE = 2 };

// JP progress.  Lives in the control block between kernels; the single-block
// kernel keeps its own copy in LDS while it runs.
struct JpState {
  int round;                   // round being coloured (L .. 1)
  int level;                   // level inside the round
  int split;                   // the round's first level is still only in L0
  int xpull;                   // the round's later-round colours are still to be pulled in
  int top;                     // L (the first round coloured)
  int done;                    // JP finished
  int levels;                  // levels and relaxation steps processed (all rounds)
  int relax;                   // the rest of the round is being relaxed
  int rit;                     // its relaxation step (0: list the uncoloured vertices)
  unsigned rstamp;             // mark stamp of the latest relaxation step (all rounds)
  unsigned long long F;        // vertices that formed a round's first level
  unsigned long long rv;       // vertices the current round's levels have coloured
  unsigned int fcnt[3];        // plain vertices per level (by level mod 3)
  unsigned int pad3;
  unsigned long long hctr[3];  // fan-out vertices (low 32 bits) and chunks (high 32 bits)
  unsigned long long psum[3];  // bitmap words summed over each level's vertices
  unsigned long long ssum[3];  // same-round successors summed over each level's vertices
};

// DEC-ADG-ITR progress (between kernels), double-buffered by iteration
// parity: the kernels of iteration k read dec[k & 1] and the last block of
// its resolve step writes dec[(k + 1) & 1], so a launch's state never
// changes while its blocks may still be starting.
struct DecState {
  int round;                   // partition being coloured (L .. 1)
  int first;                   // its first iteration: U is the partition's ORD slot
  int pull;                    // the partition still has to pull its later-round colours
  int cur;                     // U of later iterations: UL[cur]
  unsigned ucnt;               // |U|
  int done;
  long long iters;             // iterations run, all partitions
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
  unsigned long long bm_next;  // colour bitmap words handed out
  unsigned long long huge_ctr; // rows of the round cut into chunks (low 32 bits) and their chunks (high)
  unsigned long long xhuge;    // decrements done by the chunked rows
  int grid_op;                 // OP_* the grid kernel has to run next
  int num_colors;
  int pad_jp;
  // ADG-M radix selection of round l: keys whose masked bits are below
  // msel_prefix are in R, and so are those equal to it once msel_found is set
  unsigned long long msel_prefix;
  unsigned long long msel_mask;
  unsigned long long msel_k;   // rank still to find among the keys matching the prefix
  unsigned int msel_blocks;    // blocks of the current pass that have added their histogram
  int msel_found;
  JpState js;
  DecState dec[2];
  unsigned dec_unext;          // vertices that gave up their colour (the next U)
  unsigned dec_blocks;         // working blocks of k_dec_resolve done (last-block hand-off)
  // JP steps launch (k_jp_steps): registration, leader's command, completions
  unsigned long long preg;
  unsigned long long pcmd;
  unsigned long long pjoin;
  unsigned long long pnum;     // participants, published by the leader once registration is closed
  // relaxation step the steps launch's participants run: round, step, list size, stamp
  unsigned rx[4];
  // binned decrements of the current round: the targets overflow SB (then the
  // scatter pass decrements at once), the apply chunks
  int sub_direct;
  unsigned sub_chunks;
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
  int sorted;                  // ADG-O: same-round order by (D at selection, rho_R)
  int median;                  // ADG-M: R = the lower half of U by (D, rho_R)
  int dec;                     // DEC-ADG-ITR colours the partitions (bitmaps for all same-round neighbours)
  int pull;                    // UPDATE pulls: survivors lower their own D (k_update_pull)
  int relax_mode;              // RELAX_MODE_*: which rounds JP relaxes
  int binned;                  // UPDATE's decrements of D go through target bins (k_sub_*), not one atomic each
  unsigned* SB;                // the round's cut-edge targets ordered by bin
  unsigned sb_cap;             // entries of SB
  unsigned* SUBC;              // [SUB_BLOCKS][bins] targets per block and bin (then their offsets in the bin)
  unsigned* SUBS;              // [bins + 1] first entry of each bin in SB, then [bins + 1] apply chunks before each bin
  unsigned* tent;              // DEC-ADG-ITR: colour each vertex tried in its latest iteration
  unsigned* mhist;             // [MSEL_BINS] radix selection histogram
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
  int* xpred;                  // predecessors of v from later rounds (|pred(v)| less the same-round ones)
  int* nsr;                    // same-round successors of v (JP levels walk these)
  int* cnt;                    // same-round predecessors of v not yet coloured
  unsigned long long* rec;     // per vertex two words: (colour bitmap offset << 32) | |pred(v)|, and
                               // (first same-round successor entry << 24) | same-round successors
  unsigned* B;                 // colour bitmaps (bm_words(|pred|) words per vertex)
  unsigned long long bm_cap;   // words of B
  unsigned long long* pool;    // per-wavefront bitmap pools of k_update / k_part1: (end << 32) | next
  unsigned pool_chunk;         // words a pool takes from bm_next at a time
  unsigned long long* HL;      // rows of the round cut into chunks: (first chunk << 32) | vertex
  unsigned* HC;                // per such row: class counts [4] and placed counts [4]
  unsigned huge_cap;
  unsigned* L0;                // first JP level of each round, indexed like the round's ORD slot (~0: not in it)
  unsigned* F[2];              // level lists, plain vertices (by level parity)
  unsigned long long* H[2];    // level lists, fan-out vertices: (first chunk << 32) | vertex
  unsigned hub_cap;
  int* color;
  unsigned* rmark;             // relaxation: stamp of the step a position was last listed for
  int* rcol;                   // relaxation: colours of the relaxed round's vertices, by position in the round
};

// Status byte of a vertex removed in round l.  Codes repeat every 255 rounds,
// so a matching code is confirmed against the full round number.
__device__ __forceinline__ unsigned char round_code(int l) { return (unsigned char)(1 + ((l - 1) % 255)); }

// Scoped accesses for JP data.  JP's steps exchange data between
// workgroups that may sit on different XCDs (each with its own L2), inside
// one launch as well as across launches, so every access to data another
// workgroup writes or reads in the same launch is at agent scope: loads and
// stores go to the device's coherence point.  (Read-modify-write atomics are
// performed there whatever their scope.)
constexpr int SC_AGENT = __HIP_MEMORY_SCOPE_AGENT;
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
__device__ __forceinline__ void st32(unsigned* p, unsigned v) {
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
  if (blockIdx.x != 0) return;
  for (int i = threadIdx.x; i < P.upd_blocks * WPB; i += blockDim.x) P.pool[i] = 0;
  if (threadIdx.x != 0) return;
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
  c->num_colors = 0;
  c->bm_next = 0;
  c->huge_ctr = 0;
  c->xhuge = 0;
  c->msel_prefix = c->msel_mask = c->msel_k = 0;
  c->msel_blocks = 0;
  c->msel_found = 0;
  for (int k = 0; k < 2; ++k) {
    c->dec[k].done = 0;
    c->dec[k].iters = 0;
  }
  c->dec_blocks = 0;
  c->dec_unext = 0;
  JpState& j = c->js;
  j.round = 0;
  j.level = 0;
  j.split = 0;
  j.xpull = 0;
  j.top = 0;
  j.done = 0;
  j.levels = 0;
  j.F = 0;
  for (int k = 0; k < 3; ++k) {
    j.fcnt[k] = 0;
    j.hctr[k] = 0;
    j.psum[k] = 0;
    j.ssum[k] = 0;
  }
  if (P.median)
    for (int k = 0; k < MSEL_BINS; ++k) P.mhist[k] = 0;
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
    if (threadIdx.x < (unsigned)s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  c->stats_round = l;
  unsigned long long N, S;
  if (l == 1) {
    N = (unsigned long long)P.n;
    S = (unsigned long long)P.nnz;
  } else {
    const unsigned long long X = red[0] + c->xhuge;
    N = c->Nnext;
    S = c->SUnext - X;
    c->cut_edges += X;
  }
  c->xhuge = 0;
  c->huge_ctr = 0;
  if (l <= P.max_rounds + 1) {
    P.roundN[l] = (unsigned)N;
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
  // (q + p) S can pass 2^64: formed in 128 bits; D never exceeds 2^31 - 1
  const unsigned long long T = mul_div_floor_sat(P.q + P.p, S, P.q * N, 0x7fffffffull);
  c->N = N;
  c->S = S;
  c->T = (unsigned)T;
  c->round = l;
  c->sum_active += N;
  if (P.median) {
    c->msel_prefix = 0;
    c->msel_mask = 0;
    c->msel_k = (N + 1) / 2;
    c->msel_found = 0;
    c->msel_blocks = 0;
  }
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
// Selection threshold of a round: T for Algorithm 1, the radix-selected key
// for ADG-M.
struct Thr {
  unsigned T;
  int median;
  uint32_t hkey;
  unsigned long long mask, prefix;
};
__device__ __forceinline__ Thr load_thr(const Params& P, const Ctrl* c) {
  return {c->T, P.median, P.hkey, c->msel_mask, c->msel_prefix};
}
// ADG-M's key of u: D at selection, then rho_R.
__device__ __forceinline__ unsigned long long msel_key(uint32_t hkey, int u, int d) {
  return ((unsigned long long)(unsigned)d << 32) | tiebreak(hkey, (uint32_t)u);
}
__device__ __forceinline__ bool in_R(const Thr& t, int u, int d) {
  if (!t.median) return (unsigned)d <= t.T;
  return (msel_key(t.hkey, u, d) & t.mask) <= t.prefix;
}
// Element i of U_l and its D (round 1: U_1 = V, D = the degree).
__device__ __forceinline__ void u_elem(const Params& P, int l, long long i, const int* Uin, int* u, int* d) {
  if (l == 1) {
    *u = (int)i;
    *d = (int)(P.rp[i + 1] - P.rp[i]);
  } else {
    *u = Uin[i];
    *d = P.D[*u];
  }
}

__device__ __forceinline__ Sel classify(const Params& P, int l, long long i, const Thr& T, const int* Uin) {
  Sel s;
  if (l == 1) {
    s.u = (int)i;
    s.d = (int)(P.rp[i + 1] - P.rp[i]);
    if (in_R(T, s.u, s.d)) s.cat = s.d <= SMALL_DEG ? 0 : 1;
    else s.cat = 2;
  } else {
    s.u = Uin[i];
    s.d = P.D[s.u];
    if (in_R(T, s.u, s.d)) {
      int deg = (int)(P.rp[s.u + 1] - P.rp[s.u]);
      s.cat = deg <= SMALL_DEG ? 0 : 1;
    } else {
      s.cat = 2;
    }
  }
  return s;
}

// One pass of ADG-M's radix selection (pass 0 takes the top 11 bits of the
// key, pass 5 the last 9).  Every block histograms the digit of the keys of
// U_l that match the prefix chosen so far; the last block to finish picks the
// digit holding the msel_k-th smallest key, extends the prefix and clears the
// histogram for the next pass.  A pass stops the selection early when all
// keys of the picked digit are in R.
__global__ __launch_bounds__(BS) void k_msel(Params P, int l, int pass) {
  Ctrl* c = P.ctrl;
  if (c->done || c->msel_found) return;
  __shared__ unsigned hist[MSEL_BINS];
  __shared__ int last;
  const int shift = pass == MSEL_PASSES - 1 ? 0 : 64 - 11 * (pass + 1);
  const unsigned width = pass == MSEL_PASSES - 1 ? 9 : 11;
  const unsigned long long dmask = ((1ull << width) - 1) << shift;
  const unsigned long long N = c->N, mask = c->msel_mask, prefix = c->msel_prefix;
  // blocks with keys to count; the others leave at once (N does not change
  // during the selection, so every block counts them alike)
  long long active = ((long long)N + BS - 1) / BS;
  if (active < 1) active = 1;
  if (active > (long long)gridDim.x) active = gridDim.x;
  if ((long long)blockIdx.x >= active) return;
  const int* Uin = P.UL[(l + 1) & 1];
  for (int k = threadIdx.x; k < MSEL_BINS; k += BS) hist[k] = 0;
  __syncthreads();
  for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < (long long)N; i += (long long)gridDim.x * BS) {
    int u, d;
    u_elem(P, l, i, Uin, &u, &d);
    const unsigned long long key = msel_key(P.hkey, u, d);
    if ((key & mask) == prefix) atomicAdd(&hist[(key & dmask) >> shift], 1u);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < MSEL_BINS; k += BS)
    if (hist[k]) __hip_atomic_fetch_add(&P.mhist[k], hist[k], __ATOMIC_RELAXED, SC_AGENT);
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0)
    last = __hip_atomic_fetch_add(&c->msel_blocks, 1u, __ATOMIC_ACQ_REL, SC_AGENT) == (unsigned)(active - 1);
  __syncthreads();
  if (!last) return;
  __threadfence();
  // the last block: inclusive scan of the histogram, 8 bins per thread
  constexpr int PER = MSEL_BINS / BS;
  unsigned loc[PER];
  unsigned run = 0;
  for (int k = 0; k < PER; ++k) {
    loc[k] = __hip_atomic_load(&P.mhist[threadIdx.x * PER + k], __ATOMIC_RELAXED, SC_AGENT);
    run += loc[k];
  }
  __shared__ unsigned part[BS];
  part[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < BS; off <<= 1) {
    const unsigned v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  const unsigned long long want = c->msel_k;
  unsigned long long before = part[threadIdx.x] - run;
  for (int k = 0; k < PER; ++k) {
    // the bin where the running count first reaches `want`
    if (before < want && before + loc[k] >= want) {
      const unsigned long long bin = (unsigned long long)(threadIdx.x * PER + k);
      c->msel_prefix = prefix | (bin << shift);
      c->msel_mask = mask | dmask;
      c->msel_k = want - before;
      c->msel_found = (before + loc[k] == want) || pass == MSEL_PASSES - 1;
    }
    before += loc[k];
  }
  for (int k = threadIdx.x; k < MSEL_BINS; k += BS) P.mhist[k] = 0;
  if (threadIdx.x == 0) c->msel_blocks = 0;
}

__global__ __launch_bounds__(BS) void k_count(Params P, int l) {
  Ctrl* c = P.ctrl;
  if (c->done) return;
  const unsigned long long N = c->N;
  const Thr T = load_thr(P, c);
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
    for (int j = 0; j < 3; ++j) v[j] = threadIdx.x >= (unsigned)off ? part[j][threadIdx.x - off] : 0;
    if (threadIdx.x >= (unsigned)off) sv = sums[threadIdx.x - off];
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
  const Thr T = load_thr(P, c);
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
        if (P.sorted && l == 1) P.D[s.u] = s.d;   // ADG-O's same-round key
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

// Neighbour classes of v in round l: 0 = JP predecessor still in U (a later
// round), 3 = predecessor removed in round l (larger hash), 1 = same-round
// successor, 2 = successor from an earlier round.  Decrements D[w] for w
// still in U.
enum { NB_PRED = 0, NB_SUCC_SAME = 1, NB_SUCC_EARLIER = 2, NB_PRED_SAME = 3, NB_NONE = 5 };
// JP's order inside a round: rho_R, after D at selection for ADG-O.
__device__ __forceinline__ unsigned long long same_key(const Params& P, int v) {
  const unsigned long long h = tiebreak(P.hkey, (uint32_t)v);
  return P.sorted ? ((unsigned long long)(unsigned)P.D[v] << 32) | h : h;
}

// Classify UPD_UNROLL neighbours w[u] (ok[u]: entry u exists) of a vertex of
// R_l (same-round key hv[u]): NB_PRED for a neighbour still in U (a cut edge:
// counted in x when `count`, and D[w] decremented at once when `decrement`;
// otherwise the binned decrements below do it), same-round predecessor or
// successor, or earlier-round successor.  The status gathers go first, then
// the round gathers of same-round candidates, then the decisions, so that
// each kind of gather is in flight for all entries together.
template <bool FUSED>
__device__ __forceinline__ void visit_n(const Params& P, const int* w, const bool* ok, int l, unsigned char code,
                                        const unsigned long long* hv, unsigned& x, bool count, bool decrement, int* cl) {
  unsigned char st[UPD_UNROLL];
#pragma unroll
  for (int u = 0; u < UPD_UNROLL; ++u) st[u] = ok[u] ? P.status[w[u]] : 0;
  int rr[UPD_UNROLL];
#pragma unroll
  for (int u = 0; u < UPD_UNROLL; ++u) rr[u] = FUSED && ok[u] && st[u] == code ? P.round[w[u]] : 0;
#pragma unroll
  for (int u = 0; u < UPD_UNROLL; ++u) {
    if (!ok[u]) {
      cl[u] = NB_NONE;
    } else if (st[u] == 0) {
      if (count) {
        if (decrement) atomicSub(&P.D[w[u]], 1);
        x += 1;
      }
      cl[u] = NB_PRED;
    } else if (FUSED && st[u] == code && rr[u] == l) {
      cl[u] = same_key(P, w[u]) > hv[u] ? NB_PRED_SAME : NB_SUCC_SAME;
    } else {
      cl[u] = NB_SUCC_EARLIER;
    }
  }
}

__device__ __forceinline__ bool is_pred(int cl) { return cl == NB_PRED || cl == NB_PRED_SAME; }

// Colour bitmap words of a vertex with np predecessors: bits for colours
// 1 .. np+2 (GetColor's answer is at most np + 1).
__device__ __forceinline__ unsigned bm_words(int np) { return (unsigned)(np + 2 + 31) / 32; }

// A vertex's JP record: its bitmap word, and where its same-round successors
// are, in one 16-byte read.  Successor counts from 2^24 - 1 up are read from
// nsr instead.
struct JpRec {
  unsigned long long rec, sp;
};
constexpr unsigned SP_NS_MAX = (1u << 24) - 1;
__device__ __forceinline__ unsigned long long rec_of(const Params& P, int v) { return P.rec[2 * (size_t)v]; }
__device__ __forceinline__ JpRec rec_pair(const Params& P, int v) {
  const ulonglong2 x = *reinterpret_cast<const ulonglong2*>(P.rec + 2 * (size_t)v);
  return {x.x, x.y};
}
__device__ __forceinline__ long long sp_first(unsigned long long sp) { return (long long)(sp >> 24); }
__device__ __forceinline__ int sp_count(const Params& P, int v, unsigned long long sp) {
  const unsigned ns = (unsigned)sp & SP_NS_MAX;
  return ns < SP_NS_MAX ? (int)ns : P.nsr[v];
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename T>
__device__ __forceinline__ T wave_excl_scan(T x, T* total) {
  static_assert(sizeof(T) == 4, "32-bit scan");
  const unsigned incl = wave_incl_scan_u32((unsigned)x);
  *total = (T)(unsigned)__builtin_amdgcn_readlane((int)incl, WAVE - 1);
  return (T)(incl - (unsigned)x);
}

// Colour bitmap words come from one bump counter (bm_next).  A counter that
// every wavefront hits once per row serialises (one same-address atomic per
// vertex), so the kernels that build rows give each wavefront a pool: it
// takes pool_chunk words at a time and hands them out itself.  Requests
// above pool_chunk / 8 words go to the counter directly, so a chunk is at
// least 7/8 used before the next one is taken.  Pool state lives in the
// workspace by global wavefront index and carries over between launches;
// k_init empties it.
struct BmPool {
  unsigned long long next, end;   // wave-uniform
};
__device__ __forceinline__ BmPool pool_load(const Params& P, long long gw) {
  const unsigned long long s = P.pool[gw];
  return {s & 0xffffffffull, s >> 32};
}
__device__ __forceinline__ void pool_store(const Params& P, long long gw, const BmPool& b) {
  if (lane_id() == 0) P.pool[gw] = (b.end << 32) | b.next;
}
// `tot` words for the wavefront (wave-uniform); pl = nullptr: from the counter.
__device__ __forceinline__ unsigned long long pool_alloc(const Params& P, BmPool* pl, unsigned tot) {
  unsigned long long base = 0;
  if (!pl || tot > P.pool_chunk / 8) {
    if (lane_id() == 0) base = atomicAdd(&P.ctrl->bm_next, (unsigned long long)tot);
    return readlane_u64(base, 0);
  }
  if (pl->next + tot > pl->end) {
    if (lane_id() == 0) base = atomicAdd(&P.ctrl->bm_next, (unsigned long long)P.pool_chunk);
    base = readlane_u64(base, 0);
    pl->next = base;
    pl->end = base + P.pool_chunk;
  }
  const unsigned long long off = pl->next;
  pl->next += tot;
  return off;
}

// Whole wavefront: JP bookkeeping of the lanes' vertices with `has` set --
// |pred(v)| (np), same-round successors (ns), same-round predecessors still
// to be coloured (cnt = nps), and a cleared colour bitmap from the
// wavefront's pool (pl) or the bump counter (pl = nullptr);
// rec[v] = (bitmap offset << 32) | np.
__device__ __forceinline__ void jp_row(const Params& P, BmPool* pl, bool has, int v, long long first, long long np,
                                       long long ns, long long nps) {
  // JP: bits for colours 1 .. np+2; DEC-ADG-ITR: also the same-round successors
  const long long nb = P.dec ? np + ns : np;
  const unsigned w = has ? bm_words((int)nb) : 0;
  unsigned tot;
  const unsigned pre = wave_excl_scan<unsigned>(w, &tot);
  const unsigned long long base = tot ? pool_alloc(P, pl, tot) : 0;
  if (!has) return;
  unsigned long long off = base + pre;
  if (off + w > P.bm_cap) {  // cannot happen (see the capacity); keep accesses in bounds
    atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
    off = 0;
    np = 0;
    ns = 0;
    nps = 0;
  } else {
    for (unsigned k = 0; k < w; ++k) P.B[off + k] = 0;
  }
  P.xpred[v] = (int)(np - nps);
  P.nsr[v] = (int)ns;
  P.cnt[v] = (int)nps;
  P.rec[2 * (size_t)v] = (off << 32) | (unsigned)(P.dec ? np + ns : np);
  P.rec[2 * (size_t)v + 1] =
      ((unsigned long long)first << 24) | (ns < (long long)SP_NS_MAX ? (unsigned)ns : SP_NS_MAX);
}

// A vertex at position idx of its round's ORD slot (base) joins the round's
// first JP level iff it has no same-round predecessor (z).  L0 is indexed
// like the slot: it holds the vertex at that position, or ~0, so building
// it needs no counter.
__device__ __forceinline__ void l0_mark(const Params& P, long long base, long long idx, bool z, int v) {
  P.L0[base + idx] = z ? (unsigned)v : ~0u;
}

// UPDATE for a wavefront's 64 rows of at most SMALL_DEG entries each (one
// vertex per lane).  The rows' entries are spread evenly over the lanes --
// lane i of a pass takes entry p0 + i of the wavefront's concatenated rows,
// its row found by binary search over the prefix sums -- so a pass has all
// lanes busy whatever the row lengths.  Count pass: classify (and
// decrement), keeping each entry's class and the per-row class counts in
// LDS; placing pass: write the row as [predecessors from later rounds |
// same-round predecessors | same-round successors | successors from earlier
// rounds] (the order inside a part is arbitrary).
struct SmallRows {
  int off[WAVE + 1];                    // exclusive scan of the row lengths
  long long b[WAVE];                    // first entry of each row
  unsigned long long hv[WAVE];          // same-round key of each row's vertex
  unsigned cnt[WAVE][4];                // entries per class (NB_*) and row
  unsigned run[WAVE][4];                // entries placed so far
  unsigned char cls[WAVE * SMALL_DEG];  // class of each entry
};

__device__ __forceinline__ int small_owner(const SmallRows& S, int pos) {
  int lo = 0, hi = WAVE;  // the last row k with off[k] <= pos (rows before it may be empty)
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (S.off[mid] <= pos) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <bool FUSED>
__device__ void update_small(const Params& P, BmPool* pl, SmallRows& S, int v, bool valid, int l,
                             unsigned char code, unsigned& x, long long idx0) {
  const unsigned lane = lane_id();
  long long b = 0, e = 0;
  if (valid) {
    b = P.rp[v];
    e = P.rp[v + 1];
  }
  int T;
  const int off = wave_excl_scan<int>((int)(e - b), &T);
  S.off[lane] = off;
  S.b[lane] = b;
  S.hv[lane] = same_key(P, v);
  if (lane == 0) S.off[WAVE] = T;
  if (FUSED)
    for (int k = 0; k < 4; ++k) {
      S.cnt[lane][k] = 0;
      S.run[lane][k] = 0;
    }
  wave_sync();
  for (int p0 = 0; p0 < T; p0 += WAVE * UPD_UNROLL) {
    int w[UPD_UNROLL], k[UPD_UNROLL], cl[UPD_UNROLL];
    bool ok[UPD_UNROLL];
    unsigned long long hv[UPD_UNROLL];
#pragma unroll
    for (int u = 0; u < UPD_UNROLL; ++u) {
      const int pos = p0 + u * WAVE + (int)lane;
      ok[u] = pos < T;
      k[u] = ok[u] ? small_owner(S, pos) : 0;
      w[u] = ok[u] ? P.col[S.b[k[u]] + (pos - S.off[k[u]])] : 0;
      hv[u] = S.hv[k[u]];
    }
    visit_n<FUSED>(P, w, ok, l, code, hv, x, !P.pull, !P.pull && !P.binned, cl);
    if (FUSED) {
#pragma unroll
      for (int u = 0; u < UPD_UNROLL; ++u)
        if (ok[u]) {
          S.cls[p0 + u * WAVE + (int)lane] = (unsigned char)cl[u];
          atomicAdd(&S.cnt[k[u]][cl[u]], 1u);
        }
    }
  }
  if (!FUSED) return;
  wave_sync();
  const long long nl = S.cnt[lane][NB_PRED], nps = S.cnt[lane][NB_PRED_SAME], ns = S.cnt[lane][NB_SUCC_SAME];
  const long long np = nl + nps;
  for (int p0 = 0; p0 < T; p0 += WAVE * UPD_UNROLL) {
    int w[UPD_UNROLL], k[UPD_UNROLL], cl[UPD_UNROLL];
#pragma unroll
    for (int u = 0; u < UPD_UNROLL; ++u) {
      const int pos = p0 + u * WAVE + (int)lane;
      cl[u] = pos < T ? S.cls[pos] : NB_NONE;
      const bool keep = cl[u] != NB_NONE && cl[u] != NB_SUCC_EARLIER;   // earlier-round successors: never read back
      k[u] = keep ? small_owner(S, pos) : 0;
      w[u] = keep ? P.col[S.b[k[u]] + (pos - S.off[k[u]])] : 0;
      if (!keep) cl[u] = NB_NONE;
    }
#pragma unroll
    for (int u = 0; u < UPD_UNROLL; ++u)
      if (cl[u] != NB_NONE) {
        const long long bk = S.b[k[u]];
        const long long r = atomicAdd(&S.run[k[u]][cl[u]], 1u);
        const long long nlk = S.cnt[k[u]][NB_PRED], npk = nlk + S.cnt[k[u]][NB_PRED_SAME];
        const long long at = cl[u] == NB_PRED ? bk + r : cl[u] == NB_PRED_SAME ? bk + nlk + r : bk + npk + r;
        P.dag[at] = w[u];
      }
  }
  wave_sync();   // the LDS is rewritten by the wavefront's next group of rows
  jp_row(P, pl, valid, v, b + np, np, ns, nps);
  if (valid) l0_mark(P, (long long)P.n - P.roundN[l], idx0 + lane, nps == 0, v);
}

// Wave-per-vertex UPDATE for longer rows: count pass (with the decrements),
// then a placing pass.
// Class masks a wavefront keeps between its count and placing passes: per
// 64-entry chunk of a row (up to HUGE_DEG entries), the lanes holding
// predecessors from later rounds, same-round predecessors and same-round
// successors (the rest are earlier-round successors).
constexpr int ROW_CHUNKS = HUGE_DEG / WAVE;
// Per hub row, HC holds the class counts [4] and placed counts [4]; earlier
// successors are never placed, so their placed-count word holds instead the
// hub's position in its round's ORD slot (for L0).
constexpr int HC_SLOT = 4 + NB_SUCC_EARLIER;
struct RowMasks {
  uint64_t m[ROW_CHUNKS][3];
};

template <bool FUSED>
__device__ void update_big(const Params& P, BmPool* pl, RowMasks& rm, int v, long long b, long long e, int l,
                           unsigned char code, unsigned& x, long long idx) {
  if (e - b > HUGE_DEG) {  // a hub: its chunks are spread over the grid by k_update_huge_*
    if (lane_id() == 0) {
      const unsigned long long nch = (unsigned long long)((e - b + HUGE_CHUNK - 1) / HUGE_CHUNK);
      const unsigned long long old = atomicAdd(&P.ctrl->huge_ctr, (nch << 32) | 1ull);
      const unsigned h = (unsigned)old;
      if (h < P.huge_cap) {
        P.HL[h] = (old & 0xffffffff00000000ull) | (unsigned)v;
        for (int k = 0; k < 8; ++k) P.HC[8 * (size_t)h + k] = 0;
        P.HC[8 * (size_t)h + HC_SLOT] = (unsigned)idx;
        if (FUSED) l0_mark(P, (long long)P.n - P.roundN[l], idx, false, v);   // set by the hub kernels
      } else {
        atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
      }
    }
    return;
  }
  const unsigned long long hv = same_key(P, v);
  const unsigned lane = lane_id();
  long long nl = 0, nps = 0, ns = 0;
  int ch = 0;
  for (long long base = b; base < e; base += WAVE * UPD_UNROLL, ch += UPD_UNROLL) {
    int w[UPD_UNROLL], cl[UPD_UNROLL];
    bool ok[UPD_UNROLL];
    unsigned long long hvs[UPD_UNROLL];
#pragma unroll
    for (int u = 0; u < UPD_UNROLL; ++u) {
      const long long j = base + u * WAVE + lane;
      ok[u] = j < e;
      w[u] = ok[u] ? P.col[j] : 0;
      hvs[u] = hv;
    }
    visit_n<FUSED>(P, w, ok, l, code, hvs, x, !P.pull, !P.pull && !P.binned, cl);
    if (FUSED) {
#pragma unroll
      for (int u = 0; u < UPD_UNROLL; ++u) {
        const uint64_t fm = ballot(cl[u] == NB_PRED), gm = ballot(cl[u] == NB_PRED_SAME), sm = ballot(cl[u] == NB_SUCC_SAME);
        nl += __popcll(fm);
        nps += __popcll(gm);
        ns += __popcll(sm);
        if (lane == 0 && base + u * WAVE < e) {   // rows of at most HUGE_DEG entries: ch + u < ROW_CHUNKS
          rm.m[ch + u][0] = fm;
          rm.m[ch + u][1] = gm;
          rm.m[ch + u][2] = sm;
        }
      }
    }
  }
  if (!FUSED) return;
  wave_sync();
  const long long np = nl + nps;
  long long fc = 0, gc = 0, sc = 0;
  ch = 0;
  for (long long base = b; base < e; base += WAVE * UPD_UNROLL, ch += UPD_UNROLL) {
    uint64_t fm[UPD_UNROLL], gm[UPD_UNROLL], sm[UPD_UNROLL];
    int w[UPD_UNROLL];
    const uint64_t me = 1ull << lane;
#pragma unroll
    for (int u = 0; u < UPD_UNROLL; ++u) {
      const bool in = base + u * WAVE < e;
      fm[u] = in ? rm.m[ch + u][0] : 0;
      gm[u] = in ? rm.m[ch + u][1] : 0;
      sm[u] = in ? rm.m[ch + u][2] : 0;
      // earlier-round successors are never read back: their lanes load nothing
      w[u] = (fm[u] | gm[u] | sm[u]) & me ? P.col[base + u * WAVE + lane] : 0;
    }
#pragma unroll
    for (int u = 0; u < UPD_UNROLL; ++u) {
      if (fm[u] & me) P.dag[b + fc + lanes_below(fm[u])] = w[u];
      else if (gm[u] & me) P.dag[b + nl + gc + lanes_below(gm[u])] = w[u];
      else if (sm[u] & me) P.dag[b + np + sc + lanes_below(sm[u])] = w[u];
      fc += __popcll(fm[u]);
      gc += __popcll(gm[u]);
      sc += __popcll(sm[u]);
    }
  }
  wave_sync();   // the masks are rewritten by the wavefront's next row
  jp_row(P, pl, lane == 0, v, b + np, np, ns, nps);
  if (lane == 0) l0_mark(P, (long long)P.n - P.roundN[l], idx, nps == 0, v);
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
  BmPool pool = {0, 0};
  // per wavefront: the short rows' entry classes, or a long row's masks
  __shared__ union WaveUpd {
    SmallRows sr;
    RowMasks rm;
  } wu[WPB];
  WaveUpd& U = wu[threadIdx.x / WAVE];
  if (FUSED) pool = pool_load(P, gw);
  long long it = gw;
  for (; it < items && it < nsg; it += gstride) {
    long long idx = it * WAVE + lane_id();
    bool valid = idx < nRs;
    int v = valid ? RL[idx] : 0;
    update_small<FUSED>(P, &pool, U.sr, v, valid, l, code, x, it * WAVE);
  }
  // The long rows, one after the other per wavefront, with the next ones'
  // metadata in flight: the vertex of the row after next and the bounds of
  // the next row are loaded while a row is walked.
  if (it < items) {
    auto vert = [&](long long k) { return k < items ? RL[nRs + (k - nsg)] : 0; };
    int v0 = vert(it);
    long long b0 = P.rp[v0], e0 = P.rp[v0 + 1];
    int v1 = vert(it + gstride);
    for (; it < items; it += gstride) {
      const int v2 = vert(it + 2 * gstride);
      const long long b1 = P.rp[v1], e1 = P.rp[v1 + 1];
      update_big<FUSED>(P, &pool, U.rm, v0, b0, e0, l, code, x, nRs + (it - nsg));
      v0 = v1;
      b0 = b1;
      e0 = e1;
      v1 = v2;
    }
  }
  if (FUSED) pool_store(P, gw, pool);
  unsigned long long xs = wave_sum((unsigned long long)x);
  if (lane_id() == 0) xred[threadIdx.x / WAVE] = xs;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int k = 0; k < WPB; ++k) t += xred[k];
    P.xpart[blockIdx.x] = t;
  }
}

// Pull UPDATE: every vertex of U_{l+1} subtracts from its own D the number of
// its neighbours removed in round l.  Short rows are walked by their lane,
// longer ones by the whole wavefront.  The decrements per block go to xpart
// (the grid is upd_blocks, so every entry is written).
__global__ __launch_bounds__(BS) void k_update_pull(Params P, int l) {
  Ctrl* c = P.ctrl;
  if (c->done) return;
  const unsigned long long N = c->Nnext;
  const int* Un = P.UL[l & 1];
  const unsigned char code = round_code(l);
  __shared__ unsigned long long xred[WPB];
  unsigned long long x = 0;
  const long long stride = (long long)gridDim.x * BS;
  for (long long t = (long long)blockIdx.x * BS; t < (long long)N; t += stride) {
    const long long i = t + threadIdx.x;
    const bool has = i < (long long)N;
    const int v = has ? Un[i] : 0;
    long long b = 0, e = 0;
    if (has) {
      b = P.rp[v];
      e = P.rp[v + 1];
    }
    unsigned cnt = 0;
    const bool longrow = has && e - b > WAVE;
    if (has && !longrow)
      for (long long j = b; j < e; ++j) {
        const int w = P.col[j];
        cnt += P.status[w] == code && P.round[w] == l;
      }
    uint64_t m = ballot(longrow);
    while (m) {
      const int src = __ffsll((long long)m) - 1;
      m &= m - 1;
      const long long bb = readlane_i64(b, src), ee = readlane_i64(e, src);
      unsigned part = 0;
      for (long long j = bb + lane_id(); j < ee; j += WAVE) {
        const int w = P.col[j];
        part += P.status[w] == code && P.round[w] == l;
      }
      part = wave_sum(part);
      if (lane_id() == (unsigned)src) cnt = part;
    }
    if (has && cnt) {
      P.D[v] -= (int)cnt;
      x += cnt;
    }
  }
  x = wave_sum(x);
  if (lane_id() == 0) xred[threadIdx.x / WAVE] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int k = 0; k < WPB; ++k) t += xred[k];
    P.xpart[blockIdx.x] = t;
  }
}

// ---- hubs: rows longer than HUGE_DEG, cut into HUGE_CHUNK-sized chunks

// Hub entry of chunk k (entries are sorted by first chunk).
__device__ __forceinline__ unsigned huge_entry(const Params& P, unsigned nh, unsigned k, unsigned* h) {
  unsigned lo = 0, hi = nh;
  while (hi - lo > 1) {
    const unsigned mid = (lo + hi) >> 1;
    if ((unsigned)(P.HL[mid] >> 32) <= k) lo = mid;
    else hi = mid;
  }
  *h = lo;
  return (unsigned)(P.HL[lo] >> 32);
}

// Count pass over the hubs' chunks: neighbour classes (summed per hub) and
// the decrements of D.
template <bool FUSED>
__global__ __launch_bounds__(BS) void k_update_huge_count(Params P, int l) {
  Ctrl* c = P.ctrl;
  if (c->done) return;
  const unsigned long long hc = c->huge_ctr;
  const unsigned nh = (unsigned)hc < P.huge_cap ? (unsigned)hc : P.huge_cap, nch = (unsigned)(hc >> 32);
  if (nh == 0) return;
  const unsigned char code = round_code(l);
  const unsigned lane = lane_id();
  const long long gw = (long long)blockIdx.x * WPB + threadIdx.x / WAVE;
  const long long gstride = (long long)gridDim.x * WPB;
  unsigned x = 0;
  for (long long k = gw; k < nch; k += gstride) {
    unsigned h;
    const unsigned first = huge_entry(P, nh, (unsigned)k, &h);
    const int v = (int)(unsigned)P.HL[h];
    const long long b = P.rp[v], e = P.rp[v + 1];
    const long long c0 = b + ((long long)k - first) * HUGE_CHUNK;
    const long long c1 = c0 + HUGE_CHUNK < e ? c0 + HUGE_CHUNK : e;
    const unsigned long long hv = same_key(P, v);
    unsigned cnt[4] = {0, 0, 0, 0};
    for (long long base = c0; base < c1; base += WAVE * UPD_UNROLL) {
      int w[UPD_UNROLL], cl[UPD_UNROLL];
      bool ok[UPD_UNROLL];
      unsigned long long hvs[UPD_UNROLL];
#pragma unroll
      for (int u = 0; u < UPD_UNROLL; ++u) {
        const long long j = base + u * WAVE + lane;
        ok[u] = j < c1;
        w[u] = ok[u] ? P.col[j] : 0;
        hvs[u] = hv;
      }
      visit_n<FUSED>(P, w, ok, l, code, hvs, x, !P.pull, !P.pull && !P.binned, cl);
#pragma unroll
      for (int u = 0; u < UPD_UNROLL; ++u) {
        cnt[NB_PRED] += __popcll(ballot(cl[u] == NB_PRED));
        cnt[NB_PRED_SAME] += __popcll(ballot(cl[u] == NB_PRED_SAME));
        cnt[NB_SUCC_SAME] += __popcll(ballot(cl[u] == NB_SUCC_SAME));
        cnt[NB_SUCC_EARLIER] += __popcll(ballot(cl[u] == NB_SUCC_EARLIER));
      }
    }
    if (FUSED && lane < 4) atomicAdd(&P.HC[8 * (size_t)h + lane], cnt[lane]);
  }
  const unsigned long long xs = wave_sum((unsigned long long)x);
  if (lane == 0 && xs) atomicAdd(&c->xhuge, xs);
}

// Placing pass over the hubs' chunks: each chunk writes its entries at
// offsets reserved in its hub's partitions; the chunk that starts a hub also
// does the hub's JP bookkeeping.
__global__ __launch_bounds__(BS) void k_update_huge_place(Params P, int l) {
  Ctrl* c = P.ctrl;
  if (c->done) return;
  const unsigned long long hc = c->huge_ctr;
  const unsigned nh = (unsigned)hc < P.huge_cap ? (unsigned)hc : P.huge_cap, nch = (unsigned)(hc >> 32);
  if (nh == 0) return;
  const unsigned char code = round_code(l);
  const unsigned lane = lane_id();
  const long long gw = (long long)blockIdx.x * WPB + threadIdx.x / WAVE;
  const long long gstride = (long long)gridDim.x * WPB;
  unsigned x = 0;
  for (long long k = gw; k < nch; k += gstride) {
    unsigned h;
    const unsigned first = huge_entry(P, nh, (unsigned)k, &h);
    const int v = (int)(unsigned)P.HL[h];
    const long long b = P.rp[v], e = P.rp[v + 1];
    const long long c0 = b + ((long long)k - first) * HUGE_CHUNK;
    const long long c1 = c0 + HUGE_CHUNK < e ? c0 + HUGE_CHUNK : e;
    const unsigned long long hv = same_key(P, v);
    unsigned* C = P.HC + 8 * (size_t)h;
    const long long nl = C[NB_PRED], nps = C[NB_PRED_SAME], ns = C[NB_SUCC_SAME];
    const long long np = nl + nps;
    const long long start[4] = {b, b + np, 0, b + nl};   // by class (earlier successors are not kept)
    for (long long base = c0; base < c1; base += WAVE * UPD_UNROLL) {
      int w[UPD_UNROLL], cl[UPD_UNROLL];
      bool ok[UPD_UNROLL];
      unsigned long long hvs[UPD_UNROLL];
#pragma unroll
      for (int u = 0; u < UPD_UNROLL; ++u) {
        const long long j = base + u * WAVE + lane;
        ok[u] = j < c1;
        w[u] = ok[u] ? P.col[j] : 0;
        hvs[u] = hv;
      }
      visit_n<true>(P, w, ok, l, code, hvs, x, false, false, cl);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q == NB_SUCC_EARLIER) continue;   // never read back
        // one reservation for the class's entries of all UPD_UNROLL chunks
        uint64_t m[UPD_UNROLL];
        unsigned tot = 0;
#pragma unroll
        for (int u = 0; u < UPD_UNROLL; ++u) {
          m[u] = ballot(cl[u] == q);
          tot += (unsigned)__popcll(m[u]);
        }
        if (!tot) continue;
        unsigned at = 0;
        if (lane == 0) at = atomicAdd(&C[4 + q], tot);
        at = readlane_u(at, 0);
#pragma unroll
        for (int u = 0; u < UPD_UNROLL; ++u) {
          if (cl[u] == q) P.dag[start[q] + at + lanes_below(m[u])] = w[u];
          at += (unsigned)__popcll(m[u]);
        }
      }
    }
    if (k == first) {
      jp_row(P, nullptr, lane == 0, v, b + np, np, ns, nps);
      if (lane == 0) l0_mark(P, (long long)P.n - P.roundN[l], C[HC_SLOT], nps == 0, v);
    }
  }
}

// ================================================================ JP Part 1 (stand-alone)

__device__ __forceinline__ uint64_t prio(const Params& P, int w) {
  return ((uint64_t)(uint32_t)P.round[w] << 32) | tiebreak(P.hkey, (uint32_t)w);
}

// For jp_color on a given ranking: classify every neighbour by the priority
// <round, hash> and write rows [pred | succ].  All vertices form one
// pseudo-round (its L0 at offset 0), so every predecessor is counted by cnt
// and every successor is walked by the levels: nsr(v) = |succ(v)|.
__global__ __launch_bounds__(BS) void k_part1(Params P) {
  const long long gw = (long long)blockIdx.x * WPB + threadIdx.x / WAVE;
  const long long gstride = (long long)gridDim.x * WPB;
  const unsigned lane = lane_id();
  const long long groups = ((long long)P.n + WAVE - 1) / WAVE;
  BmPool pool = pool_load(P, gw);
  for (long long g = gw; g < groups; g += gstride) {
    long long idx = g * WAVE + lane;
    bool valid = idx < P.n;
    int v = valid ? (int)idx : 0;
    long long b = valid ? P.rp[v] : 0, e = valid ? P.rp[v + 1] : 0;
    const uint64_t kv = prio(P, v);
    const bool small = valid && (e - b) <= SMALL_DEG;
    long long np = 0;
    if (small) {
      long long f = b, s = e;
      for (long long j = b; j < e; ++j) {
        int w = P.col[j];
        if (prio(P, w) > kv) P.dag[f++] = w;
        else P.dag[--s] = w;
      }
      np = f - b;
    }
    jp_row(P, &pool, small, v, b + np, np, (e - b) - np, np);
    if (small) l0_mark(P, 0, v, np == 0, v);   // one pseudo-round: its slot is the identity
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
      jp_row(P, &pool, lane == 0, u, ub + fc, fc, sc, fc);
      if (lane == 0) l0_mark(P, 0, u, fc == 0, u);
    }
  }
  pool_store(P, gw, pool);
}

// ================================================================ JP Part 2
//
// Rounds are coloured from L down to 1.  Every edge of G_rho between two
// rounds points from the higher round to the lower, so once rounds above r
// are coloured, a vertex of round r waits only for its same-round
// predecessors: cnt[v] counts those not yet coloured (set by UPDATE), and the
// round's vertices with none form its first level (the list L0 of the round,
// also built by UPDATE).  Each vertex owns a bitmap of the colours its
// predecessors took (colours 1 .. |pred|+2).  When round r starts, one bulk
// step ORs in the colours of every predecessor from a later round (final by
// then).  Inside the round, a coloured vertex ORs its colour into the bitmap
// of each same-round successor and takes one unit off its cnt; whoever takes
// the last unit appends the successor to the next level.  A level's vertex
// is coloured with the first clear bit of its bitmap (GetColor), complete
// once all its predecessors have been coloured at earlier levels.
//
// Levels of at most NARROW_MAX vertices (and bounded work) run inside one
// 1024-thread block with the level lists in LDS; wider ones over the grid,
// with lists in global memory: F (vertices with at most JP_SMALL same-round
// successors, a lane each) and H (the others, whose successors are cut into
// JP_CHUNK-sized chunks that different wavefronts take).

struct JpStage {
  unsigned* buf;                // LDS staging of plain vertices (grid kernel), or null
  unsigned* cnt;                // its fill level (LDS)
  unsigned* fcnt;               // level counters (control block, or LDS)
  unsigned long long* hctr;
  unsigned long long* psum;     // bitmap words of the level's vertices
  unsigned long long* ssum;     // their same-round successors
  unsigned long long* acc;      // LDS [2]: this block's share of psum and ssum (null: sums not kept)
};

// ---- bounds on indices that come from device state
//
// The vertex ids, list positions, DAG entries and bitmap words the JP steps
// use are all derived from what earlier steps stored (level lists, DAG rows,
// JP records, counters).  They are in range whenever those steps are
// correct; these checks keep a broken state from becoming an access outside
// the workspace: the call then reports ADG_ERR_INTERNAL and the work item is
// dropped.
__device__ __forceinline__ void raise_internal(const Params& P) { atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL); }
__device__ __forceinline__ bool vid_ok(const Params& P, int v) {
  if ((unsigned)v < (unsigned)P.n) return true;
  raise_internal(P);
  return false;
}
// A same-round successor range [s0, s1) of the DAG rows.
__device__ __forceinline__ bool range_ok(const Params& P, long long s0, long long s1) {
  if (s0 >= 0 && s0 <= s1 && s1 <= P.nnz) return true;
  raise_internal(P);
  return false;
}
// A level-list slot (the lists hold at most n entries).
__device__ __forceinline__ bool slot_ok(const Params& P, unsigned at) {
  if (at < (unsigned)P.n) return true;
  raise_internal(P);
  return false;
}

// The sizes of a level's lists, and of round r's first level and slot.
__device__ __forceinline__ bool level_ok(const Params& P, unsigned nf, unsigned nh) {
  if (nf <= (unsigned)P.n && nh <= P.hub_cap) return true;
  raise_internal(P);
  return false;
}
__device__ __forceinline__ bool round_ok(const Params& P, int r) {
  if (r >= 1 && P.roundN[r] <= (unsigned)P.n && P.roundN[r + 1] <= P.roundN[r]) return true;
  raise_internal(P);
  return false;
}

// Append u (ready; JP record ur) to the global lists of level l + 1.
template <int S>
__device__ __forceinline__ void jp_append(const Params& P, JpStage& st, int l, bool rdy, int u, const JpRec& ur) {
  const long long ns = rdy ? sp_count(P, u, ur.sp) : 0;
  if (st.acc && ballot(rdy)) {
    const unsigned long long es = wave_sum((unsigned long long)ns);
    const unsigned long long ps = wave_sum((unsigned long long)(rdy ? bm_words((int)(unsigned)ur.rec) : 0));
    if (lane_id() == 0) {
      atomicAdd(&st.acc[0], ps);
      atomicAdd(&st.acc[1], es);
    }
  }
  const bool fan = rdy && ns > JP_SMALL;
  const uint64_t fm = ballot(fan);
  if (fm) {
    // one atomic per wavefront: (chunks << 32) | entries for all its fan-out vertices
    const unsigned nch = fan ? (unsigned)((ns + JP_CHUNK - 1) / JP_CHUNK) : 0;
    unsigned ctot;
    const unsigned cpre = wave_excl_scan<unsigned>(nch, &ctot);
    unsigned long long old = 0;
    if (lane_id() == 0) old = add64<S>(&st.hctr[(l + 1) % 3], ((unsigned long long)ctot << 32) | __popcll(fm));
    old = readlane_u64(old, 0);
    if (fan) {
      const unsigned pos = (unsigned)old + lanes_below(fm);
      const unsigned first = (unsigned)(old >> 32) + cpre;
      if (pos < P.hub_cap) st64<S>(&P.H[(l + 1) & 1][pos], ((unsigned long long)first << 32) | (unsigned)u);
      else atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
    }
  }
  const bool plain = rdy && !fan;
  uint64_t m = ballot(plain);
  if (!m) return;
  unsigned k = __popcll(m);
  if (!st.buf) {
    unsigned g = 0;
    if (lane_id() == 0) g = add32<S>(&st.fcnt[(l + 1) % 3], k);
    g = readlane_u(g, 0);
    if (plain && slot_ok(P, g + lanes_below(m))) sti<S>((int*)&P.F[(l + 1) & 1][g + lanes_below(m)], u);
    return;
  }
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
    if (plain && pos >= (unsigned)FB_CAP && slot_ok(P, g + lanes_below(om)))
      sti<S>((int*)&P.F[(l + 1) & 1][g + lanes_below(om)], u);
  }
}

// Block-wide: move the staged vertices to level l + 1's list.
template <int S>
__device__ __forceinline__ void jp_stage_flush(const Params& P, JpStage& st, int l) {
  __syncthreads();
  __shared__ unsigned gbase;
  unsigned k = *st.cnt;
  if (k > (unsigned)FB_CAP) k = FB_CAP;
  if (threadIdx.x == 0) {
    gbase = k ? add32<S>(&st.fcnt[(l + 1) % 3], k) : 0;
    if (st.acc) {
      if (st.acc[0]) add64<S>(&st.psum[(l + 1) % 3], st.acc[0]);
      if (st.acc[1]) add64<S>(&st.ssum[(l + 1) % 3], st.acc[1]);
      st.acc[0] = st.acc[1] = 0;
    }
  }
  __syncthreads();
  for (unsigned i = threadIdx.x; i < k; i += blockDim.x)
    if (slot_ok(P, gbase + i)) sti<S>((int*)&P.F[(l + 1) & 1][gbase + i], (int)st.buf[i]);
  __syncthreads();
  if (threadIdx.x == 0) *st.cnt = 0;
  __syncthreads();
}

// Block-wide, between the passes of a loop whose wavefronts append one
// vertex per lane and pass (this wavefront has work in the pass: `any`):
// false once no wavefront of the block has work; otherwise true, after the
// block's staged vertices (level l + 1) have gone to the global list if
// another pass could fill the staging buffer.  Without this, a long list
// (a round's first level of tens of millions of vertices) would overflow the
// buffer after a few passes, and every later wavefront would take its slots
// with an atomic on the one global counter.
__device__ __forceinline__ bool stage_pass(const Params& P, JpStage& st, int l, bool any) {
  if (!st.buf) return any;
  if (!__syncthreads_or(any)) return false;
  if (*st.cnt + blockDim.x > (unsigned)FB_CAP) jp_stage_flush<SC_AGENT>(P, st, l);
  return true;
}

// Mark colour c in the bitmap described by rec (if it can matter there).
template <int S>
__device__ __forceinline__ void bm_mark(const Params& P, unsigned long long rec, int c) {
  if (c >= 1 && c <= (int)(unsigned)rec + 2) {
    const unsigned b = (unsigned)(c - 1);
    const unsigned long long at = (rec >> 32) + (b >> 5);
    if (at < P.bm_cap) __hip_atomic_fetch_or(&P.B[at], 1u << (b & 31), __ATOMIC_RELAXED, S);
    else raise_internal(P);
  }
}

// Same-round successor u (bitmap rec) of a vertex of colour c: record c, take
// one unit off cnt[u]; true if that was u's last uncoloured same-round
// predecessor.
template <int S>
__device__ __forceinline__ bool jp_push(const Params& P, int u, unsigned long long rec, int c) {
  bm_mark<S>(P, rec, c);
  return __hip_atomic_fetch_add(&P.cnt[u], -1, __ATOMIC_RELAXED, S) == 1;
}

// A bitmap word, read at the device's coherence point (atomics update it).
__device__ __forceinline__ unsigned bm_load(const Params& P, unsigned long long at) {
  if (at < P.bm_cap) return agent_load_u32(&P.B[at]);
  raise_internal(P);
  return ~0u;
}

// Colour of a finished vertex (also read at the coherence point).
__device__ __forceinline__ int done_colour(const Params& P, int u) { return agent_load_i32(&P.color[u]); }

#ifndef ADG_XPULL_GMIN
#define ADG_XPULL_GMIN 1
#endif
constexpr long long XPULL_GMIN = ADG_XPULL_GMIN;   // fewest vertices in a pull group
constexpr int XW_WORDS = 2;   // bitmap words per vertex the cross-round pull gathers in LDS (colours 1..64)

struct WaveLds {
  int off[WAVE + 1];           // exclusive scan of the lanes' item counts
  unsigned long long rec[WAVE];
  long long pb[WAVE];
  int ffree[WAVE];             // first clear bit found in the lanes' bitmaps (then the lanes' colours)
  int soff[WAVE + 1];          // exclusive scan of the lanes' same-round successor counts
  unsigned xw[XW_WORDS * WAVE]; // cross-round pull: the first bitmap words of the lanes' vertices
};

// Lane k whose range [off[k], off[k+1]) holds position e.
__device__ __forceinline__ int wave_owner_of(const int* off, int e) {
  int lo = 0, hi = WAVE;  // last k with off[k] <= e
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= e) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int wave_owner(const WaveLds& W, int e) {
  int lo = 0, hi = WAVE;  // last k with off[k] <= e
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (W.off[mid] <= e) lo = mid;
    else hi = mid;
  }
  return lo;
}

// GetColor for every active lane (bitmap rec): the wavefront reads all the
// lanes' bitmap words, spread evenly over its lanes, and each lane takes the
// first clear bit of its own.
__device__ __forceinline__ int wave_colour(const Params& P, WaveLds& W, bool act, unsigned long long rec) {
  const unsigned lane = lane_id();
  int tot;
  const int pre = wave_excl_scan<int>(act ? (int)bm_words((int)(unsigned)rec) : 0, &tot);
  W.off[lane] = pre;
  W.rec[lane] = rec;
  W.ffree[lane] = 0x7fffffff;
  if (lane == 0) W.off[WAVE] = tot;
  wave_sync();
  for (int e0 = 0; e0 < tot; e0 += WAVE * JP_UNROLL) {
    int own[JP_UNROLL];
    unsigned wd[JP_UNROLL];
#pragma unroll
    for (int t = 0; t < JP_UNROLL; ++t) {
      const int e = e0 + t * WAVE + (int)lane;
      own[t] = -1;
      wd[t] = ~0u;
      if (e < tot) {
        own[t] = wave_owner(W, e);
        wd[t] = bm_load(P, (W.rec[own[t]] >> 32) + (unsigned)(e - W.off[own[t]]));
      }
    }
#pragma unroll
    for (int t = 0; t < JP_UNROLL; ++t)
      if (own[t] >= 0 && ~wd[t]) {
        const int e = e0 + t * WAVE + (int)lane;
        atomicMin(&W.ffree[own[t]], (e - W.off[own[t]]) * 32 + __ffs((int)~wd[t]) - 1);
      }
  }
  wave_sync();
  int col = 0;
  if (act) {
    const int f = W.ffree[lane];
    if (f == 0x7fffffff) {  // unreachable: at most |pred| of the |pred|+2 bits are set
      atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
      col = (int)(unsigned)rec + 1;
    } else {
      col = f + 1;
    }
  }
  wave_sync();
  return col;
}

// ---- D decrements by bins
//
// Each cut edge (v removed in round l, w still in U) takes one off D[w].  As
// one device atomic each, these decrements bound UPDATE: about 10^9 a second
// on targets spread over the graph, while a round of R-MAT's has 10^8 or more
// of them, concentrated on far fewer targets (hundreds per target on average
// in the middle rounds, but too spread for a small table of hot targets to
// catch most).  So UPDATE only counts them, and after it the targets -- the
// later-round predecessors that UPDATE wrote at the front of each row of R_l
// (xpred[v] of them) -- go through bins of SUB_SPAN vertices: a count pass
// (block histograms in LDS), a scan (offsets per bin and block), a scatter
// pass into SB in bin order, and an apply pass that sums each bin's targets
// in LDS and subtracts the sums from D, one atomic per target and chunk.

// The targets of round l as block blockIdx.x of SUB_BLOCKS walks them: its
// contiguous share of R_l's rows up to HUGE_DEG entries (a wavefront takes 64
// rows and spreads their targets over its lanes), then every SUB_BLOCKS-th
// chunk of HUGE_CHUNK targets of the longer rows (the hubs), the whole block
// on each.  Both passes walk the same targets in each block.  SCATTER = false:
// count them per bin in lds; true: write each to SB at the bin cursor in lds
// (or, with `direct`, decrement D at once).
#ifndef ADG_SUB_UNROLL
#define ADG_SUB_UNROLL 16
#endif
constexpr int SUB_UNROLL = ADG_SUB_UNROLL;   // 64-target chunks the binning walks load at a time
template <bool SCATTER>
__device__ __forceinline__ void sub_walk(const Params& P, WaveLds& W, unsigned* lds, bool direct) {
  Ctrl* c = P.ctrl;
  const long long nR = (long long)c->nRs + c->nRb;
  const int* RL = round_slot(P, c->N);
  const long long lo = nR * blockIdx.x / gridDim.x, hi = nR * (blockIdx.x + 1) / gridDim.x;
  const unsigned lane = lane_id();
  const int nw = blockDim.x / WAVE;
  for (long long g0 = lo + (long long)(threadIdx.x / WAVE) * WAVE; g0 < hi; g0 += (long long)nw * WAVE) {
    const long long i = g0 + lane;
    int k = 0;
    long long b = 0;
    if (i < hi) {
      const int v = RL[i];
      if (vid_ok(P, v)) {
        const long long e = P.rp[v + 1];
        b = P.rp[v];
        if (e - b <= HUGE_DEG) {
          k = P.xpred[v];
          if (k < 0 || k > e - b) {
            raise_internal(P);
            k = 0;
          }
        }
      }
    }
    int tot;
    W.off[lane] = wave_excl_scan<int>(k, &tot);
    W.pb[lane] = b;
    if (lane == 0) W.off[WAVE] = tot;
    wave_sync();
    for (int e0 = 0; e0 < tot; e0 += WAVE * SUB_UNROLL) {
      int w[SUB_UNROLL];
#pragma unroll
      for (int u = 0; u < SUB_UNROLL; ++u) {
        const int e = e0 + u * WAVE + (int)lane;
        w[u] = -1;
        if (e < tot) {
          const int own = wave_owner(W, e);
          w[u] = P.dag[W.pb[own] + (e - W.off[own])];
        }
      }
#pragma unroll
      for (int u = 0; u < SUB_UNROLL; ++u)
        if (w[u] >= 0 && vid_ok(P, w[u])) {
          if (!SCATTER) atomicAdd(&lds[w[u] >> SUB_SHIFT], 1u);
          else if (direct) atomicSub(&P.D[w[u]], 1);
          else P.SB[atomicAdd(&lds[w[u] >> SUB_SHIFT], 1u)] = (unsigned)w[u];
        }
    }
    wave_sync();   // W is rewritten by the wavefront's next rows
  }
  const unsigned long long hc = c->huge_ctr;
  const unsigned nh = (unsigned)hc < P.huge_cap ? (unsigned)hc : P.huge_cap, nch = (unsigned)(hc >> 32);
  if (nh == 0) return;
  for (long long kk = blockIdx.x; kk < nch; kk += gridDim.x) {
    unsigned h;
    const unsigned first = huge_entry(P, nh, (unsigned)kk, &h);
    const int v = (int)(unsigned)P.HL[h];
    if (!vid_ok(P, v) || first > kk) continue;
    const long long b = P.rp[v], e = P.rp[v + 1];
    long long k = P.xpred[v];
    if (k < 0 || k > e - b) {
      raise_internal(P);
      k = 0;
    }
    const long long c0 = ((long long)kk - first) * HUGE_CHUNK;
    const long long c1 = c0 + HUGE_CHUNK < k ? c0 + HUGE_CHUNK : k;
    for (long long j = c0 + threadIdx.x; j < c1; j += blockDim.x) {
      const int w = P.dag[b + j];
      if (!vid_ok(P, w)) continue;
      if (!SCATTER) atomicAdd(&lds[w >> SUB_SHIFT], 1u);
      else if (direct) atomicSub(&P.D[w], 1);
      else P.SB[atomicAdd(&lds[w >> SUB_SHIFT], 1u)] = (unsigned)w;
    }
  }
}

__device__ __forceinline__ int sub_bins(const Params& P) { return (P.n + SUB_SPAN - 1) >> SUB_SHIFT; }

// Count pass: targets per bin of this block, to SUBC[block][bin].
__global__ __launch_bounds__(SUB_BS) void k_sub_count(Params P) {
  if (P.ctrl->done) return;
  __shared__ unsigned hist[SUB_MAX_BINS];
  __shared__ WaveLds wl[SUB_BS / WAVE];
  const int nb = sub_bins(P);
  for (int k = threadIdx.x; k < nb; k += blockDim.x) hist[k] = 0;
  __syncthreads();
  sub_walk<false>(P, wl[threadIdx.x / WAVE], hist, false);
  __syncthreads();
  unsigned* out = P.SUBC + (size_t)blockIdx.x * nb;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) out[k] = hist[k];
}

// Scan, first step: per bin (a thread each), each block's offset inside the
// bin, in place in SUBC, and the bin's total to SUBS[bin] (saturated at
// 2^32 - 1: the totals fit SB, whose size is below 2^32, or the targets are
// decremented at once).
__global__ __launch_bounds__(BS) void k_sub_scan_bins(Params P) {
  if (P.ctrl->done) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int nb = sub_bins(P);
  if (k >= nb) return;
  constexpr int Q = 16;   // loads in flight
  unsigned long long t = 0;
  for (int b0 = 0; b0 < SUB_BLOCKS; b0 += Q) {
    unsigned x[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) x[q] = P.SUBC[(size_t)(b0 + q) * nb + k];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      P.SUBC[(size_t)(b0 + q) * nb + k] = (unsigned)t;
      t += x[q];
    }
  }
  P.SUBS[k] = t > 0xffffffffull ? 0xffffffffu : (unsigned)t;
}

// Exclusive scan of one value per thread of a SUB_BS-thread block (v in
// LDS, replaced by its prefix; the total returned to every thread).
__device__ __forceinline__ unsigned long long sub_block_scan(unsigned long long* v) {
  __shared__ unsigned long long wt[SUB_BS / WAVE];
  const unsigned lane = lane_id(), w = threadIdx.x / WAVE;
  if (lane == 0) {
    unsigned long long a = 0;
    for (int i = 0; i < WAVE; ++i) {
      const unsigned long long x = v[w * WAVE + i];
      v[w * WAVE + i] = a;
      a += x;
    }
    wt[w] = a;
  }
  __syncthreads();
  unsigned long long before = 0, all = 0;
  for (int k = 0; k < SUB_BS / WAVE; ++k) {
    before += k < (int)w ? wt[k] : 0ull;
    all += wt[k];
  }
  v[threadIdx.x] += before;
  __syncthreads();
  return all;
}

// Scan, second step (one block): each bin's first entry in SUBS, the apply
// chunks of the bins as a prefix after them, and whether the targets fit SB.
__global__ __launch_bounds__(SUB_BS) void k_sub_scan_total(Params P) {
  Ctrl* c = P.ctrl;
  if (c->done) return;
  __shared__ unsigned long long part[SUB_BS], cpart[SUB_BS];
  constexpr int PER = SUB_MAX_BINS / SUB_BS;   // bins per thread
  const int nb = sub_bins(P);
  unsigned long long tot[PER], chk[PER], mine = 0, mch = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int k = threadIdx.x * PER + q;
    tot[q] = k < nb ? P.SUBS[k] : 0ull;
    chk[q] = (tot[q] + SUB_CHUNK - 1) / SUB_CHUNK;
    mine += tot[q];
    mch += chk[q];
  }
  part[threadIdx.x] = mine;
  cpart[threadIdx.x] = mch;
  __syncthreads();
  const unsigned long long all = sub_block_scan(part);
  const unsigned long long chunks = sub_block_scan(cpart);
  const bool fit = all <= (unsigned long long)P.sb_cap;
  unsigned long long at = part[threadIdx.x], ct = cpart[threadIdx.x];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int k = threadIdx.x * PER + q;
    if (k < nb) {
      P.SUBS[k] = (unsigned)at;
      P.SUBS[nb + 1 + k] = (unsigned)ct;
    }
    at += tot[q];
    ct += chk[q];
  }
  if (threadIdx.x == 0) {
    P.SUBS[nb] = (unsigned)all;
    P.SUBS[nb + 1 + nb] = (unsigned)chunks;
    c->sub_direct = fit ? 0 : 1;
    c->sub_chunks = fit ? (unsigned)chunks : 0u;
  }
}

// Scatter pass: every target to SB at its bin's cursor for this block.
__global__ __launch_bounds__(SUB_BS) void k_sub_scatter(Params P) {
  Ctrl* c = P.ctrl;
  if (c->done) return;
  __shared__ unsigned cur[SUB_MAX_BINS];
  __shared__ WaveLds wl[SUB_BS / WAVE];
  const int nb = sub_bins(P);
  const bool direct = c->sub_direct != 0;
  const unsigned* off = P.SUBC + (size_t)blockIdx.x * nb;
  if (!direct)
    for (int k = threadIdx.x; k < nb; k += blockDim.x) cur[k] = P.SUBS[k] + off[k];
  __syncthreads();
  sub_walk<true>(P, wl[threadIdx.x / WAVE], cur, direct);
}

// Apply pass: chunk j of the bins' targets (chunks never span two bins)
// summed per target in LDS, the sums taken off D.  The sums are 16-bit, two
// to a word: a chunk holds fewer than 2^16 targets, so a half never carries
// into the other.
static_assert(SUB_CHUNK < 65536, "16-bit sums per chunk");
__global__ __launch_bounds__(SUB_BS) void k_sub_apply(Params P) {
  Ctrl* c = P.ctrl;
  if (c->done || c->sub_direct) return;
  __shared__ unsigned cnt[SUB_SPAN / 2];
  const unsigned nch = c->sub_chunks;
  const int nb = sub_bins(P);
  const unsigned* cpre = P.SUBS + nb + 1;
  for (unsigned j = blockIdx.x; j < nch; j += gridDim.x) {
    // its bin: the last k with cpre[k] <= j
    int lo = 0, hi = nb;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (cpre[mid] <= j) lo = mid;
      else hi = mid;
    }
    const unsigned long long b0 = P.SUBS[lo] + (unsigned long long)(j - cpre[lo]) * SUB_CHUNK;
    const unsigned long long bend = P.SUBS[lo + 1];
    const unsigned long long b1 = b0 + SUB_CHUNK < bend ? b0 + SUB_CHUNK : bend;
    for (int i = threadIdx.x; i < SUB_SPAN / 2; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    const unsigned base = (unsigned)lo << SUB_SHIFT;
    for (unsigned long long i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
      const unsigned t = P.SB[i] - base;
      if (t < (unsigned)SUB_SPAN) atomicAdd(&cnt[t >> 1], 1u << ((t & 1) * 16));
      else raise_internal(P);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < SUB_SPAN / 2; i += blockDim.x) {
      const unsigned x = cnt[i];   // non-zero halves belong to targets, so to vertices below n
      if (x & 0xffffu) atomicSub(&P.D[base + 2 * i], (int)(x & 0xffffu));
      if (x >> 16) atomicSub(&P.D[base + 2 * i + 1], (int)(x >> 16));
    }
    __syncthreads();   // cnt is cleared for the next chunk
  }
}

// ---- grid-wide steps

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

__device__ __forceinline__ long long seg_begin(const Params& P, int r) { return (long long)P.n - P.roundN[r]; }
__device__ __forceinline__ long long seg_size(const Params& P, int r) {
  return (long long)P.roundN[r] - (long long)P.roundN[r + 1];
}

// The vertex at index idx of ORD.  jp_color's one pseudo-round is every
// vertex in id order, and ORD is not written for it.
__device__ __forceinline__ int ord_at(const Params& P, long long idx) {
  return P.ord_identity ? (int)idx : P.ORD[idx];
}

// Bulk step at the start of round r: the colours of every predecessor from a
// later round into the round's bitmaps.  Wavefronts take groups of G
// consecutive vertices of the round, G spreading the round evenly over the
// wavefronts (up to 64: a small round of hubs keeps every wavefront busy),
// and spread each group's entries evenly over their lanes.
// Colours 1..64 are ORed into LDS copies of the group's first two bitmap
// words, which go out with one atomic per word; a higher colour goes
// straight to the bitmap.
template <int S>
__device__ __forceinline__ void jp_xpull_items(const Params& P, WaveLds& W, int r, long long gw, long long gstride) {
  const long long b = seg_begin(P, r), sz = seg_size(P, r);
  const unsigned lane = lane_id();
  long long G = (sz + gstride - 1) / gstride;
  if (G > WAVE) G = WAVE;
  if (G < XPULL_GMIN) G = XPULL_GMIN;
  for (long long g = gw; g * G < sz; g += gstride) {
    const long long i = g * G + lane;
    const bool ok = (long long)lane < G && i < sz;
    int x = 0;
    bool mine = false;   // the lane holds a vertex
    if (ok) {
      const int v = ord_at(P, b + i);
      if (vid_ok(P, v)) {
        mine = true;
        x = P.xpred[v];   // predecessors from later rounds
        W.rec[lane] = rec_of(P, v);
        W.pb[lane] = P.rp[v];
        if (x < 0 || x > P.rp[v + 1] - W.pb[lane]) {
          raise_internal(P);
          x = 0;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < XW_WORDS; ++k) W.xw[k * WAVE + lane] = 0;
    int tot;
    W.off[lane] = wave_excl_scan<int>(x, &tot);
    if (lane == 0) W.off[WAVE] = tot;
    wave_sync();
    for (int e0 = 0; e0 < tot; e0 += WAVE * JP_UNROLL) {
      int own[JP_UNROLL], c[JP_UNROLL];
#pragma unroll
      for (int t = 0; t < JP_UNROLL; ++t) {
        const int e = e0 + t * WAVE + (int)lane;
        own[t] = -1;
        c[t] = 0;
        if (e < tot) {
          own[t] = wave_owner(W, e);
          c[t] = P.dag[W.pb[own[t]] + (e - W.off[own[t]])];
        }
      }
#pragma unroll
      for (int t = 0; t < JP_UNROLL; ++t) c[t] = own[t] >= 0 && vid_ok(P, c[t]) ? done_colour(P, c[t]) : 0;
      // colours 1..64 gather in LDS (most of them: a vertex with few
      // predecessors has one or two words); the rest go to the bitmap
#pragma unroll
      for (int t = 0; t < JP_UNROLL; ++t)
        if (own[t] >= 0) {
          const unsigned long long rec = W.rec[own[t]];
          const int cb = c[t] - 1;
          if (c[t] >= 1 && c[t] <= (int)(unsigned)rec + 2 && cb < XW_WORDS * 32)
            atomicOr(&W.xw[(cb >> 5) * WAVE + own[t]], 1u << (cb & 31));
          else
            bm_mark<S>(P, rec, c[t]);
        }
    }
    wave_sync();
    if (mine) {   // one atomic per gathered word of the lane's vertex
      const unsigned long long rec = W.rec[lane];
#pragma unroll
      for (int k = 0; k < XW_WORDS; ++k) {
        const unsigned wd = W.xw[k * WAVE + lane];
        if (wd) {
          const unsigned long long at = (rec >> 32) + (unsigned)k;   // a set bit lies below np + 2: a word of v's bitmap
          if (at < P.bm_cap) __hip_atomic_fetch_or(&P.B[at], wd, __ATOMIC_RELAXED, S);
          else raise_internal(P);
        }
      }
    }
    wave_sync();
  }
}

// Level 0 of round r as global lists: the vertices of its slot-indexed L0
// split into F and H.
__device__ __forceinline__ void jp_split_items(const Params& P, JpStage& st, int r, long long gw, long long gstride) {
  const long long b = seg_begin(P, r), sz = seg_size(P, r);
  const unsigned lane = lane_id();
  for (long long g = gw;; g += gstride) {
    if (!stage_pass(P, st, -1, g * WAVE < sz)) break;
    if (g * WAVE >= sz) continue;
    const long long i = g * WAVE + lane;
    const bool ok = i < sz;
    int v = ok ? (int)P.L0[b + i] : -1;   // -1: not in the first level
    const bool good = v >= 0 && vid_ok(P, v);
    if (!good) v = 0;
    jp_append<SC_AGENT>(P, st, -1, good, v, good ? rec_pair(P, v) : JpRec{0, 0});
  }
}

// The work items of wide level l: groups of 64 plain vertices (colour and
// successors a lane each), then the fan-out chunks (each chunk reads its
// vertex's bitmap; the one that starts the range stores the colour).
__device__ __forceinline__ void jp_level_items(const Params& P, JpStage& st, WaveLds& W, int l, unsigned nf, unsigned long long hc,
                               long long gw, long long gstride, const unsigned long long* hlds) {
  const unsigned lane = lane_id();
  const unsigned nh = (unsigned)hc;
  const unsigned nch = nh ? (unsigned)(hc >> 32) : 0;   // chunks come with their entries
  const unsigned* Fl = P.F[l & 1];
  const unsigned long long* Hl = P.H[l & 1];
  const long long groups = ((long long)nf + WAVE - 1) / WAVE;
  for (long long it = gw; it < groups + (long long)nch; it += gstride) {
    if (it < groups) {
      const long long idx = it * WAVE + lane;
      int v = idx < nf ? (int)ld32<SC_AGENT>(&Fl[idx]) : 0;
      const bool act = idx < nf && vid_ok(P, v);
      if (!act) v = 0;
      unsigned long long rec = 0;
      long long s0 = 0, s1 = 0;
      if (act) {
        const JpRec pr = rec_pair(P, v);
        rec = pr.rec;
        s0 = sp_first(pr.sp);
        s1 = s0 + sp_count(P, v, pr.sp);
        if (!range_ok(P, s0, s1)) s1 = s0;
      }
      // The group's successors (at most JP_SMALL per vertex) spread over
      // the lanes: fetched, with their JP records, while GetColor reads
      // the bitmap words, then pushed all at once.
      int stot;
      const int spre = wave_excl_scan<int>((int)(s1 - s0), &stot);
      if (stot > JP_SMALL * WAVE) {   // plain vertices have at most JP_SMALL: a broken state
        raise_internal(P);
        stot = JP_SMALL * WAVE;
      }
      W.soff[lane] = spre;
      W.pb[lane] = s0;
      if (lane == 0) W.soff[WAVE] = stot;
      wave_sync();
      int u[JP_SMALL], own[JP_SMALL];
      bool ok[JP_SMALL];
      JpRec rc[JP_SMALL];
#pragma unroll
      for (int t = 0; t < JP_SMALL; ++t) {
        const int e = t * WAVE + (int)lane;
        ok[t] = e < stot;
        own[t] = 0;
        u[t] = 0;
        if (ok[t]) {
          own[t] = wave_owner_of(W.soff, e);
          u[t] = P.dag[W.pb[own[t]] + (e - W.soff[own[t]])];
        }
        ok[t] = ok[t] && vid_ok(P, u[t]);
      }
#pragma unroll
      for (int t = 0; t < JP_SMALL; ++t) rc[t] = ok[t] ? rec_pair(P, u[t]) : JpRec{0, 0};
      const int col = wave_colour(P, W, act, rec);
      if (act) sti<SC_AGENT>(&P.color[v], col);
      W.ffree[lane] = col;
      wave_sync();
      bool rdy[JP_SMALL];
#pragma unroll
      for (int t = 0; t < JP_SMALL; ++t) rdy[t] = ok[t] && jp_push<SC_AGENT>(P, u[t], rc[t].rec, W.ffree[own[t]]);
#pragma unroll
      for (int t = 0; t < JP_SMALL; ++t) jp_append<SC_AGENT>(P, st, l, rdy[t], u[t], rc[t]);
      wave_sync();   // W is rewritten by the wavefront's next item
    } else {
      const unsigned k = (unsigned)(it - groups);
      const unsigned long long ent = fan_entry<SC_AGENT>(Hl, nh, k, hlds);
      const int v = (int)(unsigned)ent;
      const unsigned first = (unsigned)(ent >> 32);
      if (!vid_ok(P, v) || first > k) {
        raise_internal(P);
        continue;
      }
      const JpRec pr = rec_pair(P, v);
      const unsigned long long rec = pr.rec;
      // the chunk's successors (one wavefront step) are fetched together
      // with the bitmap words
      const long long b = sp_first(pr.sp), e = b + sp_count(P, v, pr.sp);
      const long long s0 = b + (long long)(k - first) * JP_CHUNK;
      long long s1 = s0 + JP_CHUNK < e ? s0 + JP_CHUNK : e;
      if (!range_ok(P, s0, s1)) s1 = s0;
      int u[JP_CU];
      bool ok[JP_CU];
#pragma unroll
      for (int t = 0; t < JP_CU; ++t) {
        const long long j = s0 + t * WAVE + lane;
        ok[t] = j < s1;
        u[t] = ok[t] ? P.dag[j] : 0;
        ok[t] = ok[t] && vid_ok(P, u[t]);
      }
      // the whole wavefront reads v's bitmap: first clear bit
      const unsigned nw = bm_words((int)(unsigned)rec);
      int col = 0;
      for (unsigned w0 = 0; w0 < nw && !col; w0 += WAVE) {
        const unsigned w = w0 + lane;
        const unsigned wd = w < nw ? bm_load(P, (rec >> 32) + w) : ~0u;
        const int f = wave_min(~wd ? (int)(w * 32) + __ffs((int)~wd) - 1 : 0x7fffffff);
        if (f != 0x7fffffff) col = f + 1;
      }
      if (!col) {
        if (lane == 0) atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
        col = (int)(unsigned)rec + 1;
      }
      if (k == first && lane == 0) sti<SC_AGENT>(&P.color[v], col);
      JpRec rc[JP_CU];
#pragma unroll
      for (int t = 0; t < JP_CU; ++t) rc[t] = ok[t] ? rec_pair(P, u[t]) : JpRec{0, 0};
      bool rdy[JP_CU];
#pragma unroll
      for (int t = 0; t < JP_CU; ++t) rdy[t] = ok[t] && jp_push<SC_AGENT>(P, u[t], rc[t].rec, col);
#pragma unroll
      for (int t = 0; t < JP_CU; ++t) jp_append<SC_AGENT>(P, st, l, rdy[t], u[t], rc[t]);
    }
  }
}

// ---- relaxation of a deep round
//
// Colouring a round level by level costs one step per level, and the rounds
// at the top of a power-law graph hold long same-round chains (thousands of
// levels).  Their JP colours are also the unique solution of the system
//   c(v) = smallest colour neither in v's bitmap nor taken by a same-round
//          predecessor of v,
// because the same-round DAG is acyclic: going down the DAG, each equation
// fixes one colour from colours already fixed.  Repeating the equations from
// any start reaches that solution, and stops changing, in at most (longest
// chain + 1) sweeps; on these rounds it stops far sooner than the chain is
// long.  So once a round has run RELAX_AFTER levels, its uncoloured vertices
// are relaxed instead: step 0 lists them (a colour of 0: JP start clears the
// colours); step t >= 1 recomputes every vertex of its list and, where the
// colour changed, lists the same-round successors for step t + 1, each once
// (the first to raise the successor's mark to step t + 1's stamp lists it).
// The round ends with an empty list.  The vertices JP already coloured keep
// their colours: all their predecessors were coloured before them, so their
// equations hold already, and their colours are in the bitmaps of their
// successors, as the equations want.  Colours are read while other
// wavefronts may rewrite them, but every change lists its successors for the
// next step, so whatever a vertex last read was final once the lists run dry.

// A large relaxed round of a large graph works on positions in the round
// (its slice of ORD) instead of vertex ids: colours in rcol and marks in
// rmark, both indexed by position, stay small enough for the caches, where
// the colour and mark of a vertex id are scattered over arrays of n entries
// (a small round's scattered lines fit the caches anyway, and a graph of a
// few million vertices keeps its arrays in the Infinity Cache: there the
// rewrite below costs more than it saves).  Step 0 stores each
// vertex's position in cnt (free once the round's levels have stopped) and
// its colour in rcol.  In step 1 every listed vertex replaces the vertex ids
// of its own same-round predecessors and successors in the DAG by their
// positions (cnt), as it reads them: step 1 lists every uncoloured vertex,
// and each of them changes colour (from 0), so it reads both ranges.  Later
// steps read positions.  A colour that changes is stored in rcol and in the
// colour array (which nothing reads before the round ends).  Marks from an
// earlier round's positions hold older stamps, so they never look current.
// The DAG is no longer read-only here, and a later step may run on another
// XCD, whose L2 can still hold a line from before step 1: so step 1 always
// ends a launch (a grid step does anyway; the steps launch ends after it),
// and the launch boundary makes the new entries visible to plain loads.

// A position read from a list or the DAG: below the round's size (in a
// round relaxed by vertex id: below n).
__device__ __forceinline__ bool pos_ok(const Params& P, int p, unsigned sz) {
  if ((unsigned)p < sz) return true;
  raise_internal(P);
  return false;
}

// How round r is relaxed: by position (compact) or by vertex id.
struct RelaxIdx {
  bool compact;
  long long b;        // the round's first index in ORD
  unsigned lim;       // bound of the list entries and DAG values: round size, or n
  int* cols;          // colours by list entry: rcol, or the colour array
};
__device__ __forceinline__ RelaxIdx relax_idx(const Params& P, int r) {
  RelaxIdx x;
  const long long sz = seg_size(P, r);
  x.compact = sz >= RELAX_COMPACT_MIN && (long long)P.n >= RELAX_COMPACT_N;
  x.b = seg_begin(P, r);
  x.lim = x.compact ? (unsigned)sz : (unsigned)P.n;
  x.cols = x.compact ? P.rcol : P.color;
  return x;
}

// Step 0: the uncoloured vertices of the round (lane per vertex) go into
// list 1; by position, every vertex of the round gets its position (cnt)
// and colour (rcol).
__device__ __forceinline__ void jp_relax_list(const Params& P, JpStage& st, int r, long long gw, long long gstride) {
  const long long b = seg_begin(P, r), sz = seg_size(P, r);
  const bool compact = relax_idx(P, r).compact;
  const unsigned lane = lane_id();
  for (long long g = gw;; g += gstride) {
    if (!stage_pass(P, st, 0, g * WAVE < sz)) break;
    if (g * WAVE >= sz) continue;
    const long long i = g * WAVE + lane;
    int v = i < sz ? ord_at(P, b + i) : -1;
    const bool ok = v >= 0 && vid_ok(P, v);
    int c = 0;
    if (ok) {
      c = done_colour(P, v);
      if (compact) {
        sti<SC_AGENT>(&P.cnt[v], (int)i);
        sti<SC_AGENT>(&P.rcol[i], c);
      }
    }
    const bool open = ok && c == 0;
    jp_append<SC_AGENT>(P, st, 0, open, open ? (compact ? (int)i : v) : 0, JpRec{0, 0});
  }
}

// RELAX_UNROLL same-round neighbours u[k] read from dag[j[k]] (-1: none):
// in step 1 (tr) vertex ids, turned into positions and written back.
__device__ __forceinline__ void relax_translate(const Params& P, int (&u)[RELAX_UNROLL], const long long (&j)[RELAX_UNROLL]) {
#pragma unroll
  for (int k = 0; k < RELAX_UNROLL; ++k) u[k] = u[k] >= 0 && vid_ok(P, u[k]) ? ldi<SC_AGENT>(&P.cnt[u[k]]) : -1;
#pragma unroll
  for (int k = 0; k < RELAX_UNROLL; ++k)
    if (j[k] >= 0) P.dag[j[k]] = u[k];
}

// The colour equation of one vertex v (bitmap rec, np predecessors, the
// same-round ones at dag[p0, s0)), solved by the whole wavefront: windows of
// 2048 colours, each filled from v's bitmap words and then from the current
// colours of its same-round predecessors, until one has a clear bit.  (In
// step 1 the first window translates the range; a lane reads back in later
// windows what it wrote itself.)
__device__ __forceinline__ int relax_wave(const Params& P, WaveLds& W, unsigned long long rec, int np, long long p0,
                                          long long s0, bool tr, const RelaxIdx& X) {
  const unsigned lane = lane_id();
  unsigned* bits = (unsigned*)W.ffree;
  const unsigned nw = bm_words(np);
  const unsigned long long bo = rec >> 32;
  int col = 0;
  for (unsigned w0 = 0; w0 < nw && !col; w0 += WAVE) {
    bits[lane] = w0 + lane < nw ? bm_load(P, bo + w0 + lane) : ~0u;
    wave_sync();
    const int lo = (int)(w0 * 32);
    for (long long j0 = p0; j0 < s0; j0 += WAVE * RELAX_UNROLL) {
      int u[RELAX_UNROLL];
      long long jj[RELAX_UNROLL];
#pragma unroll
      for (int k = 0; k < RELAX_UNROLL; ++k) {
        const long long j = j0 + k * WAVE + lane;
        jj[k] = j < s0 ? j : -1;
        u[k] = j < s0 ? P.dag[j] : -1;
      }
      if (tr && w0 == 0) relax_translate(P, u, jj);
#pragma unroll
      for (int k = 0; k < RELAX_UNROLL; ++k) u[k] = u[k] >= 0 && pos_ok(P, u[k], X.lim) ? agent_load_i32(&X.cols[u[k]]) : 0;
#pragma unroll
      for (int k = 0; k < RELAX_UNROLL; ++k) {
        const int bit = u[k] - 1 - lo;   // colours outside 1 .. np+2 cannot be v's
        if (u[k] >= 1 && u[k] <= np + 2 && bit >= 0 && bit < WAVE * 32) atomicOr(&bits[bit >> 5], 1u << (bit & 31));
      }
    }
    wave_sync();
    const unsigned wd = bits[lane];
    const int f = wave_min(~wd ? (int)(w0 + lane) * 32 + __ffs((int)~wd) - 1 : 0x7fffffff);
    if (f != 0x7fffffff) col = f + 1;
    wave_sync();   // the window is rewritten by the next pass
  }
  if (!col) {   // unreachable: at most np of the np+2 colours are taken
    if (lane == 0) raise_internal(P);
    col = np + 1;
  }
  return col;
}

// Marks and list entries for RELAX_UNROLL same-round successors w[k]
// (positions, or vertex ids in a round relaxed by id; -1: none) of a vertex
// whose colour changed: each is listed for
// the next step unless a mark at its stamp says it already is (most are:
// listed by another changed predecessor).  A plain read of the mark, which
// can only lag behind, spares most of the atomics.
__device__ __forceinline__ void relax_mark(const Params& P, JpStage& ast, int t, unsigned stamp, unsigned lim,
                                           const int (&w)[RELAX_UNROLL]) {
  bool mk[RELAX_UNROLL];
#pragma unroll
  for (int k = 0; k < RELAX_UNROLL; ++k) mk[k] = w[k] >= 0 && pos_ok(P, w[k], lim) && P.rmark[w[k]] < stamp;
#pragma unroll
  for (int k = 0; k < RELAX_UNROLL; ++k)
    mk[k] = mk[k] && __hip_atomic_fetch_max(&P.rmark[w[k]], stamp, __ATOMIC_RELAXED, SC_AGENT) < stamp;
#pragma unroll
  for (int k = 0; k < RELAX_UNROLL; ++k) jp_append<SC_AGENT>(P, ast, t, mk[k], mk[k] ? w[k] : 0, JpRec{0, 0});
}

// The same-round successors [s0, s1) of a vertex whose colour changed, by
// the whole wavefront, RELAX_UNROLL widths at a time (translated in step 1).
__device__ __forceinline__ void relax_push_wave(const Params& P, JpStage& ast, int t, unsigned stamp, long long s0,
                                                long long s1, bool tr, unsigned lim) {
  const unsigned lane = lane_id();
  for (long long j0 = s0; j0 < s1; j0 += WAVE * RELAX_UNROLL) {
    int w[RELAX_UNROLL];
    long long jj[RELAX_UNROLL];
#pragma unroll
    for (int k = 0; k < RELAX_UNROLL; ++k) {
      const long long j = j0 + k * WAVE + lane;
      jj[k] = j < s1 ? j : -1;
      w[k] = j < s1 ? P.dag[j] : -1;
    }
    if (tr) relax_translate(P, w, jj);
    relax_mark(P, ast, t, stamp, lim, w);
  }
}

// Step t >= 1 of round r over its list of nl entries (positions, or vertex
// ids: relax_idx).  A list no longer than 2 gstride goes a wavefront per
// vertex (relax_wave, relax_push_wave).  Longer lists go G entries per
// wavefront, G spreading the list evenly over the wavefronts (up to 64),
// with lb the wavefront's LDS area of 64 x RELAX_LW words: a light vertex
// (at most RELAX_LK same-round predecessors and successors, at most
// RELAX_LW bitmap words) gets its colour from its lane's own words of lb
// (word w of lane k at lb[64 w + k]), the group's entries spread over the
// lanes; the others are solved by the whole wavefront, one after the other.
__device__ __forceinline__ void jp_relax_items(const Params& P, JpStage& st, WaveLds& W, unsigned* lb, int t, unsigned nl,
                                               unsigned stamp, long long gw, long long gstride, int r) {
  const unsigned lane = lane_id();
  const unsigned* Lin = P.F[t & 1];
  const RelaxIdx X = relax_idx(P, r);
  const bool tr = X.compact && t == 1;
  JpStage ast = st;
  ast.acc = nullptr;   // a relaxation list keeps no work sums
  if (!lb || (long long)nl <= 2 * gstride) {
    for (long long i = gw; i < (long long)nl; i += gstride) {
      const int p = __builtin_amdgcn_readfirstlane((int)ld32<SC_AGENT>(&Lin[i]));
      if (!pos_ok(P, p, X.lim)) continue;
      const int v = X.compact ? __builtin_amdgcn_readfirstlane(ord_at(P, X.b + p)) : p;
      if (!vid_ok(P, v)) continue;
      const JpRec pr = rec_pair(P, v);
      const int old = __builtin_amdgcn_readfirstlane(agent_load_i32(&X.cols[p]));
      const int np = (int)(unsigned)pr.rec;
      const long long s0 = sp_first(pr.sp);
      const long long s1 = s0 + sp_count(P, v, pr.sp);
      const long long p0 = s0 - (np - P.xpred[v]);   // same-round predecessors: [p0, s0)
      if (!range_ok(P, p0, s0) || !range_ok(P, s0, s1)) continue;
      const int col = relax_wave(P, W, pr.rec, np, p0, s0, tr, X);
      if (col == old) continue;   // (never in step 1: every listed colour is 0)
      if (lane == 0) {
        sti<SC_AGENT>(&X.cols[p], col);
        if (X.compact) sti<SC_AGENT>(&P.color[v], col);
      }
      relax_push_wave(P, ast, t, stamp, s0, s1, tr, X.lim);
    }
    return;
  }
  long long G = ((long long)nl + gstride - 1) / gstride;
  if (G > WAVE) G = WAVE;
  for (long long g = gw; g * G < (long long)nl; g += gstride) {
    const long long i = g * G + lane;
    const int p = lane < G && i < (long long)nl ? (int)ld32<SC_AGENT>(&Lin[i]) : -1;
    bool act = p >= 0 && pos_ok(P, p, X.lim);
    int v = -1;
    if (act) {
      v = X.compact ? ord_at(P, X.b + p) : p;
      act = vid_ok(P, v);
    }
    JpRec pr{0, 0};
    long long p0 = 0, s0 = 0, s1 = 0;
    int np = 0, old = 0;
    if (act) {
      pr = rec_pair(P, v);
      old = agent_load_i32(&X.cols[p]);
      np = (int)(unsigned)pr.rec;
      s0 = sp_first(pr.sp);
      s1 = s0 + sp_count(P, v, pr.sp);
      p0 = s0 - (np - P.xpred[v]);
      act = range_ok(P, p0, s0) && range_ok(P, s0, s1);
    }
    const int nw = act ? (int)bm_words(np) : 0;
    const bool lite = act && s0 - p0 <= RELAX_LK && s1 - s0 <= RELAX_LK && nw <= RELAX_LW;
    // light vertices: a vertex's words of lb belong to its lane; the
    // group's predecessor entries (then its successor entries) are spread
    // evenly over the lanes (a prefix sum of the counts and a search for
    // the owner), so that a lane with many entries does not hold the others
#pragma unroll
    for (int w = 0; w < RELAX_LW; ++w)
      lb[w * WAVE + lane] = lite && w < nw ? bm_load(P, (pr.rec >> 32) + (unsigned)w) : ~0u;
    {
      int tot;
      W.off[lane] = wave_excl_scan<int>(lite ? (int)(s0 - p0) : 0, &tot);
      if (lane == 0) W.off[WAVE] = tot;
      W.pb[lane] = p0;
      W.rec[lane] = (unsigned long long)(unsigned)np;
      wave_sync();
      for (int e0 = 0; e0 < tot; e0 += WAVE * RELAX_UNROLL) {
        int u[RELAX_UNROLL], own[RELAX_UNROLL];
        long long jj[RELAX_UNROLL];
#pragma unroll
        for (int k = 0; k < RELAX_UNROLL; ++k) {
          const int e = e0 + k * WAVE + (int)lane;
          own[k] = e < tot ? wave_owner(W, e) : -1;
          jj[k] = own[k] >= 0 ? W.pb[own[k]] + (e - W.off[own[k]]) : -1;
          u[k] = own[k] >= 0 ? P.dag[jj[k]] : -1;
        }
        if (tr) relax_translate(P, u, jj);
#pragma unroll
        for (int k = 0; k < RELAX_UNROLL; ++k) u[k] = u[k] >= 0 && pos_ok(P, u[k], X.lim) ? agent_load_i32(&X.cols[u[k]]) : 0;
#pragma unroll
        for (int k = 0; k < RELAX_UNROLL; ++k)
          if (u[k] >= 1 && u[k] <= (int)W.rec[own[k]] + 2)
            atomicOr(&lb[((u[k] - 1) >> 5) * WAVE + own[k]], 1u << ((u[k] - 1) & 31));
      }
      wave_sync();
    }
    int col = 0;
    if (lite) {
#pragma unroll
      for (int w = RELAX_LW - 1; w >= 0; --w) {
        const unsigned x = lb[w * WAVE + lane];
        if (w < nw && ~x) col = w * 32 + __ffs((int)~x);
      }
      if (!col) {   // unreachable: at most np of the np+2 colours are taken
        raise_internal(P);
        col = np + 1;
      }
    }
    const bool lchanged = lite && col != old;
    if (lchanged) {
      sti<SC_AGENT>(&X.cols[p], col);
      if (X.compact) sti<SC_AGENT>(&P.color[v], col);
    }
    {
      int tot;
      W.off[lane] = wave_excl_scan<int>(lchanged ? (int)(s1 - s0) : 0, &tot);
      if (lane == 0) W.off[WAVE] = tot;
      W.pb[lane] = s0;
      wave_sync();
      for (int e0 = 0; e0 < tot; e0 += WAVE * RELAX_UNROLL) {
        int w[RELAX_UNROLL];
        long long jj[RELAX_UNROLL];
#pragma unroll
        for (int k = 0; k < RELAX_UNROLL; ++k) {
          const int e = e0 + k * WAVE + (int)lane;
          const int own = e < tot ? wave_owner(W, e) : -1;
          jj[k] = own >= 0 ? W.pb[own] + (e - W.off[own]) : -1;
          w[k] = own >= 0 ? P.dag[jj[k]] : -1;
        }
        if (tr) relax_translate(P, w, jj);
        relax_mark(P, ast, t, stamp, X.lim, w);
      }
      wave_sync();   // W is rewritten below
    }
    // the others: the whole wavefront, one after the other
    for (uint64_t m = ballot(act && !lite); m; m &= m - 1) {
      const int src = __ffsll((long long)m) - 1;
      const long long hs0 = readlane_i64(s0, src), hs1 = readlane_i64(s1, src);
      const int c = relax_wave(P, W, readlane_u64(pr.rec, src), readlane_i(np, src), readlane_i64(p0, src), hs0, tr, X);
      if (c == readlane_i(old, src)) continue;
      if (lane == 0) {
        sti<SC_AGENT>(&X.cols[readlane_i(p, src)], c);
        if (X.compact) sti<SC_AGENT>(&P.color[readlane_i(v, src)], c);
      }
      relax_push_wave(P, ast, t, stamp, hs0, hs1, tr, X.lim);
    }
  }
}

// ---- the core mode of a small, dense round
//
// A round whose levels colour a vertex or two each (the near-cliques at the
// top of a power-law graph's order) costs a level per vertex: the ready
// vertex's bitmap, the push to its hundreds of successors, the next level,
// each a dependent round trip.  Such a round of at most CORE_MAX vertices is
// finished by one block instead: it lists the round's uncoloured vertices,
// sorts them by JP's priority inside the round (largest first) and colours
// them one after the other, each with the smallest colour in neither its
// bitmap nor the colours of its same-round predecessors (read back from
// the colour array).  Every predecessor comes earlier in that order (or was
// coloured by a level before, and its colour is in the bitmap too), so this
// is JP's colouring: the greedy colouring in priority order.
struct CoreLds {
  unsigned long long key[CORE_MAX];   // sort keys (then scratch of the compaction)
  int id[CORE_MAX];                   // the round's uncoloured vertices, in JP's order
  int col[CORE_MAX];                  // their colours, by position
  unsigned bits[3][WAVE];             // 2048-colour windows: step t fills [t % 3], sets up [(t + 1) % 3]
  unsigned long long rec[4];          // ring of the next vertices' JP records
  long long p0[4], s0[4];             // and of their same-round predecessors: dag[p0, s0)
  unsigned cnt;                       // listed vertices
};
constexpr int CORE_PF = CORE_MAX / NARROW_BS;   // predecessors a thread takes per vertex (a round has < CORE_MAX)

// JP's order inside the round (larger first): rho_R (after D at selection for
// ADG-O); jp_color's one pseudo-round orders by <given rank, rho_R>.
__device__ __forceinline__ unsigned long long core_key(const Params& P, int v) {
  return P.ord_identity ? (unsigned long long)prio(P, v) : same_key(P, v);
}

// Thread 0: the JP record of the vertex at position t into ring slot t % 4.
__device__ __forceinline__ void core_rec(const Params& P, CoreLds& K, unsigned t, unsigned m, unsigned long long rec,
                                         unsigned long long sp, int xp, int v) {
  if (t >= m) return;
  const int np = (int)(unsigned)rec;
  const long long s0 = sp_first(sp);
  long long p0 = s0 - (np - xp);
  if (!range_ok(P, p0, s0)) p0 = s0;
  K.rec[t & 3] = rec;
  K.p0[t & 3] = p0;
  K.s0[t & 3] = s0;
  (void)v;
}

// Block-wide (NARROW_BS threads): colour the uncoloured vertices of round r
// (at most CORE_MAX).  The vertices are listed and sorted; cnt[v] of each
// becomes -(position + 1), which tells a predecessor's position from its id
// (cnt is not read again in a round finished this way).  Then one vertex at
// a time, in order, with the block's loads running ahead: the record of the
// vertex four places on, the predecessor ids of the one two places on, and
// the predecessors' positions and first 64 bitmap words of the next one, so
// that a vertex's own step only reads LDS: its window of colours (set up in
// the step before) and the colours of its predecessors by position.
__device__ __forceinline__ void jp_core_round(const Params& P, CoreLds& K, int r) {
  const long long b = seg_begin(P, r), rs = seg_size(P, r);
  const unsigned tid = threadIdx.x;
  if (tid == 0) K.cnt = 0;
  __syncthreads();
  for (long long i = tid; i < rs; i += blockDim.x) {
    const int v = ord_at(P, b + i);
    if (vid_ok(P, v) && done_colour(P, v) == 0) {
      const unsigned at = atomicAdd(&K.cnt, 1u);
      if (at < (unsigned)CORE_MAX) {
        K.id[at] = v;
        K.key[at] = core_key(P, v);
      }
    }
  }
  __syncthreads();
  unsigned m = K.cnt;
  if (m > (unsigned)CORE_MAX) {   // the round was checked to fit: a broken state
    if (tid == 0) raise_internal(P);
    m = CORE_MAX;
  }
  if (m == 0) return;   // (uniform: every thread read cnt after the barrier)
  unsigned M = 1;
  while (M < m) M <<= 1;
  for (unsigned i = m + tid; i < M; i += blockDim.x) {
    K.id[i] = -1;
    K.key[i] = 0;
  }
  __syncthreads();
  // bitonic sort, largest key first
  for (unsigned k = 2; k <= M; k <<= 1)
    for (unsigned j = k >> 1; j > 0; j >>= 1) {
      for (unsigned i = tid; i < M; i += blockDim.x) {
        const unsigned o = i ^ j;
        if (o > i) {
          const unsigned long long a = K.key[i], c = K.key[o];
          if ((i & k) == 0 ? a < c : a > c) {
            K.key[i] = c;
            K.key[o] = a;
            const int x = K.id[i];
            K.id[i] = K.id[o];
            K.id[o] = x;
          }
        }
      }
      __syncthreads();
    }
  // drop the padding (it sorted among the smallest keys), keeping the order
  {
    int* tmp = (int*)K.key;
    constexpr int Q = CORE_MAX / NARROW_BS;
    int x[Q], kept = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const unsigned i = tid * Q + q;
      x[q] = i < M ? K.id[i] : -1;
      kept += x[q] >= 0;
    }
    int tot;
    const int pre = wave_excl_scan<int>(kept, &tot);
    __shared__ int wsum[NARROW_BS / WAVE];
    if (lane_id() == 0) wsum[tid / WAVE] = tot;
    __syncthreads();
    int at = pre;
    for (unsigned w = 0; w < tid / WAVE; ++w) at += wsum[w];
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (x[q] >= 0) tmp[at++] = x[q];
    __syncthreads();
    for (unsigned i = tid; i < m; i += blockDim.x) {
      const int v = tmp[i];
      K.id[i] = v;
      sti<SC_AGENT>(&P.cnt[v], -(int)i - 1);   // its position, for its successors
    }
    order_point();
    __syncthreads();
  }
  // prologue: records of positions 0..2, predecessor ids of 0 and 1, positions of 0's
  if (tid < 4) {   // every ring slot starts as an empty range
    K.rec[tid] = 0;
    K.p0[tid] = 0;
    K.s0[tid] = 0;
  }
  __syncthreads();
  if (tid == 0)
    for (unsigned t = 0; t < 3 && t < m; ++t) {
      const int v = K.id[t];
      const JpRec pr = rec_pair(P, v);
      core_rec(P, K, t, m, pr.rec, pr.sp, P.xpred[v], v);
    }
  __syncthreads();
  // The loads of the loop are straight-line code: an index out of range is
  // replaced by a valid one and the value dropped afterwards (a branch
  // around a load makes the compiler wait for every load in flight, also
  // those issued for the steps ahead).  An id out of range is remembered and
  // raised once, after the loop.
  bool bad = false;
  const unsigned long long bm_last = P.bm_cap ? P.bm_cap - 1 : 0;
  auto load_ids = [&](unsigned t, int* ids) {
    const bool live = t < m;
    long long p0 = K.p0[t & 3], s0 = K.s0[t & 3];
    const bool okr = p0 >= 0 && p0 <= s0 && s0 <= P.nnz;   // core_rec checked it
    bad |= live && !okr;
    if (!live || !okr) p0 = s0 = 0;
#pragma unroll
    for (int q = 0; q < CORE_PF; ++q) {
      const long long j = p0 + tid + (long long)q * NARROW_BS;
      const bool in = j < s0;
      const int x = P.dag[in ? j : 0];   // the round has edges: dag[0] exists
      ids[q] = in ? x : -1;
    }
  };
  auto load_pos = [&](const int* ids, int* pos) {
#pragma unroll
    for (int q = 0; q < CORE_PF; ++q) {
      const bool okv = (unsigned)ids[q] < (unsigned)P.n;
      bad |= ids[q] < -1 || ids[q] >= P.n;
      const int x = ldi<SC_AGENT>(&P.cnt[okv ? ids[q] : 0]);
      pos[q] = okv ? x : 0;
    }
  };
  // the first 64 bitmap words of position t, a word per lane of wavefront 0
  auto load_bw = [&](unsigned t) -> unsigned {
    const unsigned long long rec = K.rec[t & 3];
    const unsigned nw = t < m ? bm_words((int)(unsigned)rec) : 0;
    const bool win = tid < (unsigned)WAVE && tid < nw;
    unsigned long long at = (rec >> 32) + (win ? tid : 0);
    at = at <= bm_last ? at : bm_last;
    const unsigned x = agent_load_u32(&P.B[at]);
    return win ? x : ~0u;
  };
  // the JP record of position t (all threads load it; thread 0 files it)
  auto load_rec = [&](unsigned t, unsigned long long& rec, unsigned long long& sp, int& xp) {
    const int v = K.id[t < m ? t : m - 1];
    const JpRec pr = rec_pair(P, v);
    rec = pr.rec;
    sp = pr.sp;
    xp = P.xpred[v];
  };
  // the first clear bit of the window w (wavefront 0): its colour, 0 if none
  auto first_clear = [&](const unsigned* w, unsigned w0) -> int {
    const unsigned wd = w[tid];
    const uint64_t fm = ballot(~wd != 0u);
    if (!fm) return 0;
    const int f = __ffsll((long long)fm) - 1;
    const unsigned wf = (unsigned)__builtin_amdgcn_readlane((int)wd, f);
    return (int)(w0 + (unsigned)f) * 32 + __ffs((int)~wf);
  };
  // Step t, two barriers.  Before the first, every thread ORs the colours of
  // vertex t's same-round predecessors into its window (set up in the step
  // before).  Between them, wavefront 0 takes the first clear bit as t's
  // colour and sets up the window of t + 1.  A colour past the window
  // (rare) is found after the second, by everyone.
  // In: ids(t+1) and pos(t), loaded in the step before, bw(t+1) likewise,
  // and the record of t+3.  Out, in the other register set: ids(t+2),
  // pos(t+1), bw(t+2), the record of t+4.  The loop runs two steps per
  // iteration with the sets' roles swapped, so that no register holding a
  // load in flight is copied (a copy would wait for the load).
  auto step = [&](unsigned t, const int* ids_c, int* ids_n, const int* pos_c, int* pos_n, unsigned bw_c,
                  unsigned& bw_n, unsigned long long rec_f, unsigned long long sp_f, int xp_f,
                  unsigned long long& rec_l, unsigned long long& sp_l, int& xp_l) {
    load_rec(t + 4, rec_l, sp_l, xp_l);
    load_ids(t + 2, ids_n);
    load_pos(ids_c, pos_n);
    bw_n = load_bw(t + 2);
    const unsigned long long rec = K.rec[t & 3];
    const int np = (int)(unsigned)rec;
    const unsigned nw = bm_words(np);
    unsigned* win = K.bits[t % 3];
#pragma unroll
    for (int q = 0; q < CORE_PF; ++q)
      if (pos_c[q] < 0) {
        const unsigned p = (unsigned)(-pos_c[q] - 1);
        const int c = p < t ? K.col[p] : 0;   // a predecessor comes earlier
        if (c >= 1 && c <= np + 2 && c <= WAVE * 32) atomicOr(&win[(c - 1) >> 5], 1u << ((c - 1) & 31));
      }
    // the ring slot of t + 3 (its record was loaded in the step before);
    // the barriers below publish it before the next step reads it
    if (tid == 0) core_rec(P, K, t + 3, m, rec_f, sp_f, xp_f, 0);
    __syncthreads();
    if (tid < (unsigned)WAVE) {
      const int col = first_clear(win, 0);
      if (tid == 0) K.col[t] = col;   // 0: past the window, found below
      K.bits[(t + 1) % 3][tid] = bw_c;
    }
    __syncthreads();
    if (K.col[t] == 0) {   // (uniform) past the first 2048 colours: the next windows, their words read now
      unsigned* sw = K.bits[(t + 2) % 3];   // free until the next step sets it up
      int col = 0;
      for (unsigned w0 = WAVE; !col && w0 < nw; w0 += WAVE) {
        if (tid < (unsigned)WAVE) sw[tid] = w0 + tid < nw ? bm_load(P, (rec >> 32) + w0 + tid) : ~0u;
        __syncthreads();
        const int lo = (int)(w0 * 32);
#pragma unroll
        for (int q = 0; q < CORE_PF; ++q)
          if (pos_c[q] < 0) {
            const unsigned p = (unsigned)(-pos_c[q] - 1);
            const int c = p < t ? K.col[p] : 0;
            const int bit = c - 1 - lo;
            if (c >= 1 && c <= np + 2 && bit >= 0 && bit < WAVE * 32) atomicOr(&sw[bit >> 5], 1u << (bit & 31));
          }
        __syncthreads();
        if (tid < (unsigned)WAVE) {
          const int cf = first_clear(sw, w0);
          if (tid == 0) K.col[t] = cf;
        }
        __syncthreads();
        col = K.col[t];
        __syncthreads();   // sw is rewritten by the next window
      }
      if (!col) {   // unreachable: at most np of the np+2 colours are taken
        if (tid == 0) {
          raise_internal(P);
          K.col[t] = np + 1;
        }
        __syncthreads();
      }
    }
  };
  int idsA[CORE_PF], idsB[CORE_PF], posA[CORE_PF], posB[CORE_PF];
  unsigned bwA, bwB = ~0u;
  unsigned long long recA, spA, recB = 0, spB = 0;
  int xpA, xpB = 0;
  {   // set A for step 0: ids(1), pos(0), bw(1), the record of 3; the window of 0
    int ids0[CORE_PF];
    load_ids(0, ids0);
    load_pos(ids0, posA);
    load_ids(1, idsA);
    const unsigned b0 = load_bw(0);
    bwA = load_bw(1);
    load_rec(3, recA, spA, xpA);
    if (tid < (unsigned)WAVE) K.bits[0][tid] = b0;
    __syncthreads();
  }
  for (unsigned t = 0; t < m; t += 2) {
    step(t, idsA, idsB, posA, posB, bwA, bwB, recA, spA, xpA, recB, spB, xpB);
    if (t + 1 < m) step(t + 1, idsB, idsA, posB, posA, bwB, bwA, recB, spB, xpB, recA, spA, xpA);
  }
  if (bad) raise_internal(P);
  __syncthreads();
  // the colours, written once the round is done (nothing reads a colour of
  // this round meanwhile: same-round predecessors are read back from LDS)
  for (unsigned i = tid; i < m; i += blockDim.x) sti<SC_AGENT>(&P.color[K.id[i]], K.col[i]);
  order_point();
  __syncthreads();
}

// ---- JP state machine (plain accesses: the state is in LDS while the
// single-block kernel runs, in the control block between kernels)

__device__ __forceinline__ void jp_clear_level(JpState& j, int idx) {
  j.fcnt[idx] = 0;
  j.hctr[idx] = 0;
  j.psum[idx] = 0;
  j.ssum[idx] = 0;
}

// Start round r: its later-round colours still to be pulled in (except in
// the top round), its first level still only in L0.
__device__ __forceinline__ void jp_begin_round(JpState& j, int r) {
  j.round = r;
  j.level = 0;
  j.split = 1;
  j.xpull = r < j.top ? 1 : 0;
  j.relax = 0;
  j.rit = 0;
  j.rv = 0;
  for (int k = 0; k < 3; ++k) jp_clear_level(j, k);
  if (r <= 0) j.done = 1;
}

// Level l has been processed: level l + 1 becomes current.
__device__ __forceinline__ void jp_next_level(JpState& j) {
  j.levels += 1;
  j.level += 1;
  jp_clear_level(j, (j.level + 1) % 3);
}

// Whether the rest of round r (its levels so far in j) is worth relaxing:
// a round of at least RELAX_MIN_V vertices whose levels colour RELAX_DENSE
// or more vertices each on average (a round whose levels take a vertex or
// two is a dense core: levels cost little there, while relaxation would
// sweep its edges hundreds of times), with at least a quarter of it still
// uncoloured (listing the uncoloured vertices reads the whole round).
__device__ __forceinline__ bool relax_pays(const Params& P, const JpState& j, int r) {
  const unsigned long long rs = (unsigned long long)seg_size(P, r);
  return rs >= RELAX_MIN_V && j.rv >= (unsigned long long)RELAX_DENSE * (unsigned long long)j.level &&
         rs - (j.rv < rs ? j.rv : rs) >= rs / 4;
}

// Work of a level, as the single block sees it: bitmap words + successors.
__device__ __forceinline__ bool jp_fits_narrow(unsigned nv, unsigned long long words, unsigned long long succs) {
  return nv <= (unsigned)NARROW_MAX && words <= (unsigned long long)NARROW_WORDS &&
         succs <= (unsigned long long)NARROW_SUCC;
}

// ---- narrow levels: one block, level lists in LDS

struct NarrowLds {
  int v[2][NARROW_MAX];                  // level lists (current / next)
  long long pb[2][NARROW_MAX];           // first entry of the row in dag
  unsigned long long rec[2][NARROW_MAX]; // bitmap offset and |pred|
  int ns[2][NARROW_MAX];                 // same-round successors
  unsigned woff[NARROW_MAX + 1];         // exclusive scans of bitmap words and successors
  unsigned soff[NARROW_MAX + 1];
  int ffree[NARROW_MAX];                 // first clear bit of each vertex's bitmap
  int col[NARROW_MAX];
  unsigned wsum[2][NARROW_BS / WAVE];
  unsigned cnt[2];                       // list sizes
  WaveLds wl[NARROW_BS / WAVE];
};

// Append the ready ones among a thread's NARROW_UNROLL items (vertex u[q],
// bitmap urec[q]) to the next LDS list (slot `nx`), with their row metadata;
// past its capacity, to the global lists of level l + 1.  One LDS atomic per
// wavefront.
__device__ __forceinline__ void narrow_append(const Params& P, NarrowLds& Z, JpStage& st, int nx, int l,
                                              const bool* rdy, const int* u, const unsigned long long* urec,
                                              const unsigned long long* usp) {
  uint64_t m[NARROW_UNROLL];
  unsigned tot = 0;
#pragma unroll
  for (int q = 0; q < NARROW_UNROLL; ++q) {
    m[q] = ballot(rdy[q]);
    tot += (unsigned)__popcll(m[q]);
  }
  if (!tot) return;
  long long pb[NARROW_UNROLL];
  int ns[NARROW_UNROLL];
#pragma unroll
  for (int q = 0; q < NARROW_UNROLL; ++q) {   // row start and successors from the record
    pb[q] = rdy[q] ? sp_first(usp[q]) - (long long)(unsigned)urec[q] : 0;
    ns[q] = rdy[q] ? sp_count(P, u[q], usp[q]) : 0;
    if (rdy[q] && !range_ok(P, sp_first(usp[q]), sp_first(usp[q]) + ns[q])) ns[q] = 0;
  }
  unsigned base = 0;
  if (lane_id() == 0) base = atomicAdd(&Z.cnt[nx], tot);
  base = readlane_u(base, 0);
  unsigned run = base;
  bool over[NARROW_UNROLL];
#pragma unroll
  for (int q = 0; q < NARROW_UNROLL; ++q) {
    const unsigned pos = run + lanes_below(m[q]);
    run += (unsigned)__popcll(m[q]);
    over[q] = rdy[q] && pos >= (unsigned)NARROW_MAX;
    if (rdy[q] && !over[q]) {
      Z.v[nx][pos] = u[q];
      Z.pb[nx][pos] = pb[q];
      Z.rec[nx][pos] = urec[q];
      Z.ns[nx][pos] = ns[q];
    }
  }
  if (base + tot > (unsigned)NARROW_MAX) {
#pragma unroll
    for (int q = 0; q < NARROW_UNROLL; ++q) jp_append<SC_AGENT>(P, st, l, over[q], u[q], JpRec{urec[q], usp[q]});
  }
}

// Block-wide: the LDS entries of list `cur` (level l) to the global lists of
// level l (the level's sums are set by the caller).
__device__ __forceinline__ void narrow_flush(const Params& P, NarrowLds& Z, JpStage& st, int cur, int l) {
  const unsigned n = Z.cnt[cur] < (unsigned)NARROW_MAX ? Z.cnt[cur] : (unsigned)NARROW_MAX;
  for (unsigned b = 0; b < n; b += NARROW_BS) {
    const unsigned i = b + threadIdx.x;
    const bool ok = i < n && Z.v[cur][i] >= 0;
    const int v = ok ? Z.v[cur][i] : 0;
    const int ns = ok ? Z.ns[cur][i] : 0;
    const bool fan = ok && ns > JP_SMALL;
    if (fan) {
      unsigned long long nch = (unsigned long long)((ns + JP_CHUNK - 1) / JP_CHUNK);
      unsigned long long old = add64<SC_AGENT>(&st.hctr[l % 3], (nch << 32) | 1ull);
      unsigned pos = (unsigned)old;
      if (pos < P.hub_cap) st64<SC_AGENT>(&P.H[l & 1][pos], (old & 0xffffffff00000000ull) | (unsigned)v);
      else atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
    }
    const uint64_t m = ballot(ok && !fan);
    if (m) {
      unsigned g = 0;
      if (lane_id() == 0) g = add32<SC_AGENT>(&st.fcnt[l % 3], (unsigned)__popcll(m));
      g = readlane_u(g, 0);
      if (ok && !fan && slot_ok(P, g + lanes_below(m))) sti<SC_AGENT>((int*)&P.F[l & 1][g + lanes_below(m)], v);
    }
  }
}

// Entry i of an LDS list: vertex v with its row start, JP record and
// same-round successor count; a vertex id or successor range out of bounds
// (a broken state) becomes an empty entry (v = -1, no bitmap word beyond the
// first, no successors).
__device__ __forceinline__ void narrow_put(const Params& P, NarrowLds& Z, int cur, unsigned i, int v) {
  long long pb = 0;
  unsigned long long rec = 0;
  int ns = 0;
  if (vid_ok(P, v)) {
    const JpRec pr = rec_pair(P, v);
    ns = sp_count(P, v, pr.sp);
    if (range_ok(P, sp_first(pr.sp), sp_first(pr.sp) + ns)) {
      pb = sp_first(pr.sp) - (long long)(unsigned)pr.rec;
      rec = pr.rec;
    } else {
      ns = 0;
      v = -1;
    }
  } else {
    v = -1;
  }
  Z.v[cur][i] = v;
  Z.pb[cur][i] = pb;
  Z.rec[cur][i] = rec;
  Z.ns[cur][i] = ns;
}

// Block-wide: n vertices from a global list into LDS list `cur` at `at`.
__device__ __forceinline__ void narrow_load(const Params& P, NarrowLds& Z, int cur, const unsigned* src, unsigned n) {
  for (unsigned i = threadIdx.x; i < n; i += NARROW_BS) narrow_put(P, Z, cur, i, (int)ld32<SC_AGENT>(&src[i]));
}
__device__ __forceinline__ void narrow_load_fan(const Params& P, NarrowLds& Z, int cur, const unsigned long long* src, unsigned n,
                                unsigned at) {
  for (unsigned i = threadIdx.x; i < n; i += NARROW_BS)
    narrow_put(P, Z, cur, at + i, (int)(unsigned)ld64<SC_AGENT>(&src[i]));
}
// Block-wide: the first level of a round of n <= NARROW_MAX vertices, from
// the round's slot-indexed L0 (src), into LDS list `cur` (Z.cnt[cur] set; the
// order inside a level does not matter).
__device__ __forceinline__ void narrow_load_l0(const Params& P, NarrowLds& Z, int cur, const unsigned* src, unsigned n) {
  static_assert(NARROW_MAX <= NARROW_BS, "a thread per slot entry");
  if (threadIdx.x == 0) Z.cnt[cur] = 0;
  __syncthreads();
  const int v = threadIdx.x < n ? (int)ld32<SC_AGENT>(&src[threadIdx.x]) : -1;
  if (v >= 0) narrow_put(P, Z, cur, atomicAdd(&Z.cnt[cur], 1u), v);
  __syncthreads();
}

// Block-wide exclusive scans of two per-thread values (thread t: entry t).
__device__ void narrow_scan2(NarrowLds& Z, unsigned a0, unsigned a1, unsigned nv) {
  const unsigned lane = lane_id();
  const int w = threadIdx.x / WAVE;
  const unsigned i0 = wave_incl_scan_u32(a0), i1 = wave_incl_scan_u32(a1);
  if (lane == WAVE - 1) {
    Z.wsum[0][w] = i0;
    Z.wsum[1][w] = i1;
  }
  __syncthreads();
  unsigned p0 = 0, p1 = 0, s0 = 0, s1 = 0;
  for (int k = 0; k < NARROW_BS / WAVE; ++k) {
    const unsigned x0 = Z.wsum[0][k], x1 = Z.wsum[1][k];
    if (k < w) {
      p0 += x0;
      p1 += x1;
    }
    s0 += x0;
    s1 += x1;
  }
  const unsigned t = threadIdx.x;
  if (t < nv) {
    Z.woff[t] = p0 + i0 - a0;
    Z.soff[t] = p1 + i1 - a1;
    Z.ffree[t] = 0x7fffffff;
  }
  if (t == 0) {
    Z.woff[nv] = s0;
    Z.soff[nv] = s1;
  }
  __syncthreads();
}

__device__ __forceinline__ unsigned owner(const unsigned* off, unsigned nv, unsigned e) {
  unsigned lo = 0, hi = nv;  // last k < nv with off[k] <= e
  while (hi - lo > 1) {
    const unsigned mid = (lo + hi) >> 1;
    if (off[mid] <= e) lo = mid;
    else hi = mid;
  }
  return lo;
}

// One narrow level (list `cur`, level l): read the bitmaps and colour every
// vertex; then push the colours to the same-round successors and append the
// ready ones to list `nx`.  Returns false, having changed nothing outside
// LDS, if the level's work exceeds what one block takes.
__device__ __forceinline__ bool narrow_level(const Params& P, NarrowLds& Z, JpStage& st, int cur, int nx, int l) {
  const unsigned nv = Z.cnt[cur];
  const unsigned t = threadIdx.x;
  {
    const bool ok = t < nv;
    narrow_scan2(Z, ok ? bm_words((int)(unsigned)Z.rec[cur][t]) : 0, ok ? (unsigned)Z.ns[cur][t] : 0, nv);
  }
  const unsigned wtot = Z.woff[nv], stot = Z.soff[nv];
  if (wtot > (unsigned)NARROW_WORDS || stot > (unsigned)NARROW_SUCC) return false;
  // bitmap words -> first clear bit per vertex; successors of the first
  // pass fetched meanwhile
  int su[NARROW_UNROLL];
  unsigned sk[NARROW_UNROLL];
  unsigned long long sr[NARROW_UNROLL], ssp[NARROW_UNROLL];
#pragma unroll
  for (int q = 0; q < NARROW_UNROLL; ++q) {
    const unsigned e = q * NARROW_BS + t;
    su[q] = -1;
    sk[q] = 0;
    if (e < stot) {
      sk[q] = owner(Z.soff, nv, e);
      su[q] = P.dag[Z.pb[cur][sk[q]] + (int)(unsigned)Z.rec[cur][sk[q]] + (e - Z.soff[sk[q]])];
      if (!vid_ok(P, su[q])) su[q] = -1;
    }
  }
  for (unsigned e0 = 0; e0 < wtot; e0 += NARROW_BS * NARROW_UNROLL) {
    unsigned k[NARROW_UNROLL], wd[NARROW_UNROLL];
#pragma unroll
    for (int q = 0; q < NARROW_UNROLL; ++q) {
      const unsigned e = e0 + q * NARROW_BS + t;
      wd[q] = ~0u;
      k[q] = 0;
      if (e < wtot) {
        k[q] = owner(Z.woff, nv, e);
        wd[q] = bm_load(P, (Z.rec[cur][k[q]] >> 32) + (e - Z.woff[k[q]]));
      }
    }
#pragma unroll
    for (int q = 0; q < NARROW_UNROLL; ++q)
      if (~wd[q]) {
        const unsigned e = e0 + q * NARROW_BS + t;
        const int f = (int)((e - Z.woff[k[q]]) * 32) + __ffs((int)~wd[q]) - 1;
        if (f < Z.ffree[k[q]]) atomicMin(&Z.ffree[k[q]], f);
      }
  }
#pragma unroll
  for (int q = 0; q < NARROW_UNROLL; ++q) {
    const JpRec pr = su[q] >= 0 ? rec_pair(P, su[q]) : JpRec{0, 0};
    sr[q] = pr.rec;
    ssp[q] = pr.sp;
  }
  __syncthreads();
  // GetColor
  if (t < nv) {
    const int f = Z.ffree[t];
    int c;
    if (f == 0x7fffffff) {  // unreachable: at most |pred| of the |pred|+2 bits are set
      atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
      c = (int)(unsigned)Z.rec[cur][t] + 1;
    } else {
      c = f + 1;
    }
    Z.col[t] = c;
    if (Z.v[cur][t] >= 0) sti<SC_AGENT>(&P.color[Z.v[cur][t]], c);
  }
  __syncthreads();
  // push the colours to the same-round successors
  for (unsigned e0 = 0; e0 < stot; e0 += NARROW_BS * NARROW_UNROLL) {
    if (e0 > 0) {
#pragma unroll
      for (int q = 0; q < NARROW_UNROLL; ++q) {
        const unsigned e = e0 + q * NARROW_BS + t;
        su[q] = -1;
        sk[q] = 0;
        if (e < stot) {
          sk[q] = owner(Z.soff, nv, e);
          su[q] = P.dag[Z.pb[cur][sk[q]] + (int)(unsigned)Z.rec[cur][sk[q]] + (e - Z.soff[sk[q]])];
          if (!vid_ok(P, su[q])) su[q] = -1;
        }
      }
#pragma unroll
      for (int q = 0; q < NARROW_UNROLL; ++q) {
        const JpRec pr = su[q] >= 0 ? rec_pair(P, su[q]) : JpRec{0, 0};
        sr[q] = pr.rec;
        ssp[q] = pr.sp;
      }
    }
    bool rdy[NARROW_UNROLL];
#pragma unroll
    for (int q = 0; q < NARROW_UNROLL; ++q) rdy[q] = su[q] >= 0 && jp_push<SC_AGENT>(P, su[q], sr[q], Z.col[sk[q]]);
    narrow_append(P, Z, st, nx, l, rdy, su, sr, ssp);
  }
  order_point();
  __syncthreads();
  return true;
}

// ---- JP steps of one launch: a leader block and helper blocks
//
// Its first block to start leads: it runs the JP state machine and every
// narrow step itself, with the level lists in LDS.  The other blocks that start in
// time help: they wait for the leader's commands and take their share of
// steps too wide for one block but far too narrow for a grid launch of their
// own -- mid-sized levels, later-round colour pulls and first-level splits of
// mid-sized rounds -- as the grid kernel does, over the blocks that take
// part; the leader takes its share too and waits until every helper has
// reported the command done.  Steps wider still go to the grid kernel.
//
// Taking part.  Every block registers with one atomic add on a word of the
// control block, which the grid step launched between two steps launches
// (or k_jp_start, before the first) clears; the block that finds it empty
// leads.  The leader closes registration once every block of the launch has
// started or after a short wait, whichever comes first; blocks that start
// later leave at once.  No block ever waits for a block that has not
// registered, so the launch needs no co-residency of all its blocks.
//
// Commands are one 64-bit word (sequence << 40 | op << 32 | argument) that
// the helpers poll; completions are counted in a second word.  The leader
// ends the launch (and the helpers with it) after a bounded number of narrow
// steps without a command, so no helper waits long; every wait is bounded
// and a wait that runs out raises ADG_ERR_INTERNAL.

#ifndef ADG_STEP_BLOCKS
#define ADG_STEP_BLOCKS 64
#endif
#ifndef ADG_MID_LOG
#define ADG_MID_LOG 20
#endif
constexpr int STEP_BLOCKS = ADG_STEP_BLOCKS;    // blocks of a k_jp_steps launch (one per CU)
constexpr unsigned MID_MAX_V = ADG_MID_LOG ? 1u << 16 : 0;   // vertices of a level the launch's blocks take together
constexpr unsigned long long MID_MAX_W = ADG_MID_LOG ? 1ull << ADG_MID_LOG : 0;   // its bitmap words
constexpr unsigned long long MID_MAX_S = ADG_MID_LOG ? 1ull << ADG_MID_LOG : 0;   // its same-round successors
constexpr long long MID_MAX_XPULL = ADG_MID_LOG ? 1ll << 17 : NARROW_XPULL;   // vertices of a round whose later-round colours they pull in
constexpr unsigned MID_MAX_SPLIT = ADG_MID_LOG ? 1u << 17 : NARROW_MAX;      // first-level vertices of a round they split
constexpr int NARROW_RUN = 4096;                // narrow steps without a command before the launch ends
constexpr unsigned long long REG_CLOSED = 1ull << 32;
constexpr unsigned long long REG_SEEN = 1ull << 16;
constexpr unsigned REG_WAIT_TICKS = 2000;       // the leader waits at most 20 us (100 MHz clock) for late blocks
constexpr unsigned long long POLL_MAX = 1ull << 22;   // polls of a helper's or the leader's wait
enum { PC_LEVEL = 1, PC_XPULL = 2, PC_SPLIT = 3, PC_EXIT = 4, PC_RELAX = 5 };


// The helpers' share of a command (the leader takes part as participant 0).
__device__ __forceinline__ void steps_command(const Params& P, JpStage& st, WaveLds& W, int op, int arg, long long gw,
                                              long long gstride, unsigned long long* flds) {
  Ctrl* c = P.ctrl;
  if (op == PC_XPULL) {
    jp_xpull_items<SC_AGENT>(P, W, arg, gw, gstride);
  } else if (op == PC_SPLIT) {
    jp_split_items(P, st, arg, gw, gstride);
    jp_stage_flush<SC_AGENT>(P, st, -1);
  } else if (op == PC_LEVEL) {
    const int l = arg;
    const unsigned nf = ld32<SC_AGENT>(&c->js.fcnt[l % 3]);
    const unsigned long long hc = ld64<SC_AGENT>(&c->js.hctr[l % 3]);
    if (level_ok(P, nf, (unsigned)hc)) {
      const unsigned long long* hl = fan_stage<SC_AGENT>(P.H[l & 1], (unsigned)hc, flds);
      jp_level_items(P, st, W, l, nf, hc, gw, gstride, hl);
    }
    jp_stage_flush<SC_AGENT>(P, st, l);
  } else if (op == PC_RELAX) {
    const int rr = (int)ld32<SC_AGENT>(&c->rx[0]);
    const int t = (int)ld32<SC_AGENT>(&c->rx[1]);
    if (t == 0) jp_relax_list(P, st, rr, gw, gstride);
    else jp_relax_items(P, st, W, nullptr, t, ld32<SC_AGENT>(&c->rx[2]), ld32<SC_AGENT>(&c->rx[3]), gw, gstride, rr);
    jp_stage_flush<SC_AGENT>(P, st, t);
  }
}

// The leader's side of one command: publish it, take participant 0's share,
// wait until every helper has reported its share done.
__device__ __forceinline__ void steps_lead(const Params& P, JpStage& gst, WaveLds& W, int op, int arg,
                                           unsigned long long& seq, int nparts, long long gw, long long gstride,
                                           unsigned long long* flds, unsigned* fcntl, unsigned long long* acc,
                                           int* stop) {
  Ctrl* c = P.ctrl;
  if (threadIdx.x == 0) {
    order_point();
    st64<SC_AGENT>(&c->pcmd, ((seq + 1) << 40) | ((unsigned long long)op << 32) | (unsigned)arg);
    *fcntl = 0;
    acc[0] = acc[1] = 0;
  }
  ++seq;
  __syncthreads();
  steps_command(P, gst, W, op, arg, gw, gstride, flds);
  order_point();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long want = (unsigned long long)(nparts - 1) * seq;
    unsigned long long k = 0;
    while (ld64<SC_AGENT>(&c->pjoin) < want && ++k < POLL_MAX) __builtin_amdgcn_s_sleep(1);
    if (k >= POLL_MAX) {
      raise_internal(P);
      *stop = 1;
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(NARROW_BS) void k_jp_steps(Params P, int max_steps) {
  Ctrl* c = P.ctrl;
  __shared__ JpState S;
  __shared__ union StepsLds {
    NarrowLds z;
    CoreLds k;   // the core mode (the leader alone, with no level in LDS)
  } SL;
  NarrowLds& Z = SL.z;
  __shared__ unsigned fbuf[FB_CAP];
  __shared__ unsigned fcntl;
  __shared__ unsigned long long flds[FAN_LDS];
  __shared__ unsigned long long acc[2];
  __shared__ int have, role, nparts, pidx, cmd_op, cmd_arg, stop;
  constexpr int NW = NARROW_BS / WAVE;   // wavefronts per block
  WaveLds& W = Z.wl[threadIdx.x / WAVE];
  // ---- registration: one atomic per block on a word that the previous
  // launch of the grid step (or k_jp_start) has cleared.  The leader
  // publishes the participant count in pnum (cleared with preg): a block
  // that comes after the close still adds to preg's count, so helpers do not
  // take the count from there (another count than the leader's would split
  // the work differently, and leave items no one takes).
  if (threadIdx.x == 0) {
    const unsigned long long old = __hip_atomic_fetch_add(&c->preg, REG_SEEN + 1ull, __ATOMIC_RELAXED, SC_AGENT);
    role = (old & REG_CLOSED) ? 0 : (old & 0xffff) == 0 ? 1 : 2;   // 0: leave, 1: lead, 2: help
    pidx = (int)(old & 0xffff);
    if (role == 1) {
      // fresh command and completion words, then close registration once
      // every block has started (or after a short wait)
      st64<SC_AGENT>(&c->pcmd, 0ull);
      st64<SC_AGENT>(&c->pjoin, 0ull);
      order_point();
      const bool idle = c->js.done || c->error;
      const unsigned long long t0 = wall_clock64();
      while (!idle && ((ld64<SC_AGENT>(&c->preg) >> 16) & 0xffff) < gridDim.x &&
             wall_clock64() - t0 < REG_WAIT_TICKS)
        __builtin_amdgcn_s_sleep(2);
      nparts = (int)(__hip_atomic_fetch_or(&c->preg, REG_CLOSED, __ATOMIC_RELAXED, SC_AGENT) & 0xffff);
      st64<SC_AGENT>(&c->pnum, (unsigned long long)nparts);   // >= 1: the leader counts itself
    } else if (role == 2) {
      unsigned long long w = 0;
      for (unsigned long long k = 0; k < POLL_MAX; ++k) {
        w = ld64<SC_AGENT>(&c->pnum);
        if (w) break;
        __builtin_amdgcn_s_sleep(2);
      }
      if (!w || (unsigned long long)pidx >= w) {   // a registered helper has an index below the count
        if (!w) raise_internal(P);
        role = 0;
      }
      nparts = (int)(w & 0xffff);
    }
  }
  __syncthreads();
  if (role == 0) return;
  JpStage gst{fbuf, &fcntl, c->js.fcnt, c->js.hctr, c->js.psum, c->js.ssum, acc};   // global lists and counters
  const long long gstride = (long long)nparts * NW;
  // work items go round-robin over the participants (item k to participant
  // k mod nparts), so that the heavy items at the front of a level -- the
  // groups of plain vertices -- spread over all of them
  const long long gw = (long long)(threadIdx.x / WAVE) * nparts + pidx;
  unsigned long long seq = 0;
  if (role == 2) {
    // ---- helper: take a share of each command until told to leave
    for (;;) {
      if (threadIdx.x == 0) {
        unsigned long long w = 0;
        bool got = false;
        for (unsigned long long k = 0; k < POLL_MAX; ++k) {
          w = ld64<SC_AGENT>(&c->pcmd);
          if ((w >> 40) == seq + 1) {
            got = true;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        if (!got) raise_internal(P);
        cmd_op = got ? (int)((w >> 32) & 0xff) : PC_EXIT;
        cmd_arg = (int)(unsigned)w;
        fcntl = 0;
        acc[0] = acc[1] = 0;
      }
      __syncthreads();
      const int op = cmd_op, arg = cmd_arg;
      ++seq;
      __syncthreads();
      if (op == PC_EXIT) return;
      steps_command(P, gst, W, op, arg, gw, gstride, flds);
      order_point();
      __syncthreads();
      if (threadIdx.x == 0) __hip_atomic_fetch_add(&c->pjoin, 1ull, __ATOMIC_RELAXED, SC_AGENT);
    }
  }
  // ---- leader
  if (threadIdx.x == 0) {
    S = c->js;
    have = 0;
    stop = 0;
    if (c->error) S.done = 1;   // raised by an earlier step: JP stops
    // launches alternate (steps, grid): the op posted by the previous steps
    // launch has been run by the grid launch between them
    if (!S.done) {
      const int op = c->grid_op;
      c->grid_op = OP_NONE;
      if (op == OP_XPULL) {
        S.xpull = 0;
      } else if (op == OP_SPLIT) {
        S.split = 0;
        S.F += S.fcnt[0] + (unsigned)S.hctr[0];
      } else if (op == OP_LEVEL) {
        S.rv += S.fcnt[S.level % 3] + (unsigned)S.hctr[S.level % 3];
        jp_next_level(S);
      } else if (op == OP_RELAX) {
        S.rit += 1;
        S.levels += 1;
      }
    }
  }
  __syncthreads();
  JpStage st{nullptr, nullptr, S.fcnt, S.hctr, S.psum, S.ssum, nullptr};   // LDS counters (narrow steps)
  int cur = 0;
  int handed = OP_NONE;
  int checked = 0;          // the round whose sizes have been checked
  int since_cmd = 0;        // narrow steps since the last command
  bool in_global = false;   // the LDS level is also in the global lists
  for (int step = 0; step < max_steps; ++step) {
    if (S.done || stop) break;
    const int r = S.round;
    const int l = S.level;
    if (r != checked || !level_ok(P, S.fcnt[l % 3], (unsigned)S.hctr[l % 3])) {
      // a round's sizes are checked once, when it starts
      const bool ok = level_ok(P, S.fcnt[l % 3], (unsigned)S.hctr[l % 3]) && round_ok(P, r);
      __syncthreads();
      if (!ok) {
        if (threadIdx.x == 0) S.done = 1;   // a broken state: stop (the error is raised)
        __syncthreads();
        break;
      }
      checked = r;
    }
    if (nparts > 1 && since_cmd > NARROW_RUN) {
      // a long run of narrow steps: end the launch so that no helper waits long
      if (have && !in_global) narrow_flush(P, Z, st, cur, l);
      __syncthreads();
      if (threadIdx.x == 0) have = 0;
      __syncthreads();
      break;
    }
    if (S.xpull) {
      const long long sz = seg_size(P, r);
      if (sz > MID_MAX_XPULL) {
        handed = OP_XPULL;
        break;
      }
      if (sz > (long long)NARROW_XPULL) {
        steps_lead(P, gst, W, PC_XPULL, r, seq, nparts, gw, gstride, flds, &fcntl, acc, &stop);
        since_cmd = 0;
      } else {
        jp_xpull_items<SC_AGENT>(P, W, r, threadIdx.x / WAVE, NW);
        order_point();
        ++since_cmd;
      }
      __syncthreads();
      if (threadIdx.x == 0) S.xpull = 0;
      __syncthreads();
      continue;
    }
    if (JP_RELAX && P.relax_mode != RELAX_MODE_NONE && !S.relax && !S.split &&
        (P.relax_mode == RELAX_MODE_ALL || (S.level >= RELAX_AFTER && relax_pays(P, S, r)))) {
      // a deep round: its uncoloured vertices are relaxed from here on (a
      // level still in LDS is dropped; its vertices are uncoloured)
      __syncthreads();
      if (threadIdx.x == 0) {
        S.relax = 1;
        S.rit = 0;
        have = 0;
      }
      __syncthreads();
      in_global = false;
      continue;
    }
    if (JP_CORE && P.relax_mode == RELAX_MODE_RULE && !S.relax && !S.split && S.level >= RELAX_AFTER &&
        seg_size(P, r) <= (long long)CORE_MAX && P.nnz > 0 && P.bm_cap > 0) {
      // a small round that relaxation would not take (a dense core, or too
      // small): the rest of it in JP's order, by this block alone (a level
      // still in LDS is dropped; its vertices are uncoloured)
      __syncthreads();
      jp_core_round(P, SL.k, r);
      if (threadIdx.x == 0) {
        S.levels += 1;
        jp_begin_round(S, r - 1);
        have = 0;
      }
      __syncthreads();
      in_global = false;
      continue;
    }
    if (S.relax) {
      const int t = S.rit;
      const long long rs = seg_size(P, r);
      const unsigned nl = t == 0 ? (unsigned)rs : S.fcnt[t % 3];
      if (t > 0 && nl == 0) {   // no colour changed: the round is finished
        __syncthreads();
        if (threadIdx.x == 0) jp_begin_round(S, r - 1);
        __syncthreads();
        continue;
      }
      if ((long long)t > rs + 2 || (long long)nl > rs) {   // more steps than the longest chain needs: a broken state
        __syncthreads();
        if (threadIdx.x == 0) {
          raise_internal(P);
          S.done = 1;
        }
        __syncthreads();
        break;
      }
      const int nx = (t + 1) % 3;
      if (threadIdx.x == 0) {
        S.rstamp += 1;
        jp_clear_level(S, nx);
        st32<SC_AGENT>(&c->js.fcnt[nx], 0u);
        st64<SC_AGENT>(&c->js.hctr[nx], 0ull);
        st64<SC_AGENT>(&c->js.psum[nx], 0ull);
        st64<SC_AGENT>(&c->js.ssum[nx], 0ull);
      }
      __syncthreads();
      if (t == 0 ? rs > (long long)RELAX_MID * WAVE : nl > RELAX_MID) {
        handed = OP_RELAX;   // the grid takes the step
        break;
      }
      if (threadIdx.x == 0) {
        st32<SC_AGENT>(&c->rx[0], (unsigned)r);
        st32<SC_AGENT>(&c->rx[1], (unsigned)t);
        st32<SC_AGENT>(&c->rx[2], nl);
        st32<SC_AGENT>(&c->rx[3], S.rstamp);
      }
      steps_lead(P, gst, W, PC_RELAX, t, seq, nparts, gw, gstride, flds, &fcntl, acc, &stop);
      since_cmd = 0;
      if (threadIdx.x == 0) {
        S.fcnt[nx] = ld32<SC_AGENT>(&c->js.fcnt[nx]);
        S.rit = t + 1;
        S.levels += 1;
      }
      __syncthreads();
      if (t == 1 && relax_idx(P, r).compact) break;   // step 1 rewrote the DAG: the next steps run in a new launch
      continue;
    }
    if (!have) {
      if (S.split) {
        // the round's first level, from L0
        const long long rs = seg_size(P, r);
        if (rs > (long long)MID_MAX_SPLIT) {
          handed = OP_SPLIT;
          break;
        }
        if (rs > (long long)NARROW_MAX) {
          // split into the global lists of level 0 by all participants
          if (threadIdx.x == 0) {
            st32<SC_AGENT>(&c->js.fcnt[0], 0u);
            st64<SC_AGENT>(&c->js.hctr[0], 0ull);
            st64<SC_AGENT>(&c->js.psum[0], 0ull);
            st64<SC_AGENT>(&c->js.ssum[0], 0ull);
          }
          steps_lead(P, gst, W, PC_SPLIT, r, seq, nparts, gw, gstride, flds, &fcntl, acc, &stop);
          since_cmd = 0;
          if (threadIdx.x == 0) {
            S.fcnt[0] = ld32<SC_AGENT>(&c->js.fcnt[0]);
            S.hctr[0] = ld64<SC_AGENT>(&c->js.hctr[0]);
            S.psum[0] = ld64<SC_AGENT>(&c->js.psum[0]);
            S.ssum[0] = ld64<SC_AGENT>(&c->js.ssum[0]);
            S.split = 0;
            S.F += S.fcnt[0] + (unsigned)S.hctr[0];
          }
          __syncthreads();
          continue;
        }
        narrow_load_l0(P, Z, cur, P.L0 + seg_begin(P, r), (unsigned)rs);
        in_global = false;
        if (threadIdx.x == 0) {
          S.split = 0;
          S.F += Z.cnt[cur];
        }
      } else {
        const unsigned nf = S.fcnt[l % 3], nh = (unsigned)S.hctr[l % 3];
        if (nf + nh == 0) {  // round finished
          __syncthreads();
          if (threadIdx.x == 0) jp_begin_round(S, r - 1);
          __syncthreads();
          continue;
        }
        if (!jp_fits_narrow(nf + nh, S.psum[l % 3], S.ssum[l % 3])) {
          if (nf + nh > MID_MAX_V || S.psum[l % 3] > MID_MAX_W || S.ssum[l % 3] > MID_MAX_S) {
            handed = OP_LEVEL;
            break;
          }
          // a mid-sized level in the global lists: all participants
          if (threadIdx.x == 0) {
            st32<SC_AGENT>(&c->js.fcnt[l % 3], S.fcnt[l % 3]);
            st64<SC_AGENT>(&c->js.hctr[l % 3], S.hctr[l % 3]);
            const int nx = (l + 1) % 3;
            st32<SC_AGENT>(&c->js.fcnt[nx], 0u);
            st64<SC_AGENT>(&c->js.hctr[nx], 0ull);
            st64<SC_AGENT>(&c->js.psum[nx], 0ull);
            st64<SC_AGENT>(&c->js.ssum[nx], 0ull);
          }
          steps_lead(P, gst, W, PC_LEVEL, l, seq, nparts, gw, gstride, flds, &fcntl, acc, &stop);
          since_cmd = 0;
          if (threadIdx.x == 0) {
            const int nx = (l + 1) % 3;
            S.fcnt[nx] = ld32<SC_AGENT>(&c->js.fcnt[nx]);
            S.hctr[nx] = ld64<SC_AGENT>(&c->js.hctr[nx]);
            S.psum[nx] = ld64<SC_AGENT>(&c->js.psum[nx]);
            S.ssum[nx] = ld64<SC_AGENT>(&c->js.ssum[nx]);
            S.rv += S.fcnt[l % 3] + (unsigned)S.hctr[l % 3];
            jp_next_level(S);
          }
          __syncthreads();
          continue;
        }
        narrow_load(P, Z, cur, P.F[l & 1], nf);
        narrow_load_fan(P, Z, cur, P.H[l & 1], nh, nf);
        in_global = true;
        if (threadIdx.x == 0) Z.cnt[cur] = nf + nh;
      }
      if (threadIdx.x == 0) have = 1;
      __syncthreads();
    }
    // process level l from LDS list `cur`
    ++since_cmd;
    const int nx = cur ^ 1;
    if (threadIdx.x == 0) Z.cnt[nx] = 0;
    __syncthreads();
    if (Z.cnt[cur] == 0) {  // nothing ready: the round is finished
      __syncthreads();
      if (threadIdx.x == 0) {
        jp_begin_round(S, r - 1);
        have = 0;
      }
      __syncthreads();
      continue;
    }
    if (!narrow_level(P, Z, st, cur, nx, l)) {
      // too much work for one block: the level goes to the global lists
      // (the next pass of the loop gives it to the participants or the grid)
      if (!in_global) {
        narrow_flush(P, Z, st, cur, l);
        order_point();
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        S.psum[l % 3] = Z.woff[Z.cnt[cur]];
        S.ssum[l % 3] = Z.soff[Z.cnt[cur]];
        have = 0;
      }
      __syncthreads();
      continue;
    }
    const unsigned nn = Z.cnt[nx];
    const bool wide = nn > (unsigned)NARROW_MAX;
    if (wide) {
      // the next level leaves LDS: its overflow entries are already in the
      // global lists; add the LDS ones
      narrow_flush(P, Z, st, nx, l + 1);
      order_point();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      S.rv += Z.cnt[cur];
      jp_next_level(S);
      if (nn == 0) {
        jp_begin_round(S, r - 1);
        have = 0;
      } else if (wide) {
        have = 0;
      }
    }
    __syncthreads();
    cur = nx;
    in_global = false;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (have) {  // step bound reached with a level still in LDS: a broken state
      atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
      S.done = 1;
    }
    c->js = S;
    c->grid_op = handed;
    order_point();
    if (nparts > 1) st64<SC_AGENT>(&c->pcmd, ((seq + 1) << 40) | ((unsigned long long)PC_EXIT << 32));
  }
}

// Grid-wide: the step the single-block kernel handed over.
__global__ __launch_bounds__(BS) void k_jp_grid(Params P) {
  Ctrl* c = P.ctrl;
  // launches alternate (steps, grid): every block of the steps launch before
  // this one has finished, so its registration word can be cleared for the next
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st64<SC_AGENT>(&c->preg, 0ull);
    st64<SC_AGENT>(&c->pnum, 0ull);
  }
  // Every block decides from state no block of this launch changes: blocks
  // may start after others have finished (other streams' kernels hold CUs).
  const int op = c->grid_op;
  if (c->js.done || op == OP_NONE) return;
  {
    // blocks past the step's work leave at once (block 0 stays: it reports);
    // the round's sizes were checked by the single-block step that handed
    // the step over
    const int r = c->js.round, l = c->js.level;
    long long items;
    if (op == OP_XPULL) {
      items = seg_size(P, r);   // groups of G >= 1 vertices: at most one per vertex
    } else if (op == OP_RELAX) {
      // step 0: groups of 64 of the round's vertices; later steps: a
      // wavefront per listed vertex
      const int t = c->js.rit;
      const unsigned nl = c->js.fcnt[t % 3];
      if (t > 0 && (long long)nl > seg_size(P, r)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) raise_internal(P);
        return;
      }
      items = t == 0 ? (seg_size(P, r) + WAVE - 1) / WAVE : (long long)nl;
    } else if (op == OP_SPLIT) {
      items = (seg_size(P, r) + WAVE - 1) / WAVE;
    } else {
      if (!level_ok(P, c->js.fcnt[l % 3], (unsigned)c->js.hctr[l % 3])) return;
      items = ((long long)c->js.fcnt[l % 3] + WAVE - 1) / WAVE + (long long)(c->js.hctr[l % 3] >> 32);
    }
    if (blockIdx.x > 0 && (long long)blockIdx.x * WPB >= items) return;
  }
  __shared__ unsigned fbuf[FB_CAP];
  __shared__ unsigned fcnt;
  __shared__ unsigned long long flds[FAN_LDS];
  __shared__ WaveLds wl[WPB];
  __shared__ unsigned long long acc[2];
  if (threadIdx.x == 0) {
    fcnt = 0;
    acc[0] = acc[1] = 0;
  }
  __syncthreads();
  JpStage st{fbuf, &fcnt, c->js.fcnt, c->js.hctr, c->js.psum, c->js.ssum, acc};
  const int r = c->js.round;
  const long long gw = (long long)blockIdx.x * WPB + threadIdx.x / WAVE;
  const long long gstride = (long long)gridDim.x * WPB;
  WaveLds& W = wl[threadIdx.x / WAVE];
  if (op == OP_XPULL) {
    jp_xpull_items<SC_AGENT>(P, W, r, gw, gstride);
  } else if (op == OP_SPLIT) {
    jp_split_items(P, st, r, gw, gstride);
    jp_stage_flush<SC_AGENT>(P, st, -1);
  } else if (op == OP_RELAX) {
    const int t = c->js.rit;
    // the fan-out staging area is free: it holds the wavefronts' bits of
    // lane-solved vertices
    static_assert(sizeof(flds) >= WPB * WAVE * RELAX_LW * 4, "relaxation buffers");
    if (t == 0) jp_relax_list(P, st, r, gw, gstride);
    else jp_relax_items(P, st, W, (unsigned*)flds + (threadIdx.x / WAVE) * WAVE * RELAX_LW, t, c->js.fcnt[t % 3],
                        c->js.rstamp, gw, gstride, r);
    jp_stage_flush<SC_AGENT>(P, st, t);
  } else {
    const int l = c->js.level;
    const unsigned long long hc = c->js.hctr[l % 3];
    const unsigned long long* hl = fan_stage<SC_AGENT>(P.H[l & 1], (unsigned)hc, flds);
    jp_level_items(P, st, W, l, c->js.fcnt[l % 3], hc, gw, gstride, hl);
    jp_stage_flush<SC_AGENT>(P, st, l);
  }
}

__global__ void k_jp_start(Params P, int rounds) {
  // colours start at 0 (relaxation lists the uncoloured vertices by it),
  // and so do the relaxation marks
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < P.n; i += stride) {
    P.color[i] = 0;
    if (JP_RELAX) P.rmark[i] = 0u;
  }
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  Ctrl* c = P.ctrl;
  c->grid_op = OP_NONE;
  c->preg = 0;   // the first steps launch registers from zero
  c->pnum = 0;
  c->pcmd = 0;
  c->pjoin = 0;
  JpState& j = c->js;
  j.done = 0;
  j.levels = 0;
  j.rstamp = 0;
  j.F = 0;
  j.top = rounds;
  if (P.ord_identity) {
    P.roundN[1] = (unsigned)P.n;
    P.roundN[2] = 0;
  } else {
    P.roundN[rounds + 1] = 0;
  }
  jp_begin_round(j, rounds);
}

// Largest colour: per-block maxima, one atomic per block.
// ================================================================ DEC-ADG-ITR

__device__ __forceinline__ const int* dec_list(const Params& P, const DecState& d) {
  return d.first ? P.ORD + ((long long)P.n - P.roundN[d.round]) : P.UL[d.cur];
}

__global__ void k_dec_start(Params P, int rounds) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  DecState& d = P.ctrl->dec[0];
  d.round = rounds;
  d.first = 1;
  d.pull = 1;
  d.cur = 0;
  d.ucnt = rounds > 0 ? P.roundN[rounds] - P.roundN[rounds + 1] : 0;
  d.done = rounds == 0;
  d.iters = 0;
  P.ctrl->dec[1] = d;
  P.ctrl->dec_unext = 0;
  P.ctrl->dec_blocks = 0;
}

// Blocks of a DEC step with items to take (the others leave at once).
__device__ __forceinline__ long long dec_active(unsigned ucnt) {
  long long a = ((long long)ucnt + BS - 1) / BS;
  if (a < 1) a = 1;
  return a < (long long)gridDim.x ? a : (long long)gridDim.x;
}

// Before a partition's first iteration: OR the colours of every neighbour in
// a later round (all final) into the vertex's bitmap.
__global__ __launch_bounds__(BS) void k_dec_pull(Params P, int p) {
  const DecState d = P.ctrl->dec[p];
  if (d.done || !d.pull) return;
  const int* U = dec_list(P, d);
  const long long stride = (long long)gridDim.x * BS;
  for (long long t = (long long)blockIdx.x * BS; t < d.ucnt; t += stride) {
    const long long i = t + threadIdx.x;
    const bool has = i < d.ucnt;
    const int v = has ? U[i] : 0;
    long long b = 0, e = 0;
    unsigned long long rec = 0;
    if (has) {
      b = P.rp[v];
      e = b + P.xpred[v];
      rec = rec_of(P, v);
    }
    // the wavefront walks long rows together; each entry marks in its row's bitmap
    const bool longrow = has && e - b > WAVE;
    if (has && !longrow)
      for (long long j = b; j < e; ++j) bm_mark<SC_AGENT>(P, rec, P.color[P.dag[j]]);
    uint64_t m = ballot(longrow);
    while (m) {
      const int src = __ffsll((long long)m) - 1;
      m &= m - 1;
      const long long bb = readlane_i64(b, src), ee = readlane_i64(e, src);
      const unsigned long long rr = readlane_u64(rec, src);
      for (long long j = bb + lane_id(); j < ee; j += WAVE) bm_mark<SC_AGENT>(P, rr, P.color[P.dag[j]]);
    }
  }
}

// Part 1: every vertex of U tries the smallest colour not in its bitmap.
__global__ __launch_bounds__(BS) void k_dec_pick(Params P, int p) {
  const DecState d = P.ctrl->dec[p];
  if (d.done) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) P.ctrl->dec[p].pull = 0;
  const int* U = dec_list(P, d);
  for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < d.ucnt; i += (long long)gridDim.x * BS) {
    const int v = U[i];
    const unsigned long long rec = rec_of(P, v);
    const unsigned nw = bm_words((int)(unsigned)rec);
    unsigned c = 0;
    for (unsigned w = 0; w < nw; ++w) {
      const unsigned wd = bm_load(P, (rec >> 32) + w);
      if (wd != ~0u) {
        c = 32 * w + (unsigned)__builtin_ctz(~wd) + 1;
        break;
      }
    }
    // a vertex never has more coloured neighbours than its bitmap has bits
    if (c == 0) {
      atomicExch(&P.ctrl->error, ADG_ERR_INTERNAL);
      c = 32 * nw + 1;
    }
    P.tent[v] = c;
  }
}

// Parts 2 and 3: a vertex keeps its colour unless a same-round predecessor
// (a same-round neighbour with a larger hash) tried the same one; kept
// colours go into the bitmaps of the same-round neighbours, the others form
// the next U.  The last block moves to the next iteration or partition.
__global__ __launch_bounds__(BS) void k_dec_resolve(Params P, int p) {
  Ctrl* c = P.ctrl;
  const DecState d = c->dec[p];
  if (d.done) {   // carry the end forward to the other parity
    if (blockIdx.x == 0 && threadIdx.x == 0) c->dec[p ^ 1].done = 1;
    return;
  }
  const long long active = dec_active(d.ucnt);
  if ((long long)blockIdx.x >= active) return;
  const int* U = dec_list(P, d);
  int* Unext = P.UL[d.cur ^ 1];
  __shared__ int last;
  const long long stride = (long long)gridDim.x * BS;
  for (long long t = (long long)blockIdx.x * BS; t < d.ucnt; t += stride) {
    const long long i = t + threadIdx.x;
    const bool has = i < d.ucnt;
    int v = 0;
    unsigned tv = 0;
    long long b = 0, e = 0, e2 = 0;
    if (has) {
      v = U[i];
      tv = P.tent[v];
      const int nps = P.cnt[v];
      b = P.rp[v] + P.xpred[v];   // same-round predecessors: [b, e)
      e = b + nps;
      e2 = e + P.nsr[v];                  // and successors: [e, e2)
    }
    // Part 2: any same-round predecessor with the same tried colour?
    bool lose = false;
    const bool longrow = has && e - b > WAVE;
    if (has && !longrow)
      for (long long j = b; j < e && !lose; ++j) lose = P.tent[P.dag[j]] == tv;
    uint64_t m = ballot(longrow);
    while (m) {
      const int src = __ffsll((long long)m) - 1;
      m &= m - 1;
      const long long bb = readlane_i64(b, src), ee = readlane_i64(e, src);
      const unsigned ts = readlane_u(tv, src);
      bool hit = false;
      for (long long j = bb + lane_id(); j < ee; j += WAVE) hit |= P.tent[P.dag[j]] == ts;
      if (ballot(hit) && lane_id() == (unsigned)src) lose = true;
    }
    // Part 3: a kept colour goes to the same-round neighbours
    const bool keep = has && !lose;
    if (keep) P.color[v] = (int)tv;
    const long long pb = keep ? b : 0, pe = keep ? e2 : 0;
    const bool longpush = keep && pe - pb > WAVE;
    if (keep && !longpush)
      for (long long j = pb; j < pe; ++j) bm_mark<SC_AGENT>(P, rec_of(P, P.dag[j]), (int)tv);
    m = ballot(longpush);
    while (m) {
      const int src = __ffsll((long long)m) - 1;
      m &= m - 1;
      const long long bb = readlane_i64(pb, src), ee = readlane_i64(pe, src);
      const int ts = (int)readlane_u(tv, src);
      for (long long j = bb + lane_id(); j < ee; j += WAVE) bm_mark<SC_AGENT>(P, rec_of(P, P.dag[j]), ts);
    }
    // the others form the next U
    const uint64_t lm = ballot(has && lose);
    if (lm) {
      const int leader = __ffsll((long long)lm) - 1;
      unsigned at = 0;
      if (lane_id() == (unsigned)leader) at = atomicAdd(&c->dec_unext, (unsigned)__popcll(lm));
      at = readlane_u(at, leader);
      if (has && lose) Unext[at + lanes_below(lm)] = v;
    }
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0)
    last = __hip_atomic_fetch_add(&c->dec_blocks, 1u, __ATOMIC_ACQ_REL, SC_AGENT) == (unsigned)(active - 1);
  __syncthreads();
  if (!last || threadIdx.x != 0) return;
  __threadfence();
  DecState g = d;
  g.pull = c->dec[p].pull;
  g.iters += 1;
  const unsigned nx = __hip_atomic_load(&c->dec_unext, __ATOMIC_RELAXED, SC_AGENT);
  c->dec_unext = 0;
  c->dec_blocks = 0;
  if (nx > 0) {
    g.ucnt = nx;
    g.cur ^= 1;
    g.first = 0;
  } else if (g.round > 1) {
    g.round -= 1;
    g.first = 1;
    g.pull = 1;
    g.ucnt = P.roundN[g.round] - P.roundN[g.round + 1];
  } else {
    g.done = 1;
  }
  c->dec[p ^ 1] = g;
}

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

// ---- the total order JP colours by (adg_order_ex's pos output): rounds in
// increasing order, inside a round the same-round key (rho_R, after D at
// selection for ADG-O), as ranks 0 .. n-1.
__global__ __launch_bounds__(BS) void k_order_keys(Params P, unsigned long long* keys, unsigned* vals) {
  for (long long v = (long long)blockIdx.x * BS + threadIdx.x; v < P.n; v += (long long)gridDim.x * BS) {
    keys[v] = same_key(P, (int)v);
    vals[v] = (unsigned)v;
  }
}
__global__ __launch_bounds__(BS) void k_order_round_keys(Params P, unsigned long long* keys, const unsigned* vals) {
  for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < P.n; i += (long long)gridDim.x * BS)
    keys[i] = (unsigned)P.round[vals[i]];
}
__global__ __launch_bounds__(BS) void k_order_pos(Params P, const unsigned* vals, int* pos) {
  for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < P.n; i += (long long)gridDim.x * BS)
    pos[vals[i]] = (int)i;
}

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
                                    "jp_prep", "jp", "finish", "batched", "jp_narrow", "update_huge",
                                    "median_select", "order_sort", "dec_itr", "update_pull", "jp_phase",
                                    "dec_phase", "adg_phase", "update_sub"};
static_assert(KC_NUM <= ADG_PROFILE_CLASSES, "profile classes do not fit adg_profile_t");
struct ProfRec {
  int cls;
  hipEvent_t a, b;
  long long units;
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

// Set while an allocation-free call runs on this thread: no event is
// recorded and the loop flags are read through the caller's stack.
thread_local bool t_no_alloc = false;

hipEvent_t prof_begin(int cls, hipStream_t s) {
  if (t_no_alloc) return nullptr;
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (!(g_prof_mask & (1u << cls))) return nullptr;
  hipEvent_t a = prof_event();
  if (a && hipEventRecord(a, s) != hipSuccess) {
    g_pool.push_back(a);
    return nullptr;
  }
  return a;
}

void prof_end(int cls, hipStream_t s, hipEvent_t a, long long units) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  hipEvent_t b = prof_event();
  if (!b || hipEventRecord(b, s) != hipSuccess) {
    g_pool.push_back(a);
    if (b) g_pool.push_back(b);
    return;
  }
  g_prof.push_back({cls, a, b, units});
}

}  // namespace adg

namespace {

struct Layout {
  size_t ctrl, bcount, boff, bsum, xpart, D, status, UL0, UL1, ORD, roundN, round, dag, xpred, nsr, cnt, rec, B,
      bm_cap, L0, F0, F1, H0, H1, hub_cap, sb_cap, SUBC, SUBS, HL, HC, huge_cap, mhist, pool, pool_chunk, total;
};

constexpr int UPD_BLOCKS = 2048;
// color_graph hands graphs up to these sizes to the one-launch engine
#ifndef ADG_ONE_GRAPH_MAX_NNZ
#define ADG_ONE_GRAPH_MAX_NNZ (1 << 17)
#endif
constexpr int64_t ONE_GRAPH_MAX_NNZ = ADG_ONE_GRAPH_MAX_NNZ;
constexpr int64_t ONE_GRAPH_MAX_N = 1 << 17;

// Blocks of the UPDATE-sized launches (k_update, k_part1, the pull and DEC
// kernels): as many as the device keeps resident at once, at most
// UPD_BLOCKS.  Each block strides over its share of the rows, so blocks
// beyond what fits would only start once the first ones had finished their
// whole share, and then run with most of the chip idle.  k_update's LDS and
// registers allow 6 blocks per CU on gfx950.  Computed once per process
// (every GPU here is the same device type).
int upd_launch_blocks() {
  static const int blocks = [] {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_update<true>, BS, 0) != hipSuccess || cus <= 0 ||
        per <= 0)
      return UPD_BLOCKS;
    return std::min(UPD_BLOCKS, cus * per);
  }();
  return blocks;
}
#ifndef ADG_JP_GRID_BLOCKS
#define ADG_JP_GRID_BLOCKS 1536
#endif
constexpr int JP_GRID_BLOCKS = ADG_JP_GRID_BLOCKS;   // launch size of the grid-wide JP steps
constexpr int HUGE_BLOCKS = 1024;

// Colour bitmap words: the rows need sum over v of ceil((bits+2)/32), bits =
// |pred(v)| for JP (<= nnz/2 in total) or all non-earlier neighbours for
// DEC-ADG-ITR (<= nnz): at most base = nnz/32 + 33n/32 words.  The
// wavefront pools (pool_alloc) use at most 8/7 of what they hand out plus
// one open chunk per wavefront.
void bm_capacity(int64_t n, int64_t nnz, size_t* cap, size_t* chunk) {
  const unsigned long long base = (unsigned long long)nnz / 32 + 2ull * (unsigned long long)n + 64;
  const unsigned long long waves = (unsigned long long)UPD_BLOCKS * WPB;
  unsigned long long c = base / (8 * waves);
  c = c < 64 ? 64 : c > 8192 ? 8192 : c;
  *chunk = (size_t)c;
  *cap = (size_t)(base + base / 6 + waves * c + 64);
}

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
  L.xpred = take(4 * nn);
  L.nsr = take(4 * nn);
  L.cnt = take(4 * nn);
  L.rec = take(16 * nn);
  bm_capacity(n, nnz, &L.bm_cap, &L.pool_chunk);
  L.B = take(4 * L.bm_cap);
  L.L0 = take(4 * nn);
  L.F0 = take(4 * nn);
  L.F1 = take(4 * nn);
  // fan-out entries: vertices with more than JP_SMALL same-round successors
  // in a level, at most m / JP_SMALL of them
  L.hub_cap = (size_t)nnz / (2 * JP_SMALL) + 64;
  // JP's fan-out lists share their memory with ADG's binned cut-edge targets
  // (at most one per undirected edge and round: m = nnz / 2)
  {
    const size_t sb = (size_t)nnz / 2 + 64;
    const size_t bytes = std::max(16 * L.hub_cap, 4 * sb);
    L.H0 = take(bytes);
    L.H1 = L.H0 + 8 * L.hub_cap;
    L.sb_cap = std::min<size_t>(bytes / 4, 0xffffffffull);
  }
  {
    const size_t nb = ((size_t)n + SUB_SPAN - 1) >> SUB_SHIFT;
    L.SUBC = take(4 * (size_t)SUB_BLOCKS * nb);
    L.SUBS = take(4 * (2 * nb + 2));
  }
  // rows longer than HUGE_DEG in one round: at most nnz / HUGE_DEG
  L.huge_cap = (size_t)nnz / HUGE_DEG + 64;
  L.HL = take(8 * L.huge_cap);
  L.HC = take(4 * 8 * L.huge_cap);
  L.mhist = take(4 * MSEL_BINS);
  L.pool = take(8 * (size_t)UPD_BLOCKS * WPB);
  L.total = off;
  return L;
}

// Sort buffers of adg_order_ex's pos output, after the main layout.
struct OrderLayout {
  size_t keys0, keys1, vals0, vals1, counts, total;
};
OrderLayout make_order_layout(int64_t n, int64_t nnz) {
  OrderLayout O{};
  size_t off = make_layout(n, nnz).total;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + (bytes ? bytes : 1), 256);
    return o;
  };
  const size_t nn = (size_t)n;
  O.keys0 = take(8 * nn);
  O.keys1 = take(8 * nn);
  O.vals0 = take(4 * nn);
  O.vals1 = take(4 * nn);
  O.counts = take(rs::count_bytes());
  O.total = off;
  return O;
}

int check_graph(const adg_csr_t* g) {
  if (!g) return ADG_ERR_ARG;
  if (g->n < 0 || g->n > 0x7ffffffeLL || g->nnz < 0) return ADG_ERR_ARG;
  if (g->n > 0 && (!g->row_ptr)) return ADG_ERR_ARG;
  if (g->nnz > 0 && !g->col_idx) return ADG_ERR_ARG;
  // the colour bitmaps are addressed with 32-bit word offsets
  size_t cap = 0, chunk = 0;
  bm_capacity(g->n, g->nnz, &cap, &chunk);
  if ((unsigned long long)cap + chunk >= (1ull << 32)) return ADG_ERR_UNSUPPORTED;
  return ADG_OK;
}

int check_ws(void* ws, size_t ws_bytes, int64_t n, int64_t nnz) {
  if (!ws) return ADG_ERR_WORKSPACE;
  if (((uintptr_t)ws & 255) != 0) return ADG_ERR_WORKSPACE;
  if (ws_bytes < make_layout(n, nnz).total) return ADG_ERR_WORKSPACE;
  return ADG_OK;
}

Params make_params(const adg_csr_t* g, void* ws, uint64_t p, uint64_t q, uint64_t seed, int fused, int* round_buf,
                   int* color, uint32_t variant = 0) {
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
  P.sorted = (variant & ADG_VARIANT_SORTED) != 0;
  P.median = (variant & ADG_VARIANT_MEDIAN) != 0;
  P.dec = (variant & ADG_VARIANT_DEC_ITR) != 0;
  P.pull = (variant & ADG_VARIANT_PULL) != 0;
  P.mhist = (unsigned*)(base + L.mhist);
  P.tent = (unsigned*)(base + L.F0);   // JP's level lists are not used by DEC-ADG-ITR
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
  P.upd_blocks = upd_launch_blocks();
  P.dag = (int*)(base + L.dag);
  P.xpred = (int*)(base + L.xpred);
  P.nsr = (int*)(base + L.nsr);
  P.cnt = (int*)(base + L.cnt);
  P.rec = (unsigned long long*)(base + L.rec);
  P.B = (unsigned*)(base + L.B);
  P.bm_cap = L.bm_cap;
  P.pool = (unsigned long long*)(base + L.pool);
  P.pool_chunk = (unsigned)L.pool_chunk;
  P.L0 = (unsigned*)(base + L.L0);
  P.F[0] = (unsigned*)(base + L.F0);
  P.F[1] = (unsigned*)(base + L.F1);
  P.H[0] = (unsigned long long*)(base + L.H0);
  P.H[1] = (unsigned long long*)(base + L.H1);
  P.SB = (unsigned*)(base + L.H0);
  P.sb_cap = (unsigned)L.sb_cap;
  P.SUBC = (unsigned*)(base + L.SUBC);
  P.SUBS = (unsigned*)(base + L.SUBS);
  P.binned = ADG_SUB_BINNED && !P.pull && g->n > 0 && g->n <= (int64_t)SUB_MAX_BINS * SUB_SPAN && g->nnz >= SUB_MIN_NNZ;
  P.hub_cap = (unsigned)L.hub_cap;
  P.HL = (unsigned long long*)(base + L.HL);
  P.HC = (unsigned*)(base + L.HC);
  P.huge_cap = (unsigned)L.huge_cap;
  P.color = color;
  P.rmark = (unsigned*)(base + L.UL0);   // ADG's active lists are free once JP starts
  P.rcol = (int*)(base + L.UL1);
  // Round-count bound from the ADG depth lemma: |U| shrinks by a factor
  // 1/(1+eps) per round, so L <= ceil(log n / log(1+eps)) + 1; +1 margin.
  long long bound = (long long)g->n + 1;
  if (p > 0 && g->n > 1) {
    double b = std::ceil(std::log((double)g->n) / std::log1p((double)p / (double)q)) + 2.0;
    if (b < (double)bound) bound = (long long)b;
  }
  if (P.median) {
    // ADG-M removes ceil(|U|/2) vertices per round: L = bit length of n
    bound = 1;
    while ((1LL << bound) <= (long long)g->n) ++bound;
    bound += 1;
  }
  if (bound < 1) bound = 1;
  P.max_rounds = (int)std::min<long long>(bound, 0x7fffffff);
  return P;
}

// Pinned host words through which the host reads the device's loop flags.
// Every entry-point call takes its own from a pool (calls may run
// concurrently from several host threads on different streams) and returns
// it on exit; buffers live until the process ends.
std::mutex g_flag_mu;
std::vector<int*> g_flag_pool;

struct PinnedFlags {
  int* h = nullptr;
  int local[4] = {0, 0, 0, 0};   // pageable words for allocation-free calls
  PinnedFlags() {
    if (t_no_alloc) {
      h = local;
      return;
    }
    {
      std::lock_guard<std::mutex> g(g_flag_mu);
      if (!g_flag_pool.empty()) {
        h = g_flag_pool.back();
        g_flag_pool.pop_back();
        return;
      }
    }
    if (hipHostMalloc((void**)&h, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess) h = nullptr;
  }
  ~PinnedFlags() {
    if (!h || h == local) return;
    std::lock_guard<std::mutex> g(g_flag_mu);
    g_flag_pool.push_back(h);
  }
  PinnedFlags(const PinnedFlags&) = delete;
  PinnedFlags& operator=(const PinnedFlags&) = delete;
};

// ADG's round loop.  Synchronises the stream between chunks of rounds.
int run_adg(Params& P, hipStream_t s, bool fused, int* num_rounds_host) {
  {
    TIMED(KC_INIT, s);
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, s, P);
  }
  HIPCHK(hipGetLastError());
  *num_rounds_host = 0;
  if (P.n == 0) return ADG_OK;
  PinnedFlags pf;
  int* h = pf.h;
  if (!h) return ADG_ERR_HIP;
  int l = 1;
  int chunk = 8;
  // one event pair around the whole round loop (host round trips included)
  ProfScope phase(KC_ADG_PHASE, s);
  while (true) {
    for (int k = 0; k < chunk; ++k, ++l) {
      {
        TIMED(KC_STATS, s);
        hipLaunchKernelGGL(k_stats, dim3(1), dim3(BS), 0, s, P, l);
      }
      if (P.median) {
        TIMED(KC_MSEL, s);
        for (int pass = 0; pass < MSEL_PASSES; ++pass)
          hipLaunchKernelGGL(k_msel, dim3(MSEL_BLOCKS), dim3(BS), 0, s, P, l, pass);
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
      // (with pull UPDATE and no fusion, the push kernels have nothing to do)
      // the binned decrements read the rows' partition: the push kernels then partition even for ADG alone
      const bool part = fused || P.binned;
      if (part || !P.pull) {
        TIMED(KC_UPDATE, s);
        if (part)
          hipLaunchKernelGGL(k_update<true>, dim3(P.upd_blocks), dim3(BS), 0, s, P, l);
        else
          hipLaunchKernelGGL(k_update<false>, dim3(P.upd_blocks), dim3(BS), 0, s, P, l);
      }
      if (part || !P.pull) {
        TIMED(KC_UPDATE_HUGE, s);
        if (part) {
          hipLaunchKernelGGL(k_update_huge_count<true>, dim3(HUGE_BLOCKS), dim3(BS), 0, s, P, l);
          hipLaunchKernelGGL(k_update_huge_place, dim3(HUGE_BLOCKS), dim3(BS), 0, s, P, l);
        } else {
          hipLaunchKernelGGL(k_update_huge_count<false>, dim3(HUGE_BLOCKS), dim3(BS), 0, s, P, l);
        }
      }
      if (P.pull) {
        TIMED(KC_UPDATE_PULL, s);
        hipLaunchKernelGGL(k_update_pull, dim3(P.upd_blocks), dim3(BS), 0, s, P, l);
      }
      if (P.binned) {
        TIMED(KC_UPDATE_SUB, s);
        const int nb = (P.n + SUB_SPAN - 1) >> SUB_SHIFT;
        hipLaunchKernelGGL(k_sub_count, dim3(SUB_BLOCKS), dim3(SUB_BS), 0, s, P);
        hipLaunchKernelGGL(k_sub_scan_bins, dim3((nb + BS - 1) / BS), dim3(BS), 0, s, P);
        hipLaunchKernelGGL(k_sub_scan_total, dim3(1), dim3(SUB_BS), 0, s, P);
        hipLaunchKernelGGL(k_sub_scatter, dim3(SUB_BLOCKS), dim3(SUB_BS), 0, s, P);
        hipLaunchKernelGGL(k_sub_apply, dim3(SUB_APPLY_BLOCKS), dim3(SUB_BS), 0, s, P);
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
    const int blocks = (int)std::max<long long>(1, std::min<long long>(1024, ((long long)P.n + BS - 1) / BS));
    hipLaunchKernelGGL(k_jp_start, dim3(blocks), dim3(BS), 0, s, P, rounds);
  }
  HIPCHK(hipGetLastError());
  PinnedFlags pf;
  int* h = pf.h;
  if (!h) return ADG_ERR_HIP;
  int chunk = 2;
  long long pairs = 0;
  const long long max_pairs = std::min(4LL * ((long long)P.n + rounds + 4), (1LL << 30));
  // steps of one single-block launch: every step processes a level, loads
  // one or starts a round
  const int max_steps = (int)std::min<long long>(0x7fffffff, 3LL * ((long long)P.n + rounds) + 16);
  // grid-wide steps: no more blocks than a step can have work items (a
  // level's groups of 64 vertices plus its fan-out chunks), so that small
  // graphs do not dispatch blocks that leave at once
  const long long items = ((long long)P.n + WAVE - 1) / WAVE + (P.nnz + JP_CHUNK - 1) / JP_CHUNK;
  const int grid = (int)std::max<long long>(1, std::min<long long>(JP_GRID_BLOCKS, (items + WPB - 1) / WPB));
  // one event pair around the whole loop (host round trips between chunks
  // included), standing for the launches issued in it
  {
    ProfScope phase(KC_JP_PHASE, s);
    while (true) {
      for (int k = 0; k < chunk; ++k) {
        {
          TIMED(KC_JP_NARROW, s);
          hipLaunchKernelGGL(k_jp_steps, dim3(STEP_BLOCKS), dim3(NARROW_BS), 0, s, P, max_steps);
        }
        {
          TIMED(KC_JP, s);
          hipLaunchKernelGGL(k_jp_grid, dim3(grid), dim3(BS), 0, s, P);
        }
      }
      pairs += chunk;
      phase.units = 2 * pairs;
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(&h[0], &P.ctrl->js.done, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(&h[1], &P.ctrl->error, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (h[1]) return h[1];   // a device-side check failed (JP stops by itself)
      if (h[0]) break;
      if (pairs > max_pairs) return ADG_ERR_INTERNAL;
      chunk = std::min(chunk * 2, 256);
    }
  }
  {
    TIMED(KC_FINISH, s);
    hipLaunchKernelGGL(k_max_color, dim3(1024), dim3(BS), 0, s, P);
  }
  HIPCHK(hipGetLastError());
  return ADG_OK;
}

// DEC-ADG-ITR over the partitions, issued in growing chunks of (pull, pick,
// resolve) triples; the host reads the finish flag between chunks.  Every
// iteration colours at least the vertex of U with the largest hash, so at
// most n + L triples are needed.
int run_dec(Params& P, hipStream_t s, int rounds) {
  if (P.n == 0) return ADG_OK;
  {
    TIMED(KC_JP_PREP, s);
    hipLaunchKernelGGL(k_dec_start, dim3(1), dim3(64), 0, s, P, rounds);
  }
  HIPCHK(hipGetLastError());
  PinnedFlags pf;
  int* h = pf.h;
  if (!h) return ADG_ERR_HIP;
  int chunk = 4;
  long long triples = 0;
  const long long max_triples = (long long)P.n + rounds + 8;
  {
    ProfScope phase(KC_DEC_PHASE, s);   // as in run_jp
    while (true) {
      for (int k = 0; k < chunk; ++k) {
        TIMED(KC_DEC, s);
        const int p = (int)((triples + k) & 1);
        hipLaunchKernelGGL(k_dec_pull, dim3(P.upd_blocks), dim3(BS), 0, s, P, p);
        hipLaunchKernelGGL(k_dec_pick, dim3(P.upd_blocks), dim3(BS), 0, s, P, p);
        hipLaunchKernelGGL(k_dec_resolve, dim3(P.upd_blocks), dim3(BS), 0, s, P, p);
      }
      triples += chunk;
      phase.units = 3 * triples;
      HIPCHK(hipGetLastError());
      // the state the next triple reads (triples is even here, chunks being even)
      HIPCHK(hipMemcpyAsync(&h[0], &P.ctrl->dec[triples & 1].done, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(&h[1], &P.ctrl->error, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (h[1]) return h[1];
      if (h[0]) break;
      if (triples > max_triples) return ADG_ERR_INTERNAL;
      chunk = std::min(chunk * 2, 256);
    }
  }
  {
    TIMED(KC_FINISH, s);
    hipLaunchKernelGGL(k_max_color, dim3(1024), dim3(BS), 0, s, P);
  }
  HIPCHK(hipGetLastError());
  return ADG_OK;
}

// pos[v] = rank of v in JP's order, by a stable sort of the same-round keys
// and then of the rounds.
int run_order(Params& P, hipStream_t s, int rounds, void* ws, int32_t* pos_out) {
  TIMED(KC_ORDER, s);
  const OrderLayout O = make_order_layout(P.n, P.nnz);
  char* base = (char*)ws;
  uint64_t* keys[2] = {(uint64_t*)(base + O.keys0), (uint64_t*)(base + O.keys1)};
  uint32_t* vals[2] = {(uint32_t*)(base + O.vals0), (uint32_t*)(base + O.vals1)};
  uint32_t* counts = (uint32_t*)(base + O.counts);
  const unsigned blocks = (unsigned)std::min<long long>(((long long)P.n + BS - 1) / BS, 4096);
  hipLaunchKernelGGL(k_order_keys, dim3(blocks), dim3(BS), 0, s, P, (unsigned long long*)keys[0], vals[0]);
  HIPCHK(hipGetLastError());
  int cur = 0;
  HIPCHK(rs::sort_pairs(keys, vals, P.n, 0, P.sorted ? 64 : 32, counts, s, &cur));
  int bits = 0;
  while (bits < 31 && (1 << bits) <= rounds) ++bits;
  hipLaunchKernelGGL(k_order_round_keys, dim3(blocks), dim3(BS), 0, s, P, (unsigned long long*)keys[cur],
                     vals[cur]);
  HIPCHK(hipGetLastError());
  uint64_t* k2[2] = {keys[cur], keys[cur ^ 1]};
  uint32_t* v2[2] = {vals[cur], vals[cur ^ 1]};
  int cur2 = 0;
  HIPCHK(rs::sort_pairs(k2, v2, P.n, 0, bits, counts, s, &cur2));
  hipLaunchKernelGGL(k_order_pos, dim3(blocks), dim3(BS), 0, s, P, v2[cur2], pos_out);
  HIPCHK(hipGetLastError());
  return ADG_OK;
}

// ---- workspace of the allocation-free entry point (color_graph_static)
//
// A file-scope device array: each GPU the library runs on holds one copy
// from the time the library's code is loaded on it until the process ends.
// Host code never passes the array's name to a kernel (on the host it only
// stands for the symbol); it looks up the array's device address once per
// device with hipGetSymbolAddress and passes that address.
constexpr size_t STATIC_SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// The scratch array's address on the current device.
int static_scratch(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return ADG_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p & 255)) return ADG_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ADG_OK;
}

struct NoAllocScope {
  NoAllocScope() { t_no_alloc = true; }
  ~NoAllocScope() { t_no_alloc = false; }
};

}  // namespace

extern "C" {

size_t adg_workspace_bytes(int64_t n, int64_t nnz) {
  if (n < 0 || nnz < 0 || n > 0x7ffffffeLL) return 0;
  return make_layout(n, nnz).total;
}

size_t adg_order_workspace_bytes(int64_t n, int64_t nnz) {
  if (n < 0 || nnz < 0 || n > 0x7ffffffeLL) return 0;
  return make_order_layout(n, nnz).total;
}

int adg_order(const adg_csr_t* g, int32_t eps_num, int32_t eps_den, int32_t* round_out, int32_t* num_rounds_out,
              void* workspace, size_t ws_bytes, void* stream) {
  return adg_order_ex(g, eps_num, eps_den, 0, 0, round_out, nullptr, num_rounds_out, workspace, ws_bytes, stream);
}

int adg_order_ex(const adg_csr_t* g, int32_t eps_num, int32_t eps_den, uint64_t seed, uint32_t variant,
                 int32_t* round_out, int32_t* pos_out, int32_t* num_rounds_out, void* workspace, size_t ws_bytes,
                 void* stream) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (eps_num < 0 || eps_den < 1 || (g->n > 0 && !round_out)) return ADG_ERR_ARG;
  if (variant & ~(uint32_t)(ADG_VARIANT_SORTED | ADG_VARIANT_MEDIAN | ADG_VARIANT_PULL))
    return ADG_ERR_ARG;   // no colouring here
  if ((rc = check_ws(workspace, ws_bytes, g->n, g->nnz))) return rc;
  if (pos_out && ws_bytes < make_order_layout(g->n, g->nnz).total) return ADG_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  Params P = make_params(g, workspace, (uint64_t)eps_num, (uint64_t)eps_den, seed, 0, round_out, nullptr, variant);
  int L = 0;
  if ((rc = run_adg(P, s, false, &L))) return rc;
  if (pos_out && P.n > 0 && (rc = run_order(P, s, L, workspace, pos_out))) return rc;
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
    PinnedFlags pf;
    int* h = pf.h;
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
  return color_graph_ex(g, eps_num, eps_den, seed, 0, color_out, round_out, num_colors_out, num_rounds_out,
                        workspace, ws_bytes, stream);
}

int color_graph_ex(const adg_csr_t* g, int32_t eps_num, int32_t eps_den, uint64_t seed, uint32_t variant,
                   int32_t* color_out, int32_t* round_out, int32_t* num_colors_out, int32_t* num_rounds_out,
                   void* workspace, size_t ws_bytes, void* stream) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (eps_num < 0 || eps_den < 1 || (g->n > 0 && !color_out)) return ADG_ERR_ARG;
  if (variant & ~(uint32_t)(ADG_VARIANT_SORTED | ADG_VARIANT_MEDIAN | ADG_VARIANT_DEC_ITR | ADG_VARIANT_PULL |
                            ADG_VARIANT_MULTI_LAUNCH | ADG_VARIANT_RELAX_ALL | ADG_VARIANT_LEVELS_ONLY))
    return ADG_ERR_ARG;
  const uint32_t sched = variant & (uint32_t)(ADG_VARIANT_RELAX_ALL | ADG_VARIANT_LEVELS_ONLY);
  if (sched == (uint32_t)(ADG_VARIANT_RELAX_ALL | ADG_VARIANT_LEVELS_ONLY) || (sched && (variant & ADG_VARIANT_DEC_ITR)))
    return ADG_ERR_ARG;
  const bool multi = (variant & ADG_VARIANT_MULTI_LAUNCH) != 0 || sched != 0;
  variant &= ~(uint32_t)(ADG_VARIANT_MULTI_LAUNCH | ADG_VARIANT_RELAX_ALL | ADG_VARIANT_LEVELS_ONLY);
  if ((variant & ADG_VARIANT_DEC_ITR) && (variant & ADG_VARIANT_SORTED)) return ADG_ERR_ARG;
  if ((rc = check_ws(workspace, ws_bytes, g->n, g->nnz))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (variant == 0 && !multi && g->n > 0 && g->n <= ONE_GRAPH_MAX_N && g->nnz <= ONE_GRAPH_MAX_NNZ) {
    // a small graph: one launch of the one-workgroup engine instead of
    // several launches per round; the same result, and its counters in
    // this workspace's control block
    const Layout L = make_layout(g->n, g->nnz);
    Ctrl* c = (Ctrl*)((char*)workspace + L.ctrl);
    const StatsSink sink{&c->num_rounds, &c->num_colors, &c->sum_active, &c->cut_edges, &c->js.F, &c->js.levels,
                         &c->error, {&c->dec[0].iters, &c->dec[1].iters}};
    char* rest = (char*)workspace + L.bcount;
    if (one_graph_bytes(g->n, g->nnz) <= ws_bytes - L.bcount)
      return color_one_graph(g->n, g->nnz, g->row_ptr, g->col_idx, eps_num, eps_den, seed, color_out, round_out,
                             num_colors_out, num_rounds_out, rest, ws_bytes - L.bcount, s, sink);
  }
  Params P = make_params(g, workspace, (uint64_t)eps_num, (uint64_t)eps_den, seed, 1, round_out, color_out, variant);
  P.relax_mode = sched == ADG_VARIANT_RELAX_ALL ? RELAX_MODE_ALL : sched == ADG_VARIANT_LEVELS_ONLY ? RELAX_MODE_NONE
                                                                                                     : RELAX_MODE_RULE;
  int L = 0;
  if ((rc = run_adg(P, s, true, &L))) return rc;
  if ((rc = P.dec ? run_dec(P, s, L) : run_jp(P, s, L))) return rc;
  {
    TIMED(KC_FINISH, s);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, P, num_colors_out, num_rounds_out);
  }
  HIPCHK(hipGetLastError());
  return ADG_OK;
}

int color_graph_static(const adg_csr_t* g, int32_t eps_num, int32_t eps_den, uint64_t seed, int32_t* color_out,
                       int32_t* round_out, int32_t* num_colors_out, int32_t* num_rounds_out, void* stream) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (eps_num < 0 || eps_den < 1 || (g->n > 0 && !color_out)) return ADG_ERR_ARG;
  const size_t need = make_layout(g->n, g->nnz).total;
  if (need > STATIC_SCRATCH_BYTES) return ADG_ERR_SCRATCH;
  void* ws = nullptr;
  if ((rc = static_scratch(&ws))) return rc;
  NoAllocScope na;
  return color_graph_ex(g, eps_num, eps_den, seed, 0, color_out, round_out, num_colors_out, num_rounds_out, ws,
                        STATIC_SCRATCH_BYTES, stream);
}

size_t adg_static_scratch_bytes(void) { return STATIC_SCRATCH_BYTES; }

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
  out->frontier = (int64_t)h.js.F;
  out->jp_levels = h.js.levels + std::max(h.dec[0].iters, h.dec[1].iters);
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
      out->launches[r.cls] += r.units;
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
    case ADG_ERR_SCRATCH: return "graph too large for the allocation-free entry point's static scratch";
    default: return "unknown error";
  }
}

}  // extern "C"
