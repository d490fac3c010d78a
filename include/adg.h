/*
 * adg.h -- C ABI of libadg_hip.so: approximate degeneracy ordering (ADG) and
 * Jones-Plassmann colouring under the ADG order (JP-ADG) on AMD MI355X
 * (gfx950).
 *
 * Method: Besta et al., "High-Performance Parallel Graph Coloring with Strong
 * Guarantees on Work, Depth, and Quality" (SC 2020, arXiv 2008.11321).
 *   - adg_order:   ADG, Algorithm 1 ("Parallel Approximate Degeneracy
 *                  Ordering").
 *   - jp_color:    JP, Algorithm 3, with priority rho = <rho_ADG, rho_R>
 *                  ("Graph Coloring by Color Scheduling (JP-ADG)").
 *   - color_graph: JP-ADG end to end, with JP's Part 1 (the DAG G_rho: pred /
 *                  succ sets and |pred|) fused into ADG's UPDATE, the
 *                  "Combining JP and ADG" optimisation of the section
 *                  "Optimizations and Implementation".
 *   - color_graph_batched: JP-ADG on many independent graphs in one
 *                  persistent launch, each graph coloured exactly as alone.
 *   - adg_server_*: a serving loop with continuous batching over a device
 *                  arena.
 *
 * Conventions shared by every entry point:
 *   - Graphs are simple and undirected (symmetric adjacency, no self-loops,
 *     no duplicate entries) in CSR: row_ptr[n+1] (int64, row_ptr[0] = 0,
 *     non-decreasing, row_ptr[n] = nnz) and col_idx[nnz] (int32 in [0, n)).
 *     Vertices are numbered 0..n-1.  Row order inside a row is free: results
 *     do not depend on it.  Preconditions are not checked by the compute
 *     calls; adg_validate_csr checks them.
 *   - eps = eps_num / eps_den with eps_num >= 0, eps_den >= 1.  A vertex u
 *     is removed in an ADG round when D[u] <= (1 + eps) * avg, evaluated
 *     exactly in integers (no floating point anywhere).
 *   - Rounds are numbered 1..L.  A higher round means a higher JP priority
 *     (peeled later, coloured earlier).  Ties inside a round are broken by
 *     rho_R(v) = fmix32(v XOR k), k = low 32 bits of the first SplitMix64
 *     output from state `seed` (larger wins); fmix32 is the MurmurHash3
 *     finaliser, a bijection, so the order is total.
 *   - Colours are 1-based; num_colors = max colour (0 for an empty graph).
 *   - Every array argument is a DEVICE pointer owned by the caller; the
 *     library never allocates device memory.  Scratch space is the
 *     caller-provided workspace of at least *_workspace_bytes() bytes,
 *     256-byte aligned; its contents on entry are ignored.
 *   - Calls are issued on `stream` (a hipStream_t; NULL = default stream).
 *     The single-graph calls (adg_order, jp_color, color_graph and their _ex
 *     forms) cannot know in advance how many ADG rounds or JP levels a graph
 *     needs, so they read a finish flag from the device between chunks of
 *     launches (except color_graph on a graph small enough for the
 *     one-launch engine, see ADG_VARIANT_MULTI_LAUNCH, which never waits): they block the calling thread on hipStreamSynchronize(stream)
 *     several times (ADG: after 8 rounds, then after chunks of 16, 32, 64;
 *     JP: after chunks of 2, 4, ..., 256 kernel pairs; jp_color also once
 *     after building the DAG) and return once those loops have ended on the
 *     device.  The last kernels (num_colors, the scalar outputs, the pos
 *     sort) are still queued when they return: outputs are valid once the
 *     stream is synchronised.  Because of the waits these calls cannot be
 *     recorded into a HIP graph.  color_graph_batched never waits and can
 *     be captured; adg_get_stats and adg_validate_csr are synchronous.
 *   - Return value: ADG_OK (0) or a negative ADG_ERR_* code; no exception
 *     crosses the ABI.  adg_error_string() names a code.
 */
#ifndef ADG_H_
#define ADG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ADG_OK = 0,
  ADG_ERR_ARG = -1,         /* null pointer, negative size, bad eps, n >= 2^31 */
  ADG_ERR_WORKSPACE = -2,   /* workspace missing, misaligned or too small */
  ADG_ERR_HIP = -3,         /* a HIP runtime call failed */
  ADG_ERR_INTERNAL = -4,    /* round-count watchdog tripped or device-side check failed */
  ADG_ERR_UNSUPPORTED = -5, /* input outside the supported range: nnz / 32 + 2 n >= 2^32 for the
                               single-graph calls; a serving request larger than the arena */
  ADG_ERR_SCRATCH = -6      /* color_graph_static: the graph needs more workspace than the
                               library's static scratch (adg_static_scratch_bytes) */
};

/* CSR view of one graph; all pointers are device pointers. */
typedef struct adg_csr {
  int64_t n;               /* number of vertices, 0 <= n < 2^31 */
  int64_t nnz;             /* number of directed entries = 2m */
  const int64_t* row_ptr;  /* [n+1] */
  const int32_t* col_idx;  /* [nnz] */
} adg_csr_t;

/* Counters of the last call on a workspace, read back by adg_get_stats. */
typedef struct adg_stats {
  int64_t num_rounds;      /* L */
  int64_t num_colors;      /* max colour (0 if JP did not run) */
  int64_t sum_active;      /* sum over rounds of |U_l| */
  int64_t cut_edges;       /* decrements that hit a vertex staying in U */
  int64_t frontier;        /* vertices that started a JP level (all preds done) */
  int64_t jp_levels;       /* JP levels processed, summed over rounds; with
                              ADG_VARIANT_DEC_ITR the DEC-ADG-ITR iterations */
  int64_t error;           /* device-side error flag (0 = none) */
} adg_stats_t;

/* Workspace size in bytes for adg_order / jp_color / color_graph on a graph
 * with n vertices and nnz entries.  Returns 0 for invalid sizes. */
size_t adg_workspace_bytes(int64_t n, int64_t nnz);

/* ADG (Algorithm 1).  Writes round_out[v] in 1..L for every vertex and L to
 * num_rounds_out[0] (device int32).  Each round l: |U| and the degree sum
 * over U give the average; R = {u in U : D[u] <= (1+eps) avg}; every v in R
 * gets round l; D[w] is decremented once for every edge between R and U \ R.
 * Errors: ADG_ERR_ARG, ADG_ERR_WORKSPACE, ADG_ERR_HIP, ADG_ERR_INTERNAL
 * (round count above n or above ceil(log n / log(1+eps)) + 2). */
int adg_order(const adg_csr_t* g, int32_t eps_num, int32_t eps_den, int32_t* round_out,
              int32_t* num_rounds_out, void* workspace, size_t ws_bytes, void* stream);

/* JP (Algorithm 3) under rho = <round[v], rho_R(v)>.  round[] may be any
 * positive int32 ranking (normally adg_order's output).  Writes
 * color_out[v] >= 1 and num_colors_out[0] (device int32).  The colouring
 * equals sequential greedy colouring in decreasing priority order: each v
 * gets the smallest colour not used by its higher-priority neighbours.
 * Errors: ADG_ERR_ARG, ADG_ERR_WORKSPACE, ADG_ERR_HIP. */
int jp_color(const adg_csr_t* g, const int32_t* round, uint64_t seed, int32_t* color_out,
             int32_t* num_colors_out, void* workspace, size_t ws_bytes, void* stream);

/* JP-ADG: adg_order then jp_color, with JP Part 1 fused into ADG's update.
 * round_out and num_rounds_out may be NULL (then ADG's rounds are kept in the
 * workspace only).  Results are identical to adg_order followed by jp_color.
 * Errors: as adg_order and jp_color. */
int color_graph(const adg_csr_t* g, int32_t eps_num, int32_t eps_den, uint64_t seed,
                int32_t* color_out, int32_t* round_out, int32_t* num_colors_out,
                int32_t* num_rounds_out, void* workspace, size_t ws_bytes, void* stream);

/* ---- Variants of ADG (the _ex entry points).
 *
 * variant is a bit set:
 *   ADG_VARIANT_SORTED  ADG-O (the ADG-O listing of "Detailed Algorithm
 *       Specifications", the variant the evaluation runs): the rounds are
 *       Algorithm 1's; inside a round the order is increasing D at selection
 *       (= the degree in G[U] when the round starts), equal D by rho_R.  JP
 *       colours by this total order: larger (round, D, rho_R) first.
 *   ADG_VARIANT_MEDIAN  ADG-M (section "Degree Median Instead of Degree
 *       Average"): R is the ceil(|U|/2) vertices of U lowest by (D, rho_R).
 *       This is the paper's R = {D <= (1+eps) median} limited to half of U:
 *       at least ceil(|U|/2) vertices satisfy the bound for every eps >= 0,
 *       so the limit always decides and eps has no effect.  L is the bit
 *       length of n; JP-ADG-M uses at most 4d + 1 colours.  The tie-break
 *       seed decides which vertices of equal D fall in the lower half.
 *   ADG_VARIANT_DEC_ITR  (color_graph_ex only) colour by DEC-ADG-ITR (section
 *       "Enhancing Existing Coloring Algorithms") instead of JP: the ADG
 *       partitions R(L), ..., R(1) are coloured one after the other (the
 *       DEC-ADG listing's outer loop); inside R(l), synchronous iterations
 *       of the SIM-COL listing where every uncoloured vertex tries the
 *       smallest colour not used by its coloured neighbours, keeps it
 *       unless an uncoloured neighbour of R(l) with a larger rho_R tried
 *       the same colour, and the kept colours are final.  Deterministic for
 *       a given seed; at most 2(1+eps)d + 1 colours.  May be combined with
 *       ADG_VARIANT_MEDIAN, not with ADG_VARIANT_SORTED.
 *   ADG_VARIANT_PULL  UPDATE pulls instead of pushing (section "Using Only
 *       Concurrent Reads", and "Push vs. Pull"): every vertex that stays in U
 *       subtracts from its own D the number of its neighbours in R, so no
 *       atomics touch D; the rows of the remaining vertices are read every
 *       round.  The output is identical to pushing.  Combines with all.
 *   ADG_VARIANT_MULTI_LAUNCH  (color_graph_ex only) color_graph hands a graph
 *       with at most 2^17 entries and vertices to the one-launch engine of
 *       color_graph_batched (one workgroup colours it, in one launch and
 *       without waiting on the stream); this bit keeps such a graph on the
 *       per-round kernels.  The output is the same either way.
 *   ADG_VARIANT_RELAX_ALL, ADG_VARIANT_LEVELS_ONLY  (color_graph_ex only,
 *       not with ADG_VARIANT_DEC_ITR, not together; each keeps every graph
 *       on the per-round kernels) how JP schedules each round.  JP colours a
 *       round level by level (Algorithm 3's waves inside the round); by
 *       default, once a round of at least 2048 vertices has run 8 levels
 *       that colour 3 or more vertices each on average, with a quarter of
 *       the round still uncoloured, its other vertices are relaxed instead:
 *       every uncoloured vertex repeatedly takes the smallest colour that
 *       neither its later-round predecessors nor its current same-round
 *       predecessors have, until no colour changes.  The same-round DAG is
 *       acyclic, so these equations have one solution, which is JP's
 *       colouring: the output is the same under every schedule.
 *       RELAX_ALL relaxes every round from its start; LEVELS_ONLY never
 *       relaxes.
 * SORTED and MEDIAN may be combined.  variant = 0 is Algorithm 1 (adg_order,
 * color_graph).  Other bits or combinations: ADG_ERR_ARG. */
enum {
  ADG_VARIANT_SORTED = 1,
  ADG_VARIANT_MEDIAN = 2,
  ADG_VARIANT_DEC_ITR = 4,
  ADG_VARIANT_PULL = 8,
  ADG_VARIANT_MULTI_LAUNCH = 16,
  ADG_VARIANT_RELAX_ALL = 32,
  ADG_VARIANT_LEVELS_ONLY = 64
};

/* Workspace bytes for adg_order_ex with a pos output (adg_workspace_bytes
 * plus sort buffers of 24 n bytes); 0 for invalid sizes. */
size_t adg_order_workspace_bytes(int64_t n, int64_t nnz);

/* ADG with a variant.  round_out[v] in 1..L as adg_order; pos_out (device
 * int32[n], may be NULL) receives the total order JP colours by as ranks
 * 0..n-1 (larger = coloured first): rounds increasing, inside a round
 * increasing (D at selection, rho_R) with ADG_VARIANT_SORTED -- that is
 * ADG-O's rho, "rho(r_i) = l + i" -- else increasing rho_R(v) = the 32-bit
 * hash of v under seed.  seed matters for pos and for ADG_VARIANT_MEDIAN.
 * With pos_out, ws_bytes must be at least adg_order_workspace_bytes.
 * Errors: as adg_order. */
int adg_order_ex(const adg_csr_t* g, int32_t eps_num, int32_t eps_den, uint64_t seed, uint32_t variant,
                 int32_t* round_out, int32_t* pos_out, int32_t* num_rounds_out, void* workspace,
                 size_t ws_bytes, void* stream);

/* JP-ADG with a variant: JP (Algorithm 3) under the total order pos of
 * adg_order_ex, with JP Part 1 fused into the update as color_graph.
 * variant = 0 is color_graph.  Errors: as color_graph. */
int color_graph_ex(const adg_csr_t* g, int32_t eps_num, int32_t eps_den, uint64_t seed, uint32_t variant,
                   int32_t* color_out, int32_t* round_out, int32_t* num_colors_out,
                   int32_t* num_rounds_out, void* workspace, size_t ws_bytes, void* stream);

/* ---- Allocation-free JP-ADG, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).
 *
 * Computes exactly what color_graph computes, with the same arguments except
 * the workspace: the library's own static device array of
 * adg_static_scratch_bytes() bytes (128 MiB) serves as the workspace.  Each
 * GPU the library runs on holds one such array from when the library's code
 * is loaded on it until the process ends.  The call makes no device or host
 * memory allocation (hipMalloc, hipHostMalloc, or any allocating library
 * routine), records no profiling events, and reads the loop flags through
 * pageable memory on the calling thread's stack; it synchronises the stream
 * as color_graph does.  The caller still owns and passes every output.
 *
 * The array keeps the last call's contents; nothing in it is assumed on
 * entry.  Calls that overlap on one GPU -- from several threads or streams
 * -- share the array and race: serialise them.  A graph whose workspace
 * (adg_workspace_bytes(n, nnz)) exceeds the array returns ADG_ERR_SCRATCH
 * before any device work.  Other errors: as color_graph. */
int color_graph_static(const adg_csr_t* g, int32_t eps_num, int32_t eps_den, uint64_t seed,
                       int32_t* color_out, int32_t* round_out, int32_t* num_colors_out,
                       int32_t* num_rounds_out, void* stream);

/* Bytes of color_graph_static's static scratch (the largest workspace it takes). */
size_t adg_static_scratch_bytes(void);

/* ---- Many independent graphs in one call.
 *
 * The batch is one concatenated CSR: graph g owns global vertex slots
 * vtx_off[g] .. vtx_off[g+1]-1 and the entries row_ptr[vtx_off[g]] ..
 * row_ptr[vtx_off[g+1]]-1 of col_idx; row_ptr holds ABSOLUTE offsets into
 * col_idx, and col_idx holds LOCAL vertex ids (0 .. n_g - 1).  Each graph is
 * coloured exactly as a standalone color_graph call on it would colour it
 * (same eps, same seed, local ids): ADG's average degree is per graph, since
 * ADG on the disjoint union would select different rounds (Algorithm 1 takes
 * the average over the whole remaining graph). */
typedef struct adg_batch {
  int32_t num_graphs;      /* G >= 0 */
  int64_t total_n;         /* vtx_off[G] (host copy), < 2^31 */
  int64_t total_nnz;       /* row_ptr[total_n] (host copy) */
  const int64_t* vtx_off;  /* device [G+1], non-decreasing, vtx_off[0] = 0 */
  const int64_t* row_ptr;  /* device [total_n+1], absolute */
  const int32_t* col_idx;  /* device [total_nnz], local ids */
} adg_batch_t;

/* Launch shape of the persistent batched kernel: threads per workgroup
 * (256, 512 or 1024), resident workgroups per compute unit (1..32, with
 * block_threads * blocks_per_cu <= 2048 to be useful), and the order in which
 * workgroups take graphs (ADG_SCHED_LPT: largest work class first;
 * ADG_SCHED_NATURAL: batch order).  Results do not depend on it. */
enum { ADG_SCHED_LPT = 0, ADG_SCHED_NATURAL = 1 };
typedef struct adg_batch_config {
  int32_t block_threads;
  int32_t blocks_per_cu;
  int32_t schedule;
} adg_batch_config_t;

/* Workspace bytes for color_graph_batched; 0 for invalid sizes. */
size_t adg_batched_workspace_bytes(int32_t num_graphs, int64_t total_n, int64_t total_nnz);

/* The launch shape used when color_graph_batched gets config = NULL. */
adg_batch_config_t adg_batched_default_config(void);

/* JP-ADG (Algorithms 1 and 3, as color_graph) on every graph of the batch, in
 * one persistent launch: each workgroup colours whole graphs, one after the
 * other, taking them from a device-side queue.  Writes color_out[total_n]
 * (colour of local vertex v of graph g at vtx_off[g] + v), round_out[total_n]
 * (nullable), num_colors_out[G] and num_rounds_out[G] (nullable), all device
 * int32.  config may be NULL.  Fully asynchronous: no host synchronisation,
 * no memset, so the call can be recorded by stream capture.  Device-side
 * errors (a broken DAG, a round-count overrun) are reported by
 * adg_batched_get_stats.  Errors returned: ADG_ERR_ARG, ADG_ERR_WORKSPACE,
 * ADG_ERR_HIP. */
int color_graph_batched(const adg_batch_t* b, int32_t eps_num, int32_t eps_den, uint64_t seed,
                        int32_t* color_out, int32_t* round_out, int32_t* num_colors_out,
                        int32_t* num_rounds_out, const adg_batch_config_t* config, void* workspace,
                        size_t ws_bytes, void* stream);

/* Counters of the last color_graph_batched call on this workspace, summed
 * over the batch (num_rounds and num_colors: the largest of any graph;
 * frontier: vertices of JP's first level; error: the device-side error flag,
 * 0 = none, else an ADG_ERR_* code -- a broken DAG or a round-count
 * overrun).  Synchronises `stream`. */
int adg_batched_get_stats(const void* workspace, size_t ws_bytes, adg_stats_t* host_out, void* stream);

/* Launch-shape autotuner: runs color_graph_batched on this batch once per
 * candidate shape (block_threads x blocks_per_cu, then the schedule order for
 * the best), times each with HIP events on `stream`, and writes the fastest
 * to *best_out (and its time to *best_ms_out, nullable).  The outputs hold a
 * valid result afterwards.  The choice is cached per batch shape class
 * (G, and total_n, total_nnz rounded to powers of two) for later calls with
 * `reuse` != 0.  Synchronises `stream`. */
int adg_batched_autotune(const adg_batch_t* b, int32_t eps_num, int32_t eps_den, uint64_t seed,
                         int32_t* color_out, int32_t* num_colors_out, void* workspace, size_t ws_bytes,
                         void* stream, int32_t reuse, adg_batch_config_t* best_out, float* best_ms_out);

/* ---- Serving: a request loop with continuous batching.
 *
 * The server colours independent graphs submitted from the host (CSR in host
 * memory) with JP-ADG, each exactly as a standalone color_graph call would.
 * Requests wait in arrival order; an idle worker admits the next job that
 * fits into the device arena: a large request (nnz > small_nnz) alone, or a
 * group of up to max_group consecutive small requests packed into one
 * color_graph_batched launch.  Each worker has its own stream (default
 * priority), so jobs admitted while others run overlap on the device; arena
 * space and workers come free as jobs complete.  The oldest waiting request
 * may be overtaken by later, smaller ones at most max_bypass times.  The
 * arena is one caller-owned device buffer (256-byte aligned); the server
 * never allocates device memory. */
typedef struct adg_server adg_server_t;
typedef struct adg_server_config {
  int32_t eps_num, eps_den;  /* eps = eps_num / eps_den for every request */
  uint64_t seed;             /* tie-break seed for every request */
  int32_t workers;           /* concurrent jobs (host threads, one stream each), 1..16 */
  int64_t small_nnz;         /* requests with nnz <= small_nnz are grouped */
  int32_t max_group;         /* requests per grouped launch, >= 1 */
  int32_t max_bypass;        /* overtakes of the oldest waiting request, >= 0 */
} adg_server_config_t;
typedef struct adg_request_result {
  uint64_t tag;              /* as submitted */
  int32_t status;            /* ADG_OK or an ADG_ERR_* code */
  int32_t num_colors, num_rounds;
  int32_t group_size;        /* requests in the launch that coloured it */
  int64_t n, nnz;
  double t_submit, t_admit, t_start, t_done;  /* adg_server_clock() seconds */
} adg_request_result_t;

adg_server_config_t adg_server_default_config(void);
/* Arena bytes a request of this size needs on its own (0 for bad sizes). */
size_t adg_server_footprint(const adg_server_config_t* cfg, int64_t n, int64_t nnz);
/* Start a server on the current device.  Errors: ADG_ERR_ARG, ADG_ERR_HIP. */
int adg_server_create(const adg_server_config_t* cfg, void* arena, size_t arena_bytes, adg_server_t** out);
/* Queue one graph.  row_ptr[n+1], col_idx[nnz] and color_out[n] are HOST
 * arrays that must stay valid until the request's result has been polled;
 * color_out receives the colours.  Errors: ADG_ERR_ARG (bad sizes, row_ptr
 * not spanning [0, nnz], server stopping), ADG_ERR_UNSUPPORTED (footprint
 * larger than the whole arena). */
int adg_server_submit(adg_server_t* s, int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                      int32_t* color_out, uint64_t tag);
/* Move up to max_results finished requests to out (waiting up to wait_ms
 * for the first); *count_out = number moved. */
int adg_server_poll(adg_server_t* s, adg_request_result_t* out, int32_t max_results, int32_t wait_ms,
                    int32_t* count_out);
/* Requests submitted and not yet polled (-1 for a null server). */
int64_t adg_server_in_flight(adg_server_t* s);
/* The steady clock the result times use, in seconds. */
double adg_server_clock(void);
/* Totals over the server's successfully finished jobs. */
typedef struct adg_server_counters {
  int64_t single_jobs;       /* requests coloured by color_graph alone */
  int64_t grouped_jobs;      /* color_graph_batched launches */
  int64_t grouped_requests;  /* requests coloured in them */
  int64_t vertices, entries; /* sum of n and of nnz */
  int64_t sum_active;        /* sum over requests and ADG rounds of |U_l| */
  int64_t cut_edges;         /* sum of ADG's degree decrements */
} adg_server_counters_t;
int adg_server_get_counters(adg_server_t* s, adg_server_counters_t* out);
/* Finish every queued request, stop the workers and free the server (results
 * not polled are dropped). */
int adg_server_destroy(adg_server_t* s);

/* Copy the counters of the last adg_order / jp_color / color_graph call on
 * this workspace to host memory.  Synchronises `stream`. */
int adg_get_stats(const void* workspace, size_t ws_bytes, adg_stats_t* host_out, void* stream);

/* Check that g is a simple undirected graph in CSR form: row_ptr monotone
 * with row_ptr[0] = 0 and row_ptr[n] = nnz, col_idx in range, no self-loop,
 * no duplicate entry, symmetric.  Needs rows sorted by neighbour id to check
 * duplicates and symmetry (binary search).  Returns ADG_OK, ADG_ERR_ARG if a
 * check fails, or another error code.  Synchronises `stream`. */
int adg_validate_csr(const adg_csr_t* g, void* workspace, size_t ws_bytes, void* stream);

/* Optional timing of the library's own kernels, for measurement tools.
 * adg_profile_enable(mask) makes every later launch of a kernel class whose
 * bit is set in `mask` (classes: 0 init, 1 stats, 2 count, 3 scan,
 * 4 scatter, 5 update, 6 part1, 7 jp_prep, 8 jp (grid-wide JP steps),
 * 9 finish, 10 batched, 11 jp_narrow (single-block JP steps), 12 update_huge
 * (UPDATE of rows longer than 16384 entries, cut into chunks), 13
 * median_select (ADG-M), 14 order_sort (adg_order_ex's pos), 15 dec_itr
 * (DEC-ADG-ITR triples), 16 update_pull, 17 jp_phase, 18 dec_phase)
 * record a pair of HIP events on its launch stream; 0 disables it.  The two
 * phase classes put one pair around a call's whole JP (or DEC-ADG-ITR) loop,
 * host round trips between its chunks included, and count it as the number
 * of kernel launches issued in the loop: two events per call instead of two
 * per launch, whose host cost would slow a loop of thousands of short
 * launches.
 * adg_profile_read waits for the recorded events, adds up the elapsed time
 * and launch count per class into *out and forgets the records.  Process-wide,
 * guarded by a mutex. */
#define ADG_PROFILE_CLASSES 32
typedef struct adg_profile {
  double ms[ADG_PROFILE_CLASSES];
  int64_t launches[ADG_PROFILE_CLASSES];
} adg_profile_t;
int adg_profile_enable(uint32_t class_mask);
int adg_profile_read(adg_profile_t* out);
const char* adg_kernel_class_name(int cls);

/* Human-readable name of an ADG_* code (static string). */
const char* adg_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* ADG_H_ */
