// Host-side helpers shared by the single-graph and batched entry points:
// kernel-class timing with HIP events, the tie-break key derivation and the
// HIP error check.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace adg {

enum KClass {
  KC_INIT, KC_STATS, KC_COUNT, KC_SCAN, KC_SCATTER, KC_UPDATE, KC_PART1, KC_JP_PREP, KC_JP, KC_FINISH,
  KC_BATCH, KC_JP_NARROW, KC_UPDATE_HUGE, KC_MSEL, KC_ORDER, KC_DEC, KC_UPDATE_PULL, KC_JP_PHASE, KC_DEC_PHASE,
  KC_ADG_PHASE, KC_UPDATE_SUB, KC_NUM
};

// Event pair around one launch of class `cls` (or around a loop of
// `units` launches), recorded only while that class is enabled by
// adg_profile_enable.
hipEvent_t prof_begin(int cls, hipStream_t s);
void prof_end(int cls, hipStream_t s, hipEvent_t a, long long units);

struct ProfScope {
  int cls;
  hipStream_t s;
  hipEvent_t a;
  long long units = 1;   // launches the pair stands for
  ProfScope(int c, hipStream_t st) : cls(c), s(st), a(prof_begin(c, st)) {}
  ~ProfScope() {
    if (a) prof_end(cls, s, a, units);
  }
};
#define ADG_TIMED_CAT2(a, b) a##b
#define ADG_TIMED_CAT(a, b) ADG_TIMED_CAT2(a, b)
#define TIMED(cls, s) ::adg::ProfScope ADG_TIMED_CAT(prof_scope_, __LINE__)(cls, s)

// rho_R's key: the low 32 bits of the first SplitMix64 output from state
// `seed` (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014).
inline uint32_t hash_key_from_seed(uint64_t seed) {
  uint64_t z = seed + 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  z ^= z >> 31;
  return (uint32_t)z;
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Where the one-launch engine leaves a single graph's counters when it
// serves a color_graph call (device pointers into that call's control
// block; every field is written).
struct StatsSink {
  int* num_rounds;
  int* num_colors;
  unsigned long long* sum_active;
  unsigned long long* cut_edges;
  unsigned long long* frontier;
  int* levels;
  int* error;
  long long* zero64[2];   // counters of other colourings, cleared
};

// JP-ADG on one graph by the one-launch engine of color_graph_batched (one
// workgroup colours it; same result as the single-graph kernels).  ws holds
// one_graph_bytes(n, nnz), 256-byte aligned.
size_t one_graph_bytes(int64_t n, int64_t nnz);
int color_one_graph(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx, int32_t eps_num,
                    int32_t eps_den, uint64_t seed, int32_t* color_out, int32_t* round_out, int32_t* num_colors_out,
                    int32_t* num_rounds_out, void* ws, size_t ws_bytes, hipStream_t s, const StatsSink& sink);

#define HIPCHK(x)                              \
  do {                                         \
    if ((x) != hipSuccess) return ADG_ERR_HIP; \
  } while (0)

}  // namespace adg
