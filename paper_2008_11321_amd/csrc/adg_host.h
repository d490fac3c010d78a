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
  KC_ADG_PHASE, KC_NUM
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

#define HIPCHK(x)                              \
  do {                                         \
    if ((x) != hipSuccess) return ADG_ERR_HIP; \
  } while (0)

}  // namespace adg
