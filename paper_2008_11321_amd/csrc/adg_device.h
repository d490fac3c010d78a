// Device-side building blocks shared by the single-graph and batched paths:
// wavefront (64-lane) primitives, the JP tie-break hash and the per-vertex
// JP synchronisation word.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adg_intmath.h"

namespace adg {

constexpr int WAVE = 64;

__device__ __forceinline__ unsigned lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// Number of set bits of `mask` at lanes below the calling lane.
__device__ __forceinline__ unsigned lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int readlane_i(int x, int lane) { return __builtin_amdgcn_readlane(x, lane); }
__device__ __forceinline__ unsigned readlane_u(unsigned x, int lane) {
  return (unsigned)__builtin_amdgcn_readlane((int)x, lane);
}
__device__ __forceinline__ int64_t readlane_i64(int64_t x, int lane) {
  unsigned lo = readlane_u((unsigned)(uint64_t)x, lane);
  unsigned hi = readlane_u((unsigned)((uint64_t)x >> 32), lane);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, int lane) {
  unsigned lo = readlane_u((unsigned)x, lane);
  unsigned hi = readlane_u((unsigned)(x >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

// DPP move of a 32- or 64-bit value from the lane that CTRL selects (row and
// bank masks as in the DPP encoding); a lane whose source lies outside its
// row of 16, or is masked off, gets `old`.
template <int CTRL, int ROW, int BANK, typename T>
__device__ __forceinline__ T dpp_move(T v, T old) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v),
                                                             CTRL, ROW, BANK, false));
  } else {
    const uint64_t x = __builtin_bit_cast(uint64_t, v), o = __builtin_bit_cast(uint64_t, old);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)x, CTRL, ROW, BANK, false);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(x >> 32), CTRL, ROW, BANK, false);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}

// Inclusive scan over the 64 lanes with the associative operation `op`, by
// DPP moves (no LDS round trip): each lane combines lanes i-3 .. i of its row
// of 16, then i-7 .. i and i-15 .. i (row shifts by 4 and 8), then rows 1
// and 3 take the total of the row before them (row broadcast of lane 15) and
// rows 2 and 3 the total of rows 0-1 (row broadcast of lane 31).  Lanes with
// no source take `id`: the operation's identity for sums, or the lane's own
// value when op(v, v) == v (max, min).
template <bool IDEMPOTENT, typename T, typename Op>
__device__ __forceinline__ T wave_incl_scan(T x, Op op) {
  const T z = IDEMPOTENT ? x : T(0);
  T v = op(op(x, dpp_move<0x111, 0xf, 0xf>(x, z)), op(dpp_move<0x112, 0xf, 0xf>(x, z), dpp_move<0x113, 0xf, 0xf>(x, z)));
  v = op(v, dpp_move<0x114, 0xf, 0xe>(v, IDEMPOTENT ? v : T(0)));   // row_shr:4, lanes 4-15 of a row
  v = op(v, dpp_move<0x118, 0xf, 0xc>(v, IDEMPOTENT ? v : T(0)));   // row_shr:8, lanes 8-15 of a row
  v = op(v, dpp_move<0x142, 0xa, 0xf>(v, IDEMPOTENT ? v : T(0)));   // row_bcast:15 into rows 1 and 3
  v = op(v, dpp_move<0x143, 0xc, 0xf>(v, IDEMPOTENT ? v : T(0)));   // row_bcast:31 into rows 2 and 3
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_lane63(T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), WAVE - 1));
  } else {
    return __builtin_bit_cast(T, readlane_u64(__builtin_bit_cast(uint64_t, v), WAVE - 1));
  }
}
struct OpAdd {
  template <typename T>
  __device__ T operator()(T a, T b) const { return a + b; }
};
struct OpMax {
  template <typename T>
  __device__ T operator()(T a, T b) const { return a > b ? a : b; }
};
struct OpMin {
  template <typename T>
  __device__ T operator()(T a, T b) const { return a < b ? a : b; }
};
__device__ __forceinline__ unsigned wave_incl_scan_u32(unsigned x) { return wave_incl_scan<false>(x, OpAdd()); }
// Wave-wide sum, max and min (every lane receives the result).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) { return wave_lane63(wave_incl_scan<false>(v, OpAdd())); }
template <typename T>
__device__ __forceinline__ T wave_max(T v) { return wave_lane63(wave_incl_scan<true>(v, OpMax())); }
template <typename T>
__device__ __forceinline__ T wave_min(T v) { return wave_lane63(wave_incl_scan<true>(v, OpMin())); }

// rho_R, the random tie-break inside an ADG round: MurmurHash3's 32-bit
// finaliser applied to (v XOR key).  Each step is invertible modulo 2^32, so
// distinct vertices never tie.
__device__ __forceinline__ uint32_t tiebreak(uint32_t key, uint32_t v) {
  uint32_t h = v ^ key;
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// JP synchronisation word, one per vertex (64 bits):
//   bits  0..39  forbidden-colour mask: bit c-1 set <=> some coloured
//                predecessor has colour c (c = 1..40)
//   bits 40..63  number of predecessors not yet coloured (JP's count[v])
// A predecessor of colour c <= 40 first ORs bit c-1 into the word, then
// subtracts one count unit from the same word.  Both touch one location, so
// whoever observes the count reach zero also observes every predecessor's
// bit: the last decrementer receives the complete mask in the atomic's
// return value and can compute the vertex's colour without reading any
// other memory.
constexpr int JP_MASK_BITS = 40;
constexpr uint64_t JP_MASK = (uint64_t(1) << JP_MASK_BITS) - 1;
constexpr uint64_t JP_ONE = uint64_t(1) << JP_MASK_BITS;
constexpr int64_t JP_MAX_PRED = (int64_t(1) << (64 - JP_MASK_BITS)) - 1;

__device__ __forceinline__ unsigned long long agent_load_u64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int agent_load_i32(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned agent_load_u32(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void agent_store_i32(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void agent_store_u64(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Ordering point for the JP worklist: wait until every memory operation this
// wavefront has issued has completed, and keep the compiler from moving memory
// accesses across the point.  All data that JP wavefronts exchange is accessed
// with device-coherent atomics (read-modify-writes, and loads/stores at agent
// scope), which the hardware performs at the device's coherence point; a
// completed one is visible to every later device-coherent access.  Waiting for
// completion therefore orders a wavefront's own exchanges (e.g. a colour bit
// before the count decrement that releases a successor) without the agent-scope
// release fence, whose whole-L2 write-back costs ~100 us per fence when many
// wavefronts issue them.
__device__ __forceinline__ void order_point() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

}  // namespace adg
