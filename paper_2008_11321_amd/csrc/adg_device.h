// Device-side building blocks shared by the single-graph and batched paths:
// wavefront (64-lane) primitives, the JP tie-break hash and the per-vertex
// JP synchronisation word.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, WAVE);
    v = o > v ? o : v;
  }
  return v;
}

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
