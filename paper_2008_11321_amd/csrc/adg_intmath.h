// Exact integer helpers for ADG's threshold (Algorithm 1, the selection of
// R against (1 + eps) times the average degree of U).  With eps = p / q and
// an integer D, D <= (1 + eps) S / N holds exactly when
// D <= floor((q + p) S / (q N)); the product (q + p) S can pass 2^64 (p and q
// up to 2^31 - 1, S up to the number of adjacency entries), so it is formed
// in 128 bits.  Host and device code use the same function.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

namespace adg {

// floor(a * b / d) for d > 0, saturated at `cap`.  The 128-bit product is
// assembled from 32-bit halves; the quotient comes from a restoring long
// division of the high word's remainder (high < d) through the low word.
__host__ __device__ inline uint64_t mul_div_floor_sat(uint64_t a, uint64_t b, uint64_t d, uint64_t cap) {
  const uint64_t a0 = a & 0xffffffffu, a1 = a >> 32, b0 = b & 0xffffffffu, b1 = b >> 32;
  const uint64_t p00 = a0 * b0, p01 = a0 * b1, p10 = a1 * b0, p11 = a1 * b1;
  const uint64_t mid = (p00 >> 32) + (p01 & 0xffffffffu) + (p10 & 0xffffffffu);
  const uint64_t lo = (mid << 32) | (p00 & 0xffffffffu);
  const uint64_t hi = p11 + (p01 >> 32) + (p10 >> 32) + (mid >> 32);
  if (hi == 0) {
    const uint64_t q = lo / d;
    return q < cap ? q : cap;
  }
  if (hi >= d) return cap;   // the quotient is at least 2^64
  uint64_t r = hi, q = 0;
  for (int i = 63; i >= 0; --i) {
    const bool carry = (r >> 63) != 0;   // r << 1 would pass 2^64, so it exceeds d
    r = (r << 1) | ((lo >> i) & 1u);
    q <<= 1;
    if (carry || r >= d) {
      r -= d;
      q |= 1u;
    }
  }
  return q < cap ? q : cap;
}

}  // namespace adg
