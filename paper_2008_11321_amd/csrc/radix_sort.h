// Stable LSD radix sort of (uint64 key, uint32 value) pairs on one stream,
// 8-bit digits.  Used for orders that the library outputs, not on the
// colouring path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace adg {
namespace rs {

// Device bytes of the per-block digit counts a sort needs (any n).
size_t count_bytes();

// Sorts pairs (keys[0][i], vals[0][i]), i < n, stably by bits [begin_bit,
// end_bit) of the key (rounded up to whole digits), ping-ponging between the
// buffers [0] and [1].  Writes to *out the index of the buffer that holds the
// result.  counts: count_bytes() of device memory.  Returns hipSuccess or the
// first launch error.
hipError_t sort_pairs(uint64_t* keys[2], uint32_t* vals[2], int64_t n, int begin_bit, int end_bit,
                      uint32_t* counts, hipStream_t s, int* out);

}  // namespace rs
}  // namespace adg
