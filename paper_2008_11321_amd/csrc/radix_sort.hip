// Stable LSD radix sort (see radix_sort.h).  Each pass: per-block digit
// counts over a contiguous range of the input, one block scans them in
// digit-major order (all blocks' digit 0, then digit 1, ...), and every
// block scatters its range in input order.  Inside a block, items are taken
// 256 at a time; a lane's rank among the lanes of its wavefront with the same
// digit comes from eight ballots, and wavefronts of a block are ordered
// through per-wavefront digit counts in LDS -- so equal digits keep their
// input order and the sort is stable.

#include "radix_sort.h"

#include "adg_device.h"

namespace adg {
namespace rs {

namespace {

constexpr int RS_BS = 256;
constexpr int RS_WAVES = RS_BS / WAVE;
constexpr int RS_BLOCKS = 1024;
constexpr int RS_DIGITS = 256;

__device__ __forceinline__ void block_range(int64_t n, int64_t* b, int64_t* e) {
  int64_t per = (n + gridDim.x - 1) / gridDim.x;
  per = (per + RS_BS - 1) / RS_BS * RS_BS;
  int64_t lo = per * (int64_t)blockIdx.x;
  int64_t hi = lo + per;
  *b = lo < n ? lo : n;
  *e = hi < n ? hi : n;
}

__global__ __launch_bounds__(RS_BS) void k_rs_count(const uint64_t* keys, int64_t n, int shift, uint32_t* counts) {
  __shared__ uint32_t h[RS_DIGITS];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t b, e;
  block_range(n, &b, &e);
  for (int64_t i = b + threadIdx.x; i < e; i += RS_BS) atomicAdd(&h[(keys[i] >> shift) & 255], 1u);
  __syncthreads();
  counts[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// One block: exclusive scan of the counts in digit-major order, in place.
__global__ __launch_bounds__(RS_BS) void k_rs_scan(uint32_t* counts, int nb) {
  __shared__ uint32_t part[RS_BS];
  uint32_t* row = counts + (size_t)threadIdx.x * nb;
  uint32_t sum = 0;
  for (int k = 0; k < nb; ++k) sum += row[k];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < RS_BS; off <<= 1) {
    const uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - sum;
  for (int k = 0; k < nb; ++k) {
    const uint32_t c = row[k];
    row[k] = run;
    run += c;
  }
}

__global__ __launch_bounds__(RS_BS) void k_rs_scatter(const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                                                       uint32_t* vout, int64_t n, int shift, const uint32_t* offs) {
  __shared__ uint32_t base[RS_DIGITS];          // next output slot per digit
  __shared__ uint32_t wc[RS_WAVES][RS_DIGITS];  // per-wavefront digit counts of the current 256 items
  const int w = threadIdx.x / WAVE;
  base[threadIdx.x] = offs[(size_t)threadIdx.x * gridDim.x + blockIdx.x];
  for (int k = 0; k < RS_WAVES; ++k) wc[k][threadIdx.x] = 0;
  __syncthreads();
  int64_t b, e;
  block_range(n, &b, &e);
  for (int64_t t0 = b; t0 < e; t0 += RS_BS) {
    const int64_t i = t0 + threadIdx.x;
    const bool valid = i < e;
    const uint64_t key = valid ? kin[i] : 0;
    const uint32_t val = valid ? vin[i] : 0;
    const unsigned d = valid ? (unsigned)(key >> shift) & 255u : 0u;
    uint64_t m = ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t bb = ballot(on);
      m &= on ? bb : ~bb;
    }
    const unsigned rank = lanes_below(m);
    if (valid && rank == 0) wc[w][d] = (unsigned)__popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t at = base[d] + rank;
      for (int k = 0; k < w; ++k) at += wc[k][d];
      kout[at] = key;
      vout[at] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int k = 0; k < RS_WAVES; ++k) {
      add += wc[k][threadIdx.x];
      wc[k][threadIdx.x] = 0;
    }
    base[threadIdx.x] += add;
    __syncthreads();
  }
}

}  // namespace

size_t count_bytes() { return sizeof(uint32_t) * RS_DIGITS * RS_BLOCKS; }

hipError_t sort_pairs(uint64_t* keys[2], uint32_t* vals[2], int64_t n, int begin_bit, int end_bit,
                      uint32_t* counts, hipStream_t s, int* out) {
  int cur = 0;
  *out = 0;
  if (n <= 0) return hipSuccess;
  const int64_t tiles = (n + RS_BS - 1) / RS_BS;
  const int nb = (int)(tiles < RS_BLOCKS ? tiles : RS_BLOCKS);
  for (int shift = begin_bit; shift < end_bit && shift < 64; shift += 8) {
    hipLaunchKernelGGL(k_rs_count, dim3(nb), dim3(RS_BS), 0, s, keys[cur], n, shift, counts);
    hipLaunchKernelGGL(k_rs_scan, dim3(1), dim3(RS_BS), 0, s, counts, nb);
    hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(RS_BS), 0, s, keys[cur], vals[cur], keys[cur ^ 1],
                       vals[cur ^ 1], n, shift, counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur ^= 1;
  }
  *out = cur;
  return hipSuccess;
}

}  // namespace rs
}  // namespace adg
