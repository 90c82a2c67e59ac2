// pcf_block.h -- workgroup-level building blocks (wave64 scans, reductions,
// stable in-wave ranking) shared by the PCF Learned Sort kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcf {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l ? (~0ull >> (64 - l)) : 0ull;
}

// Inclusive scan of one uint32 across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (l >= d) x += y;
  }
  return x;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t o = __shfl_xor(v, d, 64);
    v = o < v ? o : v;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t o = __shfl_xor(v, d, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Exclusive scan of one value per thread across a workgroup of NT threads.
// `red` holds at least NT/64 + 1 words of LDS.  Returns the exclusive prefix;
// `total` receives the sum over the workgroup.  Contains barriers.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* red, uint32_t& total) {
  constexpr int NW = NT / 64;
  const int l = lane_id(), w = wave_id();
  const uint32_t x = wave_incl_scan(v);
  if (l == 63) red[w] = x;
  __syncthreads();
  if (w == 0) {
    uint32_t t = (l < NW) ? red[l] : 0u;
    t = wave_incl_scan(t);
    if (l < NW) red[l] = t;
  }
  __syncthreads();
  const uint32_t base = w ? red[w - 1] : 0u;
  total = red[NW - 1];
  __syncthreads();
  return base + x - v;
}

// In-place scan of an LDS array a[0..n) by a workgroup of NT threads.
// Each thread owns a contiguous run of ceil(n / NT) entries.  Returns the total.
template <int NT, bool INCLUSIVE>
__device__ uint32_t block_scan_array(uint32_t* a, uint32_t n, uint32_t* red) {
  const uint32_t per = (n + NT - 1) / NT;
  const uint32_t b = threadIdx.x * per;
  const uint32_t e = (b + per < n) ? b + per : n;
  uint32_t s = 0;
  for (uint32_t i = b; i < e; ++i) s += a[i];
  uint32_t total;
  uint32_t run = block_excl_scan<NT>(s, red, total);
  for (uint32_t i = b; i < e; ++i) {
    const uint32_t v = a[i];
    if (INCLUSIVE) {
      run += v;
      a[i] = run;
    } else {
      a[i] = run;
      run += v;
    }
  }
  __syncthreads();
  return total;
}

// Min and max of one uint64 per thread over the workgroup.  `red` holds at
// least 2 * NT / 64 uint64 words.  Contains barriers.
template <int NT>
__device__ __forceinline__ void block_minmax_u64(uint64_t& lo, uint64_t& hi, uint64_t* red) {
  constexpr int NW = NT / 64;
  const int l = lane_id(), w = wave_id();
  lo = wave_min_u64(lo);
  hi = wave_max_u64(hi);
  if (l == 0) {
    red[w] = lo;
    red[NW + w] = hi;
  }
  __syncthreads();
  lo = red[0];
  hi = red[NW];
#pragma unroll
  for (int i = 1; i < NW; ++i) {
    lo = red[i] < lo ? red[i] : lo;
    hi = red[NW + i] > hi ? red[NW + i] : hi;
  }
  __syncthreads();
}

// Stable ranking inside one wave round: the lanes in `active` that hold the
// same bucket id b (nbits significant bits).  Returns the mask of those peers.
__device__ __forceinline__ uint64_t wave_match(uint32_t b, uint32_t nbits, uint64_t active) {
  uint64_t peers = active;
  for (uint32_t i = 0; i < nbits; ++i) {
    const bool bit = (b >> i) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

}  // namespace pcf
