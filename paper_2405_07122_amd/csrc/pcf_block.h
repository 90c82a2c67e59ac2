// pcf_block.h -- workgroup-level building blocks (wave64 scans, reductions,
// stable in-wave ranking) shared by the PCF Learned Sort kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcf {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// Global-memory views of generic pointers.  Key and payload arrays reach the
// kernels through node and item records, so the compiler cannot prove their
// address space and emits flat loads and stores; those count against the LDS
// counter too, so every wait for an LDS result would also wait for the keys
// prefetched for the next tile.  Through these views they become global_*
// instructions, which count only against the vector-memory counter.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gld(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gst(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Workgroups are dealt to the eight XCDs round-robin by blockIdx.  A grid-
// stride loop over v in [0, 8*per) that visits unit (v % 8) * per + v / 8
// gives each XCD one contiguous run of units (per = ceil(nu / 8)), so the
// neighbouring tiles whose writes share cache lines at bucket edges meet in
// the same L2.  The map is a bijection on [0, 8*per); values >= nu are skipped.
__device__ __forceinline__ uint32_t xcd_unit(uint32_t v, uint32_t per) {
  return (v & 7u) * per + (v >> 3);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l ? (~0ull >> (64 - l)) : 0ull;
}

// Inclusive scan of one uint32 across the 64 lanes of a wave, with DPP lane
// moves (no LDS crossbar): shifts by 1, 2, 4, 8 inside each row of 16 lanes,
// then the row totals are carried by row broadcasts of lanes 15 and 31.
// Lanes that have no source keep `old` = 0, so they add nothing.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

// One step of a wave-wide min / max scan on uint64 values (two 32-bit DPP
// moves); lanes without a source see the identity `fill`.
template <int CTRL, int ROWMASK, bool MAX>
__device__ __forceinline__ uint64_t dpp_minmax_step(uint64_t v) {
  constexpr int fill = MAX ? 0 : -1;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(fill, (int)(uint32_t)v, CTRL, ROWMASK, 0xf, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp(fill, (int)(uint32_t)(v >> 32), CTRL, ROWMASK, 0xf, false);
  const uint64_t o = ((uint64_t)hi << 32) | lo;
  return MAX ? (o > v ? o : v) : (o < v ? o : v);
}

// Minimum / maximum over the wave, returned to every lane: an inclusive DPP
// scan leaves the result in lane 63, which is then read as a scalar.
template <bool MAX>
__device__ __forceinline__ uint64_t wave_reduce_u64(uint64_t v) {
  v = dpp_minmax_step<0x111, 0xf, MAX>(v);
  v = dpp_minmax_step<0x112, 0xf, MAX>(v);
  v = dpp_minmax_step<0x114, 0xf, MAX>(v);
  v = dpp_minmax_step<0x118, 0xf, MAX>(v);
  v = dpp_minmax_step<0x142, 0xa, MAX>(v);
  v = dpp_minmax_step<0x143, 0xc, MAX>(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) { return wave_reduce_u64<false>(v); }
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) { return wave_reduce_u64<true>(v); }

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

// In-place scan of an LDS array a[0..n) by a workgroup of NT threads.  Wave
// w owns a contiguous run of rows of 64 entries; a row is read by the 64
// lanes at once (consecutive words: no bank conflicts) and scanned with the
// wave scan.  A first pass sums each wave's rows; after one barrier every
// wave scans its rows from its prefix.  Returns the total.  Contains barriers.
template <int NT, bool INCLUSIVE>
__device__ uint32_t block_scan_array(uint32_t* a, uint32_t n, uint32_t* red) {
  constexpr int NW = NT / 64;
  const int l = lane_id(), w = wave_id();
  const uint32_t rows = (n + 63) / 64;
  const uint32_t rpw = (rows + NW - 1) / NW;
  const uint32_t r0 = w * rpw < rows ? w * rpw : rows;
  const uint32_t r1 = r0 + rpw < rows ? r0 + rpw : rows;
  uint32_t s = 0;
  for (uint32_t r = r0; r < r1; ++r) {
    const uint32_t i = r * 64 + l;
    s += i < n ? a[i] : 0u;
  }
  s = wave_incl_scan(s);  // lane 63: the wave's sum
  if (l == 63) red[w] = s;
  __syncthreads();
  uint32_t run = 0, total = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const uint32_t t = red[k];
    run += k < w ? t : 0u;
    total += t;
  }
  for (uint32_t r = r0; r < r1; ++r) {
    const uint32_t i = r * 64 + l;
    const uint32_t v = i < n ? a[i] : 0u;
    const uint32_t x = wave_incl_scan(v);
    if (i < n) a[i] = run + (INCLUSIVE ? x : x - v);
    run += (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
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
