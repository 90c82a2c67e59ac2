// pcf_lfail.hip -- the bucketing-failure experiment of Sec. 4.2 (Fig. 3) on the
// GPU: for every parameter cell (alpha, beta, gamma, delta) and every input
// array, one PCF bucketing (Sec. 3.3) of the whole array, and whether some
// bucket holds more than delta keys.  The lemma of Sec. 3.3 bounds the
// probability of that event; Fig. 3 compares the empirical frequency with the
// bound on uniform keys.
//
// Parameters go far beyond what a sort level uses (up to n^0.95 bins and
// buckets), so the level is evaluated without moving keys: bucket sizes are
// sums of per-bin key counts over the runs of bins that share a bucket, and
// the per-bin key counts depend only on (array, beta).  So the work is
//   1. x_min, x_max of every array;
//   2. for every distinct beta and array: the key count of every bin, then
//      its inclusive prefix P (global memory);
//   3. for every (cell, array): the alpha samples' histogram over beta + 1 bins
//      (one workgroup, global scratch), its prefix b, the bucket of each bin
//      T_i = floor(b_i gamma / alpha), and the largest bucket as the largest
//      difference of P between consecutive ends of runs of equal T.
// Samples use the same counter-based generator as the sort, with the node seed
// chained over (seed, cell, array, 0), so one run is exactly one oracle level.
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/pcfsort.h"
#include "pcf_block.h"
#include "pcf_device.h"
#include "pcf_driver.h"

namespace pcf {

constexpr int LF_NT = 1024;

__global__ __launch_bounds__(LF_NT) void k_lf_range(const double* keys, uint32_t n, uint64_t* lohi,
                                                     int32_t* bad) {
  __shared__ uint64_t red64[2 * LF_NT / 64];
  const uint32_t r = blockIdx.x;
  const uint64_t* x = reinterpret_cast<const uint64_t*>(keys) + (uint64_t)r * n;
  uint64_t lo = ~0ull, hi = 0ull;
  bool b = false;
  for (uint32_t i = threadIdx.x; i < n; i += LF_NT) {
    const uint64_t bits = x[i];
    b |= !f64_bits_valid(bits);
    const uint64_t im = img_of<KT_F64>(bits);
    lo = im < lo ? im : lo;
    hi = im > hi ? im : hi;
  }
  if (__syncthreads_or(b) && threadIdx.x == 0) *bad = 1;
  block_minmax_u64<LF_NT>(lo, hi, red64);
  if (threadIdx.x == 0) {
    lohi[2 * r] = lo;
    lohi[2 * r + 1] = hi;
  }
}

// Key count of every bin for one (beta, array): grid (chunks, arrays); the
// bins of a chunk go through LDS when they fit there.
constexpr uint32_t LF_LDS_BINS = 16384;

__global__ __launch_bounds__(LF_NT) void k_lf_keyhist(const double* keys, uint32_t n,
                                                       const uint64_t* lohi, uint32_t beta,
                                                       uint32_t* P, uint32_t chunk) {
  __shared__ uint32_t h[LF_LDS_BINS];
  const uint32_t r = blockIdx.y;
  const uint64_t* x = reinterpret_cast<const uint64_t*>(keys) + (uint64_t)r * n;
  uint32_t* out = P + (uint64_t)r * (beta + 1);
  BinFn f;
  bin_setup<KT_F64>(f, lohi[2 * r], lohi[2 * r + 1], beta);
  const uint32_t b0 = blockIdx.x * chunk, b1 = min(n, b0 + chunk);
  const bool lds = beta + 1 <= LF_LDS_BINS;
  if (lds) {
    for (uint32_t i = threadIdx.x; i <= beta; i += LF_NT) h[i] = 0u;
    __syncthreads();
    for (uint32_t i = b0 + threadIdx.x; i < b1; i += LF_NT) atomicAdd(&h[bin_of<KT_F64>(f, x[i])], 1u);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i <= beta; i += LF_NT)
      if (h[i]) atomicAdd(&out[i], h[i]);
  } else {
    for (uint32_t i = b0 + threadIdx.x; i < b1; i += LF_NT) atomicAdd(&out[bin_of<KT_F64>(f, x[i])], 1u);
  }
}

// In-place inclusive scan of one (beta, array) count array (one workgroup each).
__global__ __launch_bounds__(LF_NT) void k_lf_scan(uint32_t* P, uint32_t beta) {
  __shared__ uint32_t red[LF_NT / 64 + 1];
  uint32_t* a = P + (uint64_t)blockIdx.x * (beta + 1);
  const uint32_t m = beta + 1, per = (m + LF_NT - 1) / LF_NT;
  const uint32_t i0 = threadIdx.x * per, i1 = min(m, i0 + per);
  uint32_t s = 0;
  for (uint32_t i = i0; i < i1; ++i) s += a[i];
  uint32_t tot;
  uint32_t run = block_excl_scan<LF_NT>(s, red, tot);
  for (uint32_t i = i0; i < i1; ++i) {
    run += a[i];
    a[i] = run;
  }
}

struct LfCell {
  uint32_t alpha, beta, gamma, delta;
  uint64_t p_off;  // offset of this cell's beta block in P (arrays of beta + 1)
};

// Exclusive max-scan of one int per thread across the workgroup.
__device__ int block_excl_max(int v, int* red) {
  constexpr int NW = LF_NT / 64;
  const int l = lane_id(), w = wave_id();
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (l >= d) x = y > x ? y : x;
  }
  if (l == 63) red[w] = x;
  __syncthreads();
  if (w == 0) {
    int t = l < NW ? red[l] : -1;
#pragma unroll
    for (int d = 1; d < NW; d <<= 1) {
      const int y = __shfl_up(t, d, 64);
      if (l >= d) t = y > t ? y : t;
    }
    if (l < NW) red[l] = t;
  }
  __syncthreads();
  int before = w ? red[w - 1] : -1;
  const int prev_in_wave = __shfl_up(x, 1, 64);
  if (l > 0) before = prev_in_wave > before ? prev_in_wave : before;
  __syncthreads();
  return before;
}

__global__ __launch_bounds__(LF_NT) void k_lf_runs(const double* keys, uint32_t n, uint32_t reps,
                                                    const uint64_t* lohi, const LfCell* cells,
                                                    uint32_t ncells, const uint32_t* P,
                                                    uint32_t* scratch, uint64_t scratch_stride,
                                                    uint64_t seed, uint32_t* failures) {
  __shared__ uint32_t red[LF_NT / 64 + 1];
  __shared__ int redi[LF_NT / 64 + 1];
  __shared__ uint32_t redm[LF_NT / 64 + 1];
  uint32_t* hist = scratch + (uint64_t)blockIdx.x * scratch_stride;
  const uint64_t total = (uint64_t)ncells * reps;
  for (uint64_t run = blockIdx.x; run < total; run += gridDim.x) {
    const uint32_t ci = (uint32_t)(run / reps), r = (uint32_t)(run % reps);
    const LfCell cl = cells[ci];
    const uint32_t beta = cl.beta, alpha = cl.alpha, gamma = cl.gamma;
    const uint64_t* x = reinterpret_cast<const uint64_t*>(keys) + (uint64_t)r * n;
    const uint32_t* pk = P + cl.p_off + (uint64_t)r * (beta + 1);
    BinFn f;
    bin_setup<KT_F64>(f, lohi[2 * r], lohi[2 * r + 1], beta);
    for (uint32_t i = threadIdx.x; i <= beta; i += LF_NT) hist[i] = 0u;
    // the histogram lives in global memory and its atomics are performed in
    // L2: device-scope fences keep every thread's later loads off stale L1 lines
    __threadfence();
    __syncthreads();
    // training: alpha samples with replacement into beta + 1 bins
    const uint64_t ns = node_seed(seed, ci, r, 0);
    for (uint32_t j = threadIdx.x; j < alpha; j += LF_NT)
      atomicAdd(&hist[bin_of<KT_F64>(f, x[sample_pos(ns, j, n)])], 1u);
    __threadfence();
    __syncthreads();
    // inclusive prefix b over bins, per-thread runs
    const uint32_t m = beta + 1, per = (m + LF_NT - 1) / LF_NT;
    const uint32_t i0 = threadIdx.x * per, i1 = min(m, i0 + per);
    uint32_t s = 0;
    for (uint32_t i = i0; i < i1; ++i) s += hist[i];
    uint32_t tot;
    uint32_t run_b = block_excl_scan<LF_NT>(s, red, tot);
    for (uint32_t i = i0; i < i1; ++i) {
      run_b += hist[i];
      hist[i] = run_b;
    }
    __threadfence();
    __syncthreads();
    // runs of bins that share a bucket T_i = floor(b_i gamma / alpha): a bin
    // ends its bucket's run when the next bin's bucket differs (or it is last)
    auto T = [&](uint32_t i) {
      return (uint32_t)(((uint64_t)hist[i] * gamma) / alpha);
    };
    int last_end = -1;
    for (uint32_t i = i0; i < i1; ++i)
      if (i == beta || T(i) != T(i + 1)) last_end = (int)i;
    int prev = block_excl_max(last_end, redi);
    uint32_t mx = 0;
    for (uint32_t i = i0; i < i1; ++i) {
      if (i == beta || T(i) != T(i + 1)) {
        const uint32_t sz = pk[i] - (prev >= 0 ? pk[prev] : 0u);
        mx = sz > mx ? sz : mx;
        prev = (int)i;
      }
    }
    // block maximum of the largest bucket
    const int l = lane_id(), w = wave_id();
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const uint32_t o = __shfl_xor(mx, d, 64);
      mx = o > mx ? o : mx;
    }
    if (l == 0) redm[w] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t m2 = 0;
      for (int i = 0; i < LF_NT / 64; ++i) m2 = redm[i] > m2 ? redm[i] : m2;
      if (m2 > cl.delta) atomicAdd(&failures[ci], 1u);
    }
    __syncthreads();
  }
}

}  // namespace pcf

using namespace pcf;

extern "C" int pcf_lfail_grid(const double* d_keys, size_t n, uint32_t reps,
                              const uint32_t* h_cells, uint32_t ncells, uint64_t seed,
                              uint32_t* h_failures, void* stream) {
  if (!d_keys || !h_cells || !h_failures || n < 2 || n >= (1ull << 32) || reps == 0 || ncells == 0)
    return PCF_ERR_INVALID_ARGUMENT;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::vector<uint32_t> betas;
  std::vector<LfCell> cells(ncells);
  uint32_t beta_max = 0;
  for (uint32_t c = 0; c < ncells; ++c) {
    const uint32_t a = h_cells[4 * c], b = h_cells[4 * c + 1], g = h_cells[4 * c + 2];
    if (a == 0 || b == 0 || g == 0 || b >= (1u << 30)) return PCF_ERR_INVALID_ARGUMENT;
    cells[c] = LfCell{a, b, g, h_cells[4 * c + 3], 0};
    bool seen = false;
    for (uint32_t v : betas) seen |= v == b;
    if (!seen) betas.push_back(b);
    beta_max = b > beta_max ? b : beta_max;
  }
  // offsets of the per-beta prefix blocks (reps arrays of beta + 1 each)
  std::vector<uint64_t> boff(betas.size());
  uint64_t ptotal = 0;
  for (size_t i = 0; i < betas.size(); ++i) {
    boff[i] = ptotal;
    ptotal += (uint64_t)reps * (betas[i] + 1);
  }
  for (auto& cl : cells)
    for (size_t i = 0; i < betas.size(); ++i)
      if (betas[i] == cl.beta) cl.p_off = boff[i];
  const int cus = device_cus();
  if (cus <= 0) return PCF_ERR_UNSUPPORTED;
  const uint32_t grid = (uint32_t)cus * 2;
  const uint64_t stride = ((uint64_t)beta_max + 1 + 63) / 64 * 64;
  uint64_t *d_lohi = nullptr;
  uint32_t *d_P = nullptr, *d_scr = nullptr, *d_fail = nullptr;
  LfCell* d_cells = nullptr;
  int32_t* d_bad = nullptr;
  int rc = PCF_OK;
  auto fail = [&](hipError_t e) {
    if (rc == PCF_OK) rc = hip_fail(e, "pcf_lfail_grid", __LINE__);
  };
  hipError_t e;
  if ((e = hipMallocAsync(reinterpret_cast<void**>(&d_lohi), 16ull * reps, st)) != hipSuccess) fail(e);
  if (rc == PCF_OK && (e = hipMallocAsync(reinterpret_cast<void**>(&d_P), 4ull * ptotal, st)) != hipSuccess) fail(e);
  if (rc == PCF_OK &&
      (e = hipMallocAsync(reinterpret_cast<void**>(&d_scr), 4ull * stride * grid, st)) != hipSuccess)
    fail(e);
  if (rc == PCF_OK && (e = hipMallocAsync(reinterpret_cast<void**>(&d_fail), 4ull * ncells, st)) != hipSuccess)
    fail(e);
  if (rc == PCF_OK &&
      (e = hipMallocAsync(reinterpret_cast<void**>(&d_cells), sizeof(LfCell) * ncells, st)) != hipSuccess)
    fail(e);
  if (rc == PCF_OK && (e = hipMallocAsync(reinterpret_cast<void**>(&d_bad), 4, st)) != hipSuccess) fail(e);
  if (rc == PCF_OK) {
    (void)hipMemsetAsync(d_P, 0, 4ull * ptotal, st);
    (void)hipMemsetAsync(d_fail, 0, 4ull * ncells, st);
    (void)hipMemsetAsync(d_bad, 0, 4, st);
    (void)hipMemcpyAsync(d_cells, cells.data(), sizeof(LfCell) * ncells, hipMemcpyHostToDevice, st);
    hipLaunchKernelGGL(k_lf_range, dim3(reps), dim3(LF_NT), 0, st, d_keys, (uint32_t)n, d_lohi, d_bad);
    const uint32_t chunk = 1u << 16;
    const uint32_t nch = (uint32_t)((n + chunk - 1) / chunk);
    for (size_t i = 0; i < betas.size(); ++i) {
      hipLaunchKernelGGL(k_lf_keyhist, dim3(nch, reps), dim3(LF_NT), 0, st, d_keys, (uint32_t)n,
                         d_lohi, betas[i], d_P + boff[i], chunk);
      hipLaunchKernelGGL(k_lf_scan, dim3(reps), dim3(LF_NT), 0, st, d_P + boff[i], betas[i]);
    }
    hipLaunchKernelGGL(k_lf_runs, dim3(grid), dim3(LF_NT), 0, st, d_keys, (uint32_t)n, reps, d_lohi,
                       d_cells, ncells, d_P, d_scr, stride, seed, d_fail);
    if ((e = hipGetLastError()) != hipSuccess) fail(e);
    int32_t bad = 0;
    if (rc == PCF_OK && (e = hipMemcpyAsync(h_failures, d_fail, 4ull * ncells, hipMemcpyDeviceToHost, st)) != hipSuccess)
      fail(e);
    if (rc == PCF_OK && (e = hipMemcpyAsync(&bad, d_bad, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) fail(e);
    if (rc == PCF_OK && (e = hipStreamSynchronize(st)) != hipSuccess) fail(e);
    if (rc == PCF_OK && bad) rc = PCF_ERR_INVALID_KEY;
  }
  if (d_lohi) (void)hipFreeAsync(d_lohi, st);
  if (d_P) (void)hipFreeAsync(d_P, st);
  if (d_scr) (void)hipFreeAsync(d_scr, st);
  if (d_fail) (void)hipFreeAsync(d_fail, st);
  if (d_cells) (void)hipFreeAsync(d_cells, st);
  if (d_bad) (void)hipFreeAsync(d_bad, st);
  (void)hipStreamSynchronize(st);
  return rc;
}
