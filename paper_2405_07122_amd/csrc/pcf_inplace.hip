// pcf_inplace.hip -- PCF Learned Sort with in-place data movement.
//
// The paper's remarks on implementation (Sec. 5) note that a direct
// implementation of the bucketing step needs an auxiliary array as large as
// the input, and that sample-sort engineering gives in-place forms.  This
// variant keeps the keys in the caller's array: a node larger than a fixed
// staging capacity S is bucketed in place, and its buckets are then sorted S
// keys at a time through a staging buffer of S keys by the segmented sort.
// Auxiliary device memory is that staging buffer with its sort workspace (a
// function of S alone) plus one bit and one counter word per 64 keys of the
// node being bucketed; there is no copy of the keys.
//
// Bucketing one node in place (Algorithm 1's bucketing step, Sec. 3.3 model):
//   1. range of the node (x_min, x_max) and key validation;
//   2. the model: alpha samples histogrammed into beta + 1 equal-width bins,
//      prefix sum b, bucket table T_i = floor(b_i gamma / alpha), gamma + 1 =
//      256 buckets.  A node that failed its parent's test (|c_j| >= delta) or
//      whose scale is not finite is bucketed by the standard sort's digits
//      instead (8 bits below the top of its range);
//   3. bucket sizes, hence every bucket's final range;
//   4. eight rounds, one per bit of the bucket id from the top: every range
//      of keys that share the higher bits is split in two by the next bit.
//      A key on the wrong side of its split is "misplaced"; both sides hold
//      equally many, and the i-th misplaced key of the left side swaps with
//      the i-th of the right side.  A round marks the misplaced keys in a
//      bitmask (one word per 64 keys, counted per block of 4096 keys), scans
//      the block counts, and then each workgroup swaps the misplaced keys of
//      one left block with their partners: every position is read and written
//      by exactly one workgroup, so kernel boundaries are the only barriers
//      between workgroups.
// The swaps are not stable, so the variant sorts keys alone (equal keys are
// indistinguishable).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/pcfsort.h"
#include "pcf_block.h"
#include "pcf_device.h"
#include "pcf_driver.h"

namespace pcf {
namespace ip {

constexpr uint32_t BLK = 4096;         // keys per block (64 bitmask words)
constexpr uint32_t WPB = BLK / 64;     // bitmask words per block
constexpr uint32_t NB_IP = 256;        // buckets per in-place level
constexpr int ROUNDS = 8;              // log2(NB_IP)
constexpr uint64_t STAGE_KEYS = 1ull << 24;  // staging capacity S (keys)
constexpr int RANGE_WG = 1024;         // workgroups of the range kernel
constexpr int IP_NT = 256;

// The model of the node being bucketed (written by k_ip_fit).
struct Model {
  uint64_t lo_img, hi_img;
  double scale;
  uint32_t beta, halves, radix, shift;
  uint32_t done;  // single-valued: already in order
  uint32_t bad;   // an invalid key was found
  uint32_t pad[2];
};

// A half of a split range in one round: keys [start, end) of the node, the
// side (0 left, 1 right), its first block in this round's block list, its
// block count and the index of the other half of its split.
struct Half {
  uint32_t start, end, side, blk0, nblk, partner;
};

template <int KT>
struct BucketOf {
  BinFn f;
  uint64_t lo;
  uint32_t radix, shift;
  const uint8_t* tab;
  __device__ __forceinline__ uint32_t operator()(uint64_t bits) const {
    if (radix) return (uint32_t)((img_of<KT>(bits) - lo) >> shift);
    return tab[bin_of<KT>(f, bits)];
  }
};

template <int KT>
__device__ __forceinline__ BucketOf<KT> make_bucket_of(const Model& m, const uint8_t* tab_lds) {
  BucketOf<KT> b;
  b.radix = m.radix;
  b.shift = m.shift;
  b.lo = m.lo_img;
  b.tab = tab_lds;
  const uint64_t lob = bits_of_img<KT>(m.lo_img);
  b.f.lo_bits = lob;
  b.f.beta = m.beta;
  b.f.halves = m.halves;
  b.f.s = m.scale;
  if (KT == KT_F64) {
    b.f.lo = __longlong_as_double((long long)lob);
    b.f.lo_half = b.f.lo * 0.5;
  } else {
    b.f.lo = 0.0;
    b.f.lo_half = 0.0;
  }
  return b;
}

// 1. partial minimum / maximum images of the node, and key validation.
template <int KT>
__global__ __launch_bounds__(IP_NT) void k_ip_range(const uint64_t* keys, uint32_t n, MinMax* part,
                                                    uint32_t* bad) {
  __shared__ uint64_t red[2 * IP_NT / 64];
  uint64_t lo = ~0ull, hi = 0ull;
  bool b = false;
  for (uint32_t i = blockIdx.x * IP_NT + threadIdx.x; i < n; i += gridDim.x * IP_NT) {
    const uint64_t bits = __builtin_nontemporal_load(gld(keys) + i);
    if (KT == KT_F64) b |= !f64_bits_valid(bits);
    const uint64_t im = img_of<KT>(bits);
    lo = im < lo ? im : lo;
    hi = im > hi ? im : hi;
  }
  if (__syncthreads_or(b) && threadIdx.x == 0) atomicOr(bad, 1u);
  block_minmax_u64<IP_NT>(lo, hi, red);
  if (threadIdx.x == 0) part[blockIdx.x] = MinMax{lo, hi};
}

// 2. the model (one workgroup): range, then either the radix digit or the
// PCF table T_i = floor(b_i * 255 / alpha) over beta + 1 bins.
template <int KT>
__global__ __launch_bounds__(1024) void k_ip_fit(const uint64_t* keys, uint32_t n, const MinMax* part,
                                                 uint32_t nparts, const uint32_t* bad, uint32_t radix,
                                                 uint32_t alpha, uint32_t beta, uint64_t nseed,
                                                 Model* model, uint8_t* table) {
  __shared__ uint32_t hist[MAX_BINS + 1];
  __shared__ uint32_t red[1024 / 64 + 1];
  __shared__ uint64_t red64[2 * 1024 / 64];
  uint64_t lo = ~0ull, hi = 0ull;
  for (uint32_t i = threadIdx.x; i < nparts; i += 1024) {
    lo = part[i].lo < lo ? part[i].lo : lo;
    hi = part[i].hi > hi ? part[i].hi : hi;
  }
  block_minmax_u64<1024>(lo, hi, red64);
  Model m = {};
  m.lo_img = lo;
  m.hi_img = hi;
  m.bad = *bad;
  m.done = lo == hi ? 1u : 0u;
  BinFn f = {};
  bool rad = radix != 0;
  if (!m.done && !rad && !bin_setup<KT>(f, lo, hi, beta)) rad = true;  // scale not finite
  if (!m.done && rad) {
    const uint32_t top = 63u - (uint32_t)__clzll((long long)(hi - lo));
    m.radix = 1;
    m.shift = top + 1 > 8 ? top + 1 - 8 : 0u;
  } else if (!m.done) {
    m.beta = beta;
    m.halves = f.halves;
    m.scale = f.s;
    for (uint32_t i = threadIdx.x; i <= beta; i += 1024) hist[i] = 0u;
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < alpha; j += 1024)
      atomicAdd(&hist[bin_of<KT>(f, gld(keys)[sample_pos(nseed, j, n)])], 1u);
    __syncthreads();
    block_scan_array<1024, true>(hist, beta + 1, red);
    for (uint32_t i = threadIdx.x; i <= beta; i += 1024)
      table[i] = (uint8_t)(((uint64_t)hist[i] * (NB_IP - 1)) / alpha);
  }
  if (threadIdx.x == 0) *model = m;
}

// 3. bucket sizes: LDS histogram per workgroup, then one atomic per bucket.
template <int KT>
__global__ __launch_bounds__(IP_NT) void k_ip_count(const uint64_t* keys, uint32_t n, const Model* model,
                                                    const uint8_t* table, uint32_t* totals) {
  __shared__ uint32_t h[NB_IP];
  __shared__ uint8_t tab[MAX_BINS + 1];
  const Model m = *model;
  if (m.done || m.bad) return;
  for (uint32_t i = threadIdx.x; i < NB_IP; i += IP_NT) h[i] = 0u;
  if (!m.radix)
    for (uint32_t i = threadIdx.x; i <= m.beta; i += IP_NT) tab[i] = table[i];
  __syncthreads();
  const BucketOf<KT> bk = make_bucket_of<KT>(m, tab);
  for (uint32_t i = blockIdx.x * IP_NT + threadIdx.x; i < n; i += gridDim.x * IP_NT) {
    const uint32_t q = bk(gld(keys)[i]);
    atomicAdd(&h[q < NB_IP ? q : NB_IP - 1], 1u);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < NB_IP; i += IP_NT)
    if (h[i]) atomicAdd(&totals[i], h[i]);
}

// The half and block of this workgroup's block index (binary search over the
// halves' first blocks, held in LDS).
__device__ __forceinline__ uint32_t find_half(const Half* hs, uint32_t nh, uint32_t blk) {
  uint32_t lo = 0, hi = nh;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (hs[mid].blk0 <= blk) lo = mid;
    else hi = mid;
  }
  return lo;
}

// 4a. one round's marks: bit set for a key on the wrong side of its split
// (left side: the round's bit of its bucket is 1; right side: it is 0), and
// the number of marks of every block.
template <int KT>
__global__ __launch_bounds__(IP_NT) void k_ip_mark(const uint64_t* keys, const Model* model,
                                                   const uint8_t* table, const Half* halves,
                                                   uint32_t nh, uint32_t bit, uint64_t* mask,
                                                   uint32_t* cnt) {
  __shared__ uint8_t tab[MAX_BINS + 1];
  __shared__ Half hs[2 * NB_IP];
  __shared__ uint32_t red[IP_NT / 64 + 1];
  const Model m = *model;
  for (uint32_t i = threadIdx.x; i < nh; i += IP_NT) hs[i] = halves[i];
  if (!m.radix)
    for (uint32_t i = threadIdx.x; i <= m.beta; i += IP_NT) tab[i] = table[i];
  __syncthreads();
  const uint32_t blk = blockIdx.x;
  const Half h = hs[find_half(hs, nh, blk)];
  const uint32_t b0 = h.start + (blk - h.blk0) * BLK;
  const BucketOf<KT> bk = make_bucket_of<KT>(m, tab);
  const int l = lane_id(), w = wave_id();
  uint32_t c = 0;
  // wave w, word k: keys b0 + 64 (w * WPB / 4 + k) + lane
  for (uint32_t k = 0; k < WPB / (IP_NT / 64); ++k) {
    const uint32_t word = w * (WPB / (IP_NT / 64)) + k;
    const uint32_t i = b0 + word * 64 + l;
    bool mis = false;
    if (i < h.end) {
      const uint32_t q = bk(gld(keys)[i]);
      const uint32_t v = (q >> bit) & 1u;
      mis = h.side ? v == 0u : v == 1u;
    }
    const uint64_t bal = __ballot(mis);
    if (l == 0) mask[(uint64_t)blk * WPB + word] = bal;
    c += (uint32_t)__popcll(bal);
  }
  uint32_t tot;
  (void)block_excl_scan<IP_NT>(l == 0 ? c : 0u, red, tot);
  if (threadIdx.x == 0) cnt[blk] = tot;
}

// 4b. exclusive scan of the block counts (one workgroup, in slices).
__global__ __launch_bounds__(1024) void k_ip_scan(const uint32_t* cnt, uint32_t nblk, uint32_t* pre) {
  __shared__ uint32_t a[8192];
  __shared__ uint32_t red[1024 / 64 + 1];
  uint32_t carry = 0;
  for (uint32_t s = 0; s < nblk; s += 8192) {
    const uint32_t m = nblk - s < 8192u ? nblk - s : 8192u;
    for (uint32_t i = threadIdx.x; i < m; i += 1024) a[i] = cnt[s + i];
    __syncthreads();
    const uint32_t tot = block_scan_array<1024, false>(a, m, red);
    for (uint32_t i = threadIdx.x; i < m; i += 1024) pre[s + i] = carry + a[i];
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) pre[nblk] = carry;
}

// Positions of the marked keys of block `blk` whose rank (among the marks of
// its half, counted from the half's first block) lies in [r0, r0 + c): one
// wave, lane t reads mask word t.  out[rank - r0] = position.
__device__ __forceinline__ void wave_marked_positions(const uint64_t* mask, const uint32_t* pre,
                                                      uint32_t blk, uint32_t half_blk0,
                                                      uint32_t half_start, uint32_t r0, uint32_t c,
                                                      uint32_t* out) {
  const int l = lane_id();
  const uint64_t word = mask[(uint64_t)blk * WPB + l];
  const uint32_t pc = (uint32_t)__popcll(word);
  const uint32_t incl = wave_incl_scan(pc);
  uint32_t rank = pre[blk] - pre[half_blk0] + incl - pc;
  const uint32_t base = half_start + (blk - half_blk0) * BLK + (uint32_t)l * 64u;
  uint64_t wb = word;
  while (wb) {
    const uint32_t bi = (uint32_t)__builtin_ctzll(wb);
    wb &= wb - 1;
    if (rank >= r0 && rank < r0 + c) out[rank - r0] = base + bi;
    ++rank;
  }
}

// 4c. one round's swaps: the workgroup of a left block exchanges its marked
// keys with the marked keys of the same ranks on the right side.
__global__ __launch_bounds__(IP_NT) void k_ip_swap(uint64_t* keys, const Half* halves, uint32_t nh,
                                                   const uint64_t* mask, const uint32_t* cnt,
                                                   const uint32_t* pre, uint32_t* bad) {
  __shared__ Half hs[2 * NB_IP];
  __shared__ uint32_t posL[BLK], posR[BLK];
  for (uint32_t i = threadIdx.x; i < nh; i += IP_NT) hs[i] = halves[i];
  __syncthreads();
  const uint32_t blk = blockIdx.x;
  const Half h = hs[find_half(hs, nh, blk)];
  const uint32_t c = cnt[blk];
  if (h.side != 0 || c == 0) return;  // uniform: the whole workgroup leaves
  const Half g = hs[h.partner];
  const uint32_t r0 = pre[blk] - pre[h.blk0];  // ranks [r0, r0 + c) of this block's marks
  for (uint32_t j = threadIdx.x; j < c; j += IP_NT) posR[j] = ~0u;
  __syncthreads();
  const int w = wave_id();
  if (w == 0) wave_marked_positions(mask, pre, blk, h.blk0, h.start, r0, c, posL);
  // right blocks holding ranks [r0, r0 + c): the first one by binary search
  uint32_t lo = 0, hi = g.nblk;  // first right block whose marks end after r0
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (pre[g.blk0 + mid + 1] - pre[g.blk0] > r0) hi = mid;
    else lo = mid + 1;
  }
  for (uint32_t j = lo + (uint32_t)w; j < g.nblk; j += IP_NT / 64) {
    if (pre[g.blk0 + j] - pre[g.blk0] >= r0 + c) break;
    wave_marked_positions(mask, pre, g.blk0 + j, g.blk0, g.start, r0, c, posR);
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < c; j += IP_NT) {
    const uint32_t a = posL[j], b = posR[j];
    if (a >= h.end || b < g.start || b >= g.end) {  // cannot happen for consistent marks
      atomicOr(bad, 2u);
      continue;
    }
    const uint64_t va = gld(keys)[a], vb = gld(keys)[b];
    gst(keys)[a] = vb;
    gst(keys)[b] = va;
  }
}

}  // namespace ip

// ---- host side ---------------------------------------------------------------

namespace {

using ip::Half;
using ip::Model;

struct IpLayout {
  size_t stage, sort_ws, sort_ws_bytes, part, bad, model, table, totals, offs, halves, mask, cnt, pre;
  size_t total;
  uint64_t stage_keys, max_blocks;
};

size_t al(size_t v) { return (v + 255) / 256 * 256; }

// The staged sorts run under the call's policy (no per-node classes), so their
// workspace is the layout of S keys in up to 256 segments under that policy.
IpLayout ip_layout(size_t n, const pcf_policy& pol) {
  IpLayout L = {};
  L.stage_keys = std::min<uint64_t>(n, ip::STAGE_KEYS);
  L.max_blocks = (n + ip::BLK - 1) / ip::BLK + 2 * ip::NB_IP;
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t r = o;
    o = al(o + b);
    return r;
  };
  L.stage = take(8 * L.stage_keys);
  // (one segment reserves the root's sample buffer, many do not: take both)
  L.sort_ws_bytes = std::max(make_layout(L.stage_keys, 0, ip::NB_IP, pol, 0, 0, 0).total,
                             make_layout(L.stage_keys, 0, 1, pol, 0, 0, 0).total);
  L.sort_ws = take(L.sort_ws_bytes);
  L.part = take(sizeof(MinMax) * ip::RANGE_WG);
  L.bad = take(8);
  L.model = take(sizeof(Model));
  L.table = take(MAX_BINS + 1);
  L.totals = take(4 * ip::NB_IP);
  L.offs = take(8 * (2 * ip::NB_IP + 2));
  L.halves = take(sizeof(Half) * 2 * ip::NB_IP * ip::ROUNDS);
  L.mask = take(8 * ip::WPB * L.max_blocks);
  L.cnt = take(4 * L.max_blocks);
  L.pre = take(4 * (L.max_blocks + 1));
  L.total = o;
  return L;
}

struct IpNode {
  uint64_t off, len;
  uint32_t depth;
  int failed;  // bucket of at least delta keys of its parent: standard-sort digits
};

template <int KT>
int ip_run(uint64_t* keys, size_t n, char* ws, const IpLayout& L, const pcf_policy& pol,
           hipStream_t st) {
  uint64_t* stage = reinterpret_cast<uint64_t*>(ws + L.stage);
  void* sws = ws + L.sort_ws;
  MinMax* part = reinterpret_cast<MinMax*>(ws + L.part);
  uint32_t* bad = reinterpret_cast<uint32_t*>(ws + L.bad);
  Model* dmodel = reinterpret_cast<Model*>(ws + L.model);
  uint8_t* table = reinterpret_cast<uint8_t*>(ws + L.table);
  uint32_t* totals = reinterpret_cast<uint32_t*>(ws + L.totals);
  uint64_t* doffs = reinterpret_cast<uint64_t*>(ws + L.offs);
  Half* dhalves = reinterpret_cast<Half*>(ws + L.halves);
  uint64_t* mask = reinterpret_cast<uint64_t*>(ws + L.mask);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(ws + L.cnt);
  uint32_t* pre = reinterpret_cast<uint32_t*>(ws + L.pre);
  int32_t* sort_status = reinterpret_cast<int32_t*>(ws + L.bad + 4);
  const int kt = KT == KT_F64 ? PCF_KEY_F64 : PCF_KEY_U64;

  // Sorts keys [off, off + len) (consecutive buckets, boundaries rel[0..k],
  // rel[0] = 0) through the staging buffer with the segmented sort.
  auto stage_sort = [&](uint64_t off, const std::vector<uint64_t>& rel) -> int {
    const uint64_t len = rel.back();
    if (len == 0) return PCF_OK;
    PCF_HIP(hipMemcpyAsync(stage, keys + off, 8 * len, hipMemcpyDeviceToDevice, st));
    PCF_HIP(hipMemcpyAsync(doffs, rel.data(), 8 * rel.size(), hipMemcpyHostToDevice, st));
    SortArgs a = {};
    a.key_type = kt;
    a.keys_in = stage;
    a.keys_out = keys + off;
    a.offsets = doffs;
    a.nseg = (uint32_t)(rel.size() - 1);
    a.n = len;
    a.ws = sws;
    a.ws_bytes = L.sort_ws_bytes;
    a.d_status = sort_status;
    a.no_graph = 1;
    a.no_prof = 1;
    a.pol_override = &pol;
    a.stream = st;
    int r = run_sort(a);
    if (r != PCF_OK) return r;
    int32_t hs = 0;
    PCF_HIP(hipMemcpyAsync(&hs, sort_status, 4, hipMemcpyDeviceToHost, st));
    PCF_HIP(hipStreamSynchronize(st));  // the staging buffer is reused next
    return hs;
  };

  std::vector<IpNode> stack = {{0, n, 0, 0}};
  while (!stack.empty()) {
    const IpNode nd = stack.back();
    stack.pop_back();
    uint64_t* k = keys + nd.off;
    const uint32_t len = (uint32_t)nd.len;
    if (nd.len <= L.stage_keys) {
      int r = stage_sort(nd.off, {0, nd.len});
      if (r != PCF_OK) return r;
      continue;
    }
    // 1-2: range and model
    uint32_t nb = 0, beta = 0, alpha = 0, delta = 0;
    PolicyDev pd = {};
    pd.max_buckets = ip::NB_IP;
    pd.target_child = 1;
    pd.bins_per_bucket = pol.bins_per_bucket;
    pd.max_bins = pol.max_bins;
    pd.samples_per_bucket = pol.samples_per_bucket;
    pd.max_samples = pol.max_samples;
    node_params(len, NK_PCF, pd, nb, beta, alpha, delta);
    const uint64_t nseed = node_seed((uint64_t)pol.seed, 0, nd.depth, nd.off);
    PCF_HIP(hipMemsetAsync(bad, 0, 8, st));
    PCF_HIP(hipMemsetAsync(totals, 0, 4 * ip::NB_IP, st));
    hipLaunchKernelGGL((ip::k_ip_range<KT>), dim3(ip::RANGE_WG), dim3(ip::IP_NT), 0, st, k, len,
                       part, bad);
    hipLaunchKernelGGL((ip::k_ip_fit<KT>), dim3(1), dim3(1024), 0, st, k, len, part,
                       (uint32_t)ip::RANGE_WG, bad, (uint32_t)nd.failed, alpha, beta, nseed, dmodel,
                       table);
    hipLaunchKernelGGL((ip::k_ip_count<KT>), dim3(ip::RANGE_WG), dim3(ip::IP_NT), 0, st, k, len,
                       dmodel, table, totals);
    PCF_HIP(hipGetLastError());
    Model m;
    std::vector<uint32_t> tot(ip::NB_IP);
    PCF_HIP(hipMemcpyAsync(&m, dmodel, sizeof(Model), hipMemcpyDeviceToHost, st));
    PCF_HIP(hipMemcpyAsync(tot.data(), totals, 4 * ip::NB_IP, hipMemcpyDeviceToHost, st));
    PCF_HIP(hipStreamSynchronize(st));
    if (m.bad) return PCF_ERR_INVALID_KEY;
    if (m.done) continue;  // single-valued: already in order
    std::vector<uint32_t> B(ip::NB_IP + 1, 0);
    for (uint32_t q = 0; q < ip::NB_IP; ++q) B[q + 1] = B[q] + tot[q];
    if (B[ip::NB_IP] != len) return PCF_ERR_HIP;  // bucket sizes must add up
    // 4: the eight rounds (every round's halves known from the bucket sizes)
    std::vector<Half> all;
    std::vector<uint32_t> nh(ip::ROUNDS), nblk(ip::ROUNDS), first(ip::ROUNDS);
    for (int r = 0; r < ip::ROUNDS; ++r) {
      first[r] = (uint32_t)all.size();
      const uint32_t span = ip::NB_IP >> r;  // buckets per range of this round
      uint32_t blk = 0;
      for (uint32_t g = 0; g < (1u << r); ++g) {
        const uint32_t s = B[g * span], mid = B[g * span + span / 2], e = B[(g + 1) * span];
        if (s == mid || mid == e) continue;  // one side empty: nothing misplaced
        const uint32_t il = (uint32_t)(all.size() - first[r]);
        Half hl = {s, mid, 0, blk, (mid - s + ip::BLK - 1) / ip::BLK, il + 1};
        blk += hl.nblk;
        Half hr = {mid, e, 1, blk, (e - mid + ip::BLK - 1) / ip::BLK, il};
        blk += hr.nblk;
        all.push_back(hl);
        all.push_back(hr);
      }
      nh[r] = (uint32_t)all.size() - first[r];
      nblk[r] = blk;
      if (blk > L.max_blocks) return PCF_ERR_HIP;
    }
    if (!all.empty())
      PCF_HIP(hipMemcpyAsync(dhalves, all.data(), sizeof(Half) * all.size(), hipMemcpyHostToDevice, st));
    for (int r = 0; r < ip::ROUNDS; ++r) {
      if (nh[r] == 0) continue;
      const Half* hr = dhalves + first[r];
      const uint32_t bit = (uint32_t)(ip::ROUNDS - 1 - r);
      hipLaunchKernelGGL((ip::k_ip_mark<KT>), dim3(nblk[r]), dim3(ip::IP_NT), 0, st, k, dmodel, table,
                         hr, nh[r], bit, mask, cnt);
      hipLaunchKernelGGL(ip::k_ip_scan, dim3(1), dim3(1024), 0, st, cnt, nblk[r], pre);
      hipLaunchKernelGGL(ip::k_ip_swap, dim3(nblk[r]), dim3(ip::IP_NT), 0, st, k, hr, nh[r], mask, cnt,
                         pre, bad);
      PCF_HIP(hipGetLastError());
    }
    uint32_t hb = 0;
    PCF_HIP(hipMemcpyAsync(&hb, bad, 4, hipMemcpyDeviceToHost, st));
    PCF_HIP(hipStreamSynchronize(st));
    if (hb) return (hb & 1u) ? PCF_ERR_INVALID_KEY : PCF_ERR_HIP;
    // 5: buckets up to the staging capacity go through it in batches of
    // consecutive buckets; larger ones are bucketed in place again (a bucket
    // of at least delta keys failed: it continues with the standard sort's
    // digits, Algorithm 1)
    std::vector<uint64_t> rel = {0};
    uint64_t goff = nd.off;
    auto flush = [&]() -> int {
      const int r = stage_sort(goff, rel);
      rel.assign(1, 0);
      return r;
    };
    for (uint32_t q = 0; q < ip::NB_IP; ++q) {
      const uint64_t sz = tot[q];
      if (sz > L.stage_keys) {
        int r = flush();
        if (r != PCF_OK) return r;
        stack.push_back({nd.off + B[q], sz, nd.depth + 1, (m.radix || sz >= delta) ? 1 : 0});
        goff = nd.off + B[q + 1];
        continue;
      }
      if (rel.back() + sz > L.stage_keys) {
        int r = flush();
        if (r != PCF_OK) return r;
        goff = nd.off + B[q];
      }
      rel.push_back(rel.back() + sz);
    }
    int r = flush();
    if (r != PCF_OK) return r;
  }
  return PCF_OK;
}

}  // namespace
}  // namespace pcf

using namespace pcf;

extern "C" {

size_t pcf_inplace_workspace_bytes(int key_type, size_t n) {
  if ((key_type != PCF_KEY_F64 && key_type != PCF_KEY_U64) || n == 0) return 0;
  return ip_layout(n, policy_for(key_type, n, 0)).total;
}

int pcf_sort_inplace(int key_type, void* d_keys, size_t n, void* d_ws, size_t ws_bytes,
                     void* stream) {
  if (key_type != PCF_KEY_F64 && key_type != PCF_KEY_U64) return PCF_ERR_INVALID_ARGUMENT;
  if (n == 0) return PCF_OK;
  if (!d_keys || n >= (1ull << 32)) return PCF_ERR_INVALID_ARGUMENT;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const pcf_policy pol = policy_for(key_type, n, 0);
  const IpLayout L = ip_layout(n, pol);
  char* ws = reinterpret_cast<char*>(d_ws);
  bool own = false;
  if (!ws) {
    PCF_HIP(hipMallocAsync(reinterpret_cast<void**>(&ws), L.total, st));
    own = true;
  } else if (ws_bytes < L.total) {
    return PCF_ERR_OUT_OF_MEMORY;
  }
  uint64_t* k = reinterpret_cast<uint64_t*>(d_keys);
  int rc = key_type == PCF_KEY_F64 ? ip_run<KT_F64>(k, n, ws, L, pol, st)
                                   : ip_run<KT_U64>(k, n, ws, L, pol, st);
  if (own) {
    const hipError_t e = hipFreeAsync(ws, st);
    if (e != hipSuccess && rc == PCF_OK) rc = hip_fail(e);
    const hipError_t e2 = hipStreamSynchronize(st);
    if (e2 != hipSuccess && rc == PCF_OK) rc = hip_fail(e2);
  }
  return rc;
}

}  // extern "C"
