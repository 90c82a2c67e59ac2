// pcf_device.h -- device-side definitions of the PCF Learned Sort library:
// key images, the sampling generator, the PCF bin function and the work
// records that the kernels of one recursion level exchange through HBM.
//
// Paper: Sato & Matsui, "PCF Learned Sort", TMLR 2025.  Algorithm 1 (Sec. 3.2)
// is the recursion; Sec. 3.3 defines the PCF model used at every level.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pcf {

constexpr int KT_F64 = 0;
constexpr int KT_U64 = 1;

constexpr int MAX_LEVELS = 16;       // global recursion levels per call
constexpr int MAX_POL_CLASSES = 4;   // tuning-table size classes for node parameters
constexpr uint32_t MAX_NB = 2048;    // buckets per global node (gamma + 1)
constexpr uint32_t MAX_BINS = 16383; // beta per global node (table of beta + 1 u16)
constexpr uint32_t RADIX_NB = 256;   // buckets of a standard-sort (radix) node

// ---- order-preserving images --------------------------------------------
// fp64 keys (finite, no -0.0) map to uint64 so that unsigned order equals
// numeric order; uint64 keys are their own image.
template <int KT>
__device__ __host__ __forceinline__ uint64_t img_of(uint64_t bits) {
  if (KT == KT_F64) return (bits >> 63) ? ~bits : (bits | 0x8000000000000000ull);
  return bits;
}
template <int KT>
__device__ __host__ __forceinline__ uint64_t bits_of_img(uint64_t img) {
  if (KT == KT_F64) return (img >> 63) ? (img & 0x7fffffffffffffffull) : ~img;
  return img;
}

// fp64 keys must be finite and not -0.0 (the sorted order is then unique).
__device__ __forceinline__ bool f64_bits_valid(uint64_t bits) {
  const uint64_t exp = (bits >> 52) & 0x7ff;
  return exp != 0x7ff && bits != 0x8000000000000000ull;
}

// ---- SplitMix64 (Steele, Lea & Flood 2014) -------------------------------
// Output k (k = 0, 1, ...) of the generator whose state starts at s: the
// state advances by 0x9E3779B97F4A7C15 and passes through the published
// finalizer.  Used in counter form so any thread can draw any sample.
__device__ __host__ __forceinline__ uint64_t sm_finalize(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __host__ __forceinline__ uint64_t sm_out(uint64_t s, uint64_t k) {
  return sm_finalize(s + (k + 1) * 0x9E3779B97F4A7C15ull);
}
// A node is named by (segment, depth, offset inside the segment); its samples
// come from the generator seeded by chaining the three names.
__device__ __host__ __forceinline__ uint64_t node_seed(uint64_t seed, uint64_t seg,
                                                       uint64_t depth, uint64_t rel) {
  return sm_out(sm_out(sm_out(seed, seg), depth), rel);
}
// Sample j of a node of n keys: uniform position with replacement (Sec. 3.3),
// the high word of the 64x64 product.
__device__ __forceinline__ uint32_t sample_pos(uint64_t nseed, uint64_t j, uint32_t n) {
  return (uint32_t)__umul64hi(sm_out(nseed, j), (uint64_t)n);
}

// floor(m^{3/4}) exactly (delta of the PCF theorems, Sec. 3.3), m < 2^32.
__device__ __host__ inline uint32_t root34(uint32_t m) {
  if (m == 0) return 0;
  // m^3 as a 128-bit (hi, lo) pair
  auto mul128 = [](uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
#if defined(__HIP_DEVICE_COMPILE__)
    hi = __umul64hi(a, b);
    lo = a * b;
#else
    unsigned __int128 p = (unsigned __int128)a * b;
    hi = (uint64_t)(p >> 64);
    lo = (uint64_t)p;
#endif
  };
  uint64_t m2 = (uint64_t)m * m, m3h, m3l;
  mul128(m2, m, m3h, m3l);
  auto le = [&](uint64_t r) {  // r^4 <= m^3 ?
    uint64_t r2 = r * r, h, l;
    mul128(r2, r2, h, l);
    return h < m3h || (h == m3h && l <= m3l);
  };
  uint64_t r = (uint64_t)pow((double)m, 0.75);
  while (r > 0 && !le(r)) --r;
  while (le(r + 1)) ++r;
  return (uint32_t)r;
}

// ---- the PCF bin function i(x) (Sec. 3.3), 0-based ------------------------
// bin(v) = min(beta, floor(RN(off(v) * s))), s = RN(beta / RN(x_max - x_min)),
// off(v) = RN(v - x_min); halves of both terms when x_max - x_min overflows;
// for uint64 keys off(v) is the exact difference rounded to fp64.  All fp64
// steps are single IEEE round-to-nearest operations (built without FP
// contraction), so every key lands in the same bin as on the CPU.
struct BinFn {
  uint64_t lo_bits;
  double lo;
  double lo_half;
  double s;
  uint32_t beta;
  uint32_t halves;
};

// Position of a key in bin units, RN(RN(x - x_min) * s), before the floor.
template <int KT>
__device__ __forceinline__ double pos_of(const BinFn& f, uint64_t bits) {
  double off;
  if (KT == KT_F64) {
    const double v = __longlong_as_double((long long)bits);
    off = f.halves ? (v * 0.5 - f.lo_half) : (v - f.lo);
  } else {
    off = (double)(bits - f.lo_bits);
  }
  return off * f.s;
}

template <int KT>
__device__ __forceinline__ uint32_t bin_of(const BinFn& f, uint64_t bits) {
  const double p = pos_of<KT>(f, bits);
  const uint32_t k = (uint32_t)floor(p);
  return k < f.beta ? k : f.beta;
}

// Sets up the bin function for the range [lo, hi] (images); returns false when
// the scale is not finite (the node is then a bucketing failure).
template <int KT>
__device__ __forceinline__ bool bin_setup(BinFn& f, uint64_t lo_img, uint64_t hi_img,
                                          uint32_t beta) {
  const uint64_t lob = bits_of_img<KT>(lo_img), hib = bits_of_img<KT>(hi_img);
  f.lo_bits = lob;
  f.beta = beta;
  f.halves = 0;
  double d;
  if (KT == KT_F64) {
    const double lo = __longlong_as_double((long long)lob);
    const double hi = __longlong_as_double((long long)hib);
    f.lo = lo;
    f.lo_half = lo * 0.5;
    d = hi - lo;
    if (__builtin_isinf(d)) {
      f.halves = 1;
      d = hi * 0.5 - f.lo_half;
    }
  } else {
    f.lo = 0.0;
    f.lo_half = 0.0;
    d = (double)(hib - lob);
  }
  f.s = (double)beta / d;
  return __builtin_isfinite(f.s);
}

// ---- work records ---------------------------------------------------------
// node kinds: PCF model (Sec. 3.3), radix digits (standard sort of a failed
// bucket), spline model (App. A.5: the PCF's training, interpolated inference)
enum : uint32_t { NK_PCF = 0, NK_RADIX = 1, NK_SPLINE = 2 };
enum : uint32_t { NS_ACTIVE = 0, NS_DONE = 1 };
enum : uint32_t { IF_STD = 1, IF_ROOT = 2, IF_IOTA = 4 };

// Minimum and maximum key image of part of an array.
struct MinMax {
  uint64_t lo, hi;
};

// One array of a global level (a node of the recursion tree).  Its producer
// (the roots kernel or the parent's classify kernel) fills everything above
// `state`, including the parameters and the arena offsets; the fit kernel
// fills the rest.
struct Node {
  const void* src;          // keys of the node, element 0
  const uint32_t* vsrc;     // payload of the node, element 0 (NULL: none or iota)
  const MinMax* mmp;        // partial ranges to reduce into [min_img, max_img]
  uint64_t off;             // absolute position of element 0 in the output
  uint64_t rel;             // position inside its segment (names the node)
  uint64_t seed;            // sampling seed of the node
  uint64_t table_off, cm_off;  // arena offsets (u16 table, u32 count matrix)
  uint32_t len, seg, depth, kind;
  uint32_t nchunks, unit_base, aux_off, mmn;
  uint32_t nb, nbits, beta, alpha, delta;
  uint32_t iota;            // payload is the position inside the segment
  // filled by the fit kernel
  uint32_t state, shift, halves;
  uint32_t logd;             // radix node: digits on a log scale (keys spread over many octaves)
  uint64_t min_img, max_img;
  double scale;
};

struct Unit {
  uint32_t node, chunk;
};

// One array finished inside a workgroup's LDS.
struct Item {
  const void* src;
  const uint32_t* vsrc;
  uint64_t off;   // absolute output position of element 0
  uint64_t rel;   // position inside its segment (names the node)
  uint32_t len, depth, flags, seg;
};

struct LevelCtr {
  uint32_t num_nodes, num_units, aux_used, pad;
  unsigned long long table_used, cm_used;
  unsigned long long keys;        // keys in the level's nodes
  unsigned long long radix_keys;  // of those, keys in radix nodes (profiling)
};

struct Ctl {
  int32_t status;      // 0 or the data error (PCF_ERR_INVALID_KEY, or PCF_ERR_INVALID_ARGUMENT
                       // for CSR offsets that are not a partition of [0, n))
  uint32_t overflow;   // a capacity bound was exceeded (library bug guard); kernels
                       // read status and overflow together as one 64-bit word
  uint32_t item_count[3];
  uint32_t item_done[3];  // items below this index were finished by an earlier pass
  uint32_t n_radix_nodes, n_fail_items, n_done_nodes;
  unsigned long long item_keys[3];  // keys in the LDS items of each class (profiling)
  // profiling: keys (summed over levels) handled by the standard sort of
  // failed buckets (radix levels; bitonic in LDS) and by single-value exits
  unsigned long long radix_keys, bitonic_keys, single_keys;
  LevelCtr lv[MAX_LEVELS];
};

static_assert(offsetof(Ctl, overflow) == 4, "status and overflow form one 64-bit word");

struct PolicyDev {
  uint32_t max_buckets, target_child, bins_per_bucket, max_bins;
  uint32_t samples_per_bucket, max_samples, chunk_keys, lds_cap;
  uint32_t tau, small_cap, prof, mid_cap;
  uint32_t model;  // 0: PCF, 1: spline (kind of every model node)
};

// LDS-finish class of an array of `len` keys (0: <= small_cap, 1: <= mid_cap, 2: larger).
__device__ __host__ inline int item_class(uint32_t len, const PolicyDev& pol) {
  return len <= pol.small_cap ? 0 : (len <= pol.mid_cap ? 1 : 2);
}

// Everything a kernel of one call needs (passed by value).
struct Plan {
  Ctl* ctl;
  void* out_keys;
  uint32_t* out_vals;
  int32_t* d_status;
  uint32_t has_pay;
  uint32_t key_bytes;
  // level slots (level L uses slot L & 1)
  Node* nodes[2];
  Unit* units[2];
  uint16_t* table[2];
  uint32_t* cm[2];
  MinMax* mm[2];        // per (bucket, chunk) ranges written by the scatter
  uint32_t* bstart[2];
  int32_t* cmap[2];
  uint32_t* task_node[2];
  MinMax* mmr;          // per-unit ranges of the roots (range kernel)
  uint64_t* sbuf0;      // sample keys of a single root, gathered by the range kernel (or null)
  uint32_t sbuf0_cap;
  // global levels this call may run (levels 0 .. nlev - 1): a radix node
  // takes log-scale digits only while the levels left can still finish its
  // children with linear digits
  uint32_t nlev;
  uint32_t cap_nodes, cap_units, cap_aux, pad;
  unsigned long long cap_table, cap_cm;
  Item* items[3];
  uint32_t cap_items[3];
  // trace (level 0 only): prefix counts b of node 0
  uint32_t* trace_b;
  PolicyDev pol;
  // tuning-table classes: a node of len keys with cls_min[i] <= len <= cls_max[i]
  // takes its node parameters (buckets, bins, samples, chunk) from cls[i]
  PolicyDev cls[MAX_POL_CLASSES];
  uint32_t cls_min[MAX_POL_CLASSES], cls_max[MAX_POL_CLASSES];
  uint32_t ncls;
  uint64_t seed;
};

// The policy whose node parameters a node of `len` keys takes (the loop is
// unrolled, so the classes are read at fixed offsets of the kernel argument).
__device__ __forceinline__ PolicyDev node_pol(const Plan& p, uint32_t len) {
  PolicyDev q = p.pol;
#pragma unroll
  for (int i = 0; i < MAX_POL_CLASSES; ++i)
    if ((uint32_t)i < p.ncls && len >= p.cls_min[i] && len <= p.cls_max[i]) q = p.cls[i];
  return q;
}

// Parameters of a node of `len` keys (gamma + 1 = nb buckets, beta bins,
// alpha samples, failure threshold delta; Sec. 3.3 and the policy).
__device__ __host__ inline void node_params(uint32_t len, uint32_t kind, const PolicyDev& pol,
                                            uint32_t& nb, uint32_t& beta, uint32_t& alpha,
                                            uint32_t& delta) {
  if (kind == NK_RADIX) {
    nb = RADIX_NB;
    beta = 0;
    alpha = 0;
    delta = 0xffffffffu;
    return;
  }
  const uint32_t tgt = (len + pol.target_child - 1) / pol.target_child;
  nb = 2;
  while (nb < tgt && nb < pol.max_buckets) nb <<= 1;
  delta = root34(len);
  // Algorithm 1 pairs gamma with delta so that an expected bucket stays far
  // below the failure threshold; keep it at most delta / 4 here too (it
  // matters for arrays of a few times the LDS capacity, where len / nb from
  // the target alone would reach delta)
  const uint32_t need = (uint32_t)((4ull * len + delta - 1) / delta);
  while (nb < need && nb < pol.max_buckets) nb <<= 1;
  // bins and samples: bins_per_bucket / samples_per_bucket per bucket, and
  // on large arrays at least delta / 64 (a scaled form of the paper's
  // alpha = beta = floor(n^{3/4})), so that a dense region of a skewed
  // distribution still spreads over several bins
  beta = pol.bins_per_bucket * nb;
  if (delta / 64 > beta) beta = delta / 64;
  if (beta > pol.max_bins) beta = pol.max_bins;
  alpha = pol.samples_per_bucket * nb;
  if (beta > alpha) alpha = beta;
  if (alpha > pol.max_samples) alpha = pol.max_samples;
  // spline nodes keep the prefix counts b_i themselves in the 16-bit table
  if (kind == NK_SPLINE && alpha > 65535u) alpha = 65535u;
}

__device__ __host__ inline uint32_t bits_for(uint32_t nb) {
  uint32_t b = 0;
  while ((1u << b) < nb) ++b;
  return b;
}

// Ctl::overflow bits
constexpr uint32_t OVF_CAPACITY = 1;  // a work-list bound was exceeded
constexpr uint32_t OVF_INTERNAL = 2;  // an index failed its range check (a library bug)

}  // namespace pcf
