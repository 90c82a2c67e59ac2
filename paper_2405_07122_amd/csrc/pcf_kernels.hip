// pcf_kernels.hip -- the gfx950 kernels of one PCF Learned Sort recursion
// level and of the in-LDS finish.
//
// Paper: Sato & Matsui, "PCF Learned Sort", TMLR 2025.
//   Algorithm 1 (Sec. 3.2): Learned-Sort recursion with the small-array and
//     failed-bucket (|c_j| >= delta) exits to a standard sort.
//   Sec. 3.3: PCF training by counting alpha samples into beta equal-width
//     bins between the array's minimum and maximum, inference F(x) =
//     b_{i(x)} / alpha, bucket floor(F(x) gamma).
//
// One global level is five kernels over a list of nodes (arrays):
//   k_fit       one workgroup per node: range from the producer's partial
//               minima/maxima, alpha samples histogrammed into beta + 1 bins
//               in LDS, inclusive prefix sum, bin -> bucket table T (u16);
//   k_count     per (node, chunk) unit: T in LDS, every key's bucket, LDS
//               histogram of the gamma + 1 buckets, one column of the node's
//               bucket-major count matrix;
//   k_colscan   one wave per (node, bucket): exclusive scan over chunks;
//   k_classify  one workgroup per node: bucket starts, the paper's per-bucket
//               decision (recurse / standard sort), the next level's nodes
//               (parameters and arena space reserved once per parent) and the
//               LDS work items;
//   k_scatter   per unit: stable tile ranking with wave ballots, LDS staging
//               in bucket order, coalesced runs to HBM, per-chunk child ranges.
// k_lds_sort finishes arrays of at most a few thousand keys inside one
// workgroup's LDS with the paper's own parameters.  No kernel on the data
// path uses a same-address global atomic per key or per bucket: those
// serialize across the chip.
#include "pcf_kernels.h"
#include "pcf_block.h"

namespace pcf {

constexpr int ERR_INVALID_ARGUMENT = 1;  // PCF_ERR_INVALID_ARGUMENT
constexpr int ERR_INVALID_KEY = 2;  // PCF_ERR_INVALID_KEY
constexpr int ERR_OUT_OF_MEMORY = 3;  // PCF_ERR_OUT_OF_MEMORY
constexpr int ERR_HIP = 4;  // PCF_ERR_HIP

// No data error and no overflow so far (status and overflow are the first
// 8 bytes of the 256-byte aligned control block: one load reads both).
__device__ __forceinline__ bool ctl_ok(const Ctl* c) {
  return *reinterpret_cast<const volatile uint64_t*>(c) == 0ull;
}

__device__ __forceinline__ void flag_overflow(Ctl* c) { atomicOr(&c->overflow, OVF_CAPACITY); }
__device__ __forceinline__ void flag_internal(Ctl* c) { atomicOr(&c->overflow, OVF_INTERNAL); }

// ---------------------------------------------------------------------------
// set-up kernels
// ---------------------------------------------------------------------------

// Zeroes the control block (a fill kernel rather than a memset, so the call
// can be captured into a graph).
__global__ void k_init(Plan p) {
  uint32_t* w = reinterpret_cast<uint32_t*>(p.ctl);
  for (uint32_t i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x) w[i] = 0u;
}

__global__ void k_finish(Plan p, int32_t* d_status, int check_level) {
  if (threadIdx.x != 0) return;
  Ctl* c = p.ctl;
  if (check_level >= 0 && check_level < MAX_LEVELS && c->lv[check_level].num_nodes != 0)
    atomicOr(&c->overflow, OVF_CAPACITY);
  // the LDS items listed so far are finished: a later pass starts after them
  for (int k = 0; k < 3; ++k)
    c->item_done[k] = c->item_count[k] < p.cap_items[k] ? c->item_count[k] : p.cap_items[k];
  int32_t s = c->status;
  const uint32_t ovf = c->overflow;
  if (s == 0 && ovf) s = (ovf & OVF_INTERNAL) ? ERR_HIP : ERR_OUT_OF_MEMORY;
  if (d_status) *d_status = s;
}

__global__ void k_set_status(int32_t* d, int32_t v) {
  if (threadIdx.x == 0) *d = v;
}

// Creates the roots: one node (or one LDS item) per non-empty segment.  A
// single workgroup walks the segments in blocks and hands out indices and
// arena space with block scans, so no atomics are needed.
constexpr int ROOT_NT = 1024;

__global__ __launch_bounds__(ROOT_NT) void k_roots(Plan p, RootArgs a) {
  __shared__ uint32_t red[ROOT_NT / 64 + 1];
  __shared__ unsigned long long base[9];  // nodes, units, table, cm, aux, items 0-2, keys
  __shared__ uint32_t ush[ROOT_NT], uni[ROOT_NT], unb[ROOT_NT];
  Ctl* c = p.ctl;
  if (threadIdx.x < 9) base[threadIdx.x] = 0;
  __syncthreads();
  for (uint32_t s0 = 0; s0 < a.nseg; s0 += ROOT_NT) {
    const uint32_t s = s0 + threadIdx.x;
    uint32_t len = 0;
    uint64_t b0 = 0;
    if (s < a.nseg) {
      b0 = a.offsets ? a.offsets[s] : 0ull;
      const uint64_t b1 = a.offsets ? a.offsets[s + 1] : a.n;
      // CSR offsets must start at 0, never decrease and end at n: then the
      // segments are disjoint and every output position lies below n.  A
      // violation is a data error of the call; the segment gets no node.
      const bool bad = b1 < b0 || b1 > a.n || (s == 0 && b0 != 0) || (s + 1 == a.nseg && b1 != a.n);
      if (bad) atomicMax(&c->status, ERR_INVALID_ARGUMENT);
      len = bad ? 0u : (uint32_t)(b1 - b0);
    }
    const bool item = len > 0 && len <= p.pol.lds_cap && !a.force_global;
    const bool glob = len > 0 && !item;
    const int icls = item_class(len, p.pol);
    uint32_t nb = 0, beta = 0, alpha = 0, delta = 0, nch = 0;
    if (glob) {
      if (a.fixed_nb) {
        nb = a.fixed_nb;
        beta = a.fixed_beta;
        alpha = a.fixed_alpha;
        delta = len + 1;
        nch = (len + p.pol.chunk_keys - 1) / p.pol.chunk_keys;
      } else {
        const PolicyDev np = node_pol(p, len);
        node_params(len, p.pol.model ? NK_SPLINE : NK_PCF, np, nb, beta, alpha, delta);
        nch = (len + np.chunk_keys - 1) / np.chunk_keys;
      }
    }
    uint32_t tot;
    const uint32_t o_node = block_excl_scan<ROOT_NT>(glob ? 1u : 0u, red, tot);
    const uint32_t t_node = tot;
    const uint32_t o_unit = block_excl_scan<ROOT_NT>(nch, red, tot);
    const uint32_t t_unit = tot;
    const uint32_t o_tab = block_excl_scan<ROOT_NT>(glob ? beta + 1 : 0u, red, tot);
    const uint32_t t_tab = tot;
    const uint32_t o_cm = block_excl_scan<ROOT_NT>(nch * nb, red, tot);
    const uint32_t t_cm = tot;
    const uint32_t o_aux = block_excl_scan<ROOT_NT>(nb, red, tot);
    const uint32_t t_aux = tot;
    const uint32_t o_i0 = block_excl_scan<ROOT_NT>(item && icls == 0 ? 1u : 0u, red, tot);
    const uint32_t t_i0 = tot;
    const uint32_t o_i1 = block_excl_scan<ROOT_NT>(item && icls == 1 ? 1u : 0u, red, tot);
    const uint32_t t_i1 = tot;
    const uint32_t o_i2 = block_excl_scan<ROOT_NT>(item && icls == 2 ? 1u : 0u, red, tot);
    const uint32_t t_i2 = tot;
    const char* kb = a.seg_src ? (s < a.nseg ? reinterpret_cast<const char*>(a.seg_src[s]) : nullptr)
                               : reinterpret_cast<const char*>(a.keys) + b0 * 8ull;
    const uint32_t* vb = a.vals ? a.vals + b0 : nullptr;
    if (item) {
      const uint64_t idx = base[5 + icls] + (icls == 0 ? o_i0 : (icls == 1 ? o_i1 : o_i2));
      if (idx < p.cap_items[icls]) {
        Item it;
        it.src = kb;
        it.vsrc = vb;
        it.off = b0;
        it.rel = 0;
        it.len = len;
        it.depth = 0;
        it.flags = IF_ROOT | (a.iota ? IF_IOTA : 0u);
        it.seg = s;
        p.items[icls][idx] = it;
      } else {
        flag_overflow(c);
      }
    }
    bool glob_ok = true;
    if (glob) {
      const uint64_t ni = base[0] + o_node, ub = base[1] + o_unit, tb = base[2] + o_tab;
      const uint64_t cb = base[3] + o_cm, ab = base[4] + o_aux;
      if (ni < p.cap_nodes && ub + nch <= p.cap_units && tb + beta + 1 <= p.cap_table &&
          cb + (uint64_t)nch * nb <= p.cap_cm && ab + nb <= p.cap_aux) {
        Node nd = {};
        nd.src = kb;
        nd.vsrc = vb;
        nd.mmp = p.mmr + ub;
        nd.off = b0;
        nd.rel = 0;
        nd.seed = a.has_fixed_seed ? a.fixed_seed : node_seed(p.seed, s, 0, 0);
        nd.table_off = tb;
        nd.cm_off = cb;
        nd.len = len;
        nd.seg = s;
        nd.depth = 0;
        nd.kind = p.pol.model ? NK_SPLINE : NK_PCF;
        nd.nchunks = nch;
        nd.unit_base = (uint32_t)ub;
        nd.aux_off = (uint32_t)ab;
        nd.mmn = nch;
        nd.nb = nb;
        nd.nbits = bits_for(nb);
        nd.beta = beta;
        nd.alpha = alpha;
        nd.delta = delta;
        nd.iota = a.iota;
        p.nodes[0][ni] = nd;
      } else {
        flag_overflow(c);
        glob_ok = false;
      }
    }
    // unit records of this block's roots, written by the whole workgroup
    ush[threadIdx.x] = (glob && glob_ok) ? nch : 0u;
    uni[threadIdx.x] = (uint32_t)(base[0] + o_node);
    unb[threadIdx.x] = (uint32_t)(base[1] + o_unit);
    __syncthreads();
    // this block's units are consecutive from base[1]: unit k belongs to the
    // last root whose first unit is at or before k (a search over unb)
    const uint32_t ub0 = (uint32_t)base[1];
    for (uint32_t k = threadIdx.x; k < t_unit; k += ROOT_NT) {
      uint32_t lo = 0, hi = ROOT_NT;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (unb[mid] - ub0 <= k) lo = mid;
        else hi = mid;
      }
      const uint32_t i = k - (unb[lo] - ub0);
      if (i < ush[lo]) p.units[0][unb[lo] + i] = Unit{uni[lo], i};
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      base[0] += t_node;
      base[1] += t_unit;
      base[2] += t_tab;
      base[3] += t_cm;
      base[4] += t_aux;
      base[5] += t_i0;
      base[6] += t_i1;
      base[7] += t_i2;
    }
    if (glob) atomicAdd(&base[8], (unsigned long long)len);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    c->lv[0].num_nodes = (uint32_t)base[0];
    c->lv[0].num_units = (uint32_t)base[1];
    c->lv[0].table_used = base[2];
    c->lv[0].cm_used = base[3];
    c->lv[0].aux_used = (uint32_t)base[4];
    c->item_count[0] = (uint32_t)base[5];
    c->item_count[1] = (uint32_t)base[6];
    c->item_count[2] = (uint32_t)base[7];
    c->lv[0].keys = base[8];
  }
}

// Chunk [b, e) of a unit: the node's keys split into nchunks equal parts.
__device__ __forceinline__ void chunk_range(const Node& nd, uint32_t chunk, uint32_t& b,
                                            uint32_t& e) {
  b = (uint32_t)(((uint64_t)nd.len * chunk) / nd.nchunks);
  e = (uint32_t)(((uint64_t)nd.len * (chunk + 1)) / nd.nchunks);
}

// ---------------------------------------------------------------------------
// K0: range of the level-0 nodes (x_min, x_max of Sec. 3.3) + key validation
// ---------------------------------------------------------------------------
// Each unit writes its own partial minimum and maximum; the fit kernel
// reduces them (no atomics on the node).
template <int KT, int NT>
__global__ __launch_bounds__(NT) void k_range(Plan p) {
  __shared__ uint64_t red[2 * NT / 64];
  __shared__ uint32_t bad_sh;
  const uint32_t nu = p.ctl->lv[0].num_units;
  constexpr int U = 8;
  for (uint32_t u = blockIdx.x; u < nu; u += gridDim.x) {
    const Unit un = p.units[0][u];
    const Node& nd = p.nodes[0][un.node];
    uint32_t b, e;
    chunk_range(nd, un.chunk, b, e);
    const uint64_t* src = reinterpret_cast<const uint64_t*>(nd.src);
    uint64_t lo = ~0ull, hi = 0ull;
    bool bad = false;
    for (uint32_t base = b; base < e; base += U * NT) {
      uint64_t v[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const uint32_t i = base + k * NT + threadIdx.x;
        v[k] = i < e ? __builtin_nontemporal_load(gld(src) + i) : 0ull;
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const uint32_t i = base + k * NT + threadIdx.x;
        if (i < e) {
          if (KT == KT_F64) bad |= !f64_bits_valid(v[k]);
          const uint64_t im = img_of<KT>(v[k]);
          lo = im < lo ? im : lo;
          hi = im > hi ? im : hi;
        }
      }
    }
    // a single root: this unit's share of its samples (positions depend only
    // on the node seed), so the fit reads them contiguously instead of
    // gathering them from one workgroup
    if (p.sbuf0 && p.ctl->lv[0].num_nodes == 1 && nd.kind != NK_RADIX && nd.alpha <= p.sbuf0_cap) {
      const uint32_t jb = (uint32_t)(((uint64_t)nd.alpha * un.chunk) / nd.nchunks);
      const uint32_t je = (uint32_t)(((uint64_t)nd.alpha * (un.chunk + 1)) / nd.nchunks);
      for (uint32_t j = jb + threadIdx.x; j < je; j += NT)
        gst(p.sbuf0)[j] = gld(src)[sample_pos(nd.seed, j, nd.len)];
    }
    if (threadIdx.x == 0) bad_sh = 0;
    __syncthreads();
    if (bad) bad_sh = 1;
    block_minmax_u64<NT>(lo, hi, red);
    if (threadIdx.x == 0) {
      if (bad_sh) atomicMax(&p.ctl->status, ERR_INVALID_KEY);
      p.mmr[u] = MinMax{lo, hi};
    }
  }
}

// ---------------------------------------------------------------------------
// K1: fit -- range, sample, histogram, prefix sum, bin -> bucket table
// ---------------------------------------------------------------------------
template <int KT, int NT>
__global__ __launch_bounds__(NT) void k_fit(Plan p, int L, int trace) {
  __shared__ uint32_t hist[MAX_BINS + 1];
  __shared__ uint32_t red[NT / 64 + 1];
  __shared__ uint64_t red64[2 * NT / 64];
  constexpr uint32_t RS = 256;  // samples that choose a radix node's digit scale
  __shared__ uint64_t rs_x[RS];
  __shared__ uint32_t rs_cnt[RS];
  __shared__ uint64_t rs_q[2];
  __shared__ uint32_t rs_dom[2];
  const int s = L & 1;
  Ctl* c = p.ctl;
  const uint32_t nn = c->lv[L].num_nodes;
  if (!ctl_ok(c)) return;  // status is fixed while this kernel runs
  for (uint32_t ni = blockIdx.x; ni < nn; ni += gridDim.x) {
    Node& nd = p.nodes[s][ni];
    // units and tasks of the node (also for a single-valued node: its units copy it)
    for (uint32_t i = threadIdx.x; i < nd.nchunks; i += NT)
      p.units[s][nd.unit_base + i] = Unit{ni, i};
    for (uint32_t q = threadIdx.x; q < nd.nb; q += NT) p.task_node[s][nd.aux_off + q] = ni;
    // range: reduce the producer's partial minima / maxima
    uint64_t lo = ~0ull, hi = 0ull;
    for (uint32_t i = threadIdx.x; i < nd.mmn; i += NT) {
      const uint64_t mlo = gld(nd.mmp)[i].lo, mhi = gld(nd.mmp)[i].hi;
      lo = mlo < lo ? mlo : lo;
      hi = mhi > hi ? mhi : hi;
    }
    block_minmax_u64<NT>(lo, hi, red64);
    if (lo == hi) {
      if (threadIdx.x == 0) {
        nd.min_img = lo;
        nd.max_img = hi;
        nd.state = NS_DONE;
        if (p.pol.prof) atomicAdd(&c->single_keys, (unsigned long long)nd.len);
      }
      __syncthreads();
      continue;
    }
    uint32_t kind = nd.kind, shift = 0, logd = 0;
    const uint32_t nb = nd.nb, beta = nd.beta, alpha = nd.alpha;
    BinFn f = {};
    if (kind != NK_RADIX && !bin_setup<KT>(f, lo, hi, beta)) kind = NK_RADIX;  // scale not finite
    if (kind == NK_RADIX) {
      // standard sort by most-significant digits of the range: nb buckets
      const uint64_t range = hi - lo;
      const uint32_t top = 63u - (uint32_t)__clzll((long long)range);
      const uint32_t nbits = nd.nbits;
      shift = top + 1 > nbits ? top + 1 - nbits : 0u;
      // Level budget.  A linear digit leaves its children at most
      // bl - nbits = bl - 8 bits of range (bl = top + 1), so a radix node of
      // bl bits finishes within ceil(bl / 8) levels plus the level that marks
      // its single-valued children done.  A log digit fixes only the leading
      // one and the two bits after it: children keep up to bl - 3 bits.  Log
      // digits are therefore taken only when the levels after this one can
      // still finish such a child linearly; every radix node then finishes
      // inside the call's nlev levels.
      const uint32_t left = p.nlev > (uint32_t)L + 1 ? p.nlev - (uint32_t)L - 1 : 0u;
      const bool log_fits = (top + 1 - 3 + 7) / 8 + 1 <= left;
      if (top >= 16 && nd.len >= RS && log_fits) {
        // RS samples: if most of them share one digit and, inside it, span
        // eight octaves or more between their 10th and 90th percentiles,
        // the keys spread over scales (clusters at log-uniform offsets) and
        // digits on a log scale split them; a point mass or a narrow range
        // keeps the linear digits
        const uint32_t t = threadIdx.x;
        if (t < RS) rs_cnt[t] = 0u;
        __syncthreads();
        uint64_t xs = 0;
        uint32_t dg = 0;
        if (t < RS) {
          xs = img_of<KT>(gld(reinterpret_cast<const uint64_t*>(nd.src))[sample_pos(nd.seed, t, nd.len)]) - lo;
          dg = (uint32_t)(xs >> shift);
          rs_x[t] = xs;
          atomicAdd(&rs_cnt[dg], 1u);
        }
        __syncthreads();
        if (t == 0) {
          uint32_t best = 0, bc = 0;
          for (uint32_t d = 0; d < RS; ++d)
            if (rs_cnt[d] > bc) {
              bc = rs_cnt[d];
              best = d;
            }
          rs_dom[0] = best;
          rs_dom[1] = bc;
          rs_q[0] = rs_q[1] = 0;
        }
        __syncthreads();
        const uint32_t dom = rs_dom[0], dcnt = rs_dom[1];
        if (dcnt >= RS / 2) {
          if (t < RS && dg == dom) {
            uint32_t rk = 0;  // rank among the dominant digit's samples (ties by index)
            for (uint32_t j = 0; j < RS; ++j) {
              const uint64_t xj = rs_x[j];
              rk += ((uint32_t)(xj >> shift) == dom) && (xj < xs || (xj == xs && j < t));
            }
            if (rk == dcnt / 10) rs_q[0] = xs;
            if (rk == dcnt - 1 - dcnt / 10) rs_q[1] = xs;
          }
          __syncthreads();
          const uint64_t q0 = rs_q[0], q1 = rs_q[1];
          const uint32_t e0 = q0 ? 64u - (uint32_t)__clzll((long long)q0) : 0u;
          const uint32_t e1 = q1 ? 64u - (uint32_t)__clzll((long long)q1) : 0u;
          logd = e1 >= e0 + 8 ? 1u : 0u;
        }
      }
    } else {
      for (uint32_t i = threadIdx.x; i <= beta; i += NT) hist[i] = 0u;
      __syncthreads();
      const uint64_t* src = reinterpret_cast<const uint64_t*>(nd.src);
      // a single root's samples were gathered by the range kernel
      const bool pre = L == 0 && p.sbuf0 && nn == 1 && alpha <= p.sbuf0_cap;
      // samples in batches of 8 per thread: all loads issued before any atomic
      constexpr int SB = 8;
      for (uint32_t j0 = 0; j0 < alpha; j0 += SB * NT) {
        uint64_t v[SB];
#pragma unroll
        for (int k = 0; k < SB; ++k) {
          const uint32_t j = j0 + k * NT + threadIdx.x;
          v[k] = j < alpha ? (pre ? gld(p.sbuf0)[j] : gld(src)[sample_pos(nd.seed, j, nd.len)])
                           : 0ull;
        }
#pragma unroll
        for (int k = 0; k < SB; ++k)
          if (j0 + k * NT + threadIdx.x < alpha) atomicAdd(&hist[bin_of<KT>(f, v[k])], 1u);
      }
      __syncthreads();
      block_scan_array<NT, true>(hist, beta + 1, red);
      if (trace && L == 0 && ni == 0 && p.trace_b)
        for (uint32_t i = threadIdx.x; i <= beta; i += NT) p.trace_b[i] = hist[i];
      const uint32_t gamma = nb - 1;
      uint16_t* tab = p.table[s] + nd.table_off;
      if (kind == NK_SPLINE) {
        // the spline interpolates between prefix counts: keep b_i itself
        for (uint32_t i = threadIdx.x; i <= beta; i += NT) tab[i] = (uint16_t)hist[i];
      } else if (alpha <= (1u << 21)) {
        // b_i <= alpha and gamma < 2^11: the product fits 32 bits and the
        // exact quotient takes the cheaper 32-bit division
        for (uint32_t i = threadIdx.x; i <= beta; i += NT)
          tab[i] = (uint16_t)((hist[i] * gamma) / alpha);
      } else {
        for (uint32_t i = threadIdx.x; i <= beta; i += NT)
          tab[i] = (uint16_t)(((uint64_t)hist[i] * gamma) / alpha);
      }
    }
    if (threadIdx.x == 0) {
      if (p.pol.prof && kind == NK_RADIX) {
        atomicAdd(&c->radix_keys, (unsigned long long)nd.len);
        atomicAdd(&c->lv[L].radix_keys, (unsigned long long)nd.len);
      }
      nd.kind = kind;
      nd.state = NS_ACTIVE;
      nd.shift = shift;
      nd.logd = logd;
      nd.halves = f.halves;
      nd.scale = f.s;
      nd.min_img = lo;
      nd.max_img = hi;
    }
    __syncthreads();
  }
}

// Bucket of a key in an active node.  index() is pure arithmetic (the bin,
// or the radix digit); finish() maps a bin through the LDS table, so callers
// can batch the table reads of many keys.
template <int KT>
struct Bucketer {
  BinFn f;
  uint64_t lo_img;
  uint32_t shift;
  uint32_t radix;
  uint32_t logd;        // radix digits on a log scale
  uint32_t narrow;      // T held as bytes (at most 256 buckets)
  uint32_t spline;      // the table holds prefix counts b_i (App. A.5)
  double alpha, gamma;  // spline: sample count and last bucket index
  const void* tab;      // LDS copy of T (or of b for the spline)
  __device__ __forceinline__ uint32_t index(uint64_t bits) const {
    if (radix) {
      const uint64_t x = img_of<KT>(bits) - lo_img;
      if (!logd) return (uint32_t)(x >> shift);
      // four digits per octave: the octave, then the two bits after the
      // leading one (monotone in x; at most 251)
      const uint32_t e = x ? 64u - (uint32_t)__clzll((long long)x) : 0u;
      return e <= 2 ? (uint32_t)x : (e - 2) * 4 + (uint32_t)((x >> (e - 3)) & 3u);
    }
    return bin_of<KT>(f, bits);
  }
  __device__ __forceinline__ uint32_t finish(uint32_t idx) const {
    if (radix) return idx;
    return narrow ? (uint32_t) reinterpret_cast<const uint8_t*>(tab)[idx]
                  : (uint32_t) reinterpret_cast<const uint16_t*>(tab)[idx];
  }
  // Spline bucket (App. A.5), 0-based: bin k, frac = p - k, and
  // floor((b_{k-1} + frac (b_k - b_{k-1})) gamma / alpha), one IEEE
  // round-to-nearest step per operation in the order t = frac * c,
  // v = b_{k-1} + t, u = v * gamma, w = u / alpha.
  __device__ __forceinline__ uint32_t spline_bucket(uint64_t bits) const {
    const uint16_t* b = reinterpret_cast<const uint16_t*>(tab);
    const double p = pos_of<KT>(f, bits);
    uint32_t k = (uint32_t)floor(p);
    k = k < f.beta ? k : f.beta;
    const double frac = p - (double)k;
    const uint32_t lo = k ? (uint32_t)b[k - 1] : 0u;
    const uint32_t cnt = (uint32_t)b[k] - lo;
    const double t = frac * (double)cnt;
    const double v = (double)lo + t;
    const double u = v * gamma;
    const double w = u / alpha;
    const uint32_t q = (uint32_t)floor(w);
    const uint32_t g = (uint32_t)gamma;
    return q < g ? q : g;
  }
  // bucket of a key whose index() was `idx`
  __device__ __forceinline__ uint32_t finish2(uint32_t idx, uint64_t bits) const {
    return spline ? spline_bucket(bits) : finish(idx);
  }
  __device__ __forceinline__ uint32_t operator()(uint64_t bits) const {
    return spline ? spline_bucket(bits) : finish(index(bits));
  }
};

template <int KT>
__device__ __forceinline__ Bucketer<KT> make_bucketer(const Node& nd, const void* tab_lds,
                                                     bool narrow = false) {
  Bucketer<KT> bk;
  bk.lo_img = nd.min_img;
  bk.shift = nd.shift;
  bk.logd = nd.logd;
  bk.radix = nd.kind == NK_RADIX;
  bk.spline = nd.kind == NK_SPLINE;
  bk.narrow = (narrow && !bk.spline) ? 1u : 0u;
  bk.alpha = (double)nd.alpha;
  bk.gamma = (double)(nd.nb - 1);
  bk.tab = tab_lds;
  const uint64_t lob = bits_of_img<KT>(nd.min_img);
  bk.f.lo_bits = lob;
  bk.f.beta = nd.beta;
  bk.f.halves = nd.halves;
  bk.f.s = nd.scale;
  if (KT == KT_F64) {
    bk.f.lo = __longlong_as_double((long long)lob);
    bk.f.lo_half = bk.f.lo * 0.5;
  } else {
    bk.f.lo = 0.0;
    bk.f.lo_half = 0.0;
  }
  return bk;
}

// ---------------------------------------------------------------------------
// K2: count -- bucket histogram of every (node, chunk) unit
// ---------------------------------------------------------------------------
template <int KT, int NT>
__global__ __launch_bounds__(NT) void k_count(Plan p, int L) {
  extern __shared__ __align__(16) unsigned char lds[];
  uint16_t* tab = reinterpret_cast<uint16_t*>(lds);                       // MAX_BINS + 1
  uint32_t* hist = reinterpret_cast<uint32_t*>(lds + 2 * (MAX_BINS + 1));  // MAX_NB
  const int s = L & 1;
  Ctl* c = p.ctl;
  const uint32_t nu = c->lv[L].num_units;
  if (!ctl_ok(c)) return;
  const int l = lane_id();
  uint32_t tab_node = 0xffffffffu;  // node whose table the LDS holds
  for (uint32_t u = blockIdx.x; u < nu; u += gridDim.x) {
    const Unit un = p.units[s][u];
    const Node& nd = p.nodes[s][un.node];
    if (nd.state != NS_ACTIVE) continue;
    const uint32_t nb = nd.nb;
    if (nd.kind != NK_RADIX && un.node != tab_node) {
      for (uint32_t i = threadIdx.x; i <= nd.beta; i += NT) tab[i] = p.table[s][nd.table_off + i];
      tab_node = un.node;
    }
    for (uint32_t i = threadIdx.x; i < nb; i += NT) hist[i] = 0u;
    __syncthreads();
    const Bucketer<KT> bk = make_bucketer<KT>(nd, tab);
    uint32_t b, e;
    chunk_range(nd, un.chunk, b, e);
    const uint64_t* src = reinterpret_cast<const uint64_t*>(nd.src);
    // software pipeline: the next block's keys are loaded while this one is
    // counted; table reads and LDS atomics of a block are issued back to back
    constexpr int U = 8;
    uint64_t v[U], nv[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint32_t i = b + k * NT + threadIdx.x;
      nv[k] = i < e ? __builtin_nontemporal_load(gld(src) + i) : 0ull;
    }
    for (uint32_t base = b; base < e; base += U * NT) {
#pragma unroll
      for (int k = 0; k < U; ++k) v[k] = nv[k];
      const uint32_t nb2 = base + U * NT;
      if (nb2 < e) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
          const uint32_t i = nb2 + k * NT + threadIdx.x;
          nv[k] = i < e ? __builtin_nontemporal_load(gld(src) + i) : 0ull;
        }
      }
      uint32_t q[U];
#pragma unroll
      for (int k = 0; k < U; ++k) q[k] = bk.index(v[k]);
#pragma unroll
      for (int k = 0; k < U; ++k) q[k] = bk.finish2(q[k], v[k]);
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const uint32_t i = base + k * NT + threadIdx.x;
        const bool valid = i < e;
        uint32_t qk = valid ? q[k] : 0u;
        if (qk >= nb) {
          flag_internal(c);
          qk = nb - 1;
        }
        // a whole wave in one bucket (runs of duplicates): one add
        const uint32_t q0 = __builtin_amdgcn_readfirstlane(qk);
        const uint64_t act = __ballot(valid);
        if (act == ~0ull && __all(qk == q0)) {
          if (l == 0) atomicAdd(&hist[q0], 64u);
        } else if (valid) {
          atomicAdd(&hist[qk], 1u);
        }
      }
    }
    __syncthreads();
    uint32_t* col = p.cm[s] + nd.cm_off;
    for (uint32_t q = threadIdx.x; q < nb; q += NT) col[(uint64_t)q * nd.nchunks + un.chunk] = hist[q];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// K3a: column scan -- for every (node, bucket): exclusive scan over chunks
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(NT) void k_colscan(Plan p, int L) {
  const int s = L & 1;
  Ctl* c = p.ctl;
  const uint32_t nt = c->lv[L].aux_used;
  if (!ctl_ok(c)) return;
  constexpr int NW = NT / 64;
  const int l = lane_id();
  for (uint32_t t = blockIdx.x * NW + wave_id(); t < nt; t += gridDim.x * NW) {
    const uint32_t ni = p.task_node[s][t];
    const Node& nd = p.nodes[s][ni];
    if (nd.state != NS_ACTIVE) continue;
    const uint32_t q = t - nd.aux_off;
    const uint32_t C = nd.nchunks;
    uint32_t* col = p.cm[s] + nd.cm_off + (uint64_t)q * C;
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < C; c0 += 64) {
      const uint32_t v = (c0 + l < C) ? col[c0 + l] : 0u;
      const uint32_t x = wave_incl_scan(v);
      if (c0 + l < C) col[c0 + l] = carry + x - v;
      carry += __shfl(x, 63, 64);
    }
    if (l == 0) p.bstart[s][nd.aux_off + q] = carry;  // bucket total for now
  }
}

// ---------------------------------------------------------------------------
// K3b: classify -- bucket starts and the paper's per-bucket decision
// ---------------------------------------------------------------------------
enum : uint32_t { BC_EMPTY = 0, BC_LDS_PCF = 1, BC_LDS_STD = 2, BC_GLB_PCF = 3, BC_GLB_RADIX = 4 };

template <int NT>
__global__ __launch_bounds__(NT) void k_classify(Plan p, int L, LevelIO io) {
  __shared__ uint32_t st[MAX_NB + 1];
  __shared__ uint32_t pre[MAX_NB];
  __shared__ uint8_t cls[MAX_NB];
  __shared__ uint8_t istart[MAX_NB];
  __shared__ uint32_t red[NT / 64 + 1];
  __shared__ unsigned long long base[8];
  const int s = L & 1, s1 = (L + 1) & 1;
  Ctl* c = p.ctl;
  const uint32_t nn = c->lv[L].num_nodes;
  if (!ctl_ok(c)) return;
  const uint32_t cap = p.pol.lds_cap;
  const uint32_t half = p.pol.small_cap / 2 ? p.pol.small_cap / 2 : 1;
  const bool has_next = L + 1 < MAX_LEVELS;
  LevelCtr* ln = &c->lv[has_next ? L + 1 : L];
  for (uint32_t ni = blockIdx.x; ni < nn; ni += gridDim.x) {
    const Node& nd = p.nodes[s][ni];
    if (nd.state != NS_ACTIVE) continue;
    const uint32_t nb = nd.nb;
    uint32_t* bs = p.bstart[s] + nd.aux_off;
    int32_t* cmap = p.cmap[s] + nd.aux_off;
    for (uint32_t q = threadIdx.x; q < nb; q += NT) st[q] = bs[q];
    __syncthreads();
    block_scan_array<NT, false>(st, nb, red);
    if (threadIdx.x == 0) st[nb] = nd.len;
    __syncthreads();
    // buckets of a radix node that fit LDS are finished by the in-LDS PCF
    // levels, which are themselves a correct standard sort of them
    const uint32_t lds_grp = BC_LDS_PCF;
    for (uint32_t q = threadIdx.x; q < nb; q += NT) {
      bs[q] = st[q];
      const uint32_t sz = st[q + 1] - st[q];
      uint32_t k;
      if (sz == 0) {
        k = BC_EMPTY;
      } else if (nd.kind == NK_RADIX) {
        k = sz <= cap ? BC_LDS_PCF : BC_GLB_RADIX;
      } else {
        const bool fail = sz >= nd.delta;  // Algorithm 1: |c_j| >= delta
        k = sz <= cap ? (fail ? BC_LDS_STD : BC_LDS_PCF) : (fail ? BC_GLB_RADIX : BC_GLB_PCF);
      }
      cls[q] = (uint8_t)k;
      pre[q] = (k == BC_EMPTY || k == BC_LDS_PCF || k == BC_LDS_STD) ? sz : 0u;
    }
    __syncthreads();
    block_scan_array<NT, false>(pre, nb, red);
    // LDS items: consecutive small buckets of one class packed up to small_cap
    // keys (sorting the union of consecutive buckets equals concatenating the
    // sorted buckets, because bucket ranges are disjoint and ordered).
    for (uint32_t q = threadIdx.x; q < nb; q += NT) {
      const uint32_t k = cls[q];
      uint32_t start = 0;
      if (k <= BC_LDS_STD) {
        const uint32_t g = k == BC_EMPTY ? lds_grp : k;
        const uint32_t sz = st[q + 1] - st[q];
        if (q == 0) {
          start = 1;
        } else {
          const uint32_t kp = cls[q - 1];
          const uint32_t gp = kp == BC_EMPTY ? lds_grp : kp;
          const uint32_t szp = st[q] - st[q - 1];
          start = (kp > BC_LDS_STD) || gp != g || sz > half || szp > half ||
                  (pre[q] / half) != (pre[q - 1] / half);
        }
      }
      istart[q] = (uint8_t)start;
    }
    __syncthreads();
    // per bucket: item length (0 if none) and the child's arena needs; the
    // LDS arrays are reused for the scans (pre: item class 0, st kept)
    constexpr int PER = (MAX_NB + NT - 1) / NT;
    uint32_t ilen[PER], icl[PER];
    uint32_t cnb[PER], cbeta[PER], calpha[PER], cdelta[PER], cnch[PER];
    uint32_t n_i0 = 0, n_i1 = 0, n_i2 = 0, n_node = 0, n_unit = 0, n_tab = 0, n_cm = 0, n_aux = 0, n_key = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const uint32_t q = threadIdx.x * PER + k;  // contiguous runs per thread
      ilen[k] = 0;
      icl[k] = 0;
      cnb[k] = 0;
      cnch[k] = 0;
      cbeta[k] = 0;
      if (q < nb) {
        const uint32_t kq = cls[q];
        if (istart[q]) {
          uint32_t e = q + 1;
          while (e < nb && cls[e] <= BC_LDS_STD && !istart[e]) ++e;
          ilen[k] = st[e] - st[q];
          icl[k] = (uint32_t)item_class(ilen[k], p.pol);
          if (ilen[k]) {
            if (icl[k] == 0) ++n_i0;
            else if (icl[k] == 1) ++n_i1;
            else ++n_i2;
          }
        }
        if (kq >= BC_GLB_PCF && has_next) {
          const uint32_t sz = st[q + 1] - st[q];
          const PolicyDev np = node_pol(p, sz);
          node_params(sz, kq == BC_GLB_RADIX ? NK_RADIX : (p.pol.model ? NK_SPLINE : NK_PCF), np,
                      cnb[k], cbeta[k], calpha[k], cdelta[k]);
          cnch[k] = (sz + np.chunk_keys - 1) / np.chunk_keys;
          ++n_node;
          n_unit += cnch[k];
          n_tab += kq == BC_GLB_PCF ? cbeta[k] + 1 : 0u;
          n_cm += cnch[k] * cnb[k];
          n_aux += cnb[k];
          n_key += sz;
        }
      }
    }
    uint32_t t0, t1, t2, t3, t4, t5, t6, t7;
    const uint32_t o_i0 = block_excl_scan<NT>(n_i0, red, t0);
    const uint32_t o_i1 = block_excl_scan<NT>(n_i1, red, t1);
    const uint32_t o_i2 = block_excl_scan<NT>(n_i2, red, t7);
    const uint32_t o_node = block_excl_scan<NT>(n_node, red, t2);
    const uint32_t o_unit = block_excl_scan<NT>(n_unit, red, t3);
    const uint32_t o_tab = block_excl_scan<NT>(n_tab, red, t4);
    const uint32_t o_cm = block_excl_scan<NT>(n_cm, red, t5);
    const uint32_t o_aux = block_excl_scan<NT>(n_aux, red, t6);
    uint32_t tk;
    block_excl_scan<NT>(n_key, red, tk);
    if (threadIdx.x == 0) {
      // one reservation per parent node and list
      base[0] = t0 ? atomicAdd(&c->item_count[0], t0) : 0u;
      base[1] = t1 ? atomicAdd(&c->item_count[1], t1) : 0u;
      base[7] = t7 ? atomicAdd(&c->item_count[2], t7) : 0u;
      base[2] = t2 ? atomicAdd(&ln->num_nodes, t2) : 0u;
      base[3] = t3 ? atomicAdd(&ln->num_units, t3) : 0u;
      base[4] = t4 ? atomicAdd(&ln->table_used, (unsigned long long)t4) : 0ull;
      base[5] = t5 ? atomicAdd(&ln->cm_used, (unsigned long long)t5) : 0ull;
      base[6] = t6 ? atomicAdd(&ln->aux_used, t6) : 0u;
      if (tk) atomicAdd(&ln->keys, (unsigned long long)tk);
    }
    __syncthreads();
    uint64_t bi0 = base[0] + o_i0, bi1 = base[1] + o_i1, bi2 = base[7] + o_i2,
             bn = base[2] + o_node,
             bu = base[3] + o_unit, bt = base[4] + o_tab, bc = base[5] + o_cm,
             ba = base[6] + o_aux;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const uint32_t q = threadIdx.x * PER + k;
      if (q >= nb) break;
      cmap[q] = -1;
      if (ilen[k]) {
        const int ic = (int)icl[k];
        const uint64_t idx = ic == 0 ? bi0++ : (ic == 1 ? bi1++ : bi2++);
        if (idx >= p.cap_items[ic]) {
          flag_overflow(c);
        } else {
          const uint32_t kq = cls[q];
          const uint32_t g = kq == BC_EMPTY ? lds_grp : kq;
          Item it;
          const uint64_t off = nd.off + st[q];
          it.src = reinterpret_cast<const char*>(io.dst_keys) + off * 8ull;
          it.vsrc = p.has_pay ? io.dst_vals + off : nullptr;
          it.off = off;
          it.rel = nd.rel + st[q];
          it.len = ilen[k];
          it.depth = nd.depth + 1;
          it.flags = g == BC_LDS_STD ? IF_STD : 0u;
          it.seg = nd.seg;
          p.items[ic][idx] = it;
        }
      }
      if (cnb[k]) {
        const uint32_t kq = cls[q];
        const uint32_t sz = st[q + 1] - st[q];
        const uint64_t ci = bn++, ub = bu, tb = bt, cb = bc, ab = ba;
        const bool radix = kq == BC_GLB_RADIX;
        bu += cnch[k];
        bt += radix ? 0u : cbeta[k] + 1;
        bc += (uint64_t)cnch[k] * cnb[k];
        ba += cnb[k];
        if (ci >= p.cap_nodes || ub + cnch[k] > p.cap_units || tb + cbeta[k] + 1 > p.cap_table ||
            cb + (uint64_t)cnch[k] * cnb[k] > p.cap_cm || ab + cnb[k] > p.cap_aux) {
          flag_overflow(c);
          continue;
        }
        Node ch = {};
        const uint64_t off = nd.off + st[q];
        ch.src = reinterpret_cast<const char*>(io.dst_keys) + off * 8ull;
        ch.vsrc = p.has_pay ? io.dst_vals + off : nullptr;
        ch.mmp = p.mm[s] + nd.cm_off + (uint64_t)q * nd.nchunks;  // filled by the scatter
        ch.mmn = nd.nchunks;
        ch.off = off;
        ch.rel = nd.rel + st[q];
        ch.seed = node_seed(p.seed, nd.seg, nd.depth + 1, ch.rel);
        ch.table_off = tb;
        ch.cm_off = cb;
        ch.len = sz;
        ch.seg = nd.seg;
        ch.depth = nd.depth + 1;
        ch.kind = radix ? NK_RADIX : (p.pol.model ? NK_SPLINE : NK_PCF);
        ch.nchunks = cnch[k];
        ch.unit_base = (uint32_t)ub;
        ch.aux_off = (uint32_t)ab;
        ch.nb = cnb[k];
        ch.nbits = bits_for(cnb[k]);
        ch.beta = cbeta[k];
        ch.alpha = calpha[k];
        ch.delta = cdelta[k];
        p.nodes[s1][ci] = ch;
        cmap[q] = (int32_t)ci;
      }
    }
    if (!has_next) {
      for (uint32_t q = threadIdx.x; q < nb; q += NT)
        if (cls[q] >= BC_GLB_PCF) flag_overflow(c);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// K4: scatter -- LDS-staged, coalesced; stable when a payload travels
// ---------------------------------------------------------------------------
// With a payload the tile ranking is stable (wave ballots + per-wave bucket
// counters) so that equal keys keep their input order.  Keys alone need no
// stability (equal keys are the same bits), so their tile ranks come from LDS
// atomics, which is several times cheaper.
// The second launch bound is waves per SIMD: 4 keeps two 512-thread
// workgroups resident per CU (at most 128 VGPRs); the stable variant needs
// more registers and runs one workgroup per CU.
template <int KT, int NT, int TS, int PAY>
__global__ __launch_bounds__(NT, (PAY && TS > 2048) ? 2 : 4) void k_scatter(Plan p, int L, LevelIO io, uint32_t max_bins,
                                                uint32_t nbmax) {
  constexpr int NW = NT / 64;
  constexpr int PW = TS / NW;   // keys of a wave per tile
  constexpr int R = PW / 64;    // rounds per wave
  static_assert(PW % 64 == 0, "tile must split into whole wave rounds");
  extern __shared__ __align__(16) unsigned char lds[];
  const ScatterLds lay = scatter_lds(max_bins, nbmax, NW, TS, PAY, (int)p.pol.model);
  unsigned char* tab = lds + lay.tab;  // T as bytes when nbmax <= 256, else uint16
  const bool tab8 = nbmax <= 256 && !p.pol.model;  // spline tables hold b_i: 16 bits
  uint16_t* wcnt = reinterpret_cast<uint16_t*>(lds + lay.wcnt);
  uint32_t* runoff = reinterpret_cast<uint32_t*>(lds + lay.runoff);
  uint32_t* tstart = reinterpret_cast<uint32_t*>(lds + lay.tstart);
  uint32_t* tcnt = reinterpret_cast<uint32_t*>(lds + lay.tcnt);
  unsigned long long* mmlo = reinterpret_cast<unsigned long long*>(lds + lay.mmlo);
  unsigned long long* mmhi = reinterpret_cast<unsigned long long*>(lds + lay.mmhi);
  uint8_t* cmapf = reinterpret_cast<uint8_t*>(lds + lay.cmapf);
  uint64_t* sk = reinterpret_cast<uint64_t*>(lds + lay.sk);
  uint32_t* sv = reinterpret_cast<uint32_t*>(lds + lay.sv);
  uint16_t* sb = reinterpret_cast<uint16_t*>(lds + lay.sb);
  __shared__ uint32_t red[NW + 1];

  const int s = L & 1;
  Ctl* c = p.ctl;
  const uint32_t nu = c->lv[L].num_units;
  if (!ctl_ok(c)) return;
  const int l = lane_id(), w = wave_id();
  uint64_t* dk = reinterpret_cast<uint64_t*>(io.dst_keys);
  uint32_t tab_node = 0xffffffffu;  // node whose table the LDS holds
  uint32_t* dv = io.dst_vals;
  uint64_t* ok_ = reinterpret_cast<uint64_t*>(p.out_keys);

  const uint32_t per = (nu + 7) / 8;
  for (uint32_t v = blockIdx.x; v < 8 * per; v += gridDim.x) {
    const uint32_t u = xcd_unit(v, per);
    if (u >= nu) continue;
    const Unit un = p.units[s][u];
    const Node& nd = p.nodes[s][un.node];
    uint32_t cb, ce;
    chunk_range(nd, un.chunk, cb, ce);
    const uint64_t* src = reinterpret_cast<const uint64_t*>(nd.src);
    if (nd.state == NS_DONE) {
      // single-valued node: already in order; move it to the output if needed
      uint64_t* o = ok_ + nd.off;
      if ((const void*)o != nd.src)
        for (uint32_t i = cb + threadIdx.x; i < ce; i += NT) gst(o)[i] = gld(src)[i];
      if (PAY) {
        uint32_t* ov = p.out_vals + nd.off;
        if (nd.vsrc == nullptr) {
          for (uint32_t i = cb + threadIdx.x; i < ce; i += NT) ov[i] = (uint32_t)nd.rel + i;
        } else if (ov != nd.vsrc) {
          for (uint32_t i = cb + threadIdx.x; i < ce; i += NT) gst(ov)[i] = gld(nd.vsrc)[i];
        }
      }
      continue;
    }
    const uint32_t nb = nd.nb, nbits = nd.nbits, C = nd.nchunks;
    if (nd.kind != NK_RADIX && un.node != tab_node) {
      tab_node = un.node;
      const uint16_t* tg = p.table[s] + nd.table_off;
      if (tab8)
        for (uint32_t i = threadIdx.x; i <= nd.beta; i += NT) tab[i] = (unsigned char)tg[i];
      else
        for (uint32_t i = threadIdx.x; i <= nd.beta; i += NT)
          reinterpret_cast<uint16_t*>(tab)[i] = tg[i];
    }
    const uint32_t* bs = p.bstart[s] + nd.aux_off;
    const int32_t* cm = p.cmap[s] + nd.aux_off;
    const uint32_t* col = p.cm[s] + nd.cm_off;
    for (uint32_t q = threadIdx.x; q < nb; q += NT) {
      runoff[q] = bs[q] + col[(uint64_t)q * C + un.chunk];
      cmapf[q] = cm[q] >= 0 ? 1 : 0;
      mmlo[q] = ~0ull;
      mmhi[q] = 0ull;
      tcnt[q] = 0u;
    }
    if (PAY)
      for (uint32_t q = threadIdx.x; q < NW * nb; q += NT) wcnt[q] = 0;
    bool glb = false;
    for (uint32_t q = threadIdx.x; q < nb; q += NT) glb |= cm[q] >= 0;
    const bool any_glb = __syncthreads_or(glb) != 0;
    const Bucketer<KT> bk = make_bucketer<KT>(nd, tab, tab8);
    const uint32_t* vsrc = nd.vsrc;
    const bool iota = PAY && vsrc == nullptr;

    // software pipeline: the next tile's keys are in flight while this one
    // is ranked, staged and written.  Every tile issues the same vector-memory
    // instructions (clamped addresses, no branch around them; positions of
    // an argsort's first level are read from the keys as a dummy and
    // replaced), so the wait for the prefetched tile leaves the previous
    // tile's stores in flight.  Range-check failures are reported after the
    // unit.
    bool bad = false;
    uint64_t key[R], nkey[R];
    uint32_t val[R], nval[R];
    // (chunks of a node are never empty; the clamped addresses below need a
    // key: an empty chunk skips the tiles and leaves neutral ranges)
    if (cb < ce) {
      const uint32_t* vld = iota ? reinterpret_cast<const uint32_t*>(src) : vsrc;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t i = cb + w * PW + r * 64 + l;
        const uint32_t ii = i < ce ? i : ce - 1;
        nkey[r] = __builtin_nontemporal_load(gld(src) + ii);
        if (PAY) {
          const uint32_t lv = gld(vld)[ii];
          nval[r] = iota ? (uint32_t)nd.rel + ii : lv;
        }
      }
      for (uint32_t t0 = cb; t0 < ce; t0 += TS) {
        const uint32_t tn = (ce - t0 < (uint32_t)TS) ? ce - t0 : (uint32_t)TS;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          key[r] = nkey[r];
          if (PAY) val[r] = nval[r];
        }
        const uint32_t t1 = t0 + TS;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t i = t1 + w * PW + r * 64 + l;  // past the chunk: the last key again
          const uint32_t ii = i < ce ? i : ce - 1;
          nkey[r] = __builtin_nontemporal_load(gld(src) + ii);
          if (PAY) {
            const uint32_t lv = gld(vld)[ii];
            nval[r] = iota ? (uint32_t)nd.rel + ii : lv;
          }
        }
        // bucket and rank of every key of the tile; wave w owns keys
        // [w*PW, (w+1)*PW), round r lane l
        uint32_t code[R];  // bucket << 16 | rank
        uint16_t* wc = wcnt + w * nb;
        // every table read of the tile is issued before the rank atomics
        uint32_t qq[R];
#pragma unroll
        for (int r = 0; r < R; ++r) qq[r] = bk.index(key[r]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t i = w * PW + r * 64 + l;
          uint32_t q = i < tn ? bk.finish2(qq[r], key[r]) : 0u;
          bad |= q >= nb;  // range check: cannot happen for a consistent model
          qq[r] = q < nb ? q : nb - 1;
        }
        if (any_glb) {
          // child ranges (lanes here hold unrelated buckets: few LDS conflicts)
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const uint32_t i = w * PW + r * 64 + l;
            if (i < tn && cmapf[qq[r]]) {
              const unsigned long long im = img_of<KT>(key[r]);
              atomicMin(&mmlo[qq[r]], im);
              atomicMax(&mmhi[qq[r]], im);
            }
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t i = w * PW + r * 64 + l;
          const bool valid = i < tn;
          const uint32_t q = qq[r];
          if (PAY) {
            // stable: rank among equal buckets in lane order, per-wave counters
            const uint64_t act = __ballot(valid);
            const uint64_t peers = wave_match(q, nbits, act);
            const uint32_t rk = (uint32_t)__popcll(peers & lanemask_lt());
            uint32_t base = 0;
            if (valid) base = wc[q];
            if (valid && rk == 0) wc[q] = (uint16_t)(base + (uint32_t)__popcll(peers));
            code[r] = (q << 16) | (base + rk);
          } else {
            // keys only: any order inside a bucket is the same output
            const uint32_t q0 = __builtin_amdgcn_readfirstlane(q);
            const uint64_t act = __ballot(valid);
            uint32_t rk = 0;
            if (act == ~0ull && __all(q == q0)) {
              uint32_t b0 = 0;
              if (l == 0) b0 = atomicAdd(&tcnt[q0], 64u);
              rk = __builtin_amdgcn_readfirstlane(b0) + l;
            } else if (valid) {
              rk = atomicAdd(&tcnt[q], 1u);
            }
            code[r] = (q << 16) | rk;
          }
        }
        __syncthreads();
        if (PAY) {
          // per bucket: wave offsets (exclusive over waves) and tile counts
          for (uint32_t q = threadIdx.x; q < nb; q += NT) {
            uint32_t run = 0;
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) {
              const uint32_t v = wcnt[ww * nb + q];
              wcnt[ww * nb + q] = (uint16_t)run;
              run += v;
            }
            tcnt[q] = run;
          }
          __syncthreads();
        }
        for (uint32_t q = threadIdx.x; q < nb; q += NT) tstart[q] = tcnt[q];
        __syncthreads();
        block_scan_array<NT, false>(tstart, nb, red);
        // stage keys in bucket order
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t i = w * PW + r * 64 + l;
          if (i < tn) {
            const uint32_t q = code[r] >> 16;
            const uint32_t pos = tstart[q] + (PAY ? wc[q] : 0u) + (code[r] & 0xffffu);
            if (pos < (uint32_t)TS) {
              sk[pos] = key[r];
              if (PAY) sv[pos] = val[r];
              sb[pos] = (uint16_t)q;
            } else {
              bad = true;
            }
          }
        }
        __syncthreads();
        // write runs: consecutive staged keys of one bucket are consecutive in
        // HBM.  A lane past the tile's end repeats the store of the tile's last
        // staged key (same values, same addresses).
        {
          constexpr int WPT = TS / NT;
#pragma unroll
          for (int k = 0; k < WPT; ++k) {
            const uint32_t i = threadIdx.x + k * NT;
            const uint32_t ic = i < tn ? i : tn - 1;
            const uint32_t q = sb[ic];
            const uint32_t rel = runoff[q] + (ic - tstart[q]);
            bad |= rel >= nd.len;
            const uint64_t dst = nd.off + (rel < nd.len ? rel : nd.len - 1);
            gst(dk)[dst] = sk[ic];
            if (PAY) gst(dv)[dst] = sv[ic];
          }
        }
        __syncthreads();
        for (uint32_t q = threadIdx.x; q < nb; q += NT) {
          runoff[q] += tcnt[q];
          tcnt[q] = 0u;
          if (PAY) {
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) wcnt[ww * nb + q] = 0;
          }
        }
        __syncthreads();
      }
    }
    if (bad) flag_internal(c);
    // this chunk's range of every child that is a node of the next level
    MinMax* mm = p.mm[s] + nd.cm_off;
    for (uint32_t q = threadIdx.x; q < nb; q += NT)
      if (cmapf[q]) mm[(uint64_t)q * C + un.chunk] = MinMax{mmlo[q], mmhi[q]};
    __syncthreads();
  }
}


// Keys only: tile ranks from LDS atomics (order inside a bucket is not
// observable for keys alone).  A tile costs three barriers:
//   rank (LDS atomics) | wave 0: tile bucket starts, write bases, run offsets |
//   stage in bucket order | write runs (overlaps the next tile's rank phase).
template <int KT, int NT, int TS>
__global__ __launch_bounds__(NT, (TS / NT >= 16 ? 2 : 4)) void k_scatter_keys(Plan p, int L, LevelIO io, uint32_t max_bins,
                                                     uint32_t nbmax) {
  constexpr int NW = NT / 64;
  constexpr int PW = TS / NW;
  constexpr int R = PW / 64;
  static_assert(PW % 64 == 0, "tile must split into whole wave rounds");
  extern __shared__ __align__(16) unsigned char lds[];
  const ScatterKeysLds lay = scatter_keys_lds(max_bins, nbmax, TS, (int)p.pol.model);
  unsigned char* tab = lds + lay.tab;  // T as bytes when nbmax <= 256, else uint16
  const bool tab8 = nbmax <= 256 && !p.pol.model;  // spline tables hold b_i: 16 bits
  uint32_t* runoff = reinterpret_cast<uint32_t*>(lds + lay.runoff);
  uint32_t* tstart = reinterpret_cast<uint32_t*>(lds + lay.tstart);
  uint32_t* wbase = reinterpret_cast<uint32_t*>(lds + lay.wbase);
  uint32_t* tcnt = reinterpret_cast<uint32_t*>(lds + lay.tcnt);
  unsigned long long* mmlo = reinterpret_cast<unsigned long long*>(lds + lay.mmlo);
  unsigned long long* mmhi = reinterpret_cast<unsigned long long*>(lds + lay.mmhi);
  uint8_t* cmapf = reinterpret_cast<uint8_t*>(lds + lay.cmapf);
  uint64_t* sk = reinterpret_cast<uint64_t*>(lds + lay.sk);
  uint16_t* sb = reinterpret_cast<uint16_t*>(lds + lay.sb);

  const int s = L & 1;
  Ctl* c = p.ctl;
  const uint32_t nu = c->lv[L].num_units;
  if (!ctl_ok(c)) return;
  const int l = lane_id(), w = wave_id();
  uint64_t* dk = reinterpret_cast<uint64_t*>(io.dst_keys);
  uint32_t tab_node = 0xffffffffu;  // node whose table the LDS holds
  uint64_t* ok_ = reinterpret_cast<uint64_t*>(p.out_keys);

  const uint32_t per = (nu + 7) / 8;
  for (uint32_t v = blockIdx.x; v < 8 * per; v += gridDim.x) {
    const uint32_t u = xcd_unit(v, per);
    if (u >= nu) continue;
    const Unit un = p.units[s][u];
    const Node& nd = p.nodes[s][un.node];
    uint32_t cb, ce;
    chunk_range(nd, un.chunk, cb, ce);
    const uint64_t* src = reinterpret_cast<const uint64_t*>(nd.src);
    if (nd.state == NS_DONE) {
      // single-valued node: already in order; move it to the output if needed
      uint64_t* o = ok_ + nd.off;
      if ((const void*)o != nd.src)
        for (uint32_t i = cb + threadIdx.x; i < ce; i += NT) gst(o)[i] = gld(src)[i];
      continue;
    }
    const uint32_t nb = nd.nb, C = nd.nchunks;
    if (nd.kind != NK_RADIX && un.node != tab_node) {
      tab_node = un.node;
      const uint16_t* tg = p.table[s] + nd.table_off;
      if (tab8)
        for (uint32_t i = threadIdx.x; i <= nd.beta; i += NT) tab[i] = (unsigned char)tg[i];
      else
        for (uint32_t i = threadIdx.x; i <= nd.beta; i += NT)
          reinterpret_cast<uint16_t*>(tab)[i] = tg[i];
    }
    const uint32_t* bs = p.bstart[s] + nd.aux_off;
    const int32_t* cm = p.cmap[s] + nd.aux_off;
    const uint32_t* col = p.cm[s] + nd.cm_off;
    bool glb = false;
    for (uint32_t q = threadIdx.x; q < nb; q += NT) {
      runoff[q] = bs[q] + col[(uint64_t)q * C + un.chunk];
      tcnt[q] = 0u;
      const bool g = cm[q] >= 0;
      cmapf[q] = g ? 1 : 0;
      glb |= g;
      mmlo[q] = ~0ull;
      mmhi[q] = 0ull;
    }
    const bool any_glb = __syncthreads_or(glb) != 0;
    const Bucketer<KT> bk = make_bucketer<KT>(nd, tab, tab8);

    // software pipeline: the next tile's keys are in flight while this one
    // is ranked, staged and written.  Every tile issues the same vector-memory
    // instructions (R loads, then R stores, with clamped addresses and no
    // branch around them), so the wait for the prefetched keys is a fixed
    // count that leaves the previous tile's stores in flight.  Range-check
    // failures are collected and reported after the unit.
    bool bad = false;
    uint64_t key[R], nkey[R];
    // the common case: a PCF node with a byte table and an unhalved range,
    // whose bucket needs none of the general Bucketer's per-key tests (same
    // arithmetic, same result)
    const bool fast = KT == KT_F64 && nd.kind == NK_PCF && tab8 && !bk.f.halves;
    // (chunks of a node are never empty; the clamped addresses below need a
    // key: an empty chunk skips the tiles and leaves neutral ranges)
    if (cb < ce) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t i = cb + w * PW + r * 64 + l;
        nkey[r] = __builtin_nontemporal_load(gld(src) + (i < ce ? i : ce - 1));
      }
      for (uint32_t t0 = cb; t0 < ce; t0 += TS) {
        const uint32_t tn = (ce - t0 < (uint32_t)TS) ? ce - t0 : (uint32_t)TS;
#pragma unroll
        for (int r = 0; r < R; ++r) key[r] = nkey[r];
        const uint32_t t1 = t0 + TS;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t i = t1 + w * PW + r * 64 + l;  // past the chunk: the last key again
          nkey[r] = __builtin_nontemporal_load(gld(src) + (i < ce ? i : ce - 1));
        }
        // A: bucket of every key (all table reads issued before any atomic),
        // rank inside the tile's bucket, child ranges
        uint32_t qq[R];
        if (fast) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const double pos = KT == KT_F64
                                   ? (__longlong_as_double((long long)key[r]) - bk.f.lo) * bk.f.s
                                   : (double)(key[r] - bk.f.lo_bits) * bk.f.s;
            const uint32_t k = (uint32_t)floor(pos);
            qq[r] = k < bk.f.beta ? k : bk.f.beta;
          }
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const uint32_t i = w * PW + r * 64 + l;
            const uint32_t q = tab[qq[r]];  // T_i <= gamma < nb
            qq[r] = i < tn ? q : 0u;
          }
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) qq[r] = bk.index(key[r]);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const uint32_t i = w * PW + r * 64 + l;
            uint32_t q = i < tn ? bk.finish2(qq[r], key[r]) : 0u;
            bad |= q >= nb;  // range check: cannot happen for a consistent model
            qq[r] = q < nb ? q : nb - 1;
          }
        }
        uint32_t code[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t i = w * PW + r * 64 + l;
          const bool valid = i < tn;
          const uint32_t q = qq[r];
          const uint32_t q0 = __builtin_amdgcn_readfirstlane(q);
          const uint64_t act = __ballot(valid);
          uint32_t rk = 0;
          if (act == ~0ull && __all(q == q0)) {
            // the whole wave in one bucket (runs of near-equal keys)
            uint32_t b0 = 0;
            if (l == 0) b0 = atomicAdd(&tcnt[q0], 64u);
            rk = __builtin_amdgcn_readfirstlane(b0) + l;
            if (any_glb && cmapf[q0]) {
              const uint64_t im = img_of<KT>(key[r]);
              const uint64_t wlo = wave_min_u64(im), whi = wave_max_u64(im);
              if (l == 0) {
                atomicMin(&mmlo[q0], (unsigned long long)wlo);
                atomicMax(&mmhi[q0], (unsigned long long)whi);
              }
            }
          } else if (valid) {
            rk = atomicAdd(&tcnt[q], 1u);
            if (any_glb && cmapf[q]) {
              const unsigned long long im = img_of<KT>(key[r]);
              atomicMin(&mmlo[q], im);
              atomicMax(&mmhi[q], im);
            }
          }
          code[r] = (q << 16) | rk;
        }
        __syncthreads();
        // B (wave 0): tile bucket starts, write bases, next run offsets, counters
        if (w == 0) {
          uint32_t carry = 0;
          for (uint32_t q0 = 0; q0 < nb; q0 += 64) {
            const uint32_t q = q0 + l;
            const uint32_t v = q < nb ? tcnt[q] : 0u;
            const uint32_t x = wave_incl_scan(v);
            if (q < nb) {
              const uint32_t st = carry + x - v;
              const uint32_t ro = runoff[q];
              tstart[q] = st;
              wbase[q] = ro - st;
              runoff[q] = ro + v;
              tcnt[q] = 0u;
            }
            carry += (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
          }
        }
        __syncthreads();
        // C: stage keys in bucket order
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t i = w * PW + r * 64 + l;
          if (i < tn) {
            const uint32_t q = code[r] >> 16;
            const uint32_t pos = tstart[q] + (code[r] & 0xffffu);
            if (pos < (uint32_t)TS) {
              sk[pos] = key[r];
              sb[pos] = (uint16_t)q;
            } else {
              bad = true;
            }
          }
        }
        __syncthreads();
        // D: write runs (consecutive staged keys of one bucket go to consecutive
        // addresses); no barrier after it: the next tile's rank phase touches
        // only tcnt and the min/max, and its bucket-start phase comes after the
        // next barrier
        // (per half: the staged ids, then their write bases, then the keys,
        // each a batch of independent LDS reads).  A lane past the tile's end
        // repeats the store of the tile's last key: same value, same address.
        {
          constexpr int H = R / 2 > 0 ? R / 2 : 1;
#pragma unroll
          for (int h = 0; h < R; h += H) {
            uint32_t qd[H], wb[H], ic[H];
            uint64_t kd[H];
#pragma unroll
            for (int r = 0; r < H; ++r) {
              const uint32_t i = (h + r) * NT + threadIdx.x;
              ic[r] = i < tn ? i : tn - 1;
              qd[r] = sb[ic[r]];
            }
#pragma unroll
            for (int r = 0; r < H; ++r) wb[r] = wbase[qd[r]];
#pragma unroll
            for (int r = 0; r < H; ++r) kd[r] = sk[ic[r]];
#pragma unroll
            for (int r = 0; r < H; ++r) {
              const uint32_t rel = wb[r] + ic[r];
              bad |= rel >= nd.len;
              gst(dk)[nd.off + (rel < nd.len ? rel : nd.len - 1)] = kd[r];
            }
          }
        }
      }
    }
    if (bad) flag_internal(c);
    __syncthreads();
    if (any_glb) {
      MinMax* mm = p.mm[s] + nd.cm_off;
      for (uint32_t q = threadIdx.x; q < nb; q += NT)
        if (cmapf[q]) mm[(uint64_t)q * C + un.chunk] = MinMax{mmlo[q], mmhi[q]};
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// K5: finish an array inside one workgroup's LDS
// ---------------------------------------------------------------------------
// Algorithm 1 inside LDS.  Every level trains the PCF on all m keys of its
// array (alpha = m: Sec. 3.2 allows training on all elements) with beta = m
// equal-width bins, the top bin folded into bin m - 1, and gamma = alpha, so
// the bucket of a key, floor(b_{i(x)} gamma / alpha) = b_{i(x)}, is its bin:
// buckets hold about one key.  Buckets below tau get a counting rank, buckets
// of tau keys or more recurse, failed buckets (>= delta = floor(m^{3/4})) get
// the standard sort (in-LDS bitonic).  Ties are ordered by the key's position
// in the item when a payload makes order observable (the global scatters
// before this one are then stable); keys alone break ties by LDS index.
//
// The first level of an item runs from registers: keys are loaded once
// (coalesced), bucketed with LDS-atomic ranks, and written to LDS already in
// bin order, so an item whose bins all stay below tau costs five barriers.

// Exact floor(n^{3/4}) for the failure test of the (rare) big bins: an fp64
// estimate through two square roots, corrected with exact integer steps.
__device__ __forceinline__ uint32_t k5_root34(uint32_t n) {
  const double m = (double)n;
  uint64_t r = (uint64_t)sqrt(sqrt(m * m * m));
  auto le = [&](uint64_t x) {  // x^4 <= n^3 (both below 2^128: compare as 128-bit)
    const uint64_t x2 = x * x, n2 = (uint64_t)n * n;
    const uint64_t ah = __umul64hi(x2, x2), al = x2 * x2;
    const uint64_t bh = __umul64hi(n2, (uint64_t)n), bl = n2 * (uint64_t)n;
    return ah < bh || (ah == bh && al <= bl);
  };
  while (r > 0 && !le(r)) --r;
  while (le(r + 1)) ++r;
  return (uint32_t)r;
}

template <int KT, int CAP, int NT, int PAY>
__device__ void k5_bitonic(K5Smem<KT, CAP, NT, PAY>& sm, uint32_t s, uint32_t e) {
  const uint32_t n = e - s;
  uint32_t P = 1;
  while (P < n) P <<= 1;
  auto cmpswap = [&](uint32_t i, uint32_t j) {
    const uint64_t ki = sm.key[s + i], kj = sm.key[s + j];
    bool sw = kj < ki;
    if (PAY) sw = sw || (kj == ki && sm.pos[s + j] < sm.pos[s + i]);
    if (sw) {
      sm.key[s + i] = kj;
      sm.key[s + j] = ki;
      if (PAY) {
        const uint16_t pi = sm.pos[s + i];
        sm.pos[s + i] = sm.pos[s + j];
        sm.pos[s + j] = pi;
      }
    }
  };
  for (uint32_t k = 2; k <= P; k <<= 1) {
    const uint32_t hk = k >> 1;
    for (uint32_t t = threadIdx.x; t < P / 2; t += NT) {
      const uint32_t blk = t / hk, o = t % hk;
      const uint32_t i = blk * k + o, j = blk * k + k - 1 - o;
      if (j < n) cmpswap(i, j);
    }
    __syncthreads();
    for (uint32_t d = hk >> 1; d >= 1; d >>= 1) {
      for (uint32_t t = threadIdx.x; t < P / 2; t += NT) {
        const uint32_t blk = t / d, o = t % d;
        const uint32_t i = blk * 2 * d + o, j = i + d;
        if (j < n) cmpswap(i, j);
      }
      __syncthreads();
    }
  }
  for (uint32_t i = s + threadIdx.x; i < e; i += NT) sm.seg[i] = i | ((i + 1) << 16);
  __syncthreads();
}

// Exclusive scan, in place, of the bin counts cnt[0..CAP) of a level on the
// LDS range [s, s + n) (bins at or beyond n are zero); cnt[CAP] = n.  Bins of
// tau keys or more are pushed on the range stack, flagged as failed when they
// hold delta = floor(n^{3/4}) keys or more.  Two barriers.
template <int KT, int CAP, int NT, int PAY>
__device__ __forceinline__ void k5_scan_bins(K5Smem<KT, CAP, NT, PAY>& sm, uint32_t s, uint32_t n,
                                             uint32_t depth, uint32_t tau) {
  constexpr int EC = CAP / NT;
  static_assert(EC % 4 == 0, "bin runs are read as uint4");
  const int l = lane_id(), w = wave_id();
  uint4* p4 = reinterpret_cast<uint4*>(sm.cnt + threadIdx.x * EC);
  uint32_t c[EC];
#pragma unroll
  for (int j = 0; j < EC / 4; ++j) {
    const uint4 v = p4[j];
    c[4 * j] = v.x;
    c[4 * j + 1] = v.y;
    c[4 * j + 2] = v.z;
    c[4 * j + 3] = v.w;
  }
  uint32_t sum = 0;
  bool big = false;
#pragma unroll
  for (int j = 0; j < EC; ++j) {
    sum += c[j];
    big |= c[j] >= tau;
  }
  const uint32_t incl = wave_incl_scan(sum);
  if (l == 63) sm.red[w] = incl;
  __syncthreads();
  uint32_t run = incl - sum;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i)
    if (i < w) run += sm.red[i];
  uint32_t st[EC];
#pragma unroll
  for (int j = 0; j < EC; ++j) {
    st[j] = run;
    run += c[j];
  }
#pragma unroll
  for (int j = 0; j < EC / 4; ++j)
    p4[j] = make_uint4(st[4 * j], st[4 * j + 1], st[4 * j + 2], st[4 * j + 3]);
  if (big) {  // rare: a bin of at least tau keys
    const uint32_t delta = k5_root34(n);
#pragma unroll
    for (int j = 0; j < EC; ++j) {
      if (c[j] >= tau) {
        const uint32_t slot = atomicAdd(&sm.nstk, 1u);
        if (slot < K5Cfg<CAP>::SMAX) {
          sm.stk[slot][0] = s + st[j];
          sm.stk[slot][1] = s + st[j] + c[j];
          sm.stk[slot][2] = (depth + 1) | (c[j] >= delta ? 0x80000000u : 0u);
        } else {
          sm.flag = 1;  // cannot happen: ranges of >= tau keys are disjoint
        }
      }
    }
  }
  if (threadIdx.x == 0) sm.cnt[CAP] = n;
  __syncthreads();
}

// One PCF level on the LDS range [s, e) (a node of depth `depth`) with all of
// its keys as the training set and one bin per key.
template <int KT, int CAP, int NT, int PAY>
__device__ void k5_level(K5Smem<KT, CAP, NT, PAY>& sm, uint32_t s, uint32_t e, uint32_t depth,
                         uint64_t lo, uint64_t hi, uint32_t tau) {
  constexpr int EPT = (CAP + NT - 1) / NT;
  constexpr int EC = CAP / NT;
  const uint32_t n = e - s;
  BinFn f;
  if (!bin_setup<KT>(f, lo, hi, n)) {
    k5_bitonic<KT, CAP, NT, PAY>(sm, s, e);
    return;
  }
  uint4* p4 = reinterpret_cast<uint4*>(sm.cnt + threadIdx.x * EC);
#pragma unroll
  for (int j = 0; j < EC / 4; ++j) p4[j] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  uint64_t kk[EPT];
  uint32_t bp[EPT];  // bin | rank << 16 (both below 2^16)
  uint16_t ps[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const uint32_t i = s + threadIdx.x + k * NT;
    if (i < e) {
      kk[k] = sm.key[i];
      if (PAY) ps[k] = sm.pos[i];
      uint32_t b = bin_of<KT>(f, bits_of_img<KT>(kk[k]));
      b = b < n - 1 ? b : n - 1;
      bp[k] = b | (atomicAdd(&sm.cnt[b], 1u) << 16);
    }
  }
  __syncthreads();
  k5_scan_bins<KT, CAP, NT, PAY>(sm, s, n, depth, tau);
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const uint32_t i = s + threadIdx.x + k * NT;
    if (i < e) {
      const uint32_t b = bp[k] & 0xffffu;
      const uint32_t a = sm.cnt[b], z = sm.cnt[b + 1];
      const uint32_t d = s + a + (bp[k] >> 16);
      if (d >= e) continue;  // range check: cannot happen for consistent counts
      sm.key[d] = kk[k];
      if (PAY) sm.pos[d] = ps[k];
      sm.seg[d] = (s + a) | ((s + z) << 16);
    }
  }
  __syncthreads();
}

template <int KT, int CAP, int NT, int PAY>
__global__ __launch_bounds__(NT, (K5Occ<KT, CAP, PAY, NT>::v)) void k_lds_sort(Plan p, int cls) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  K5Smem<KT, CAP, NT, PAY>& sm = *reinterpret_cast<K5Smem<KT, CAP, NT, PAY>*>(lds_raw);
  constexpr int EPT = CAP / NT;
  constexpr int NW = NT / 64;
  Ctl* c = p.ctl;
  // the status is fixed while this kernel runs, except for invalid root keys
  // found here, which concern only their own item
  if (!ctl_ok(c)) return;
  const uint32_t total = c->item_count[cls] < p.cap_items[cls] ? c->item_count[cls]
                                                                : p.cap_items[cls];
  const uint32_t first = c->item_done[cls];  // items of earlier passes are done
  const uint32_t tau = p.pol.tau;
  uint64_t* ok_ = reinterpret_cast<uint64_t*>(p.out_keys);
  const int l = lane_id(), w = wave_id();
  unsigned long long done_keys = 0, bit_keys = 0, one_keys = 0;
  // static assignment of items to workgroups (a shared work counter would be
  // a same-address atomic per item)
  // fp64 keys: the next item's descriptor is loaded while this one is
  // sorted (its latency otherwise starts every item: 10 % of the small
  // class's time).  The uint64 instantiations keep the plain load: holding
  // the descriptor there raised their register spills and slowed them.
  constexpr bool IPF = KT == KT_F64;
  Item nit = {};
  if (IPF && first + blockIdx.x < total) nit = p.items[cls][first + blockIdx.x];
  for (uint32_t ii = first + blockIdx.x; ii < total; ii += gridDim.x) {
    const Item it = IPF ? nit : p.items[cls][ii];
    if (IPF && ii + gridDim.x < total) nit = p.items[cls][ii + gridDim.x];
    const uint32_t m = it.len;
    done_keys += m;
    uint64_t kk[EPT];
    {
      const uint64_t* s0 = reinterpret_cast<const uint64_t*>(it.src);
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const uint32_t i = threadIdx.x + k * NT;
        kk[k] = i < m ? __builtin_nontemporal_load(gld(s0) + i) : 0ull;
      }
    }
    // validate (roots), images, range; clear the bins
    uint64_t lo = ~0ull, hi = 0ull;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const uint32_t i = threadIdx.x + k * NT;
      if (i < m) {
        if (KT == KT_F64 && (it.flags & IF_ROOT)) bad |= !f64_bits_valid(kk[k]);
        kk[k] = img_of<KT>(kk[k]);
        lo = kk[k] < lo ? kk[k] : lo;
        hi = kk[k] > hi ? kk[k] : hi;
      }
    }
    {
      uint4* p4 = reinterpret_cast<uint4*>(sm.cnt + threadIdx.x * EPT);
#pragma unroll
      for (int j = 0; j < EPT / 4; ++j) p4[j] = make_uint4(0u, 0u, 0u, 0u);
    }
    lo = wave_min_u64(lo);
    hi = wave_max_u64(hi);
    const bool wbad = __ballot(bad) != 0ull;
    if (l == 0) {
      sm.red64[w] = lo;
      sm.red64[NW + w] = hi;
      sm.red[NW] = 0u;
    }
    if (threadIdx.x == 0) {
      sm.nstk = 0;
      sm.flag = 0;
    }
    __syncthreads();
    if (wbad && l == 0) sm.red[NW] = 1u;  // read after the next barrier
    lo = sm.red64[0];
    hi = sm.red64[NW];
#pragma unroll
    for (int i = 1; i < NW; ++i) {
      lo = sm.red64[i] < lo ? sm.red64[i] : lo;
      hi = sm.red64[NW + i] > hi ? sm.red64[NW + i] : hi;
    }
    uint64_t* ok = ok_ + it.off;
    if (lo == hi) one_keys += m;
    if (lo == hi && KT == KT_U64) {
      // single-valued: input order is the answer (a u64 range cannot be bad)
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const uint32_t i = threadIdx.x + k * NT;
        if (i < m) {
          ok[i] = bits_of_img<KT>(kk[k]);
          if (PAY) p.out_vals[it.off + i] = it.vsrc ? gld(it.vsrc)[i] : (uint32_t)it.rel + i;
        }
      }
      __syncthreads();  // the range was read from red64, which the next item rewrites
      continue;
    }
    BinFn f;
    const bool fast = m >= tau && lo != hi && !(it.flags & IF_STD) && bin_setup<KT>(f, lo, hi, m);
    if (fast) {
      // first level from registers: bin, rank inside the bin
      uint32_t bp[EPT];
      if (KT == KT_F64 && !f.halves) {
        // an unhalved fp64 range: the bin without bin_of's per-key select
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          const uint32_t i = threadIdx.x + k * NT;
          if (i < m) {
            const double v = __longlong_as_double((long long)bits_of_img<KT>(kk[k]));
            const uint32_t b0 = (uint32_t)floor((v - f.lo) * f.s);
            const uint32_t b = b0 < m - 1 ? b0 : m - 1;
            bp[k] = b | (atomicAdd(&sm.cnt[b], 1u) << 16);
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          const uint32_t i = threadIdx.x + k * NT;
          if (i < m) {
            uint32_t b = bin_of<KT>(f, bits_of_img<KT>(kk[k]));
            b = b < m - 1 ? b : m - 1;
            bp[k] = b | (atomicAdd(&sm.cnt[b], 1u) << 16);
          }
        }
      }
      __syncthreads();
      if (sm.red[NW]) {  // invalid key in a root item
        if (threadIdx.x == 0) atomicMax(&c->status, ERR_INVALID_KEY);
        __syncthreads();
        continue;
      }
      k5_scan_bins<KT, CAP, NT, PAY>(sm, 0, m, it.depth, tau);
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const uint32_t i = threadIdx.x + k * NT;
        if (i < m) {
          const uint32_t b = bp[k] & 0xffffu;
          const uint32_t a = sm.cnt[b], z = sm.cnt[b + 1];
          const uint32_t d = a + (bp[k] >> 16);
          if (d >= m) continue;  // range check: cannot happen for consistent counts
          sm.key[d] = kk[k];
          if (PAY) sm.pos[d] = (uint16_t)i;
          sm.seg[d] = a | (z << 16);
        }
      }
      __syncthreads();
    } else {
      // standard sort (tiny, failed or unbucketable arrays) or, for fp64,
      // a single value: everything goes through LDS; a range that needs the
      // standard sort goes on the stack as a failed range
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const uint32_t i = threadIdx.x + k * NT;
        if (i < m) {
          sm.key[i] = kk[k];
          if (PAY) sm.pos[i] = (uint16_t)i;
          sm.seg[i] = lo == hi ? (i | ((i + 1) << 16)) : (m << 16);
        }
      }
      if (threadIdx.x == 0 && lo != hi && m >= tau) {
        sm.stk[0][0] = 0;
        sm.stk[0][1] = m;
        sm.stk[0][2] = (uint32_t)it.depth | 0x80000000u;
        sm.nstk = 1;
      }
      __syncthreads();
      if (sm.red[NW]) {
        if (threadIdx.x == 0) atomicMax(&c->status, ERR_INVALID_KEY);
        __syncthreads();
        continue;
      }
    }
    // ranges still at or above tau: recurse (or standard sort if failed)
    while (sm.nstk != 0) {
      __syncthreads();
      if (threadIdx.x == 0) {
        const uint32_t k = sm.nstk < K5Cfg<CAP>::SMAX ? sm.nstk : K5Cfg<CAP>::SMAX;
        if (k > 0) {
          sm.sh[0] = sm.stk[k - 1][0];
          sm.sh[1] = sm.stk[k - 1][1];
          sm.sh[2] = sm.stk[k - 1][2];
          sm.sh[3] = 1;
          sm.nstk = k - 1;
        } else {
          sm.sh[3] = 0;
        }
      }
      __syncthreads();
      if (!sm.sh[3]) break;
      const uint32_t rs = sm.sh[0], re = sm.sh[1];
      const uint32_t rdepth = sm.sh[2] & 0x7fffffffu;
      const bool rfail = (sm.sh[2] >> 31) != 0;
      uint64_t rlo = ~0ull, rhi = 0ull;
      for (uint32_t i = rs + threadIdx.x; i < re; i += NT) {
        const uint64_t im = sm.key[i];
        rlo = im < rlo ? im : rlo;
        rhi = im > rhi ? im : rhi;
      }
      block_minmax_u64<NT>(rlo, rhi, sm.red64);
      if (rlo == rhi) one_keys += re - rs;
      else if (rfail) bit_keys += re - rs;
      if (rlo == rhi && !PAY) {
        // equal keys alone: any order is the sorted order
        for (uint32_t i = rs + threadIdx.x; i < re; i += NT) sm.seg[i] = i | ((i + 1) << 16);
        __syncthreads();
      } else if (rlo == rhi || rfail) {
        // equal keys (ordered by position) or a failed bucket: standard sort
        k5_bitonic<KT, CAP, NT, PAY>(sm, rs, re);
      } else {
        k5_level<KT, CAP, NT, PAY>(sm, rs, re, rdepth, rlo, rhi, tau);
      }
    }
    if (!PAY) {
      // final ranks inside the segments: a key alone in its segment already
      // sits at its rank; the others count the keys of their segment that
      // precede them (ties by position).  All LDS reads of this pass come
      // before a barrier; then the keys that are not in place move to their
      // ranks in LDS, and after a second barrier the item leaves in coalesced
      // rows, with nontemporal stores: nothing reads the output again here,
      // and lines left dirty in L2 slowed the next sort's first scatter.  The
      // next item writes keys only after its first barrier.
      uint64_t kv[EPT];
      uint32_t rk[EPT];
#pragma unroll
      for (int kq = 0; kq < EPT; ++kq) {
        const uint32_t i = threadIdx.x + kq * NT;
        rk[kq] = i;
        if (i < m) {
          const uint32_t sg = sm.seg[i];
          const uint32_t a = sg & 0xffffu, b = sg >> 16;
          const uint64_t k = sm.key[i];
          uint32_t rnk = a;
          if (b - a > 1) {
            for (uint32_t q = a; q < b; ++q) {
              const uint64_t kq2 = sm.key[q];
              rnk += (kq2 < k) || (kq2 == k && q < i);
            }
          }
          kv[kq] = k;
          rk[kq] = rnk;
        }
      }
      __syncthreads();
#pragma unroll
      for (int kq = 0; kq < EPT; ++kq) {
        const uint32_t i = threadIdx.x + kq * NT;
        if (i < m && rk[kq] != i) {
          if (rk[kq] < m) sm.key[rk[kq]] = kv[kq];
          else flag_internal(c);
        }
      }
      __syncthreads();
#pragma unroll
      for (int kq = 0; kq < EPT; ++kq) {
        const uint32_t i = threadIdx.x + kq * NT;
        if (i < m) __builtin_nontemporal_store(bits_of_img<KT>(sm.key[i]), ok + i);
      }
      continue;
    }
    // with a payload: counting rank inside final segments, then the
    // write-out.  All reads (LDS keys and the payload, which may live in the
    // very range being written) happen before a barrier and all writes after
    // it: ranks and payload words are staged in LDS at each key's own
    // position (seg and cnt are free by now).  Keys in segments of several
    // keys are ranked in a second, non-unrolled pass.  Outputs are written
    // with nontemporal stores, as for keys alone.  (Moving keys and payload
    // words to their ranks in LDS for a coalesced write-out, as for keys
    // alone, holds registers across a barrier and spilled here.)
    uint32_t multi = 0;  // bit kq: the key sits in a segment of several keys
#pragma unroll
    for (int kq = 0; kq < EPT; ++kq) {
      const uint32_t i = threadIdx.x + kq * NT;
      if (i < m) {
        const uint32_t sg = sm.seg[i];
        const uint32_t a = sg & 0xffffu, b = sg >> 16;
        if (b - a > 1) {
          multi |= 1u << kq;
        } else {
          const uint32_t ps = sm.pos[i];
          sm.cnt[i] = it.vsrc ? gld(it.vsrc)[ps] : (uint32_t)it.rel + ps;
          sm.seg[i] = a;
        }
      }
    }
#pragma unroll 1
    for (uint32_t mm = multi; mm != 0; mm &= mm - 1) {
      const int kq = __builtin_ctz(mm);
      const uint32_t i = threadIdx.x + kq * NT;
      const uint32_t sg = sm.seg[i];
      const uint32_t a = sg & 0xffffu, b = sg >> 16;
      const uint64_t k = sm.key[i];
      const uint32_t ps = sm.pos[i];
      uint32_t rnk = a;
      for (uint32_t q = a; q < b; ++q) {
        const uint64_t kq2 = sm.key[q];
        const uint32_t pq = sm.pos[q];
        rnk += (kq2 < k) || (kq2 == k && pq < ps);
      }
      // a thread reads seg only at its own positions: the rank can take
      // their place
      sm.cnt[i] = it.vsrc ? gld(it.vsrc)[ps] : (uint32_t)it.rel + ps;
      sm.seg[i] = rnk;
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < EPT; ++kq) {
      const uint32_t i = threadIdx.x + kq * NT;
      if (i < m) {
        const uint32_t rnk = sm.seg[i];
        if (rnk >= m) {
          flag_internal(c);
          continue;
        }
        __builtin_nontemporal_store(bits_of_img<KT>(sm.key[i]), ok + rnk);
        __builtin_nontemporal_store(sm.cnt[i], p.out_vals + it.off + rnk);
      }
    }
    __syncthreads();
  }
  if (p.pol.prof && threadIdx.x == 0 && done_keys) {
    atomicAdd(&c->item_keys[cls], done_keys);
    if (bit_keys) atomicAdd(&c->bitonic_keys, bit_keys);
    if (one_keys) atomicAdd(&c->single_keys, one_keys);
  }
}

// ---------------------------------------------------------------------------
// explicit instantiations used by the driver
// ---------------------------------------------------------------------------
#define PCF_INST_KT(KT)                                                                  \
  template __global__ void k_range<KT, 256>(Plan);                                       \
  template __global__ void k_fit<KT, 1024>(Plan, int, int);                              \
  template __global__ void k_count<KT, 512>(Plan, int);                                  \
  template __global__ void k_scatter_keys<KT, 1024, 8192>(Plan, int, LevelIO, uint32_t,  \
                                                         uint32_t);                      \
  template __global__ void k_scatter_keys<KT, 512, 4096>(Plan, int, LevelIO, uint32_t,   \
                                                         uint32_t);                      \
  template __global__ void k_scatter<KT, 512, 1024, 1>(Plan, int, LevelIO, uint32_t,     \
                                                       uint32_t);                        \
  template __global__ void k_scatter<KT, 512, 2048, 1>(Plan, int, LevelIO, uint32_t,     \
                                                       uint32_t);                        \
  template __global__ void k_lds_sort<KT, 2048, 256, 0>(Plan, int);                      \
  template __global__ void k_lds_sort<KT, 2048, 256, 1>(Plan, int);                      \
  template __global__ void k_lds_sort<KT, 4096, 512, 0>(Plan, int);            \
  template __global__ void k_lds_sort<KT, 4096, 512, 1>(Plan, int);            \
  template __global__ void k_lds_sort<KT, 8192, 1024, 0>(Plan, int);            \
  template __global__ void k_lds_sort<KT, 8192, 1024, 1>(Plan, int);

PCF_INST_KT(KT_F64)
PCF_INST_KT(KT_U64)
template __global__ void k_colscan<256>(Plan, int);
template __global__ void k_classify<512>(Plan, int, LevelIO);

}  // namespace pcf
