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
//   k_fit       one workgroup per node: range checks, parameters, alpha
//               samples histogrammed into beta + 1 bins in LDS, inclusive
//               prefix sum, bin -> bucket table T (u16) written to HBM;
//   k_count     per (node, chunk) unit: T in LDS, every key's bucket,
//               LDS histogram of the gamma + 1 buckets, one column of the
//               node's bucket-major count matrix;
//   k_colscan   one wave per (node, bucket): exclusive scan over chunks;
//   k_classify  one workgroup per node: bucket starts, the paper's per-bucket
//               decision (recurse / standard sort) and the work lists of the
//               next level and of the LDS finish;
//   k_scatter   per unit: stable tile ranking with wave ballots, LDS staging
//               in bucket order, coalesced runs to HBM, per-child min/max.
// k_lds_sort finishes arrays of at most a few thousand keys inside one
// workgroup's LDS with the paper's own parameters.
#include "pcf_kernels.h"
#include "pcf_block.h"

namespace pcf {

constexpr int ERR_INVALID_KEY = 2;  // PCF_ERR_INVALID_KEY

__device__ __forceinline__ uint64_t load_bits(const void* base, uint64_t i) {
  return reinterpret_cast<const uint64_t*>(base)[i];
}

__device__ __forceinline__ bool ctl_ok(const Ctl* c) {
  return *reinterpret_cast<const volatile int32_t*>(&c->status) == 0;
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

__global__ void k_roots(Plan p, RootArgs a) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.nseg) return;
  const uint64_t b0 = a.offsets ? a.offsets[s] : 0ull;
  const uint64_t b1 = a.offsets ? a.offsets[s + 1] : a.n;
  if (b1 <= b0) return;
  const uint32_t len = (uint32_t)(b1 - b0);
  const char* kb = reinterpret_cast<const char*>(a.keys) + b0 * 8ull;
  const uint32_t* vb = a.vals ? a.vals + b0 : nullptr;
  Ctl* c = p.ctl;
  if (len <= p.pol.lds_cap && !a.force_global) {
    const int cls = len <= p.pol.small_cap ? 0 : 1;
    const uint32_t idx = atomicAdd(&c->item_count[cls], 1u);
    if (idx >= p.cap_items[cls]) {
      flag_overflow(c);
      return;
    }
    Item it;
    it.src = kb;
    it.vsrc = vb;
    it.off = b0;
    it.rel = 0;
    it.len = len;
    it.depth = 0;
    it.flags = IF_ROOT | (a.iota ? IF_IOTA : 0u);
    it.seg = s;
    p.items[cls][idx] = it;
    return;
  }
  const uint32_t ni = atomicAdd(&c->lv[0].num_nodes, 1u);
  if (ni >= p.cap_nodes) {
    flag_overflow(c);
    return;
  }
  const uint32_t nch = (len + p.pol.chunk_keys - 1) / p.pol.chunk_keys;
  const uint32_t ub = atomicAdd(&c->lv[0].num_units, nch);
  if (ub + nch > p.cap_units) {
    flag_overflow(c);
    return;
  }
  for (uint32_t i = 0; i < nch; ++i) p.units[0][ub + i] = Unit{ni, i};
  Node nd = {};
  nd.src = kb;
  nd.vsrc = vb;
  nd.off = b0;
  nd.rel = 0;
  nd.seed = a.has_fixed_seed ? a.fixed_seed : node_seed(p.seed, s, 0, 0);
  nd.min_img = ~0ull;
  nd.max_img = 0ull;
  nd.len = len;
  nd.seg = s;
  nd.depth = 0;
  nd.kind = NK_PCF;
  nd.nchunks = nch;
  nd.unit_base = ub;
  nd.fixed = a.fixed_nb ? 1u : 0u;
  nd.alpha = a.fixed_alpha;
  nd.beta = a.fixed_beta;
  nd.nb = a.fixed_nb;
  nd.iota = a.iota;
  p.nodes[0][ni] = nd;
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
template <int KT, int NT>
__global__ __launch_bounds__(NT) void k_range(Plan p) {
  __shared__ uint64_t red[2 * NT / 64];
  __shared__ uint32_t bad_sh;
  const uint32_t nu = p.ctl->lv[0].num_units;
  for (uint32_t u = blockIdx.x; u < nu; u += gridDim.x) {
    const Unit un = p.units[0][u];
    Node& nd = p.nodes[0][un.node];
    uint32_t b, e;
    chunk_range(nd, un.chunk, b, e);
    const uint64_t* src = reinterpret_cast<const uint64_t*>(nd.src);
    uint64_t lo = ~0ull, hi = 0ull;
    bool bad = false;
    for (uint32_t i = b + threadIdx.x; i < e; i += NT) {
      const uint64_t bits = __builtin_nontemporal_load(src + i);
      if (KT == KT_F64) bad |= !f64_bits_valid(bits);
      const uint64_t im = img_of<KT>(bits);
      lo = im < lo ? im : lo;
      hi = im > hi ? im : hi;
    }
    if (threadIdx.x == 0) bad_sh = 0;
    __syncthreads();
    if (bad) bad_sh = 1;
    block_minmax_u64<NT>(lo, hi, red);
    if (threadIdx.x == 0) {
      if (bad_sh) atomicMax(&p.ctl->status, ERR_INVALID_KEY);
      atomicMin(&nd.min_img, (unsigned long long)lo);
      atomicMax(&nd.max_img, (unsigned long long)hi);
    }
  }
}

// ---------------------------------------------------------------------------
// K1: fit -- sample, histogram, prefix sum, bin -> bucket table
// ---------------------------------------------------------------------------
template <int KT, int NT>
__global__ __launch_bounds__(NT) void k_fit(Plan p, int L, int trace) {
  __shared__ uint32_t hist[MAX_BINS + 1];
  __shared__ uint32_t red[NT / 64 + 1];
  __shared__ uint64_t alloc_sh[4];
  __shared__ uint32_t ok_sh;
  const int s = L & 1;
  Ctl* c = p.ctl;
  LevelCtr& lc = c->lv[L];
  const uint32_t nn = lc.num_nodes;
  for (uint32_t ni = blockIdx.x; ni < nn; ni += gridDim.x) {
    if (!ctl_ok(c)) return;
    Node& nd = p.nodes[s][ni];
    const uint64_t lo = nd.min_img, hi = nd.max_img;
    if (lo == hi) {
      if (threadIdx.x == 0) {
        nd.state = NS_DONE;
        atomicAdd(&c->n_done_nodes, 1u);
      }
      continue;
    }
    uint32_t kind = nd.kind, nb, nbits, beta = 0, alpha = 0, delta, shift = 0;
    BinFn f = {};
    if (kind == NK_PCF) {
      if (nd.fixed) {
        nb = nd.nb;
        beta = nd.beta;
        alpha = nd.alpha;
        delta = nd.len + 1;
      } else {
        const uint32_t tgt = (nd.len + p.pol.target_child - 1) / p.pol.target_child;
        nb = 2;
        while (nb < tgt && nb < p.pol.max_buckets) nb <<= 1;
        beta = p.pol.bins_per_bucket * nb;
        if (beta > p.pol.max_bins) beta = p.pol.max_bins;
        alpha = p.pol.samples_per_bucket * nb;
        if (alpha > p.pol.max_samples) alpha = p.pol.max_samples;
        delta = root34(nd.len);
      }
      if (!bin_setup<KT>(f, lo, hi, beta)) {
        kind = NK_RADIX;  // scale not finite: a bucketing failure
        if (threadIdx.x == 0) atomicAdd(&c->n_radix_nodes, 1u);
      }
    }
    if (kind == NK_RADIX) {
      const uint64_t range = hi - lo;
      const uint32_t top = 63u - (uint32_t)__clzll((long long)range);
      shift = top >= 7 ? top - 7 : 0u;
      nb = RADIX_NB;
      delta = 0xffffffffu;
    }
    nbits = 32u - (uint32_t)__clz((int)(nb - 1));
    if (nb == 1) nbits = 0;
    // allocate the node's share of the level arenas
    if (threadIdx.x == 0) {
      const uint64_t tsz = kind == NK_PCF ? (uint64_t)beta + 1 : 0;
      const uint64_t t0 = atomicAdd(&lc.table_used, (unsigned long long)tsz);
      const uint64_t msz = (uint64_t)nd.nchunks * nb;
      const uint64_t m0 = atomicAdd(&lc.cm_used, (unsigned long long)msz);
      const uint32_t a0 = atomicAdd(&lc.aux_used, nb);
      const uint32_t k0 = atomicAdd(&lc.tasks, nb);
      uint32_t ok = 1;
      if (t0 + tsz > p.cap_table || m0 + msz > p.cap_cm || a0 + nb > p.cap_aux ||
          k0 + nb > p.cap_tasks) {
        flag_overflow(c);
        ok = 0;
      }
      alloc_sh[0] = t0;
      alloc_sh[1] = m0;
      alloc_sh[2] = a0;
      alloc_sh[3] = k0;
      ok_sh = ok;
    }
    __syncthreads();
    if (!ok_sh) return;
    const uint64_t t0 = alloc_sh[0], m0 = alloc_sh[1];
    const uint32_t a0 = (uint32_t)alloc_sh[2], k0 = (uint32_t)alloc_sh[3];
    for (uint32_t b = threadIdx.x; b < nb; b += NT) p.task_node[s][k0 + b] = ni;
    if (kind == NK_PCF) {
      for (uint32_t i = threadIdx.x; i <= beta; i += NT) hist[i] = 0u;
      __syncthreads();
      const uint64_t* src = reinterpret_cast<const uint64_t*>(nd.src);
      for (uint32_t j = threadIdx.x; j < alpha; j += NT) {
        const uint32_t pos = sample_pos(nd.seed, j, nd.len);
        atomicAdd(&hist[bin_of<KT>(f, src[pos])], 1u);
      }
      __syncthreads();
      block_scan_array<NT, true>(hist, beta + 1, red);
      if (trace && L == 0 && ni == 0 && p.trace_b)
        for (uint32_t i = threadIdx.x; i <= beta; i += NT) p.trace_b[i] = hist[i];
      const uint32_t gamma = nb - 1;
      uint16_t* tab = p.table[s] + t0;
      for (uint32_t i = threadIdx.x; i <= beta; i += NT)
        tab[i] = (uint16_t)(((uint64_t)hist[i] * gamma) / alpha);
    }
    if (threadIdx.x == 0) {
      nd.kind = kind;
      nd.state = NS_ACTIVE;
      nd.nb = nb;
      nd.nbits = nbits;
      nd.beta = beta;
      nd.alpha = alpha;
      nd.delta = delta;
      nd.shift = shift;
      nd.halves = f.halves;
      nd.scale = f.s;
      nd.table_off = t0;
      nd.cm_off = m0;
      nd.aux_off = a0;
      nd.task_base = k0;
    }
    __syncthreads();
  }
}

// Bucket of a key in an active node.
template <int KT>
struct Bucketer {
  BinFn f;
  uint64_t lo_img;
  uint32_t shift;
  uint32_t radix;
  const uint16_t* tab;  // LDS copy of T
  __device__ __forceinline__ uint32_t operator()(uint64_t bits) const {
    if (radix) return (uint32_t)((img_of<KT>(bits) - lo_img) >> shift);
    return tab[bin_of<KT>(f, bits)];
  }
};

template <int KT>
__device__ __forceinline__ Bucketer<KT> make_bucketer(const Node& nd, const uint16_t* tab_lds) {
  Bucketer<KT> bk;
  bk.lo_img = nd.min_img;
  bk.shift = nd.shift;
  bk.radix = nd.kind == NK_RADIX;
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
  uint16_t* tab = reinterpret_cast<uint16_t*>(lds);                    // MAX_BINS + 1
  uint32_t* hist = reinterpret_cast<uint32_t*>(lds + 2 * (MAX_BINS + 1));  // MAX_NB
  const int s = L & 1;
  Ctl* c = p.ctl;
  const uint32_t nu = c->lv[L].num_units;
  for (uint32_t u = blockIdx.x; u < nu; u += gridDim.x) {
    if (!ctl_ok(c)) return;
    const Unit un = p.units[s][u];
    const Node& nd = p.nodes[s][un.node];
    if (nd.state != NS_ACTIVE) continue;
    const uint32_t nb = nd.nb;
    if (nd.kind == NK_PCF)
      for (uint32_t i = threadIdx.x; i <= nd.beta; i += NT) tab[i] = p.table[s][nd.table_off + i];
    for (uint32_t i = threadIdx.x; i < nb; i += NT) hist[i] = 0u;
    __syncthreads();
    const Bucketer<KT> bk = make_bucketer<KT>(nd, tab);
    uint32_t b, e;
    chunk_range(nd, un.chunk, b, e);
    const uint64_t* src = reinterpret_cast<const uint64_t*>(nd.src);
    constexpr int U = 4;
    const int l = lane_id();
    for (uint32_t base = b; base < e; base += U * NT) {
      uint64_t v[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const uint32_t i = base + k * NT + threadIdx.x;
        v[k] = i < e ? __builtin_nontemporal_load(src + i) : 0ull;
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const uint32_t i = base + k * NT + threadIdx.x;
        const bool valid = i < e;
        uint32_t q = valid ? bk(v[k]) : 0u;
        if (q >= nb) {
          flag_internal(c);
          q = nb - 1;
        }
        // a whole wave in one bucket (runs of duplicates): one add
        const uint32_t q0 = __shfl(q, 0, 64);
        const uint64_t act = __ballot(valid);
        if (act == ~0ull && __all(q == q0)) {
          if (l == 0) atomicAdd(&hist[q0], 64u);
        } else if (valid) {
          atomicAdd(&hist[q], 1u);
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
  const uint32_t nt = c->lv[L].tasks;
  constexpr int NW = NT / 64;
  const int l = lane_id();
  for (uint32_t t = blockIdx.x * NW + wave_id(); t < nt; t += gridDim.x * NW) {
    if (!ctl_ok(c)) return;
    const uint32_t ni = p.task_node[s][t];
    const Node& nd = p.nodes[s][ni];
    const uint32_t q = t - nd.task_base;
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
  const int s = L & 1, s1 = (L + 1) & 1;
  Ctl* c = p.ctl;
  const uint32_t nn = c->lv[L].num_nodes;
  const uint32_t cap = p.pol.lds_cap;
  const uint32_t half = p.pol.small_cap / 2 ? p.pol.small_cap / 2 : 1;
  for (uint32_t ni = blockIdx.x; ni < nn; ni += gridDim.x) {
    if (!ctl_ok(c)) return;
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
    const uint32_t lds_grp = nd.kind == NK_RADIX ? BC_LDS_STD : BC_LDS_PCF;
    for (uint32_t q = threadIdx.x; q < nb; q += NT) {
      bs[q] = st[q];
      const uint32_t sz = st[q + 1] - st[q];
      uint32_t k;
      if (sz == 0) {
        k = BC_EMPTY;
      } else if (nd.kind == NK_RADIX) {
        k = sz <= cap ? BC_LDS_STD : BC_GLB_RADIX;
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
      const bool lds = k <= BC_LDS_STD;
      uint32_t start = 0;
      if (lds) {
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
    LevelCtr* ln = &c->lv[L + 1 < MAX_LEVELS ? L + 1 : MAX_LEVELS - 1];
    for (uint32_t q = threadIdx.x; q < nb; q += NT) {
      const uint32_t k = cls[q];
      cmap[q] = -1;
      if (istart[q]) {
        uint32_t e = q + 1;
        while (e < nb && cls[e] <= BC_LDS_STD && !istart[e]) ++e;
        const uint32_t ilen = st[e] - st[q];
        if (ilen > 0) {
          const uint32_t g = k == BC_EMPTY ? lds_grp : k;
          const int ic = ilen <= p.pol.small_cap ? 0 : 1;
          const uint32_t idx = atomicAdd(&c->item_count[ic], 1u);
          if (idx >= p.cap_items[ic]) {
            flag_overflow(c);
          } else {
            Item it;
            const uint64_t off = nd.off + st[q];
            it.src = reinterpret_cast<const char*>(io.dst_keys) + off * 8ull;
            it.vsrc = p.has_pay ? io.dst_vals + off : nullptr;
            it.off = off;
            it.rel = nd.rel + st[q];
            it.len = ilen;
            it.depth = nd.depth + 1;
            it.flags = g == BC_LDS_STD ? IF_STD : 0u;
            it.seg = nd.seg;
            p.items[ic][idx] = it;
            if (g == BC_LDS_STD) atomicAdd(&c->n_fail_items, 1u);
          }
        }
      }
      if (k >= BC_GLB_PCF) {
        const uint32_t sz = st[q + 1] - st[q];
        if (L + 1 >= MAX_LEVELS) {
          flag_overflow(c);
          continue;
        }
        const uint32_t ci = atomicAdd(&ln->num_nodes, 1u);
        const uint32_t nch = (sz + p.pol.chunk_keys - 1) / p.pol.chunk_keys;
        const uint32_t ub = atomicAdd(&ln->num_units, nch);
        if (ci >= p.cap_nodes || ub + nch > p.cap_units) {
          flag_overflow(c);
          continue;
        }
        for (uint32_t i = 0; i < nch; ++i) p.units[s1][ub + i] = Unit{ci, i};
        Node ch = {};
        const uint64_t off = nd.off + st[q];
        ch.src = reinterpret_cast<const char*>(io.dst_keys) + off * 8ull;
        ch.vsrc = p.has_pay ? io.dst_vals + off : nullptr;
        ch.off = off;
        ch.rel = nd.rel + st[q];
        ch.seed = node_seed(p.seed, nd.seg, nd.depth + 1, ch.rel);
        ch.min_img = ~0ull;
        ch.max_img = 0ull;
        ch.len = sz;
        ch.seg = nd.seg;
        ch.depth = nd.depth + 1;
        ch.kind = k == BC_GLB_RADIX ? NK_RADIX : NK_PCF;
        ch.nchunks = nch;
        ch.unit_base = ub;
        p.nodes[s1][ci] = ch;
        cmap[q] = (int32_t)ci;
        if (k == BC_GLB_RADIX) atomicAdd(&c->n_radix_nodes, 1u);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// K4: scatter -- stable, LDS-staged, coalesced
// ---------------------------------------------------------------------------
template <int KT, int NT, int TS, int PAY>
__global__ __launch_bounds__(NT) void k_scatter(Plan p, int L, LevelIO io, uint32_t max_bins,
                                                uint32_t nbmax) {
  constexpr int NW = NT / 64;
  constexpr int PW = TS / NW;   // keys of a wave per tile
  constexpr int R = PW / 64;    // rounds per wave
  static_assert(PW % 64 == 0, "tile must split into whole wave rounds");
  extern __shared__ __align__(16) unsigned char lds[];
  const ScatterLds lay = scatter_lds(max_bins, nbmax, NW, TS, PAY);
  uint16_t* tab = reinterpret_cast<uint16_t*>(lds + lay.tab);
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

  const int s = L & 1, s1 = (L + 1) & 1;
  Ctl* c = p.ctl;
  const uint32_t nu = c->lv[L].num_units;
  const int l = lane_id(), w = wave_id();
  uint64_t* dk = reinterpret_cast<uint64_t*>(io.dst_keys);
  uint32_t* dv = io.dst_vals;
  uint64_t* ok_ = reinterpret_cast<uint64_t*>(p.out_keys);

  for (uint32_t u = blockIdx.x; u < nu; u += gridDim.x) {
    if (!ctl_ok(c)) return;
    const Unit un = p.units[s][u];
    const Node& nd = p.nodes[s][un.node];
    uint32_t cb, ce;
    chunk_range(nd, un.chunk, cb, ce);
    const uint64_t* src = reinterpret_cast<const uint64_t*>(nd.src);
    if (nd.state == NS_DONE) {
      // single-valued node: already in order; move it to the output if needed
      uint64_t* o = ok_ + nd.off;
      if ((const void*)o != nd.src)
        for (uint32_t i = cb + threadIdx.x; i < ce; i += NT) o[i] = src[i];
      if (PAY) {
        uint32_t* ov = p.out_vals + nd.off;
        if (nd.vsrc == nullptr) {
          for (uint32_t i = cb + threadIdx.x; i < ce; i += NT) ov[i] = (uint32_t)nd.rel + i;
        } else if (ov != nd.vsrc) {
          for (uint32_t i = cb + threadIdx.x; i < ce; i += NT) ov[i] = nd.vsrc[i];
        }
      }
      continue;
    }
    const uint32_t nb = nd.nb, nbits = nd.nbits, C = nd.nchunks;
    if (nd.kind == NK_PCF)
      for (uint32_t i = threadIdx.x; i <= nd.beta; i += NT) tab[i] = p.table[s][nd.table_off + i];
    const uint32_t* bs = p.bstart[s] + nd.aux_off;
    const int32_t* cm = p.cmap[s] + nd.aux_off;
    const uint32_t* col = p.cm[s] + nd.cm_off;
    for (uint32_t q = threadIdx.x; q < nb; q += NT) {
      runoff[q] = bs[q] + col[(uint64_t)q * C + un.chunk];
      cmapf[q] = cm[q] >= 0 ? 1 : 0;
      mmlo[q] = ~0ull;
      mmhi[q] = 0ull;
    }
    for (uint32_t q = threadIdx.x; q < NW * nb; q += NT) wcnt[q] = 0;
    __syncthreads();
    const Bucketer<KT> bk = make_bucketer<KT>(nd, tab);
    const uint32_t* vsrc = nd.vsrc;
    const bool iota = PAY && vsrc == nullptr;

    for (uint32_t t0 = cb; t0 < ce; t0 += TS) {
      const uint32_t tn = (ce - t0 < (uint32_t)TS) ? ce - t0 : (uint32_t)TS;
      // 1. load: wave w owns keys [w*PW, (w+1)*PW) of the tile, round r lane l
      uint64_t key[R];
      uint32_t val[R];
      uint32_t code[R];  // bucket << 16 | rank inside the wave's part
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t i = w * PW + r * 64 + l;
        key[r] = i < tn ? __builtin_nontemporal_load(src + t0 + i) : 0ull;
        if (PAY) val[r] = i < tn ? (iota ? (uint32_t)nd.rel + t0 + i : vsrc[t0 + i]) : 0u;
      }
      // 2. bucket + stable rank inside the wave (ballot match per round)
      uint16_t* wc = wcnt + w * nb;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t i = w * PW + r * 64 + l;
        const bool valid = i < tn;
        uint32_t q = valid ? bk(key[r]) : 0u;
        if (q >= nb) {  // range check: cannot happen for a consistent model
          flag_internal(c);
          q = nb - 1;
        }
        const uint64_t act = __ballot(valid);
        const uint64_t peers = wave_match(q, nbits, act);
        const uint32_t rk = (uint32_t)__popcll(peers & lanemask_lt());
        uint32_t base = 0;
        if (valid) base = wc[q];
        if (valid && rk == 0) wc[q] = (uint16_t)(base + (uint32_t)__popcll(peers));
        code[r] = (q << 16) | (base + rk);
      }
      __syncthreads();
      // 3. per bucket: wave offsets (exclusive over waves) and tile counts
      for (uint32_t q = threadIdx.x; q < nb; q += NT) {
        uint32_t run = 0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
          const uint32_t v = wcnt[ww * nb + q];
          wcnt[ww * nb + q] = (uint16_t)run;
          run += v;
        }
        tcnt[q] = run;
        tstart[q] = run;
      }
      __syncthreads();
      block_scan_array<NT, false>(tstart, nb, red);
      // 4. stage keys in bucket order
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t i = w * PW + r * 64 + l;
        if (i < tn) {
          const uint32_t q = code[r] >> 16;
          const uint32_t pos = tstart[q] + wc[q] + (code[r] & 0xffffu);
          if (pos < (uint32_t)TS) {
            sk[pos] = key[r];
            if (PAY) sv[pos] = val[r];
            sb[pos] = (uint16_t)q;
          } else {
            flag_internal(c);
          }
        }
      }
      __syncthreads();
      // 5. write runs: consecutive staged keys of one bucket are consecutive in HBM
      for (uint32_t i = threadIdx.x; i < tn; i += NT) {
        const uint32_t q = sb[i];
        const uint64_t dst = nd.off + runoff[q] + (i - tstart[q]);
        const uint64_t kv = sk[i];
        if (dst >= nd.off + nd.len) {
          flag_internal(c);
          continue;
        }
        dk[dst] = kv;
        if (PAY) dv[dst] = sv[i];
        if (cmapf[q]) {
          const unsigned long long im = img_of<KT>(kv);
          atomicMin(&mmlo[q], im);
          atomicMax(&mmhi[q], im);
        }
      }
      __syncthreads();
      for (uint32_t q = threadIdx.x; q < nb; q += NT) {
        runoff[q] += tcnt[q];
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) wcnt[ww * nb + q] = 0;
      }
      __syncthreads();
    }
    // child ranges for the next level
    for (uint32_t q = threadIdx.x; q < nb; q += NT) {
      if (cmapf[q] && mmlo[q] != ~0ull) {
        Node& ch = p.nodes[s1][cm[q]];
        atomicMin(&ch.min_img, mmlo[q]);
        atomicMax(&ch.max_img, mmhi[q]);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// K5: finish an array inside one workgroup's LDS
// ---------------------------------------------------------------------------
// Algorithm 1 with the paper's parameters alpha = beta = gamma = delta =
// floor(m^{3/4}) and tau: PCF levels run in LDS (out-of-order bucket writes
// through LDS atomics), buckets below tau get a counting rank, failed buckets
// (>= delta) an in-LDS bitonic sort.  Ties are ordered by the key's position
// in the item, which is the input order because every global scatter before
// this one was stable.
template <int KT, int CAP, int NT>
__device__ void k5_bitonic(K5Smem<KT, CAP, NT>& sm, uint32_t s, uint32_t e) {
  const uint32_t n = e - s;
  uint32_t P = 1;
  while (P < n) P <<= 1;
  for (uint32_t k = 2; k <= P; k <<= 1) {
    const uint32_t hk = k >> 1;
    for (uint32_t t = threadIdx.x; t < P / 2; t += NT) {
      const uint32_t blk = t / hk, o = t % hk;
      const uint32_t i = blk * k + o, j = blk * k + k - 1 - o;
      if (j < n) {
        const uint64_t ki = sm.key[s + i], kj = sm.key[s + j];
        const uint16_t pi = sm.pos[s + i], pj = sm.pos[s + j];
        if (kj < ki || (kj == ki && pj < pi)) {
          sm.key[s + i] = kj; sm.key[s + j] = ki;
          sm.pos[s + i] = pj; sm.pos[s + j] = pi;
        }
      }
    }
    __syncthreads();
    for (uint32_t d = hk >> 1; d >= 1; d >>= 1) {
      for (uint32_t t = threadIdx.x; t < P / 2; t += NT) {
        const uint32_t blk = t / d, o = t % d;
        const uint32_t i = blk * 2 * d + o, j = i + d;
        if (j < n) {
          const uint64_t ki = sm.key[s + i], kj = sm.key[s + j];
          const uint16_t pi = sm.pos[s + i], pj = sm.pos[s + j];
          if (kj < ki || (kj == ki && pj < pi)) {
            sm.key[s + i] = kj; sm.key[s + j] = ki;
            sm.pos[s + i] = pj; sm.pos[s + j] = pi;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t i = s + threadIdx.x; i < e; i += NT) sm.seg[i] = i | ((i + 1) << 16);
  __syncthreads();
}

// One PCF level on the LDS range [s, e) (a node of depth `depth`).
template <int KT, int CAP, int NT>
__device__ void k5_level(K5Smem<KT, CAP, NT>& sm, uint32_t s, uint32_t e, uint64_t nseed,
                         uint32_t depth, uint64_t lo, uint64_t hi, uint32_t tau) {
  constexpr int EPT = (CAP + NT - 1) / NT;
  const uint32_t n = e - s;
  const uint32_t r = root34(n);
  const uint32_t alpha = r, beta = r, gamma = r, delta = r, nb = r + 1;
  BinFn f;
  if (!bin_setup<KT>(f, lo, hi, beta)) {
    k5_bitonic<KT, CAP, NT>(sm, s, e);
    return;
  }
  for (uint32_t i = threadIdx.x; i <= nb; i += NT) {
    sm.hist[i] = 0u;
    sm.cnt[i] = 0u;
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < alpha; j += NT) {
    const uint32_t q = s + sample_pos(nseed, j, n);
    atomicAdd(&sm.hist[bin_of<KT>(f, bits_of_img<KT>(sm.key[q]))], 1u);
  }
  __syncthreads();
  block_scan_array<NT, true>(sm.hist, beta + 1, sm.red);
  for (uint32_t i = threadIdx.x; i <= beta; i += NT)
    sm.tab[i] = (uint16_t)(((uint64_t)sm.hist[i] * gamma) / alpha);
  __syncthreads();
  uint64_t kk[EPT];
  uint32_t pc[EPT];  // pos | bucket << 16
  uint32_t rk[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const uint32_t i = s + threadIdx.x + k * NT;
    if (i < e) {
      kk[k] = sm.key[i];
      const uint32_t q = sm.tab[bin_of<KT>(f, bits_of_img<KT>(kk[k]))];
      pc[k] = (uint32_t)sm.pos[i] | (q << 16);
      rk[k] = atomicAdd(&sm.cnt[q], 1u);
    }
  }
  __syncthreads();
  block_scan_array<NT, false>(sm.cnt, nb, sm.red);
  if (threadIdx.x == 0) sm.cnt[nb] = n;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const uint32_t i = s + threadIdx.x + k * NT;
    if (i < e) {
      const uint32_t q = pc[k] >> 16;
      const uint32_t d = s + sm.cnt[q] + rk[k];
      if (d >= e) continue;  // range check: cannot happen for consistent counts
      sm.key[d] = kk[k];
      sm.pos[d] = (uint16_t)(pc[k] & 0xffffu);
      sm.seg[d] = (s + sm.cnt[q]) | ((s + sm.cnt[q + 1]) << 16);
    }
  }
  // buckets of at least tau keys need more work (recursion or, when they
  // failed, the standard sort)
  for (uint32_t q = threadIdx.x; q < nb; q += NT) {
    const uint32_t a = sm.cnt[q], b = sm.cnt[q + 1];
    if (b - a >= tau) {
      const uint32_t slot = atomicAdd(&sm.nstk, 1u);
      if (slot < K5Cfg<CAP>::SMAX) {
        sm.stk[slot][0] = s + a;
        sm.stk[slot][1] = s + b;
        sm.stk[slot][2] = (depth + 1) | ((b - a >= delta) ? 0x80000000u : 0u);
      } else {
        sm.flag = 1;  // cannot happen: ranges >= tau are disjoint
      }
    }
  }
  __syncthreads();
}

template <int KT, int CAP, int NT, int PAY>
__global__ __launch_bounds__(NT) void k_lds_sort(Plan p, int cls) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  K5Smem<KT, CAP, NT>& sm = *reinterpret_cast<K5Smem<KT, CAP, NT>*>(lds_raw);
  Ctl* c = p.ctl;
  const uint32_t total = c->item_count[cls] < p.cap_items[cls] ? c->item_count[cls]
                                                                : p.cap_items[cls];
  const uint32_t tau = p.pol.tau;
  uint64_t* ok_ = reinterpret_cast<uint64_t*>(p.out_keys);
  while (true) {
    if (threadIdx.x == 0) {
      sm.item = atomicAdd(&c->item_next[cls], 1u);
      sm.sh[3] = ctl_ok(c) ? 1u : 0u;
    }
    __syncthreads();
    const uint32_t ii = sm.item;
    const bool go = sm.sh[3] != 0;
    __syncthreads();
    if (ii >= total || !go) return;
    const Item it = p.items[cls][ii];
    const uint32_t m = it.len;
    const uint64_t* src = reinterpret_cast<const uint64_t*>(it.src);
    // load, validate (roots), range
    uint64_t lo = ~0ull, hi = 0ull;
    bool bad = false;
    for (uint32_t i = threadIdx.x; i < m; i += NT) {
      const uint64_t bits = src[i];
      if (KT == KT_F64 && (it.flags & IF_ROOT)) bad |= !f64_bits_valid(bits);
      const uint64_t im = img_of<KT>(bits);
      sm.key[i] = im;
      sm.pos[i] = (uint16_t)i;
      sm.seg[i] = 0u | (m << 16);
      lo = im < lo ? im : lo;
      hi = im > hi ? im : hi;
    }
    if (threadIdx.x == 0) {
      sm.flag = 0;
      sm.nstk = 0;
    }
    __syncthreads();
    if (bad) sm.flag = 2;
    block_minmax_u64<NT>(lo, hi, sm.red64);
    if (sm.flag == 2) {
      if (threadIdx.x == 0) atomicMax(&c->status, ERR_INVALID_KEY);
      __syncthreads();
      continue;
    }
    const uint64_t seed0 = node_seed(p.seed, it.seg, it.depth, it.rel);
    if (lo == hi) {
      // single-valued: input order is the answer
      for (uint32_t i = threadIdx.x; i < m; i += NT) sm.seg[i] = i | ((i + 1) << 16);
      __syncthreads();
    } else if (it.flags & IF_STD) {
      k5_bitonic<KT, CAP, NT>(sm, 0, m);
    } else if (m >= tau) {
      k5_level<KT, CAP, NT>(sm, 0, m, seed0, it.depth, lo, hi, tau);
      // ranges still at or above tau: recurse (or standard sort if failed)
      while (true) {
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
        if (rlo == rhi) {
          if (rfail) k5_bitonic<KT, CAP, NT>(sm, rs, re);
          // else: the counting rank orders equal keys by position
        } else if (rfail) {
          k5_bitonic<KT, CAP, NT>(sm, rs, re);
        } else {
          const uint64_t ns = node_seed(p.seed, it.seg, rdepth, it.rel + rs);
          k5_level<KT, CAP, NT>(sm, rs, re, ns, rdepth, rlo, rhi, tau);
        }
      }
    }
    __syncthreads();
    // counting rank inside final segments; all reads (LDS keys and the
    // payload, which may live in the very range being written) happen before
    // the barrier, all writes after it
    constexpr int EPT = (CAP + NT - 1) / NT;
    uint32_t rr[EPT], vv[EPT];
#pragma unroll
    for (int kq = 0; kq < EPT; ++kq) {
      const uint32_t i = threadIdx.x + kq * NT;
      rr[kq] = 0xffffffffu;
      vv[kq] = 0u;
      if (i < m) {
        const uint32_t sg = sm.seg[i];
        const uint32_t a = sg & 0xffffu, b = sg >> 16;
        const uint64_t k = sm.key[i];
        const uint32_t ps = sm.pos[i];
        uint32_t rnk = a;
        if (b - a > 1) {
          for (uint32_t q = a; q < b; ++q) {
            const uint64_t kq2 = sm.key[q];
            rnk += (kq2 < k) || (kq2 == k && sm.pos[q] < ps);
          }
        }
        rr[kq] = rnk;
        if (PAY) vv[kq] = it.vsrc ? it.vsrc[ps] : (uint32_t)it.rel + ps;
      }
    }
    __syncthreads();
    uint64_t* ok = ok_ + it.off;
#pragma unroll
    for (int kq = 0; kq < EPT; ++kq) {
      const uint32_t i = threadIdx.x + kq * NT;
      if (i < m) {
        const uint32_t rnk = rr[kq];
        if (rnk >= m) {
          flag_internal(c);
          continue;
        }
        ok[rnk] = bits_of_img<KT>(sm.key[i]);
        if (PAY) p.out_vals[it.off + rnk] = vv[kq];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// explicit instantiations used by the driver
// ---------------------------------------------------------------------------
#define PCF_INST_KT(KT)                                                                  \
  template __global__ void k_range<KT, 256>(Plan);                                       \
  template __global__ void k_fit<KT, 1024>(Plan, int, int);                              \
  template __global__ void k_count<KT, 512>(Plan, int);                                  \
  template __global__ void k_scatter<KT, 512, 4096, 0>(Plan, int, LevelIO, uint32_t,     \
                                                       uint32_t);                        \
  template __global__ void k_scatter<KT, 512, 4096, 1>(Plan, int, LevelIO, uint32_t,     \
                                                       uint32_t);                        \
  template __global__ void k_scatter<KT, 512, 2048, 0>(Plan, int, LevelIO, uint32_t,     \
                                                       uint32_t);                        \
  template __global__ void k_scatter<KT, 512, 2048, 1>(Plan, int, LevelIO, uint32_t,     \
                                                       uint32_t);                        \
  template __global__ void k_lds_sort<KT, 2048, 256, 0>(Plan, int);                      \
  template __global__ void k_lds_sort<KT, 2048, 256, 1>(Plan, int);                      \
  template __global__ void k_lds_sort<KT, 8192, 512, 0>(Plan, int);                      \
  template __global__ void k_lds_sort<KT, 8192, 512, 1>(Plan, int);

PCF_INST_KT(KT_F64)
PCF_INST_KT(KT_U64)
template __global__ void k_colscan<256>(Plan, int);
template __global__ void k_classify<512>(Plan, int, LevelIO);

}  // namespace pcf
