// pcf_driver.hip -- host driver and C ABI of the PCF Learned Sort library.
//
// Runs Algorithm 1 (Sec. 3.2) of the paper on the GPU: the recursion is
// unrolled into a chain of global levels (each: fit, count, column scan,
// classify, scatter over a device-resident node list) followed by the in-LDS
// finish of every small array.  The host never reads keys; between levels it
// reads back only the size of the next level's node list, once the number of
// levels that the paper's delta rule allows for the input size has run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "pcf_driver.h"
#include "pcf_kernels.h"

namespace pcf {

static thread_local int g_last_hip_error = 0;

int hip_fail(hipError_t e, const char* what, int line) {
  g_last_hip_error = (int)e;
  static const bool dbg = getenv("PCF_DEBUG") != nullptr;
  if (dbg && what)
    fprintf(stderr, "pcfsort: %s failed at line %d: %s\n", what, line, hipGetErrorString(e));
  return PCF_ERR_HIP;
}

static std::mutex g_pol_mu;
static pcf_policy g_pol = {
    /*max_buckets*/ 256,
    /*target_child*/ 2048,
    /*bins_per_bucket*/ 16,
    /*max_bins*/ 16383,
    /*samples_per_bucket*/ 16,
    /*max_samples*/ 65536,
    /*chunk_keys*/ 16384,
    /*lds_cap*/ 8192,
    /*tau*/ 100,
    /*seed*/ 0x5eed,
    /*model*/ 0,
    /*scatter_tile*/ 0,
};

pcf_policy current_policy() {
  std::lock_guard<std::mutex> g(g_pol_mu);
  return g_pol;
}

// Tuned policies per size class (pcf_load_tuning); sizes no entry covers use
// g_pol.  The version changes with every install (graph cache key).
static std::vector<TuneEntry> g_table;
static uint64_t g_table_version = 0;

pcf_policy policy_for(int key_type, size_t n, int has_pay) {
  std::lock_guard<std::mutex> g(g_pol_mu);
  for (const TuneEntry& e : g_table)
    if (e.key_type == key_type && e.with_payload == (has_pay ? 1 : 0) && n >= e.min_n && n < e.max_n)
      return e.pol;
  return g_pol;
}

void install_table(const std::vector<TuneEntry>& t) {
  std::lock_guard<std::mutex> g(g_pol_mu);
  g_table = t;
  ++g_table_version;
}

// The policies of one call: the call's own (by its total size) and the table's
// classes of its kind, from which every global node takes its node parameters
// by its length.  `cover` bounds what any node can use (most buckets, bins and
// samples, fewest keys per chunk): the workspace layout is sized from it.
struct CallPolicy {
  pcf_policy pol, cover;
  std::vector<TuneEntry> cls;
  uint64_t version = 0;
};

static CallPolicy call_policy(int key_type, size_t n, int has_pay, const pcf_policy* override_pol) {
  CallPolicy c;
  c.pol = override_pol ? *override_pol : policy_for(key_type, n, has_pay);
  if (!override_pol) {
    std::lock_guard<std::mutex> g(g_pol_mu);
    for (const TuneEntry& e : g_table)
      if (e.key_type == key_type && e.with_payload == (has_pay ? 1 : 0) &&
          c.cls.size() < (size_t)MAX_POL_CLASSES)
        c.cls.push_back(e);
    c.version = g_table_version;
  }
  c.cover = c.pol;
  for (const TuneEntry& e : c.cls) {
    c.cover.max_buckets = std::max(c.cover.max_buckets, e.pol.max_buckets);
    c.cover.max_bins = std::max(c.cover.max_bins, e.pol.max_bins);
    c.cover.bins_per_bucket = std::max(c.cover.bins_per_bucket, e.pol.bins_per_bucket);
    c.cover.max_samples = std::max(c.cover.max_samples, e.pol.max_samples);
    c.cover.target_child = std::min(c.cover.target_child, e.pol.target_child);
    c.cover.chunk_keys = std::min(c.cover.chunk_keys, e.pol.chunk_keys);
  }
  return c;
}

int check_policy(const pcf_policy& p) {
  if (p.max_buckets < 2 || p.max_buckets > MAX_NB || (p.max_buckets & (p.max_buckets - 1)))
    return PCF_ERR_INVALID_ARGUMENT;
  if (p.target_child < 16 || p.bins_per_bucket < 1 || p.max_bins < 2 || p.max_bins > MAX_BINS)
    return PCF_ERR_INVALID_ARGUMENT;
  if (p.samples_per_bucket < 1 || p.max_samples < 2 || p.max_samples > (1u << 20))
    return PCF_ERR_INVALID_ARGUMENT;
  if (p.chunk_keys < 1024 || p.lds_cap < 2048 || p.lds_cap > 8192) return PCF_ERR_INVALID_ARGUMENT;
  if (p.tau < 16 || p.tau > 1024) return PCF_ERR_INVALID_ARGUMENT;
  if (p.model > 1) return PCF_ERR_INVALID_ARGUMENT;
  if (p.scatter_tile != 0 && p.scatter_tile != 1024 && p.scatter_tile != 2048 &&
      p.scatter_tile != 4096 && p.scatter_tile != 8192)
    return PCF_ERR_INVALID_ARGUMENT;
  return PCF_OK;
}

static int g_cus = 0;
static std::mutex g_dev_mu;

int device_cus() {
  std::lock_guard<std::mutex> g(g_dev_mu);
  if (g_cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return 0;
    g_cus = pr.multiProcessorCount > 0 ? pr.multiProcessorCount : 1;
  }
  return g_cus;
}

// ---- opt-in per-kernel profile ---------------------------------------------
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static uint32_t g_prof_mask = (1u << PCF_K_RADIX_KEYS) - 1;  // timed kinds
static pcf_kernel_stat g_prof[PCF_K_COUNT_KINDS];

struct ProfMark {
  int kind, level;
  hipEvent_t a, b;
};

// Event pairs of the calls of one thread; events are pooled.  A call that
// waits for its stream folds its marks into the global counters at once; a
// call that only enqueues (a device status word is given) leaves them
// pending, with a copy of its control block made on the stream, until the
// thread's next waiting call or pcf_profile_read.
struct CallProf {
  bool on = false;
  uint32_t mask = 0;  // kinds whose launches get events
  bool rec = false;   // the open mark records events
  hipStream_t st = nullptr;
  std::vector<ProfMark> marks;
  size_t used = 0;   // marks in use (pending calls' and this call's)
  size_t first = 0;  // this call's first mark
  struct Pending {
    size_t b, e;
    Ctl* pin;
    uint64_t n;
    hipStream_t st;
  };
  std::vector<Pending> pend;
  std::vector<Ctl*> pins;  // pinned control-block copies, one per pending call
  void start(hipStream_t s, bool on_, uint32_t mask_) {
    st = s;
    on = on_;
    mask = mask_;
    if (pend.empty()) used = 0;
    first = used;
  }
  int begin(int kind, int level) {
    rec = on && ((mask >> kind) & 1u);
    if (!rec) return PCF_OK;
    if (used == marks.size()) {
      ProfMark m = {kind, level, nullptr, nullptr};
      PCF_HIP(hipEventCreate(&m.a));
      PCF_HIP(hipEventCreate(&m.b));
      marks.push_back(m);
    }
    marks[used].kind = kind;
    marks[used].level = level;
    PCF_HIP(hipEventRecord(marks[used].a, st));
    return PCF_OK;
  }
  int end() {
    if (!rec) return PCF_OK;
    PCF_HIP(hipEventRecord(marks[used].b, st));
    ++used;
    return PCF_OK;
  }
  // marks [b, e) of a finished call, with its control block
  int fold(size_t b, size_t e, const Ctl& hc, uint64_t n) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof[PCF_K_RADIX_KEYS].keys += (double)hc.radix_keys;
    g_prof[PCF_K_BITONIC_KEYS].keys += (double)hc.bitonic_keys;
    g_prof[PCF_K_SINGLE_KEYS].keys += (double)hc.single_keys;
    for (size_t i = b; i < e; ++i) {
      float ms = 0.f;
      PCF_HIP(hipEventElapsedTime(&ms, marks[i].a, marks[i].b));
      const int k = marks[i].kind, L = marks[i].level;
      double keys = 0, share = 0;
      const double ik = (double)(hc.item_keys[0] + hc.item_keys[1] + hc.item_keys[2]);
      if (k == PCF_K_SETUP) {
        keys = (double)n;
      } else if (k == PCF_K_LDS_SMALL || k == PCF_K_LDS_BIG) {
        keys = k == PCF_K_LDS_SMALL ? (double)hc.item_keys[0]
                                    : (double)(hc.item_keys[1] + hc.item_keys[2]);
        share = ik > 0 ? std::min(1.0, (double)hc.bitonic_keys / ik) : 0.0;
      } else {
        keys = (double)hc.lv[L].keys;
        if (k != PCF_K_RANGE && keys > 0) share = (double)hc.lv[L].radix_keys / keys;
      }
      g_prof[k].launches += 1;
      g_prof[k].ms += ms;
      g_prof[k].keys += keys;
      g_prof[k].fallback_ms += ms * share;
    }
    return PCF_OK;
  }
  // this call only enqueues: copy its control block on the stream, fold later
  int defer(const Ctl* dctl, uint64_t n) {
    if (!on) return PCF_OK;
    if (pend.size() == pins.size()) {
      Ctl* pin = nullptr;
      PCF_HIP(hipHostMalloc(reinterpret_cast<void**>(&pin), sizeof(Ctl), hipHostMallocPortable));
      pins.push_back(pin);
    }
    Ctl* pin = pins[pend.size()];
    PCF_HIP(hipMemcpyAsync(pin, dctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    pend.push_back({first, used, pin, n, st});
    return PCF_OK;
  }
  // waits for the pending calls' streams and folds their marks
  int drain() {
    for (const Pending& pc : pend) PCF_HIP(hipStreamSynchronize(pc.st));
    for (const Pending& pc : pend) {
      const int r = fold(pc.b, pc.e, *pc.pin, pc.n);
      if (r != PCF_OK) return r;
    }
    pend.clear();
    used = first = 0;
    return PCF_OK;
  }
  // after this call's stream is synchronized
  int commit(const Ctl& hc, uint64_t n) {
    if (on) {
      const int r = fold(first, used, hc, n);
      if (r != PCF_OK) return r;
    }
    return drain();
  }
};
static thread_local CallProf t_prof;

#define PCF_MARK(kind, level, launch)                 \
  do {                                                \
    int r_ = t_prof.begin((kind), (level));           \
    if (r_ != PCF_OK) return r_;                      \
    launch;                                           \
    r_ = t_prof.end();                                \
    if (r_ != PCF_OK) return r_;                      \
  } while (0)

// LDS-finish classes (LDS capacity and workgroup size).
constexpr int K5_SMALL_CAP = 2048, K5_SMALL_NT = 256;
constexpr int K5_MID_CAP = 4096, K5_MID_NT = 512;
constexpr int K5_BIG_CAP = 8192, K5_BIG_NT = 1024;
// Scatter workgroup and tile: keys only (unstable ranks) / with a payload (stable).
constexpr int SC_NT = 512, SC_TS_KEYS = 8192, SC_TS_PAY = 2048;

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// A capacity overflow reports PCF_ERR_OUT_OF_MEMORY; a failed device range
// check reports PCF_ERR_HIP with pcf_last_hip_error() == -2.
static int overflow_status(uint32_t ovf) {
  if (ovf & OVF_INTERNAL) {
    g_last_hip_error = -2;
    return PCF_ERR_HIP;
  }
  return PCF_ERR_OUT_OF_MEMORY;
}

Layout make_layout(size_t n, int has_pay, uint32_t nseg, const pcf_policy& pol, int int_keys,
                   uint32_t trace_nb, uint32_t trace_beta) {
  Layout L = {};
  const uint64_t cap = pol.lds_cap;
  const uint64_t nodes = n / (cap + 1) + 64;
  const uint64_t nbmax = std::max<uint64_t>(std::max<uint64_t>(pol.max_buckets, RADIX_NB), trace_nb);
  const uint64_t units = n / std::max<uint64_t>(pol.chunk_keys, 1) + nodes + 16;
  // buckets over the nodes of a level: radix nodes have 256, PCF nodes fewer
  // than 2 ceil(len / target) + 2
  const uint64_t aux = std::max<uint64_t>(nodes * RADIX_NB,
                                          2 * n / pol.target_child + 4 * nodes + trace_nb) + 64;
  // bin tables of a level: a node has max(bins_per_bucket * buckets, delta / 64)
  // bins (at most max_bins); delta / 64 exceeds 16 * 256 bins only for nodes of
  // more than 2^24 keys
  const uint64_t table = std::min<uint64_t>(
      nodes * (pol.max_bins + 1) + trace_beta + 1,
      nodes + (uint64_t)pol.bins_per_bucket * aux + (n / (1ull << 24) + 1) * (pol.max_bins + 1) +
          trace_beta + 1);
  const uint64_t cmc = aux + nbmax * (n / std::max<uint64_t>(pol.chunk_keys, 1) + 1);
  // LDS items: every key belongs to one item; items start at window crossings
  // or big buckets (<= 2n/half), failed buckets (>= delta > cap^{3/4}), runs
  // after a global child (<= 2 nodes per level) and roots
  const uint64_t half = std::max<uint64_t>(pol.lds_cap / 4, 1);  // small_cap / 2
  const uint64_t items0 = 2 * n / half + 2 * n / 700 + 2 * MAX_LEVELS * nodes + nseg + 1024;
  const uint64_t items1 = n / (K5_SMALL_CAP + 1) + nseg + 1024;
  const uint64_t items2 = n / (K5_MID_CAP + 1) + nseg + 1024;
  L.cap_nodes = (uint32_t)std::min<uint64_t>(nodes, 0xffffffffu);
  L.cap_units = (uint32_t)std::min<uint64_t>(units, 0xffffffffu);
  L.cap_aux = (uint32_t)std::min<uint64_t>(aux, 0xffffffffu);
  L.cap_table = table;
  L.cap_cm = cmc;
  L.cap_items[0] = (uint32_t)std::min<uint64_t>(items0, 0xffffffffu);
  L.cap_items[1] = (uint32_t)std::min<uint64_t>(items1, 0xffffffffu);
  L.cap_items[2] = (uint32_t)std::min<uint64_t>(items2, 0xffffffffu);
  L.nbmax = (uint32_t)nbmax;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + bytes, 256);
    return r;
  };
  L.ctl = take(sizeof(Ctl));
  L.tmp_keys = take(n * 8);
  L.tmp_vals = take(has_pay ? n * 4 : 0);
  L.int_keys = take(int_keys ? n * 8 : 0);
  L.trace_b = take(trace_beta ? 4ull * (trace_beta + 1) : 0);
  L.mmr = take(sizeof(MinMax) * (size_t)L.cap_units);
  // a single root's samples (plain calls): gathered while its range is read
  L.sbuf0 = take(nseg == 1 ? 8ull * pol.max_samples : 0);
  for (int s = 0; s < 2; ++s) {
    L.nodes[s] = take(sizeof(Node) * (size_t)L.cap_nodes);
    L.units[s] = take(sizeof(Unit) * (size_t)L.cap_units);
    L.table[s] = take(2 * (size_t)L.cap_table);
    L.cm[s] = take(4 * (size_t)L.cap_cm);
    L.mm[s] = take(sizeof(MinMax) * (size_t)L.cap_cm);
    L.bstart[s] = take(4 * (size_t)L.cap_aux);
    L.cmap[s] = take(4 * (size_t)L.cap_aux);
    L.task_node[s] = take(4 * (size_t)L.cap_aux);
  }
  for (int k = 0; k < 3; ++k) L.items[k] = take(sizeof(Item) * (size_t)L.cap_items[k]);
  L.total = o;
  return L;
}

// Number of global levels the delta rule allows before every array that
// recursed is small enough for the LDS finish: a bucket that recurses holds
// fewer than delta = floor(len^{3/4}) keys (worst-case lemma, Sec. 3.2).
static int planned_levels(uint64_t n, uint32_t cap) {
  int d = 0;
  uint64_t m = n;
  while (m > cap && d < MAX_LEVELS - 1) {
    m = root34((uint32_t)std::min<uint64_t>(m, 0xffffffffu));
    ++d;
  }
  return d;
}

// Levels of a fixed launch chain (graph capture) that cover every input of n
// keys: PCF levels shrink an array of m keys below root34(m), so PCF nodes
// live only on the first `planned` levels; a failed bucket becomes a radix
// node whose children's key range loses at least 8 of the 64 bits per level,
// so at most 8 radix levels follow, plus one level on which single-valued
// nodes are marked done.
static int chain_levels(uint64_t n, uint32_t cap) {
  return std::min(planned_levels(n, cap) + 9, MAX_LEVELS - 1);
}

// A pinned copy of the control block and an event, per device and thread,
// for reading the block back without draining the stream.  Both live until
// the process ends.
static int ctl_readback_slot(Ctl** pin, hipEvent_t* ev) {
  struct Slot {
    Ctl* pin = nullptr;
    hipEvent_t ev = nullptr;
  };
  static thread_local Slot slots[16];
  int dev = 0;
  PCF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 16) return PCF_ERR_UNSUPPORTED;
  Slot& sl = slots[dev];
  if (!sl.pin)
    PCF_HIP(hipHostMalloc(reinterpret_cast<void**>(&sl.pin), sizeof(Ctl), hipHostMallocPortable));
  if (!sl.ev) PCF_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
  *pin = sl.pin;
  *ev = sl.ev;
  return PCF_OK;
}

// Enqueues one sort on a.stream.  fixed_levels == 0: the planned levels run
// without host reads; a copy of the control block is then read back while
// the LDS finish of the items so far already runs, and only if a further
// level holds nodes (failed buckets of skewed inputs) do more levels follow,
// each with a host read, and a second finish pass for their items.
// fixed_levels > 0: exactly that many levels are launched with no host
// synchronization (empty levels exit at once), then one finish pass; with
// `capture` the function returns right there (the launches are being
// captured into a graph), otherwise it ends like any call: deferred profile
// marks with a status word, a wait for the outcome without one.
template <int KT, int PAY>
static int run_typed(const SortArgs& a, const Layout& lay, char* ws, const CallPolicy& cp,
                     int fixed_levels, bool capture) {
  const pcf_policy& pol = cp.pol;
  hipStream_t st = a.stream;
  const int cus = device_cus();
  if (cus <= 0) return PCF_ERR_UNSUPPORTED;
  Plan p = {};
  p.ctl = reinterpret_cast<Ctl*>(ws + lay.ctl);
  void* out_keys = a.keys_out ? a.keys_out : (void*)(ws + lay.int_keys);
  void* tmp_keys = ws + lay.tmp_keys;
  uint32_t* tmp_vals = PAY ? reinterpret_cast<uint32_t*>(ws + lay.tmp_vals) : nullptr;
  p.out_keys = out_keys;
  p.out_vals = PAY ? a.vals_out : nullptr;
  p.d_status = a.d_status;
  p.has_pay = PAY;
  p.key_bytes = 8;
  for (int s = 0; s < 2; ++s) {
    p.nodes[s] = reinterpret_cast<Node*>(ws + lay.nodes[s]);
    p.units[s] = reinterpret_cast<Unit*>(ws + lay.units[s]);
    p.table[s] = reinterpret_cast<uint16_t*>(ws + lay.table[s]);
    p.cm[s] = reinterpret_cast<uint32_t*>(ws + lay.cm[s]);
    p.mm[s] = reinterpret_cast<MinMax*>(ws + lay.mm[s]);
    p.bstart[s] = reinterpret_cast<uint32_t*>(ws + lay.bstart[s]);
    p.cmap[s] = reinterpret_cast<int32_t*>(ws + lay.cmap[s]);
    p.task_node[s] = reinterpret_cast<uint32_t*>(ws + lay.task_node[s]);
  }
  for (int k = 0; k < 3; ++k) {
    p.items[k] = reinterpret_cast<Item*>(ws + lay.items[k]);
    p.cap_items[k] = lay.cap_items[k];
  }
  p.mmr = reinterpret_cast<MinMax*>(ws + lay.mmr);
  p.sbuf0 = (a.nseg == 1 && !a.trace) ? reinterpret_cast<uint64_t*>(ws + lay.sbuf0) : nullptr;
  p.sbuf0_cap = cp.cover.max_samples;
  p.cap_nodes = lay.cap_nodes;
  p.cap_units = lay.cap_units;
  p.cap_aux = lay.cap_aux;
  p.cap_table = lay.cap_table;
  p.cap_cm = lay.cap_cm;
  p.trace_b = a.trace ? reinterpret_cast<uint32_t*>(ws + lay.trace_b) : nullptr;
  // scatter work per level: enough units to give every workgroup a few
  const uint32_t bins_lds = std::max<uint32_t>(cp.cover.max_bins, a.trace ? a.trace_beta : 0u);
  // keys only: the LDS-atomic scatter; with a payload: the stable one
  int sc_ts;
  uint32_t sc_lds;
  if (PAY) {
    // 2048-key tiles by default (two 512-thread workgroups per CU); the
    // policy may ask for 1024
    sc_ts = pol.scatter_tile == 1024 ? 1024 : SC_TS_PAY;
    sc_lds = scatter_lds(bins_lds, lay.nbmax, SC_NT / 64, sc_ts, PAY, (int)pol.model).total;
    if (sc_lds > 160 * 1024 - 1024) {  // many buckets: halve the tile
      sc_ts /= 2;
      sc_lds = scatter_lds(bins_lds, lay.nbmax, SC_NT / 64, sc_ts, PAY, (int)pol.model).total;
    }
  } else {
    // 8192-key tiles, 1024 threads, one workgroup per CU by default: the
    // same scatter time as two 512-thread workgroups with 4096-key tiles,
    // half the bucket-edge lines, and longer work units for the count and
    // fit; the policy may ask for 4096
    sc_ts = pol.scatter_tile == 4096 ? 4096 : 8192;
    sc_lds = scatter_keys_lds(bins_lds, lay.nbmax, sc_ts, (int)pol.model).total;
    if (sc_lds > 160 * 1024 - 1024) {
      sc_ts = 4096;
      sc_lds = scatter_keys_lds(bins_lds, lay.nbmax, sc_ts, (int)pol.model).total;
    }
  }
  if (sc_lds > 160 * 1024 - 1024) return PCF_ERR_INVALID_ARGUMENT;
  struct {
    uint32_t total;
  } sl = {sc_lds};
  // resident workgroups per CU: what LDS allows, capped by the registers the
  // launch bounds give (tiles of at most 4096 keys, or 2048 with a payload:
  // 4 waves per SIMD = two 512-thread workgroups; larger tiles: one)
  const int sc_per_cu = std::max(1, (int)(160 * 1024 / sl.total));
  const int sc_reg_cap = ((PAY && sc_ts > 2048) || sc_ts >= 8192) ? 1 : 2;
  const int g_sc = cus * std::min(sc_per_cu, sc_reg_cap);
  PolicyDev pd;
  pd.max_buckets = pol.max_buckets;
  pd.target_child = pol.target_child;
  pd.bins_per_bucket = pol.bins_per_bucket;
  pd.max_bins = pol.max_bins;
  pd.samples_per_bucket = pol.samples_per_bucket;
  pd.max_samples = pol.max_samples;
  pd.chunk_keys =
      (uint32_t)std::max<uint64_t>(pol.chunk_keys, (a.n + 8ull * g_sc - 1) / (8ull * g_sc));
  pd.lds_cap = pol.lds_cap;
  pd.tau = pol.tau;
  pd.model = pol.model;
  pd.small_cap = K5_SMALL_CAP;
  pd.mid_cap = K5_MID_CAP;
  {
    std::lock_guard<std::mutex> g(g_prof_mu);
    pd.prof = (g_prof_on && !a.no_prof) ? 1u : 0u;
  }
  p.pol = pd;
  // the table's classes: node parameters by node length (the same floor on
  // keys per chunk as the call's, so a level never has more units than the
  // layout holds)
  p.ncls = 0;
  for (const TuneEntry& e : cp.cls) {
    if (e.min_n > 0xffffffffull) continue;
    PolicyDev q = pd;
    q.max_buckets = e.pol.max_buckets;
    q.target_child = e.pol.target_child;
    q.bins_per_bucket = e.pol.bins_per_bucket;
    q.max_bins = e.pol.max_bins;
    q.samples_per_bucket = e.pol.samples_per_bucket;
    q.max_samples = e.pol.max_samples;
    q.chunk_keys = (uint32_t)std::max<uint64_t>(e.pol.chunk_keys, (a.n + 8ull * g_sc - 1) / (8ull * g_sc));
    p.cls[p.ncls] = q;
    p.cls_min[p.ncls] = (uint32_t)e.min_n;
    p.cls_max[p.ncls] = (uint32_t)std::min<uint64_t>(e.max_n - 1, 0xffffffffull);
    ++p.ncls;
  }
  p.seed = (uint64_t)pol.seed;
  p.nlev = fixed_levels > 0 ? (uint32_t)fixed_levels : (a.trace ? 1u : (uint32_t)(MAX_LEVELS - 1));

  RootArgs ra = {};
  ra.keys = a.keys_in;
  ra.seg_src = a.seg_src;
  ra.vals = a.vals_in;
  ra.offsets = a.offsets;
  ra.n = a.n;
  ra.nseg = a.nseg;
  ra.iota = a.iota ? 1u : 0u;
  if (a.trace) {
    ra.fixed_alpha = a.trace_alpha;
    ra.fixed_beta = a.trace_beta;
    ra.fixed_nb = a.trace_nb;
    ra.force_global = 1;
    ra.fixed_seed = a.trace_seed;
    ra.has_fixed_seed = 1;
  }

  // level L writes into dst[L & 1] (absolute positions); sources are recorded
  // per node, so keys and payload may alternate independently
  void* kdst[2];
  uint32_t* vdst[2];
  kdst[0] = (a.keys_in == out_keys) ? tmp_keys : out_keys;
  kdst[1] = (kdst[0] == out_keys) ? tmp_keys : out_keys;
  vdst[0] = nullptr;
  vdst[1] = nullptr;
  if (PAY) {
    vdst[0] = (a.vals_in == a.vals_out) ? tmp_vals : a.vals_out;
    vdst[1] = (vdst[0] == a.vals_out) ? tmp_vals : a.vals_out;
  }

  {
    std::lock_guard<std::mutex> g(g_prof_mu);
    t_prof.start(st, g_prof_on && !a.no_prof, g_prof_mask);
  }
  PCF_MARK(PCF_K_SETUP, 0, {
    hipLaunchKernelGGL(k_init, dim3(1), dim3(256), 0, st, p);
    hipLaunchKernelGGL(k_roots, dim3(1), dim3(1024), 0, st, p, ra);
  });
  PCF_MARK(PCF_K_RANGE, 0,
           hipLaunchKernelGGL((k_range<KT, 256>), dim3(cus * 8), dim3(256), 0, st, p));
  PCF_HIP(hipGetLastError());

  const size_t cnt_lds = 2 * (MAX_BINS + 1) + 4 * MAX_NB;
  const int planned = a.trace ? 1 : planned_levels(a.n, pol.lds_cap);
  int levels = 0;
  Ctl hc;
  // one level of fit, count, column scan, classify and scatter
  auto level = [&](int L) -> int {
    LevelIO io;
    io.dst_keys = kdst[L & 1];
    io.dst_vals = vdst[L & 1];
    PCF_MARK(PCF_K_FIT, L,
             hipLaunchKernelGGL((k_fit<KT, 1024>), dim3(cus * 2), dim3(1024), 0, st, p, L,
                                a.trace));
    PCF_MARK(PCF_K_COUNT, L,
             hipLaunchKernelGGL((k_count<KT, 512>), dim3(cus * 3), dim3(512), cnt_lds, st, p, L));
    PCF_MARK(PCF_K_COLSCAN, L,
             hipLaunchKernelGGL((k_colscan<256>), dim3(cus * 4), dim3(256), 0, st, p, L));
    PCF_MARK(PCF_K_CLASSIFY, L,
             hipLaunchKernelGGL((k_classify<512>), dim3(cus * 2), dim3(512), 0, st, p, L, io));
    PCF_MARK(PCF_K_SCATTER, L, {
      if (PAY) {
        if (sc_ts == SC_TS_PAY)
          hipLaunchKernelGGL((k_scatter<KT, SC_NT, SC_TS_PAY, 1>), dim3(g_sc), dim3(SC_NT),
                             sl.total, st, p, L, io, bins_lds, lay.nbmax);
        else
          hipLaunchKernelGGL((k_scatter<KT, SC_NT, SC_TS_PAY / 2, 1>), dim3(g_sc), dim3(SC_NT),
                             sl.total, st, p, L, io, bins_lds, lay.nbmax);
      } else {
        if (sc_ts == 8192)
          hipLaunchKernelGGL((k_scatter_keys<KT, 2 * SC_NT, 8192>), dim3(g_sc), dim3(2 * SC_NT),
                             sl.total, st, p, L, io, bins_lds, lay.nbmax);
        else
          hipLaunchKernelGGL((k_scatter_keys<KT, SC_NT, 4096>), dim3(g_sc), dim3(SC_NT), sl.total,
                             st, p, L, io, bins_lds, lay.nbmax);
      }
    });
    PCF_HIP(hipGetLastError());
    ++levels;
    return PCF_OK;
  };
  // one pass of the LDS finish over the items listed since the last pass,
  // then the status word
  auto finish = [&](int check_level) -> int {
    // finish every small array inside LDS
    PCF_MARK(PCF_K_LDS_SMALL, 0,
             hipLaunchKernelGGL((k_lds_sort<KT, K5_SMALL_CAP, K5_SMALL_NT, PAY>),
                                dim3(cus * k5_wg_per_cu<KT, K5_SMALL_CAP, PAY, K5_SMALL_NT>()),
                                dim3(K5_SMALL_NT), sizeof(K5Smem<KT, K5_SMALL_CAP, K5_SMALL_NT, PAY>), st,
                                p, 0));
    PCF_MARK(PCF_K_LDS_BIG, 0, {
      hipLaunchKernelGGL((k_lds_sort<KT, K5_MID_CAP, K5_MID_NT, PAY>),
                         dim3(cus * k5_wg_per_cu<KT, K5_MID_CAP, PAY, K5_MID_NT>()),
                         dim3(K5_MID_NT), sizeof(K5Smem<KT, K5_MID_CAP, K5_MID_NT, PAY>), st, p, 1);
      hipLaunchKernelGGL((k_lds_sort<KT, K5_BIG_CAP, K5_BIG_NT, PAY>),
                         dim3(cus * k5_wg_per_cu<KT, K5_BIG_CAP, PAY, K5_BIG_NT>()), dim3(K5_BIG_NT),
                         sizeof(K5Smem<KT, K5_BIG_CAP, K5_BIG_NT, PAY>), st, p, 2);
    });
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, st, p, a.d_status, check_level);
    PCF_HIP(hipGetLastError());
    return PCF_OK;
  };
  // the control block as it stands after the work enqueued so far (a pinned
  // copy on the stream, waited for through an event)
  auto readback = [&]() -> int {
    Ctl* pin = nullptr;
    hipEvent_t ev = nullptr;
    const int rr = ctl_readback_slot(&pin, &ev);
    if (rr != PCF_OK) return rr;
    PCF_HIP(hipMemcpyAsync(pin, p.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    PCF_HIP(hipEventRecord(ev, st));
    PCF_HIP(hipEventSynchronize(ev));
    std::memcpy(&hc, pin, sizeof(Ctl));
    return PCF_OK;
  };
  int r = PCF_OK;
  if (a.trace) {
    // one level with the caller's parameters, then its model and partition
    if ((r = level(0)) != PCF_OK) return r;
    if (a.levels_run) *a.levels_run = (uint32_t)levels;
    if ((r = readback()) != PCF_OK) return r;
    if (hc.status) return hc.status;
    if (hc.overflow) return overflow_status(hc.overflow);
    t_prof.used = t_prof.first;  // a trace level is not profiled
    // the level's model and bucket sizes for the caller
    Node nd;
    PCF_HIP(hipMemcpyAsync(&nd, p.nodes[0], sizeof(Node), hipMemcpyDeviceToHost, st));
    PCF_HIP(hipStreamSynchronize(st));
    const uint32_t beta = a.trace_beta, nb = a.trace_nb;
    if (a.h_scalars) {
      uint64_t sb;
      std::memcpy(&sb, &nd.scale, 8);
      a.h_scalars[0] = bits_of_img<KT>(nd.min_img);
      a.h_scalars[1] = bits_of_img<KT>(nd.max_img);
      a.h_scalars[2] = sb;
      a.h_scalars[3] = nd.halves;
      a.h_scalars[4] = nd.state == NS_DONE ? 1 : (nd.kind == NK_RADIX ? 2 : 0);
    }
    if (nd.state == NS_ACTIVE && nd.kind != NK_RADIX) {
      std::vector<uint32_t> hb(beta + 1), st32(nb);
      std::vector<uint16_t> ht(beta + 1);
      PCF_HIP(hipMemcpy(hb.data(), p.trace_b, 4ull * (beta + 1), hipMemcpyDeviceToHost));
      PCF_HIP(hipMemcpy(ht.data(), p.table[0] + nd.table_off, 2ull * (beta + 1),
                        hipMemcpyDeviceToHost));
      PCF_HIP(hipMemcpy(st32.data(), p.bstart[0] + nd.aux_off, 4ull * nb, hipMemcpyDeviceToHost));
      for (uint32_t i = 0; i <= beta; ++i) {
        if (a.h_b) a.h_b[i] = hb[i];
        if (a.h_T) a.h_T[i] = ht[i];
      }
      if (a.h_sizes)
        for (uint32_t q = 0; q < nb; ++q)
          a.h_sizes[q] = (q + 1 < nb ? st32[q + 1] : nd.len) - st32[q];
    }
    return PCF_OK;
  }
  if (fixed_levels > 0) {
    // a fixed chain: every level, one finish pass, no host reads
    for (int L = 0; L < fixed_levels; ++L)
      if ((r = level(L)) != PCF_OK) return r;
    if (a.levels_run) *a.levels_run = (uint32_t)levels;
    if ((r = finish(fixed_levels)) != PCF_OK) return r;
    if (capture) return PCF_OK;
  } else {
    // the planned levels run without host reads; the control block is then
    // copied back while the LDS finish of the items so far already runs, so
    // the device does not wait for the host's decision on further levels
    for (int L = 0; L < planned; ++L)
      if ((r = level(L)) != PCF_OK) return r;
    Ctl* pin = nullptr;
    hipEvent_t ev = nullptr;
    if ((r = ctl_readback_slot(&pin, &ev)) != PCF_OK) return r;
    PCF_HIP(hipMemcpyAsync(pin, p.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    PCF_HIP(hipEventRecord(ev, st));
    if ((r = finish(-1)) != PCF_OK) return r;
    PCF_HIP(hipEventSynchronize(ev));
    std::memcpy(&hc, pin, sizeof(Ctl));
    if (hc.status) return hc.status;
    if (hc.overflow) return overflow_status(hc.overflow);
    if (hc.lv[planned].num_nodes != 0) {
      // rare (failed buckets of skewed inputs): more levels, one host read each
      for (int L = planned;; ++L) {
        if (L >= MAX_LEVELS - 1) return PCF_ERR_OUT_OF_MEMORY;
        if ((r = level(L)) != PCF_OK) return r;
        if ((r = readback()) != PCF_OK) return r;
        if (hc.status) return hc.status;
        if (hc.overflow) return overflow_status(hc.overflow);
        if (hc.lv[L + 1].num_nodes == 0) break;
      }
      if ((r = finish(-1)) != PCF_OK) return r;
    }
    if (a.levels_run) *a.levels_run = (uint32_t)levels;
  }
  PCF_HIP(hipGetLastError());
  if (a.d_status) return t_prof.defer(p.ctl, a.n);  // errors reach the status word
  PCF_HIP(hipMemcpyAsync(&hc, p.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  PCF_HIP(hipStreamSynchronize(st));
  {
    const int r = t_prof.commit(hc, a.n);
    if (r != PCF_OK) return r;
  }
  if (hc.status) return hc.status;
  if (hc.overflow) return overflow_status(hc.overflow);
  return PCF_OK;
}

static bool g_attr_done = false;
static std::mutex g_attr_mu;

// Raises a kernel's dynamic-LDS limit to what its launches use (the static
// LDS of the kernel counts against the same 160 KiB).
static int allow_lds(const void* fn, size_t dynamic_bytes) {
  if (dynamic_bytes <= 64 * 1024) return PCF_OK;
  hipFuncAttributes fa;
  PCF_HIP(hipFuncGetAttributes(&fa, fn));
  if (fa.sharedSizeBytes + dynamic_bytes > 160 * 1024) return PCF_ERR_UNSUPPORTED;
  PCF_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dynamic_bytes));
  return PCF_OK;
}

template <int KT, int PAY>
static int set_attrs_typed() {
  int r;
  if ((r = allow_lds(reinterpret_cast<const void*>(&k_lds_sort<KT, K5_BIG_CAP, K5_BIG_NT, PAY>),
                     sizeof(K5Smem<KT, K5_BIG_CAP, K5_BIG_NT, PAY>))) != PCF_OK)
    return r;
  if ((r = allow_lds(reinterpret_cast<const void*>(&k_lds_sort<KT, K5_MID_CAP, K5_MID_NT, PAY>),
                     sizeof(K5Smem<KT, K5_MID_CAP, K5_MID_NT, PAY>))) != PCF_OK)
    return r;
  if ((r = allow_lds(reinterpret_cast<const void*>(&k_lds_sort<KT, K5_SMALL_CAP, K5_SMALL_NT, PAY>),
                     sizeof(K5Smem<KT, K5_SMALL_CAP, K5_SMALL_NT, PAY>))) != PCF_OK)
    return r;
  const size_t sc_max = 160 * 1024 - 1024;  // scatter launches stay below this
  if (PAY) {
    if ((r = allow_lds(reinterpret_cast<const void*>(&k_scatter<KT, SC_NT, SC_TS_PAY, 1>),
                       sc_max)) != PCF_OK)
      return r;
    if ((r = allow_lds(reinterpret_cast<const void*>(&k_scatter<KT, SC_NT, SC_TS_PAY / 2, 1>),
                       sc_max)) != PCF_OK)
      return r;
  } else {
    if ((r = allow_lds(reinterpret_cast<const void*>(&k_scatter_keys<KT, 2 * SC_NT, 8192>), sc_max)) !=
        PCF_OK)
      return r;
    if ((r = allow_lds(reinterpret_cast<const void*>(&k_scatter_keys<KT, SC_NT, 4096>), sc_max)) !=
        PCF_OK)
      return r;
  }
  return PCF_OK;
}

static int set_attrs() {
  std::lock_guard<std::mutex> g(g_attr_mu);
  if (g_attr_done) return PCF_OK;
  int r;
  if ((r = set_attrs_typed<KT_F64, 0>()) != PCF_OK) return r;
  if ((r = set_attrs_typed<KT_F64, 1>()) != PCF_OK) return r;
  if ((r = set_attrs_typed<KT_U64, 0>()) != PCF_OK) return r;
  if ((r = set_attrs_typed<KT_U64, 1>()) != PCF_OK) return r;
  g_attr_done = true;
  return PCF_OK;
}

static int dispatch(const SortArgs& a, const Layout& lay, char* ws, const CallPolicy& cp,
                    int has_pay, int fixed_levels, bool capture = false) {
  if (a.key_type == PCF_KEY_F64)
    return has_pay ? run_typed<KT_F64, 1>(a, lay, ws, cp, fixed_levels, capture)
                   : run_typed<KT_F64, 0>(a, lay, ws, cp, fixed_levels, capture);
  return has_pay ? run_typed<KT_U64, 1>(a, lay, ws, cp, fixed_levels, capture)
                 : run_typed<KT_U64, 0>(a, lay, ws, cp, fixed_levels, capture);
}

// ---- graph replay of segmented sorts ----------------------------------------
// A segmented call with a caller workspace is captured once per argument set
// (device, key type, buffers, sizes, policy) as the fixed launch chain and
// replayed from then on; the executable graphs live in a small LRU cache.
struct GraphKey {
  int dev, kt, pay;
  const void* kin;
  void* kout;
  const uint32_t* vin;
  uint32_t* vout;
  const uint64_t* off;
  uint32_t nseg;
  uint64_t n;
  void* ws;
  int32_t* dst;
  pcf_policy pol;
  uint64_t table_version;  // the tuning table the node parameters came from
};

struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec;
  hipEvent_t done;  // recorded after the latest launch
  uint64_t tick;
};

constexpr size_t GRAPH_CACHE = 16;
static std::mutex g_graph_mu;
static std::vector<GraphEntry> g_graphs;
static uint64_t g_graph_tick = 0, g_graph_captures = 0, g_graph_replays = 0;
static hipStream_t g_cap_stream[16] = {};

static bool graphs_enabled() {
  static const bool off = getenv("PCF_NO_GRAPH") != nullptr;
  return !off;
}

static bool use_graph(const SortArgs& a) {
  if (!a.offsets || a.trace || a.no_graph || !graphs_enabled()) return false;
  std::lock_guard<std::mutex> g(g_prof_mu);
  return !g_prof_on;  // profiling records events per launch: eager path
}

static int run_graph(const SortArgs& a, const Layout& lay, char* ws, const CallPolicy& cp,
                     int has_pay) {
  const pcf_policy& pol = cp.pol;
  GraphKey k;
  std::memset(&k, 0, sizeof(k));  // padding takes part in the comparison
  PCF_HIP(hipGetDevice(&k.dev));
  if (k.dev < 0 || k.dev >= 16) return PCF_ERR_UNSUPPORTED;
  k.kt = a.key_type;
  k.pay = has_pay;
  k.kin = a.keys_in;
  k.kout = a.keys_out;
  k.vin = a.vals_in;
  k.vout = a.vals_out;
  k.off = a.offsets;
  k.nseg = a.nseg;
  k.n = a.n;
  k.ws = ws;
  k.dst = a.d_status;
  k.pol = pol;
  k.table_version = cp.cls.empty() ? 0 : cp.version;
  std::lock_guard<std::mutex> g(g_graph_mu);
  GraphEntry* e = nullptr;
  for (auto& x : g_graphs)
    if (std::memcmp(&x.key, &k, sizeof(k)) == 0) e = &x;
  if (!e) {
    if (!g_cap_stream[k.dev]) PCF_HIP(hipStreamCreateWithFlags(&g_cap_stream[k.dev], hipStreamNonBlocking));
    hipStream_t cs = g_cap_stream[k.dev];
    PCF_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    SortArgs b = a;
    b.stream = cs;
    const int rc = dispatch(b, lay, ws, cp, has_pay, chain_levels(a.n, pol.lds_cap), true);
    hipGraph_t gr = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &gr);
    if (rc != PCF_OK) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture", __LINE__);
    GraphEntry ne = {};
    ne.key = k;
    const hipError_t ei = hipGraphInstantiate(&ne.exec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiate", __LINE__);
    const hipError_t ev = hipEventCreateWithFlags(&ne.done, hipEventDisableTiming);
    if (ev != hipSuccess) {
      (void)hipGraphExecDestroy(ne.exec);
      return hip_fail(ev, "hipEventCreate", __LINE__);
    }
    if (g_graphs.size() >= GRAPH_CACHE) {  // evict the least recently used
      size_t v = 0;
      for (size_t i = 1; i < g_graphs.size(); ++i)
        if (g_graphs[i].tick < g_graphs[v].tick) v = i;
      PCF_HIP(hipEventSynchronize(g_graphs[v].done));
      (void)hipGraphExecDestroy(g_graphs[v].exec);
      (void)hipEventDestroy(g_graphs[v].done);
      g_graphs.erase(g_graphs.begin() + (long)v);
    }
    g_graphs.push_back(ne);
    e = &g_graphs.back();
    ++g_graph_captures;
  } else {
    ++g_graph_replays;
  }
  e->tick = ++g_graph_tick;
  PCF_HIP(hipGraphLaunch(e->exec, a.stream));
  PCF_HIP(hipEventRecord(e->done, a.stream));
  if (a.d_status) return PCF_OK;
  // no status word: wait and report the outcome
  Ctl hc;
  PCF_HIP(hipMemcpyAsync(&hc, ws + lay.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, a.stream));
  PCF_HIP(hipStreamSynchronize(a.stream));
  if (hc.status) return hc.status;
  if (hc.overflow) return overflow_status(hc.overflow);
  return PCF_OK;
}

int graph_stats(uint64_t* captures, uint64_t* replays, uint64_t* cached) {
  std::lock_guard<std::mutex> g(g_graph_mu);
  if (captures) *captures = g_graph_captures;
  if (replays) *replays = g_graph_replays;
  if (cached) *cached = g_graphs.size();
  return PCF_OK;
}

int graph_clear() {
  std::lock_guard<std::mutex> g(g_graph_mu);
  for (auto& x : g_graphs) {
    PCF_HIP(hipEventSynchronize(x.done));
    (void)hipGraphExecDestroy(x.exec);
    (void)hipEventDestroy(x.done);
  }
  g_graphs.clear();
  return PCF_OK;
}

size_t workspace_for(int key_type, size_t n, int has_pay, uint32_t nseg, int int_keys) {
  const CallPolicy cp = call_policy(key_type, n, has_pay, nullptr);
  return make_layout(n, has_pay, nseg ? nseg : 1, cp.cover, int_keys, 0, 0).total;
}

// Debugging switches, read from the environment once:
//   PCF_SYNC=1   every call waits for its work and returns its data status
//                (also a call given a status word, which otherwise returns
//                after enqueue);
//   PCF_TRACE=1  the same, and one line per call on stderr: keys, segments,
//                payload, nodes / units / keys of every level that ran, LDS
//                items per class, status and overflow flags.
// Neither applies while the caller's stream is being captured into a graph.
struct DebugEnv {
  bool sync, trace;
};
static bool env_on(const char* name) {
  const char* v = getenv(name);
  return v && *v && strcmp(v, "0") != 0;
}
static const DebugEnv& debug_env() {
  static const DebugEnv e = {env_on("PCF_SYNC") || env_on("PCF_TRACE"), env_on("PCF_TRACE")};
  return e;
}

// Waits for a finished call's work, prints its trace line if asked, and
// returns its data status (PCF_OK when it has none).
static int debug_finish(const SortArgs& a, const Layout& lay, const char* ws) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  PCF_HIP(hipStreamIsCapturing(a.stream, &cs));
  if (cs != hipStreamCaptureStatusNone) return PCF_OK;
  PCF_HIP(hipStreamSynchronize(a.stream));
  Ctl hc;
  PCF_HIP(hipMemcpy(&hc, ws + lay.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  int32_t st = hc.status;
  if (st == 0 && hc.overflow) st = (hc.overflow & OVF_INTERNAL) ? PCF_ERR_HIP : PCF_ERR_OUT_OF_MEMORY;
  if (debug_env().trace) {
    char line[1024];
    int o = snprintf(line, sizeof line, "pcf: %s n=%llu segments=%u payload=%d levels=[",
                     a.key_type == PCF_KEY_F64 ? "f64" : "u64", (unsigned long long)a.n, a.nseg,
                     a.vals_out != nullptr ? 1 : 0);
    for (int L = 0; L < MAX_LEVELS && o < (int)sizeof line - 64; ++L) {
      if (hc.lv[L].num_nodes == 0) break;
      o += snprintf(line + o, sizeof line - o, "%s%u/%u/%llu", L ? " " : "", hc.lv[L].num_nodes,
                    hc.lv[L].num_units, (unsigned long long)hc.lv[L].keys);
    }
    snprintf(line + o, sizeof line - o, "] items=[%u %u %u] status=%d overflow=%u\n", hc.item_count[0],
             hc.item_count[1], hc.item_count[2], (int)hc.status, hc.overflow);
    fputs(line, stderr);
  }
  return st;
}

int run_sort(const SortArgs& a) {
  if (a.key_type != PCF_KEY_F64 && a.key_type != PCF_KEY_U64) return PCF_ERR_INVALID_ARGUMENT;
  if (a.n == 0) {
    // a kernel rather than a memset, so a captured call holds no memset node
    if (a.d_status) {
      hipLaunchKernelGGL(k_set_status, dim3(1), dim3(64), 0, a.stream, a.d_status, 0);
      PCF_HIP(hipGetLastError());
    }
    return PCF_OK;
  }
  if (!a.keys_in && !a.seg_src) return PCF_ERR_INVALID_ARGUMENT;
  if (a.seg_src && (!a.offsets || !a.keys_out)) return PCF_ERR_INVALID_ARGUMENT;
  if (a.n >= (1ull << 32)) return PCF_ERR_INVALID_ARGUMENT;
  const int has_pay = a.vals_out != nullptr;
  if (has_pay && !a.iota && !a.vals_in) return PCF_ERR_INVALID_ARGUMENT;
  if (!has_pay && !a.keys_out) return PCF_ERR_INVALID_ARGUMENT;
  const CallPolicy cp = call_policy(a.key_type, a.n, has_pay, a.pol_override);
  const pcf_policy& pol = cp.pol;
  int r = set_attrs();
  if (r != PCF_OK) return r;
  const Layout lay = make_layout(a.n, has_pay, a.nseg, cp.cover, a.keys_out == nullptr,
                                 a.trace ? a.trace_nb : 0, a.trace ? a.trace_beta : 0);
  char* ws = reinterpret_cast<char*>(a.ws);
  bool own = false;
  if (!ws) {
    PCF_HIP(hipMallocAsync(reinterpret_cast<void**>(&ws), lay.total, a.stream));
    own = true;
  } else if (a.ws_bytes < lay.total) {
    return PCF_ERR_OUT_OF_MEMORY;
  }
  int rc;
  if (!own && use_graph(a))
    rc = run_graph(a, lay, ws, cp, has_pay);
  else if (a.d_status && !a.trace)
    // data errors reach the status word, so nothing needs the host: the
    // fixed chain is enqueued and the call returns (a caller may capture it)
    rc = dispatch(a, lay, ws, cp, has_pay, chain_levels(a.n, pol.lds_cap));
  else
    rc = dispatch(a, lay, ws, cp, has_pay, 0);
  if (rc == PCF_OK && debug_env().sync) rc = debug_finish(a, lay, ws);
  if (own) {
    hipError_t e = hipFreeAsync(ws, a.stream);
    if (e != hipSuccess && rc == PCF_OK) rc = hip_fail(e);
  }
  return rc;
}

// ---- scratch of the allocation-free entry point ------------------------------
// pcf_sort_f64_static takes its workspace from this array instead of a
// caller buffer or a stream-ordered allocation.  Every device the library
// runs on holds its own copy (at its own address) until the process ends.
constexpr size_t STATIC_SCRATCH_BYTES = PCF_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_addr[16] = {};  // device address of `scratch`, per device

// The device address of `scratch` on the current device, looked up once per
// device with that device current.  (In host code the array's name is only a
// stand-in for the symbol; kernels are given this address.)
static int static_scratch(void** out) {
  int dev = 0;
  PCF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 16) return PCF_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)", __LINE__);
    if (!ptr) return PCF_ERR_HIP;
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return PCF_OK;
}

}  // namespace pcf

using namespace pcf;

extern "C" {

const char* pcf_status_string(int s) {
  switch (s) {
    case PCF_OK: return "ok";
    case PCF_ERR_INVALID_ARGUMENT: return "invalid argument";
    case PCF_ERR_INVALID_KEY: return "invalid key (NaN, infinity or -0.0)";
    case PCF_ERR_OUT_OF_MEMORY: return "out of memory";
    case PCF_ERR_HIP: return "HIP runtime error";
    case PCF_ERR_UNSUPPORTED: return "unsupported";
    case PCF_PENDING: return "pending";
    case PCF_ERR_UNKNOWN_TICKET: return "unknown ticket";
    case PCF_ERR_SHUTDOWN: return "server shutting down";
    default: return "unknown status";
  }
}

int pcf_last_hip_error(void) { return g_last_hip_error; }

const char* pcf_version(void) { return "pcfsort 0.1 (gfx950)"; }

size_t pcf_workspace_bytes(int key_type, size_t n, int with_payload, uint32_t num_segments) {
  const CallPolicy cp = call_policy(key_type, n, with_payload, nullptr);
  // argsort may need internal keys: include them
  return make_layout(n, with_payload, num_segments ? num_segments : 1, cp.cover, with_payload, 0, 0)
      .total;
}

int pcf_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_on = on != 0;
  return PCF_OK;
}

int pcf_profile_select(uint32_t kind_mask) {
  if (kind_mask >> PCF_K_RADIX_KEYS) return PCF_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_mask = kind_mask;
  return PCF_OK;
}

int pcf_profile_read(pcf_kernel_stat* out, int reset) {
  if (!out) return PCF_ERR_INVALID_ARGUMENT;
  {
    const int r = t_prof.drain();  // this thread's calls that only enqueued
    if (r != PCF_OK) return r;
  }
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (int i = 0; i < PCF_K_COUNT_KINDS; ++i) out[i] = g_prof[i];
  if (reset) std::memset(g_prof, 0, sizeof(g_prof));
  return PCF_OK;
}

const char* pcf_kernel_name(int kind) {
  static const char* names[PCF_K_COUNT_KINDS] = {
      "setup",   "range",     "fit",        "count",        "colscan",      "classify",
      "scatter", "lds_small", "lds_big",    "radix_keys",   "bitonic_keys", "single_keys"};
  return (kind >= 0 && kind < PCF_K_COUNT_KINDS) ? names[kind] : "unknown";
}

int pcf_get_policy(pcf_policy* out) {
  if (!out) return PCF_ERR_INVALID_ARGUMENT;
  *out = current_policy();
  return PCF_OK;
}

int pcf_policy_for(int key_type, size_t n, int with_payload, pcf_policy* out) {
  if (!out || (key_type != PCF_KEY_F64 && key_type != PCF_KEY_U64)) return PCF_ERR_INVALID_ARGUMENT;
  *out = policy_for(key_type, n, with_payload);
  return PCF_OK;
}

int pcf_set_policy(const pcf_policy* p) {
  if (!p) return PCF_ERR_INVALID_ARGUMENT;
  int r = check_policy(*p);
  if (r != PCF_OK) return r;
  std::lock_guard<std::mutex> g(g_pol_mu);
  g_pol = *p;
  return PCF_OK;
}

static int sort_keys(int kt, const void* in, void* out, size_t n, void* ws, size_t wsb,
                     int32_t* d_status, void* stream) {
  if (n > 0 && (!in || !out)) return PCF_ERR_INVALID_ARGUMENT;
  SortArgs a = {};
  a.key_type = kt;
  a.keys_in = in;
  a.keys_out = out;
  a.nseg = 1;
  a.n = n;
  a.ws = ws;
  a.ws_bytes = wsb;
  a.d_status = d_status;
  a.stream = reinterpret_cast<hipStream_t>(stream);
  return run_sort(a);
}

int pcf_sort_f64(const double* d_in, double* d_out, size_t n, void* d_ws, size_t ws_bytes,
                 int32_t* d_status, void* stream) {
  return sort_keys(PCF_KEY_F64, d_in, d_out, n, d_ws, ws_bytes, d_status, stream);
}

int pcf_sort_u64(const uint64_t* d_in, uint64_t* d_out, size_t n, void* d_ws, size_t ws_bytes,
                 int32_t* d_status, void* stream) {
  return sort_keys(PCF_KEY_U64, d_in, d_out, n, d_ws, ws_bytes, d_status, stream);
}

int pcf_sort_f64_static(const double* d_in, double* d_out, size_t n, int32_t* d_status,
                        void* stream) {
  if (!d_status || (n > 0 && (!d_in || !d_out))) return PCF_ERR_INVALID_ARGUMENT;
  if (n > 0 && workspace_for(PCF_KEY_F64, n, 0, 1, 0) > STATIC_SCRATCH_BYTES)
    return PCF_ERR_OUT_OF_MEMORY;  // beyond the static scratch
  void* ws = nullptr;
  const int r = static_scratch(&ws);
  if (r != PCF_OK) return r;
  SortArgs a = {};
  a.key_type = PCF_KEY_F64;
  a.keys_in = d_in;
  a.keys_out = d_out;
  a.nseg = 1;
  a.n = n;
  a.ws = ws;
  a.ws_bytes = STATIC_SCRATCH_BYTES;
  a.d_status = d_status;  // the fixed chain: no host read, no pinned buffer
  a.no_prof = 1;          // profile events are created on demand: none here
  a.stream = reinterpret_cast<hipStream_t>(stream);
  return run_sort(a);
}

int pcf_argsort(int key_type, const void* d_keys_in, void* d_keys_out, uint32_t* d_idx_out,
                size_t n, void* d_ws, size_t ws_bytes, int32_t* d_status, void* stream) {
  if (n > 0 && (!d_keys_in || !d_idx_out)) return PCF_ERR_INVALID_ARGUMENT;
  SortArgs a = {};
  a.key_type = key_type;
  a.keys_in = d_keys_in;
  a.keys_out = d_keys_out;
  a.vals_out = d_idx_out;
  a.iota = 1;
  a.nseg = 1;
  a.n = n;
  a.ws = d_ws;
  a.ws_bytes = ws_bytes;
  a.d_status = d_status;
  a.stream = reinterpret_cast<hipStream_t>(stream);
  return run_sort(a);
}

int pcf_sort_segmented(int key_type, const void* d_keys_in, void* d_keys_out,
                       const uint32_t* d_vals_in, uint32_t* d_vals_out, const uint64_t* d_offsets,
                       uint32_t num_segments, size_t total_keys, void* d_ws, size_t ws_bytes,
                       int32_t* d_status, void* stream) {
  if (num_segments == 0 || total_keys == 0) return PCF_OK;
  if (!d_keys_in || !d_keys_out || !d_offsets) return PCF_ERR_INVALID_ARGUMENT;
  if ((d_vals_in == nullptr) != (d_vals_out == nullptr)) return PCF_ERR_INVALID_ARGUMENT;
  SortArgs a = {};
  a.key_type = key_type;
  a.keys_in = d_keys_in;
  a.keys_out = d_keys_out;
  a.vals_in = d_vals_in;
  a.vals_out = d_vals_out;
  a.offsets = d_offsets;
  a.nseg = num_segments;
  a.n = total_keys;
  a.ws = d_ws;
  a.ws_bytes = ws_bytes;
  a.d_status = d_status;
  a.stream = reinterpret_cast<hipStream_t>(stream);
  return run_sort(a);
}

int pcf_graph_stats(uint64_t* captures, uint64_t* replays, uint64_t* cached) {
  return graph_stats(captures, replays, cached);
}

int pcf_graph_clear(void) { return graph_clear(); }

int pcf_level_trace(int key_type, const void* d_keys_in, const uint32_t* d_vals_in, size_t n,
                    uint64_t node_seed_v, uint32_t alpha, uint32_t beta, uint32_t gamma,
                    void* d_part_keys, uint32_t* d_part_vals, uint64_t* h_b, uint64_t* h_T,
                    uint64_t* h_sizes, uint64_t* h_scalars, void* stream) {
  if (n == 0 || !d_keys_in || !d_part_keys) return PCF_ERR_INVALID_ARGUMENT;
  if (alpha == 0 || beta == 0 || beta > MAX_BINS || gamma + 1 > MAX_NB || alpha > (1u << 24))
    return PCF_ERR_INVALID_ARGUMENT;
  if ((d_vals_in == nullptr) != (d_part_vals == nullptr)) return PCF_ERR_INVALID_ARGUMENT;
  if (current_policy().model != 0 && alpha > 65535u) return PCF_ERR_INVALID_ARGUMENT;
  SortArgs a = {};
  a.key_type = key_type;
  a.keys_in = d_keys_in;
  a.keys_out = d_part_keys;
  a.vals_in = d_vals_in;
  a.vals_out = d_part_vals;
  a.nseg = 1;
  a.n = n;
  a.stream = reinterpret_cast<hipStream_t>(stream);
  a.trace = 1;
  a.trace_seed = node_seed_v;
  a.trace_alpha = alpha;
  a.trace_beta = beta;
  a.trace_nb = gamma + 1;
  a.h_b = h_b;
  a.h_T = h_T;
  a.h_sizes = h_sizes;
  a.h_scalars = h_scalars;
  int r = run_sort(a);
  if (r == PCF_OK) {
    hipError_t e = hipStreamSynchronize(a.stream);
    if (e != hipSuccess) return hip_fail(e);
  }
  return r;
}

}  // extern "C"
