// pcf_tune.cpp -- the autotuner and the tuning-table loader.
//
// The GPU recursion has free parameters the paper leaves to the implementer
// (Sec. 5 suggests tuning alpha, beta, gamma dynamically): the number of
// buckets per global level, the samples and bins per bucket, the keys per
// count/scatter work unit and the bucket size aimed at.  pcf_autotune times
// candidate policies on synthetic arrays of one representative size per size
// class (coordinate descent from the built-in defaults, hipEvent-timed, median
// of repeats, summed over three distributions) and writes the winners as JSON;
// pcf_load_tuning installs such a file as the per-size-class policy table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pcfsort.h"
#include "pcf_driver.h"

namespace {

using pcf::TuneEntry;

// ---- synthetic inputs (host): SplitMix64 stream, Box-Muller normals ---------
uint64_t sm64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double unit_open(uint64_t& s) { return ((double)(sm64(s) >> 11) + 0.5) * 0x1.0p-53; }

// dist 0: uniform [0,1); 1: normal; 2: lognormal.  u64 keys: floor((x - lo) 2^32).
void make_keys(int kt, int dist, uint64_t seed, std::vector<uint64_t>& out) {
  uint64_t s = seed;
  const double lo = dist == 1 ? -10.0 : 0.0;
  for (size_t i = 0; i < out.size(); ++i) {
    double x;
    if (dist == 0) {
      x = (double)(sm64(s) >> 11) * 0x1.0p-53;
    } else {
      const double u1 = unit_open(s), u2 = unit_open(s);
      x = std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
      if (dist == 2) x = std::exp(x);
    }
    x += 0.0;  // no negative zero
    if (kt == PCF_KEY_F64) {
      std::memcpy(&out[i], &x, 8);
    } else {
      const double y = std::max(x - lo, 0.0) * 4294967296.0;
      out[i] = (uint64_t)std::floor(y);
    }
  }
}

// A size class and what it is timed on: one array of rep_n keys, or (seg_lo <
// seg_hi) a segmented batch of rep_n keys in segments of floor(2^U[seg_lo,
// seg_hi]) keys, so that a class of small arrays is timed by its throughput
// (the batched use) rather than by the launch latency of one small sort.
struct Class {
  uint64_t min_n, max_n, rep_n;
  double seg_lo, seg_hi;
};

const Class kClasses[] = {
    {0, 1ull << 18, 1ull << 25, 10.0, 18.0},
    {1ull << 18, 1ull << 22, 1ull << 25, 18.0, 22.0},
    {1ull << 22, 1ull << 25, 1ull << 23, 0.0, 0.0},
    {1ull << 25, 1ull << 32, 1ull << 26, 0.0, 0.0},
};

struct Bench {
  int kt, pay;
  void* keys[3] = {nullptr, nullptr, nullptr};
  void* out = nullptr;
  uint32_t* idx = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  uint64_t* offs = nullptr;  // device CSR offsets of the current class's batch (or none)
  uint32_t nseg = 1;

  ~Bench() {
    if (offs) (void)hipFree(offs);
    for (void* k : keys)
      if (k) (void)hipFree(k);
    if (out) (void)hipFree(out);
    if (idx) (void)hipFree(idx);
    if (ws) (void)hipFree(ws);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
  }

  // milliseconds of one sort of `n` keys of distribution d under `pol`, or <0
  double time_one(const pcf_policy& pol, int d, size_t n) {
    pcf::SortArgs a = {};
    a.key_type = kt;
    a.keys_in = keys[d];
    a.keys_out = out;
    a.vals_out = pay ? idx : nullptr;
    a.iota = pay ? 1 : 0;
    a.nseg = nseg;
    a.offsets = nseg > 1 ? offs : nullptr;
    a.no_graph = 1;
    a.n = n;
    a.ws = ws;
    a.ws_bytes = ws_bytes;
    a.stream = st;
    a.pol_override = &pol;
    if (hipEventRecord(e0, st) != hipSuccess) return -1.0;
    if (pcf::run_sort(a) != PCF_OK) return -1.0;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
    return ms;
  }

  // median over `reps` of the summed time over the three distributions
  double score(const pcf_policy& pol, size_t n, int reps) {
    if (pcf::check_policy(pol) != PCF_OK) return -1.0;
    if (pcf::make_layout(n, pay, nseg, pol, 0, 0, 0).total > ws_bytes) return -1.0;
    std::vector<double> v;
    for (int r = 0; r < reps; ++r) {
      double t = 0;
      for (int d = 0; d < 3; ++d) {
        const double x = time_one(pol, d, n);
        if (x < 0) return -1.0;
        t += x;
      }
      v.push_back(t);
    }
    std::sort(v.begin(), v.end());
    return v[v.size() / 2];
  }
};

// ---- a small JSON reader (objects, arrays, numbers, strings, literals) ------
struct JVal {
  enum Kind { NUL, NUM, STR, ARR, OBJ, BOOL } kind = NUL;
  double num = 0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal* get(const char* k) const {
    for (const auto& kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

struct JParser {
  const char* p;
  const char* end;
  bool ok = true;
  void ws() {
    while (p < end && std::isspace((unsigned char)*p)) ++p;
  }
  bool lit(const char* s) {
    const size_t n = std::strlen(s);
    if ((size_t)(end - p) >= n && std::strncmp(p, s, n) == 0) {
      p += n;
      return true;
    }
    return false;
  }
  std::string string() {
    std::string s;
    ++p;  // opening quote
    while (p < end && *p != '"') {
      if (*p == '\\' && p + 1 < end) ++p;
      s.push_back(*p++);
    }
    if (p >= end) ok = false;
    else ++p;
    return s;
  }
  JVal value(int depth = 0) {
    JVal v;
    ws();
    if (p >= end || depth > 32) {
      ok = false;
      return v;
    }
    if (*p == '{') {
      v.kind = JVal::OBJ;
      ++p;
      ws();
      if (p < end && *p == '}') {
        ++p;
        return v;
      }
      while (ok) {
        ws();
        if (p >= end || *p != '"') {
          ok = false;
          break;
        }
        std::string k = string();
        ws();
        if (p >= end || *p != ':') {
          ok = false;
          break;
        }
        ++p;
        v.obj.emplace_back(k, value(depth + 1));
        ws();
        if (p < end && *p == ',') {
          ++p;
          continue;
        }
        if (p < end && *p == '}') {
          ++p;
          break;
        }
        ok = false;
      }
    } else if (*p == '[') {
      v.kind = JVal::ARR;
      ++p;
      ws();
      if (p < end && *p == ']') {
        ++p;
        return v;
      }
      while (ok) {
        v.arr.push_back(value(depth + 1));
        ws();
        if (p < end && *p == ',') {
          ++p;
          continue;
        }
        if (p < end && *p == ']') {
          ++p;
          break;
        }
        ok = false;
      }
    } else if (*p == '"') {
      v.kind = JVal::STR;
      v.str = string();
    } else if (lit("true")) {
      v.kind = JVal::BOOL;
      v.num = 1;
    } else if (lit("false")) {
      v.kind = JVal::BOOL;
    } else if (lit("null")) {
      v.kind = JVal::NUL;
    } else {
      char* e = nullptr;
      v.kind = JVal::NUM;
      v.num = std::strtod(p, &e);
      if (e == p) ok = false;
      p = e;
    }
    return v;
  }
};

constexpr int kNumFields = 12;
const char* kFields[kNumFields] = {"max_buckets", "target_child", "bins_per_bucket", "max_bins",
                                   "samples_per_bucket", "max_samples", "chunk_keys", "lds_cap",
                                   "tau", "seed", "model", "scatter_tile"};

uint32_t* field(pcf_policy& p, int i) {
  uint32_t* f[kNumFields] = {&p.max_buckets, &p.target_child,       &p.bins_per_bucket,
                             &p.max_bins,    &p.samples_per_bucket, &p.max_samples,
                             &p.chunk_keys,  &p.lds_cap,            &p.tau,
                             &p.seed,        &p.model,              &p.scatter_tile};
  return f[i];
}

bool whole(const JVal* v, double lo, double hi, uint64_t* out) {
  if (!v || v->kind != JVal::NUM || v->num < lo || v->num > hi || v->num != std::floor(v->num))
    return false;
  *out = (uint64_t)v->num;
  return true;
}

}  // namespace

extern "C" {

int pcf_autotune(int key_type, int with_payload, const char* out_json) {
  if ((key_type != PCF_KEY_F64 && key_type != PCF_KEY_U64) || !out_json)
    return PCF_ERR_INVALID_ARGUMENT;
  const int pay = with_payload ? 1 : 0;
  Bench b;
  b.kt = key_type;
  b.pay = pay;
  const size_t nmax = kClasses[3].rep_n;
  if (hipStreamCreateWithFlags(&b.st, hipStreamNonBlocking) != hipSuccess) return PCF_ERR_HIP;
  if (hipEventCreate(&b.e0) != hipSuccess || hipEventCreate(&b.e1) != hipSuccess) return PCF_ERR_HIP;
  {
    std::vector<uint64_t> h(nmax);
    for (int d = 0; d < 3; ++d) {
      make_keys(key_type, d, 0x5eed7ull + 977ull * (uint64_t)d, h);
      if (hipMalloc(&b.keys[d], nmax * 8) != hipSuccess) return PCF_ERR_OUT_OF_MEMORY;
      if (hipMemcpy(b.keys[d], h.data(), nmax * 8, hipMemcpyHostToDevice) != hipSuccess)
        return PCF_ERR_HIP;
    }
  }
  if (hipMalloc(&b.out, nmax * 8) != hipSuccess) return PCF_ERR_OUT_OF_MEMORY;
  if (pay && hipMalloc(reinterpret_cast<void**>(&b.idx), nmax * 4) != hipSuccess)
    return PCF_ERR_OUT_OF_MEMORY;

  // candidate values per parameter (coordinate descent, two passes)
  struct Dim {
    int field;
    std::vector<uint32_t> vals;
  };
  const std::vector<Dim> dims = {
      {0, {64, 128, 256, 512}},      // max_buckets
      {4, {8, 16, 32}},              // samples_per_bucket
      {2, {8, 16, 32}},              // bins_per_bucket
      {6, {8192, 16384, 32768}},     // chunk_keys
      {1, {1024, 2048, 4096, 8192}}, // target_child
      {11, pay ? std::vector<uint32_t>{1024, 2048} : std::vector<uint32_t>{4096, 8192}},  // scatter_tile
  };
  // the workspace must hold every candidate's layout at the largest size
  const pcf_policy base = pcf::current_policy();
  b.ws_bytes = 0;
  for (uint32_t mb : dims[0].vals)
    for (uint32_t sp : dims[1].vals)
      for (uint32_t bp : dims[2].vals)
        for (uint32_t ck : dims[3].vals)
          for (uint32_t tc : dims[4].vals) {
            pcf_policy c = base;
            c.max_buckets = mb;
            c.samples_per_bucket = sp;
            c.bins_per_bucket = bp;
            c.chunk_keys = ck;
            c.target_child = tc;
            b.ws_bytes = std::max(b.ws_bytes, pcf::make_layout(nmax, pay, 4096, c, 0, 0, 0).total);
          }
  if (hipMalloc(&b.ws, b.ws_bytes) != hipSuccess) return PCF_ERR_OUT_OF_MEMORY;

  std::vector<TuneEntry> table;
  for (const Class& c : kClasses) {
    const size_t n = c.rep_n;
    // the class's batch: segment sizes from a fixed SplitMix64 stream
    b.nseg = 1;
    if (c.seg_lo < c.seg_hi) {
      std::vector<uint64_t> off(1, 0);
      uint64_t rs = 0x5e65ull + (uint64_t)c.min_n;
      while (off.back() < n && off.size() < 4096) {
        const double u = (double)(sm64(rs) >> 11) * 0x1.0p-53;
        const uint64_t len = (uint64_t)std::floor(std::exp2(c.seg_lo + u * (c.seg_hi - c.seg_lo)));
        off.push_back(std::min<uint64_t>(n, off.back() + std::max<uint64_t>(len, 1)));
      }
      off.back() = n;
      if (b.offs) (void)hipFree(b.offs);
      b.offs = nullptr;
      if (hipMalloc(reinterpret_cast<void**>(&b.offs), off.size() * 8) != hipSuccess)
        return PCF_ERR_OUT_OF_MEMORY;
      if (hipMemcpy(b.offs, off.data(), off.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
        return PCF_ERR_HIP;
      b.nseg = (uint32_t)(off.size() - 1);
    }
    const int reps = n >= (1u << 23) ? 3 : 5;
    pcf_policy best = base;
    (void)b.score(best, n, 1);  // warm-up
    double best_ms = b.score(best, n, reps);
    if (best_ms < 0) return PCF_ERR_HIP;
    for (int pass = 0; pass < 2; ++pass) {
      for (const Dim& d : dims) {
        for (uint32_t v : d.vals) {
          if (v == *field(best, d.field)) continue;
          pcf_policy cand = best;
          *field(cand, d.field) = v;
          const double t = b.score(cand, n, reps);
          if (t > 0 && t < best_ms * 0.98) {  // keep a change only when it clearly helps
            best = cand;
            best_ms = t;
          }
        }
      }
    }
    TuneEntry e;
    e.key_type = key_type;
    e.with_payload = pay;
    e.min_n = c.min_n;
    e.max_n = c.max_n;
    e.pol = best;
    e.ms = best_ms / 3.0;
    table.push_back(e);
  }

  hipDeviceProp_t pr;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const bool have_pr = hipGetDeviceProperties(&pr, dev) == hipSuccess;
  FILE* f = std::fopen(out_json, "w");
  if (!f) return PCF_ERR_INVALID_ARGUMENT;
  std::fprintf(f, "{\n  \"format\": \"pcfsort-tuning-1\",\n  \"device\": \"%s\",\n  \"arch\": \"%s\",\n",
               have_pr ? pr.name : "unknown", have_pr ? pr.gcnArchName : "unknown");
  std::fprintf(f, "  \"entries\": [\n");
  for (size_t i = 0; i < table.size(); ++i) {
    const TuneEntry& e = table[i];
    std::fprintf(f,
                 "    {\"key_type\": %d, \"with_payload\": %d, \"min_n\": %llu, \"max_n\": %llu, "
                 "\"rep_n\": %llu, \"ms_per_sort\": %.5f,\n     \"policy\": {",
                 e.key_type, e.with_payload, (unsigned long long)e.min_n,
                 (unsigned long long)e.max_n, (unsigned long long)kClasses[i].rep_n, e.ms);
    pcf_policy p = e.pol;
    for (int k = 0; k < kNumFields; ++k)
      std::fprintf(f, "%s\"%s\": %u", k ? ", " : "", kFields[k], *field(p, k));
    std::fprintf(f, "}}%s\n", i + 1 < table.size() ? "," : "");
  }
  std::fprintf(f, "  ]\n}\n");
  std::fclose(f);
  return PCF_OK;
}

int pcf_load_tuning(const char* json_path) {
  if (!json_path) {
    pcf::install_table({});
    return PCF_OK;
  }
  FILE* f = std::fopen(json_path, "rb");
  if (!f) return PCF_ERR_INVALID_ARGUMENT;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) {
    text.append(buf, got);
    if (text.size() > (1u << 22)) break;
  }
  std::fclose(f);
  JParser jp{text.data(), text.data() + text.size()};
  const JVal root = jp.value();
  if (!jp.ok || root.kind != JVal::OBJ) return PCF_ERR_INVALID_ARGUMENT;
  const JVal* fmt = root.get("format");
  if (!fmt || fmt->kind != JVal::STR || fmt->str != "pcfsort-tuning-1") return PCF_ERR_INVALID_ARGUMENT;
  const JVal* ents = root.get("entries");
  if (!ents || ents->kind != JVal::ARR) return PCF_ERR_INVALID_ARGUMENT;
  std::vector<TuneEntry> t;
  for (const JVal& e : ents->arr) {
    if (e.kind != JVal::OBJ) return PCF_ERR_INVALID_ARGUMENT;
    TuneEntry te = {};
    uint64_t kt, wp;
    if (!whole(e.get("key_type"), 0, 1, &kt) || !whole(e.get("with_payload"), 0, 1, &wp) ||
        !whole(e.get("min_n"), 0, 4294967296.0, &te.min_n) ||
        !whole(e.get("max_n"), 1, 4294967296.0, &te.max_n) || te.min_n >= te.max_n)
      return PCF_ERR_INVALID_ARGUMENT;
    te.key_type = (int)kt;
    te.with_payload = (int)wp;
    const JVal* pol = e.get("policy");
    if (!pol || pol->kind != JVal::OBJ) return PCF_ERR_INVALID_ARGUMENT;
    te.pol = pcf::current_policy();  // fields the file omits keep the defaults
    for (int k = 0; k < kNumFields; ++k) {
      const JVal* v = pol->get(kFields[k]);
      if (!v) continue;
      uint64_t x;
      if (!whole(v, 0, 4294967295.0, &x)) return PCF_ERR_INVALID_ARGUMENT;
      *field(te.pol, k) = (uint32_t)x;
    }
    if (pcf::check_policy(te.pol) != PCF_OK) return PCF_ERR_INVALID_ARGUMENT;
    // overlapping classes of one kind are ambiguous
    for (const TuneEntry& o : t)
      if (o.key_type == te.key_type && o.with_payload == te.with_payload && te.min_n < o.max_n &&
          o.min_n < te.max_n)
        return PCF_ERR_INVALID_ARGUMENT;
    t.push_back(te);
  }
  pcf::install_table(t);
  return PCF_OK;
}

}  // extern "C"
