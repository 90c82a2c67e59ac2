// Host-memory executor for the serving scheduler: lets CPU tests drive the
// real admission, batching, budget and ticket logic of pcf_serve_core.
// "Device" memory is host memory; a batch is sorted with std::stable_sort per
// segment, after an optional delay that keeps slots busy.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#include "pcf_serve_core.h"

using namespace pcfserve;

namespace {

std::atomic<int> g_running{0}, g_max_running{0};
std::atomic<uint64_t> g_batches{0}, g_max_batch{0};
// while closed, a batch that has started waits before it sorts (bounded)
std::atomic<int> g_gate_closed{0};

uint64_t ordered(int kt, uint64_t b) {
  if (kt == 1) return b;
  return (b >> 63) ? ~b : (b | (1ull << 63));
}

class MockExecutor : public Executor {
 public:
  explicit MockExecutor(uint32_t delay_us) : delay_us_(delay_us) {}
  int init(int, uint32_t, uint64_t budget, uint32_t, void** base) override {
    mem_.assign(budget, 0);
    *base = mem_.data();
    return S_OK;
  }
  uint64_t work_bytes(int, uint64_t total, int, uint32_t nseg) override {
    return 16 * total + 64 * (uint64_t)nseg + 1024;
  }
  int run(uint32_t, const BatchDesc& d) override {
    const int now = ++g_running;
    int prev = g_max_running.load();
    while (now > prev && !g_max_running.compare_exchange_weak(prev, now)) {}
    uint64_t pb = g_max_batch.load();
    while (d.nseg > pb && !g_max_batch.compare_exchange_weak(pb, d.nseg)) {}
    ++g_batches;
    for (int i = 0; i < 20000 && g_gate_closed.load(); ++i)
      std::this_thread::sleep_for(std::chrono::milliseconds(1));
    if (delay_us_) std::this_thread::sleep_for(std::chrono::microseconds(delay_us_));
    // the work area must be writable over its whole declared size
    memset(d.work, 0xab, d.work_bytes);
    int rc = S_OK;
    std::vector<std::pair<uint64_t, uint32_t>> v;
    for (uint32_t s = 0; s < d.nseg && rc == S_OK; ++s) {
      const uint64_t a = d.offsets[s], n = d.offsets[s + 1] - a;
      const uint64_t* src = reinterpret_cast<const uint64_t*>((uintptr_t)d.src[s]);
      v.resize(n);
      for (uint64_t i = 0; i < n; ++i) {
        const uint64_t b = src[i];
        if (d.key_type == 0) {
          double x;
          memcpy(&x, &b, 8);
          if (!isfinite(x) || b == (1ull << 63)) rc = S_INVALID_KEY;
        }
        v[i] = {ordered(d.key_type, b), (uint32_t)i};
      }
      std::stable_sort(v.begin(), v.end(),
                       [](const std::pair<uint64_t, uint32_t>& x,
                          const std::pair<uint64_t, uint32_t>& y) { return x.first < y.first; });
      uint64_t* ok = reinterpret_cast<uint64_t*>(d.out_keys) + a;
      for (uint64_t i = 0; i < n; ++i) {
        ok[i] = src[v[i].second];
        if (d.out_idx) d.out_idx[a + i] = v[i].second;
      }
    }
    --g_running;
    return rc;
  }
  void shutdown() override {}

 private:
  uint32_t delay_us_;
  std::vector<char> mem_;
};

}  // namespace

extern "C" {

struct mock_result {
  uint64_t keys, idx, n, latency_ns, queue_ns;
  int32_t status;
  uint32_t batch_requests;
};

void* mock_create(uint64_t budget, uint32_t slots, uint32_t maxreq, uint64_t maxkeys,
                  uint32_t delay_us) {
  g_running = 0;
  g_max_running = 0;
  g_batches = 0;
  g_max_batch = 0;
  g_gate_closed = 0;
  ServeConfig c = {budget, slots, maxreq, maxkeys, 0};
  auto* s = new Server(c, std::unique_ptr<Executor>(new MockExecutor(delay_us)));
  if (s->start() != S_OK) {
    delete s;
    return nullptr;
  }
  return s;
}

int mock_submit(void* s, int kt, const void* keys, uint64_t n, int argsort, uint64_t* ticket) {
  return static_cast<Server*>(s)->submit(kt, keys, n, argsort, ticket);
}

static void conv(const Result& r, mock_result* o) {
  o->keys = (uint64_t)(uintptr_t)r.keys;
  o->idx = (uint64_t)(uintptr_t)r.idx;
  o->n = r.n;
  o->latency_ns = r.latency_ns;
  o->queue_ns = r.queue_ns;
  o->status = r.status;
  o->batch_requests = r.batch_requests;
}

int mock_poll(void* s, uint64_t t, mock_result* o) {
  Result r;
  const int rc = static_cast<Server*>(s)->poll(t, &r);
  if (rc == S_OK) conv(r, o);
  return rc;
}

int mock_wait(void* s, uint64_t t, uint32_t ms, mock_result* o) {
  Result r;
  const int rc = static_cast<Server*>(s)->wait(t, ms, &r);
  if (rc == S_OK) conv(r, o);
  return rc;
}

int mock_release(void* s, uint64_t t) { return static_cast<Server*>(s)->release(t); }

void mock_stats(void* s, uint64_t* out8) {
  const Stats t = static_cast<Server*>(s)->stats();
  const uint64_t v[8] = {t.submitted, t.completed, t.released, t.batches,
                         t.budget,    t.in_use,    t.high_water, t.queued};
  memcpy(out8, v, sizeof(v));
}

void mock_stop(void* s) { static_cast<Server*>(s)->stop(); }

void mock_destroy(void* s) { delete static_cast<Server*>(s); }

int mock_max_running(void) { return g_max_running.load(); }
uint64_t mock_max_batch(void) { return g_max_batch.load(); }
uint64_t mock_batches_started(void) { return g_batches.load(); }
void mock_gate(int closed) { g_gate_closed = closed ? 1 : 0; }

}  // extern "C"
