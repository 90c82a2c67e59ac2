// pcf_serve.cpp -- the serving C ABI: the continuous-batching scheduler of
// pcf_serve_core driven by a HIP executor.
//
// Every batch is one segmented sort whose roots read each request's keys in
// place (per-segment source addresses), so requests are never gathered into a
// staging copy; the sorted keys (and argsort positions) land in server-owned
// arena memory.  Each slot has its own worker thread and its own stream, so
// batches of different slots overlap on the device.
#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "../../include/pcfsort.h"
#include "pcf_driver.h"
#include "pcf_serve_core.h"

namespace {

using pcfserve::BatchDesc;

uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

class HipExecutor : public pcfserve::Executor {
 public:
  ~HipExecutor() override { shutdown(); }

  int init(int device, uint32_t slots, uint64_t budget, uint32_t max_batch_requests,
           void** arena_base) override {
    dev_ = device;
    maxreq_ = max_batch_requests;
    if (hipSetDevice(dev_) != hipSuccess) return PCF_ERR_HIP;
    if (hipMalloc(&arena_, budget) != hipSuccess) {
      (void)hipGetLastError();
      arena_ = nullptr;
      return PCF_ERR_OUT_OF_MEMORY;
    }
    for (uint32_t s = 0; s < slots; ++s) {
      hipStream_t st = nullptr;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return PCF_ERR_HIP;
      streams_.push_back(st);
      void* pin = nullptr;
      if (hipHostMalloc(&pin, staging_bytes(), hipHostMallocDefault) != hipSuccess) return PCF_ERR_HIP;
      pinned_.push_back(pin);
    }
    *arena_base = arena_;
    return PCF_OK;
  }

  uint64_t work_bytes(int key_type, uint64_t total, int argsort, uint32_t nseg) override {
    return round_up(pcf::workspace_for(key_type, total, argsort, nseg, 0), 256) + meta_bytes(nseg);
  }

  int run(uint32_t slot, const BatchDesc& d) override {
    if (hipSetDevice(dev_) != hipSuccess) return PCF_ERR_HIP;
    hipStream_t st = streams_[slot];
    const uint64_t ws_bytes =
        round_up(pcf::workspace_for(d.key_type, d.total, d.argsort, d.nseg, 0), 256);
    if (ws_bytes + meta_bytes(d.nseg) > d.work_bytes || d.nseg > maxreq_) return PCF_ERR_INVALID_ARGUMENT;
    char* w = reinterpret_cast<char*>(d.work);
    // metadata after the workspace: offsets (nseg + 1), sources (nseg)
    uint64_t* m_dev = reinterpret_cast<uint64_t*>(w + ws_bytes);
    uint64_t* m_host = reinterpret_cast<uint64_t*>(pinned_[slot]);
    for (uint32_t s = 0; s <= d.nseg; ++s) m_host[s] = d.offsets[s];
    for (uint32_t s = 0; s < d.nseg; ++s) m_host[d.nseg + 1 + s] = d.src[s];
    // the producers' work on the request keys comes first
    for (uint32_t s = 0; s < d.nseg; ++s)
      if (d.ready && d.ready[s] &&
          hipStreamWaitEvent(st, reinterpret_cast<hipEvent_t>((uintptr_t)d.ready[s]), 0) != hipSuccess)
        return PCF_ERR_HIP;
    if (hipMemcpyAsync(m_dev, m_host, 8ull * (2 * d.nseg + 1), hipMemcpyHostToDevice, st) != hipSuccess)
      return PCF_ERR_HIP;
    pcf::SortArgs a = {};
    a.key_type = d.key_type;
    a.keys_out = d.out_keys;
    a.vals_out = d.out_idx;
    a.iota = d.argsort ? 1 : 0;
    a.offsets = m_dev;
    a.seg_src = m_dev + d.nseg + 1;
    a.no_graph = 1;
    a.nseg = d.nseg;
    a.n = d.total;
    a.ws = w;
    a.ws_bytes = ws_bytes;
    a.stream = st;
    // no status word: the worker waits for the batch anyway, so the call takes
    // the levels the input needs (the host reads the level counts) and
    // returns the data status itself
    int rc = pcf::run_sort(a);
    // the staging buffer and the batch memory are reused after this returns
    if (hipStreamSynchronize(st) != hipSuccess && rc == PCF_OK) rc = PCF_ERR_HIP;
    return rc;
  }

  void shutdown() override {
    if (dev_ >= 0) (void)hipSetDevice(dev_);
    for (auto st : streams_) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
    streams_.clear();
    for (auto p : pinned_) (void)hipHostFree(p);
    pinned_.clear();
    if (arena_) (void)hipFree(arena_);
    arena_ = nullptr;
  }

 private:
  uint64_t meta_bytes(uint32_t nseg) const { return round_up(8ull * (2 * nseg + 1), 256) + 256; }
  uint64_t staging_bytes() const { return 8ull * (2 * maxreq_ + 2) + 64; }

  int dev_ = -1;
  uint32_t maxreq_ = 0;
  void* arena_ = nullptr;
  std::vector<hipStream_t> streams_;
  std::vector<void*> pinned_;
};

}  // namespace

struct pcf_server {
  std::unique_ptr<pcfserve::Server> srv;
};

extern "C" {

int pcf_serve_create(const pcf_serve_config* cfg, pcf_server** out) {
  if (!cfg || !out) return PCF_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (cfg->hbm_budget_bytes < 4096 || cfg->max_streams < 1 || cfg->max_streams > 8 ||
      cfg->max_batch_requests < 1 || cfg->max_batch_requests > (1u << 20) ||
      cfg->max_batch_keys < 1 || cfg->flags != 0)
    return PCF_ERR_INVALID_ARGUMENT;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) return PCF_ERR_HIP;
  if (cfg->device < 0 || cfg->device >= ndev) return PCF_ERR_INVALID_ARGUMENT;
  pcfserve::ServeConfig c;
  c.budget = cfg->hbm_budget_bytes;
  c.slots = cfg->max_streams;
  c.max_batch_requests = cfg->max_batch_requests;
  c.max_batch_keys = cfg->max_batch_keys;
  c.device = cfg->device;
  std::unique_ptr<pcf_server> s(new pcf_server);
  s->srv.reset(new pcfserve::Server(c, std::unique_ptr<pcfserve::Executor>(new HipExecutor)));
  const int rc = s->srv->start();
  if (rc != PCF_OK) return rc;
  *out = s.release();
  return PCF_OK;
}

int pcf_serve_submit(pcf_server* s, int key_type, const void* d_keys, size_t n, int want_argsort,
                     uint64_t* ticket) {
  if (!s) return PCF_ERR_INVALID_ARGUMENT;
  return s->srv->submit(key_type, d_keys, n, want_argsort, ticket);
}

int pcf_serve_submit_after(pcf_server* s, int key_type, const void* d_keys, size_t n,
                           int want_argsort, void* ready_event, uint64_t* ticket) {
  if (!s) return PCF_ERR_INVALID_ARGUMENT;
  return s->srv->submit(key_type, d_keys, n, want_argsort, ticket, ready_event);
}

static void to_c(const pcfserve::Result& r, pcf_result* out) {
  out->d_keys_sorted = r.keys;
  out->d_idx = r.idx;
  out->n = r.n;
  out->latency_ns = r.latency_ns;
  out->queue_ns = r.queue_ns;
  out->status = r.status;
  out->batch_requests = r.batch_requests;
}

int pcf_serve_poll(pcf_server* s, uint64_t ticket, pcf_result* out) {
  if (!s) return PCF_ERR_INVALID_ARGUMENT;
  pcfserve::Result r;
  const int rc = s->srv->poll(ticket, &r);
  if (rc == PCF_OK && out) to_c(r, out);
  return rc;
}

int pcf_serve_wait(pcf_server* s, uint64_t ticket, uint32_t timeout_ms, pcf_result* out) {
  if (!s) return PCF_ERR_INVALID_ARGUMENT;
  pcfserve::Result r;
  const int rc = s->srv->wait(ticket, timeout_ms, &r);
  if (rc == PCF_OK && out) to_c(r, out);
  return rc;
}

int pcf_serve_release(pcf_server* s, uint64_t ticket) {
  if (!s) return PCF_ERR_INVALID_ARGUMENT;
  return s->srv->release(ticket);
}

int pcf_serve_get_stats(pcf_server* s, pcf_serve_stats* out) {
  if (!s || !out) return PCF_ERR_INVALID_ARGUMENT;
  const pcfserve::Stats t = s->srv->stats();
  out->submitted = t.submitted;
  out->completed = t.completed;
  out->released = t.released;
  out->batches = t.batches;
  out->budget_bytes = t.budget;
  out->budget_in_use = t.in_use;
  out->budget_high_water = t.high_water;
  out->queued = t.queued;
  return PCF_OK;
}

int pcf_serve_destroy(pcf_server* s) {
  if (!s) return PCF_ERR_INVALID_ARGUMENT;
  s->srv->stop();
  delete s;
  return PCF_OK;
}

}  // extern "C"
