// pcf_serve_core.h -- continuous-batching sort server (host logic only).
//
// The scheduler knows nothing of HIP: it admits requests, packs them into
// batches (one segmented sort each), places every batch's memory inside one
// arena whose size is the HBM budget, and hands batches to an Executor that
// runs them on the device (one worker thread and one stream per slot).  A
// mock executor over host memory drives the same scheduler in CPU tests.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace pcfserve {

// Status codes shared with the C ABI (same values as pcf_status).
enum {
  S_OK = 0,
  S_INVALID_ARGUMENT = 1,
  S_INVALID_KEY = 2,
  S_OUT_OF_MEMORY = 3,
  S_HIP = 4,
  S_UNSUPPORTED = 5,
  S_PENDING = 6,
  S_UNKNOWN_TICKET = 7,
  S_SHUTDOWN = 8,
};

// First-fit allocator over [0, size) with coalescing; offsets are aligned to
// `align` bytes.  Not thread-safe (the server holds its lock).
class Arena {
 public:
  explicit Arena(uint64_t size = 0, uint64_t align = 256);
  // returns false when no free block fits
  bool alloc(uint64_t bytes, uint64_t* off);
  void free(uint64_t off);
  uint64_t in_use() const { return used_; }
  uint64_t high_water() const { return high_; }
  uint64_t size() const { return size_; }
  // largest free block (for admission decisions)
  uint64_t largest_free() const;
  size_t free_blocks() const { return free_.size(); }

 private:
  uint64_t size_, align_, used_ = 0, high_ = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> length
  std::map<uint64_t, uint64_t> live_;  // offset -> length
};

// One batch as the executor sees it: segment s of the output holds the sorted
// keys of request s, whose input starts at src[s] (device address) and has
// offsets[s+1] - offsets[s] keys.  All pointers are arena addresses except src.
struct BatchDesc {
  int key_type;
  int argsort;
  uint32_t nseg;
  uint64_t total;
  const uint64_t* offsets;  // host, nseg + 1 entries
  const uint64_t* src;      // host, nseg device addresses
  const uint64_t* ready;    // host, nseg opaque event handles (0: none) the
                            // batch must wait for before it reads src[s]
  void* out_keys;           // total keys
  uint32_t* out_idx;        // total indices or NULL
  void* work;               // work_bytes of scratch (workspace + metadata)
  uint64_t work_bytes;
};

class Executor {
 public:
  virtual ~Executor() {}
  // Allocates the arena (budget bytes) and the per-slot resources.
  virtual int init(int device, uint32_t slots, uint64_t budget, uint32_t max_batch_requests,
                   void** arena_base) = 0;
  // Scratch one batch needs besides its outputs.
  virtual uint64_t work_bytes(int key_type, uint64_t total, int argsort, uint32_t nseg) = 0;
  // Runs one batch on the slot's stream and returns when it has completed.
  virtual int run(uint32_t slot, const BatchDesc& b) = 0;
  // Frees what init allocated; called after every worker has stopped.
  virtual void shutdown() = 0;
};

struct ServeConfig {
  uint64_t budget;
  uint32_t slots;
  uint32_t max_batch_requests;
  uint64_t max_batch_keys;
  int device;
};

struct Result {
  void* keys;
  uint32_t* idx;
  uint64_t n;
  uint64_t latency_ns;
  uint64_t queue_ns;
  int32_t status;
  uint32_t batch_requests;
};

struct Stats {
  uint64_t submitted, completed, released, batches, budget, in_use, high_water, queued;
};

class Server {
 public:
  Server(const ServeConfig& cfg, std::unique_ptr<Executor> ex);
  ~Server();
  int start();  // S_OK or an executor error
  // `ready` is an opaque event handle the executor waits for before the batch
  // reads d_keys (NULL: the keys are ready now)
  int submit(int key_type, const void* d_keys, uint64_t n, int argsort, uint64_t* ticket,
             const void* ready = nullptr);
  int poll(uint64_t ticket, Result* out);
  int wait(uint64_t ticket, uint32_t timeout_ms, Result* out);
  int release(uint64_t ticket);
  Stats stats();
  void stop();  // drains running batches, fails queued requests with S_SHUTDOWN

 private:
  struct Batch;
  struct Request {
    uint64_t ticket;
    int key_type, argsort;
    const void* src;
    const void* ready;
    uint64_t n;
    uint64_t t_submit, t_start, t_done;
    int32_t status;
    bool done, released;
    Batch* batch;
    uint64_t out_pos;  // position of the result inside the batch's output
    uint32_t batch_requests;
  };
  struct Batch {
    uint64_t out_off, idx_off, work_off;
    bool has_idx;
    uint32_t live;  // requests of the batch not yet released
  };

  uint64_t out_bytes(uint64_t n, int argsort) const;
  uint64_t alone_bytes(int key_type, uint64_t n, int argsort);
  void worker(uint32_t slot);
  // under mu_: takes the next batch that fits the arena, or returns false
  bool form_batch(std::vector<Request*>& reqs, Batch*& b, uint64_t& total);
  void fill_result(const Request& r, Result* out) const;
  void drop_request(Request* r);  // under mu_: frees the result if the batch is fully released

  ServeConfig cfg_;
  std::unique_ptr<Executor> ex_;
  void* base_ = nullptr;
  Arena arena_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<Request*> queue_;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs_;
  std::vector<std::thread> workers_;
  uint64_t next_ticket_ = 1;
  bool stopping_ = false, started_ = false;
  Stats st_ = {};
};

uint64_t now_ns();

}  // namespace pcfserve
