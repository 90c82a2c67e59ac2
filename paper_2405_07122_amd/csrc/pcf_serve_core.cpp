// pcf_serve_core.cpp -- continuous-batching sort server (host logic only).
#include "pcf_serve_core.h"

#include <algorithm>
#include <chrono>

namespace pcfserve {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

static uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// ---- Arena -------------------------------------------------------------------

Arena::Arena(uint64_t size, uint64_t align) : size_(size / align * align), align_(align) {
  if (size_) free_[0] = size_;
}

bool Arena::alloc(uint64_t bytes, uint64_t* off) {
  const uint64_t need = round_up(std::max<uint64_t>(bytes, 1), align_);
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < need) continue;
    const uint64_t o = it->first, len = it->second;
    free_.erase(it);
    if (len > need) free_[o + need] = len - need;
    live_[o] = need;
    used_ += need;
    high_ = std::max(high_, used_);
    *off = o;
    return true;
  }
  return false;
}

void Arena::free(uint64_t off) {
  auto lv = live_.find(off);
  if (lv == live_.end()) return;
  uint64_t o = off, len = lv->second;
  live_.erase(lv);
  used_ -= len;
  auto nx = free_.lower_bound(o);
  if (nx != free_.end() && nx->first == o + len) {  // merge with the next block
    len += nx->second;
    nx = free_.erase(nx);
  }
  if (nx != free_.begin()) {  // merge with the previous block
    auto pv = std::prev(nx);
    if (pv->first + pv->second == o) {
      pv->second += len;
      return;
    }
  }
  free_[o] = len;
}

uint64_t Arena::largest_free() const {
  uint64_t m = 0;
  for (const auto& kv : free_) m = std::max(m, kv.second);
  return m;
}

// ---- Server ------------------------------------------------------------------

Server::Server(const ServeConfig& cfg, std::unique_ptr<Executor> ex)
    : cfg_(cfg), ex_(std::move(ex)), arena_(cfg.budget) {
  st_.budget = arena_.size();
}

Server::~Server() {
  stop();
  // batches whose results were never released
  std::vector<Batch*> held;
  for (auto& kv : reqs_)
    if (kv.second->batch &&
        std::find(held.begin(), held.end(), kv.second->batch) == held.end())
      held.push_back(kv.second->batch);
  for (Batch* b : held) delete b;
}

int Server::start() {
  const int rc = ex_->init(cfg_.device, cfg_.slots, arena_.size(), cfg_.max_batch_requests, &base_);
  if (rc != S_OK) return rc;
  started_ = true;
  for (uint32_t s = 0; s < cfg_.slots; ++s) workers_.emplace_back(&Server::worker, this, s);
  return S_OK;
}

uint64_t Server::out_bytes(uint64_t n, int argsort) const {
  return round_up(8 * n, 256) + (argsort ? round_up(4 * n, 256) : 0);
}

uint64_t Server::alone_bytes(int key_type, uint64_t n, int argsort) {
  return out_bytes(n, argsort) + round_up(ex_->work_bytes(key_type, n, argsort, 1), 256);
}

int Server::submit(int key_type, const void* d_keys, uint64_t n, int argsort, uint64_t* ticket,
                   const void* ready) {
  if (!ticket || (key_type != 0 && key_type != 1)) return S_INVALID_ARGUMENT;
  if (n > 0 && !d_keys) return S_INVALID_ARGUMENT;
  if (n >= (1ull << 32)) return S_INVALID_ARGUMENT;
  const uint64_t need = n ? alone_bytes(key_type, n, argsort) : 0;
  std::lock_guard<std::mutex> g(mu_);
  if (stopping_ || !started_) return S_SHUTDOWN;
  if (need > arena_.size()) return S_OUT_OF_MEMORY;
  auto r = std::make_unique<Request>();
  r->ticket = next_ticket_++;
  r->key_type = key_type;
  r->argsort = argsort ? 1 : 0;
  r->src = d_keys;
  r->ready = ready;
  r->n = n;
  r->t_submit = now_ns();
  r->status = S_PENDING;
  Request* rp = r.get();
  reqs_[rp->ticket] = std::move(r);
  ++st_.submitted;
  *ticket = rp->ticket;
  if (n == 0) {  // nothing to sort
    rp->t_start = rp->t_done = rp->t_submit;
    rp->status = S_OK;
    rp->done = true;
    ++st_.completed;
    cv_done_.notify_all();
    return S_OK;
  }
  queue_.push_back(rp);
  cv_work_.notify_one();
  return S_OK;
}

bool Server::form_batch(std::vector<Request*>& reqs, Batch*& b, uint64_t& total) {
  reqs.clear();
  total = 0;
  if (queue_.empty()) return false;
  const Request* head = queue_.front();
  // FIFO from the head: every queued request of the head's kind, within the
  // per-batch limits (segment sizes stay below 2^32 in the sum)
  for (Request* r : queue_) {
    if (reqs.size() >= cfg_.max_batch_requests) break;
    if (r->key_type != head->key_type || r->argsort != head->argsort) continue;
    if (!reqs.empty() && (total + r->n > cfg_.max_batch_keys || total + r->n >= (1ull << 32)))
      break;
    reqs.push_back(r);
    total += r->n;
  }
  // shrink from the tail until the batch's memory fits the arena
  while (!reqs.empty()) {
    uint64_t o_out = 0, o_idx = 0, o_work = 0;
    const int as = head->argsort;
    const uint64_t wb = ex_->work_bytes(head->key_type, total, as, (uint32_t)reqs.size());
    bool ok = arena_.alloc(8 * total, &o_out);
    bool ok_idx = ok && (!as || arena_.alloc(4 * total, &o_idx));
    bool ok_work = ok_idx && arena_.alloc(wb, &o_work);
    if (ok_work) {
      b = new Batch{o_out, o_idx, o_work, as != 0, (uint32_t)reqs.size()};
      break;
    }
    if (ok_idx && as) arena_.free(o_idx);
    if (ok) arena_.free(o_out);
    total -= reqs.back()->n;
    reqs.pop_back();
  }
  if (reqs.empty()) return false;  // the head waits for memory
  st_.high_water = arena_.high_water();
  // remove the chosen requests from the queue, keeping the others' order
  size_t k = 0;
  std::deque<Request*> rest;
  for (Request* r : queue_) {
    if (k < reqs.size() && r == reqs[k]) {
      ++k;
      continue;
    }
    rest.push_back(r);
  }
  queue_.swap(rest);
  return true;
}

void Server::worker(uint32_t slot) {
  std::vector<Request*> reqs;
  std::vector<uint64_t> offs, srcs, readys;
  for (;;) {
    Batch* b = nullptr;
    uint64_t total = 0;
    {
      std::unique_lock<std::mutex> lk(mu_);
      for (;;) {
        if (stopping_) return;
        if (form_batch(reqs, b, total)) break;
        cv_work_.wait(lk);
      }
      const uint64_t t = now_ns();
      uint64_t pos = 0;
      for (Request* r : reqs) {
        r->t_start = t;
        r->batch = b;
        r->out_pos = pos;
        r->batch_requests = (uint32_t)reqs.size();
        pos += r->n;
      }
    }
    const int kt = reqs[0]->key_type, as = reqs[0]->argsort;
    char* base = reinterpret_cast<char*>(base_);
    auto run_group = [&](size_t i0, size_t i1) {
      offs.assign(1, 0);
      srcs.clear();
      readys.clear();
      for (size_t i = i0; i < i1; ++i) {
        offs.push_back(offs.back() + reqs[i]->n);
        srcs.push_back((uint64_t)(uintptr_t)reqs[i]->src);
        readys.push_back((uint64_t)(uintptr_t)reqs[i]->ready);
      }
      BatchDesc d;
      d.key_type = kt;
      d.argsort = as;
      d.nseg = (uint32_t)(i1 - i0);
      d.total = offs.back();
      d.offsets = offs.data();
      d.src = srcs.data();
      d.ready = readys.data();
      d.out_keys = base + b->out_off + 8 * reqs[i0]->out_pos;
      d.out_idx = as ? reinterpret_cast<uint32_t*>(base + b->idx_off) + reqs[i0]->out_pos : nullptr;
      d.work = base + b->work_off;
      d.work_bytes = ex_->work_bytes(kt, total, as, (uint32_t)reqs.size());
      return ex_->run(slot, d);
    };
    std::vector<int> rcs(reqs.size(), S_OK);
    const int rc = run_group(0, reqs.size());
    for (auto& x : rcs) x = rc;
    if (rc == S_INVALID_KEY && reqs.size() > 1) {
      // isolate the request(s) with invalid keys: rerun each one alone in
      // its own slice of the batch's memory
      for (size_t i = 0; i < reqs.size(); ++i) rcs[i] = run_group(i, i + 1);
    }
    {
      std::lock_guard<std::mutex> g(mu_);
      arena_.free(b->work_off);
      const uint64_t t = now_ns();
      for (size_t i = 0; i < reqs.size(); ++i) {
        Request* r = reqs[i];
        r->t_done = t;
        r->status = rcs[i];
        r->done = true;
        ++st_.completed;
        if (r->released) drop_request(r);
      }
      ++st_.batches;
      cv_done_.notify_all();
      cv_work_.notify_all();
    }
  }
}

void Server::drop_request(Request* r) {
  Batch* b = r->batch;
  const uint64_t t = r->ticket;
  if (b && --b->live == 0) {
    arena_.free(b->out_off);
    if (b->has_idx) arena_.free(b->idx_off);
    delete b;
    cv_work_.notify_all();
  }
  reqs_.erase(t);
}

void Server::fill_result(const Request& r, Result* out) const {
  char* base = reinterpret_cast<char*>(base_);
  out->n = r.n;
  out->keys = (r.batch && r.n) ? base + r.batch->out_off + 8 * r.out_pos : nullptr;
  out->idx = (r.batch && r.n && r.batch->has_idx)
                 ? reinterpret_cast<uint32_t*>(base + r.batch->idx_off) + r.out_pos
                 : nullptr;
  out->latency_ns = r.t_done - r.t_submit;
  out->queue_ns = r.t_start - r.t_submit;
  out->status = r.status;
  out->batch_requests = r.batch_requests;
}

int Server::poll(uint64_t ticket, Result* out) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = reqs_.find(ticket);
  if (it == reqs_.end() || it->second->released) return S_UNKNOWN_TICKET;
  if (!it->second->done) return S_PENDING;
  if (out) fill_result(*it->second, out);
  return S_OK;
}

int Server::wait(uint64_t ticket, uint32_t timeout_ms, Result* out) {
  std::unique_lock<std::mutex> lk(mu_);
  // a system_clock deadline waits through pthread_cond_timedwait, which thread
  // sanitizers understand (the steady_clock form uses pthread_cond_clockwait)
  const auto until = std::chrono::system_clock::now() + std::chrono::milliseconds(timeout_ms);
  for (;;) {
    auto it = reqs_.find(ticket);
    if (it == reqs_.end() || it->second->released) return S_UNKNOWN_TICKET;
    if (it->second->done) {
      if (out) fill_result(*it->second, out);
      return S_OK;
    }
    if (cv_done_.wait_until(lk, until) == std::cv_status::timeout) {
      auto jt = reqs_.find(ticket);
      if (jt != reqs_.end() && jt->second->done && !jt->second->released) {
        if (out) fill_result(*jt->second, out);
        return S_OK;
      }
      return jt == reqs_.end() ? S_UNKNOWN_TICKET : S_PENDING;
    }
  }
}

int Server::release(uint64_t ticket) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = reqs_.find(ticket);
  if (it == reqs_.end() || it->second->released) return S_UNKNOWN_TICKET;
  Request* r = it->second.get();
  r->released = true;
  ++st_.released;
  if (!r->done) {
    // still queued: drop it now; running: dropped when its batch completes
    auto q = std::find(queue_.begin(), queue_.end(), r);
    if (q != queue_.end()) {
      queue_.erase(q);
      r->batch = nullptr;
      drop_request(r);
    }
    return S_OK;
  }
  drop_request(r);
  return S_OK;
}

Stats Server::stats() {
  std::lock_guard<std::mutex> g(mu_);
  Stats s = st_;
  s.in_use = arena_.in_use();
  s.high_water = arena_.high_water();
  s.queued = queue_.size();
  return s;
}

void Server::stop() {
  {
    std::lock_guard<std::mutex> g(mu_);
    if (stopping_ && workers_.empty()) return;
    stopping_ = true;
    // queued requests never run
    for (Request* r : queue_) {
      r->status = S_SHUTDOWN;
      r->done = true;
      r->t_start = r->t_done = now_ns();
    }
    queue_.clear();
    cv_work_.notify_all();
    cv_done_.notify_all();
  }
  for (auto& t : workers_) t.join();  // a running batch finishes first
  workers_.clear();
  if (started_) ex_->shutdown();
  started_ = false;
}

}  // namespace pcfserve
