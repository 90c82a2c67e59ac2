// Multi-threaded stress of the serving scheduler over the mock executor.
// Built with -fsanitize=thread by the CPU tests: client threads submit, poll,
// wait and release concurrently with the workers; every result must be
// sorted, and every byte of the budget must be returned at the end.
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <random>
#include <thread>
#include <vector>

#include "pcf_serve_core.h"

extern "C" {
void* mock_create(uint64_t budget, uint32_t slots, uint32_t maxreq, uint64_t maxkeys,
                  uint32_t delay_us);
void mock_destroy(void* s);
}

using namespace pcfserve;

int main(int argc, char** argv) {
  const int clients = argc > 1 ? atoi(argv[1]) : 4;
  const int per_client = argc > 2 ? atoi(argv[2]) : 200;
  Server* s = static_cast<Server*>(mock_create(4 << 20, 3, 16, 1 << 16, 50));
  if (!s) return 2;
  std::atomic<int> bad{0}, done{0};
  std::vector<std::thread> th;
  for (int c = 0; c < clients; ++c) {
    th.emplace_back([&, c] {
      std::mt19937_64 rng(1000 + c);
      std::vector<std::vector<uint64_t>> bufs(per_client);
      std::vector<uint64_t> tickets;
      for (int i = 0; i < per_client; ++i) {
        const uint64_t n = rng() % 5000;
        bufs[i].resize(n);
        for (auto& x : bufs[i]) x = rng() >> (rng() % 60);
        uint64_t t = 0;
        int rc = s->submit(1, n ? bufs[i].data() : nullptr, n, (int)(rng() & 1), &t);
        if (rc != S_OK) {
          ++bad;
          continue;
        }
        tickets.push_back(t);
        if (rng() % 4 == 0) {  // sometimes release before completion
          s->release(t);
          tickets.back() = 0;
        }
      }
      for (uint64_t t : tickets) {
        if (!t) continue;
        Result r;
        if (s->wait(t, 60000, &r) != S_OK || r.status != S_OK) {
          ++bad;
          continue;
        }
        const uint64_t* k = static_cast<const uint64_t*>(r.keys);
        for (uint64_t i = 1; i < r.n; ++i)
          if (k[i - 1] > k[i]) {
            ++bad;
            break;
          }
        if (s->release(t) != S_OK) ++bad;
        ++done;
      }
    });
  }
  for (auto& t : th) t.join();
  const Stats st = s->stats();
  printf("done=%d bad=%d batches=%llu in_use=%llu high=%llu budget=%llu\n", done.load(), bad.load(),
         (unsigned long long)st.batches, (unsigned long long)st.in_use,
         (unsigned long long)st.high_water, (unsigned long long)st.budget);
  const bool ok = bad == 0 && st.in_use == 0 && st.high_water <= st.budget && st.queued == 0;
  mock_destroy(s);
  return ok ? 0 : 1;
}
