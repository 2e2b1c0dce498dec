// Host unit test of the server's scheduling core: batching policy, admission
// by budget, rejection, and nearest-rank percentiles.  Built with g++ by
// tests/test_serve_core_cpu.py; exits nonzero on the first failed check.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "../../paper_2606_21791_amd/csrc/serve_core.h"

using namespace sgserve;

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                \
    }                                                              \
  } while (0)

static Request req(uint64_t t, int kind, int view, int nv, int64_t arr, size_t bytes) {
  Request r;
  r.ticket = t; r.kind = kind; r.view = view; r.n_variants = nv; r.arrival_ns = arr; r.bytes = bytes;
  return r;
}

int main() {
  // continuous batching: campaigns on the same view merge up to max_batch, in order
  {
    Scheduler s(0, 0, 64, 100);
    CHECK(s.submit(req(1, kCampaign, 0, 32, 10, 1)) == 0);
    CHECK(s.submit(req(2, kGuardedRender, 0, 1, 11, 1)) == 0);
    CHECK(s.submit(req(3, kCampaign, 1, 32, 12, 1)) == 0);
    CHECK(s.submit(req(4, kCampaign, 0, 32, 13, 1)) == 0);
    CHECK(s.submit(req(5, kCampaign, 0, 32, 14, 1)) == 0);
    Batch b;
    CHECK(s.next(&b));
    CHECK(b.view == 0 && b.kind == kCampaign && b.reqs.size() == 2 && b.reqs[0].ticket == 1 && b.reqs[1].ticket == 4);
    CHECK(b.n_variants == 64);
    Batch c;
    CHECK(s.next(&c));
    CHECK(c.kind == kGuardedRender && c.reqs.size() == 1 && c.reqs[0].ticket == 2);   // never merged
    Batch d;
    CHECK(s.next(&d));
    CHECK(d.view == 1 && d.reqs.size() == 1);
    Batch e;
    CHECK(s.next(&e));
    CHECK(e.reqs.size() == 1 && e.reqs[0].ticket == 5);
    Batch f;
    CHECK(!s.next(&f));
    s.finish(b, 1010);
    s.finish(c, 2011);
    Percentiles p = s.latency(kCampaign);
    CHECK(p.n == 2 && p.p50 == 0.997 && p.p99 == 1.0);
  }
  // admission: a request that cannot fit even on an idle device is rejected at submit;
  // one that fits waits while running work holds memory
  {
    Scheduler s(1000, 600, 64, 100);
    CHECK(s.submit(req(1, kGuardedRender, 0, 1, 0, 500)) == -2);
    CHECK(s.submit(req(2, kGuardedRender, 0, 1, 0, 300)) == 0);
    CHECK(s.submit(req(3, kGuardedRender, 0, 1, 0, 300)) == 0);
    Batch a, b;
    CHECK(s.next(&a) && a.reqs[0].ticket == 2);
    CHECK(!s.next(&b));                      // 600 + 300 + 300 > 1000: waits
    s.finish(a, 10);
    CHECK(s.next(&b) && b.reqs[0].ticket == 3);
    Scheduler::Counters k = s.counters();
    CHECK(k.rejected == 1 && k.submitted == 2);
  }
  // merging respects the budget too
  {
    Scheduler s(1000, 0, 64, 100);
    CHECK(s.submit(req(1, kCampaign, 0, 8, 0, 400)) == 0);
    CHECK(s.submit(req(2, kCampaign, 0, 8, 0, 400)) == 0);
    CHECK(s.submit(req(3, kCampaign, 0, 8, 0, 400)) == 0);
    Batch a;
    CHECK(s.next(&a) && a.reqs.size() == 2 && a.bytes == 800);
  }
  // queue depth
  {
    Scheduler s(0, 0, 64, 2);
    CHECK(s.submit(req(1, kCampaign, 0, 1, 0, 0)) == 0);
    CHECK(s.submit(req(2, kCampaign, 0, 1, 0, 0)) == 0);
    CHECK(s.submit(req(3, kCampaign, 0, 1, 0, 0)) == -1);
  }
  // no merging in the reference FIFO mode
  {
    Scheduler s(0, 0, 64, 100, false);
    CHECK(s.submit(req(1, kCampaign, 0, 4, 0, 0)) == 0);
    CHECK(s.submit(req(2, kCampaign, 0, 4, 0, 0)) == 0);
    Batch a;
    CHECK(s.next(&a) && a.reqs.size() == 1);
  }
  // nearest-rank percentiles
  {
    std::vector<double> v;
    for (int i = 1; i <= 100; ++i) v.push_back((double)i);
    CHECK(percentile(v, 0.5) == 50.0 && percentile(v, 0.99) == 99.0 && percentile(v, 1.0) == 100.0);
  }
  // concurrent use, as by the server: producer threads submit while worker
  // threads take launches and finish them; every accepted request completes
  // exactly once and the memory held by running work returns to zero
  {
    constexpr int kProducers = 4, kWorkers = 4, kPerProducer = 3000;
    Scheduler s(1 << 20, 1 << 18, 64, 1 << 20);
    std::atomic<int> accepted{0}, refused{0}, done_reqs{0}, producers_left{kProducers};
    std::vector<std::thread> th;
    for (int p = 0; p < kProducers; ++p)
      th.emplace_back([&, p] {
        for (int i = 0; i < kPerProducer; ++i) {
          const uint64_t t = (uint64_t)p * kPerProducer + (uint64_t)i + 1;
          const size_t bytes = (t % 7 == 0) ? (size_t)1 << 20 : (size_t)(t % 5 + 1) << 12;   // 1 in 7 never fits
          const int rc = s.submit(req(t, (int)(t % 3 == 0), (int)(t % 4), 1 + (int)(t % 16), (int64_t)t, bytes));
          (rc == 0 ? accepted : refused).fetch_add(1);
        }
        producers_left.fetch_sub(1);
      });
    for (int w = 0; w < kWorkers; ++w)
      th.emplace_back([&] {
        for (;;) {
          Batch b;
          if (s.next(&b)) {
            if (!b.rejected) {
              CHECK(b.n_variants <= 64 || b.reqs.size() == 1);
              done_reqs.fetch_add((int)b.reqs.size());
            }
            s.finish(b, (int64_t)1 << 40);
          } else if (producers_left.load() == 0 && s.pending() == 0) {
            return;
          } else {
            std::this_thread::yield();
          }
        }
      });
    for (std::thread& t : th) t.join();
    Scheduler::Counters k = s.counters();
    CHECK(accepted.load() + refused.load() == kProducers * kPerProducer);
    CHECK((int)k.submitted == accepted.load() && (int)k.completed == done_reqs.load());
    CHECK(k.completed + (k.rejected - (uint64_t)refused.load()) == k.submitted);
    CHECK(s.running_bytes() == 0 && s.pending() == 0);
    CHECK(s.latency(kCampaign).n + s.latency(kGuardedRender).n == k.completed);
  }
  std::printf("serve core ok\n");
  return 0;
}
