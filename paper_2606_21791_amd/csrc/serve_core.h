// Scheduling core of the libsg server, free of any device API so that it can
// be unit-tested on the host: the pending-request queue, the batching policy
// (continuous batching of injection campaigns per resident view), admission by
// a device-memory budget, and latency statistics.
//
// Requests are admitted in arrival order.  A worker that becomes free takes
// the oldest pending request; if it is a campaign, every other pending
// campaign on the same view is merged into the same launch while the launch
// stays within max_batch variants.  A request whose device bytes would push
// the total above the budget waits until running work releases memory, and
// is rejected outright if it could not fit even on an idle device.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <deque>
#include <mutex>
#include <vector>

namespace sgserve {

enum Kind { kCampaign = 0, kGuardedRender = 1 };

struct Request {
  uint64_t ticket = 0;
  int kind = kCampaign;
  int view = 0;
  int n_variants = 1;          // variants the request adds to a launch
  int64_t arrival_ns = 0;
  size_t bytes = 0;            // device bytes the request needs while it runs
};

struct Batch {
  int view = -1;
  int kind = kCampaign;
  bool rejected = false;       // the request can no longer fit the budget
  std::vector<Request> reqs;
  int n_variants = 0;
  size_t bytes = 0;
};

struct Percentiles {
  double p50 = 0.0, p99 = 0.0, mean = 0.0;
  uint64_t n = 0;
};

// Nearest-rank percentile of a sample (sorted copy).
inline double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  size_t k = (size_t)std::ceil(q * (double)v.size());
  if (k == 0) k = 1;
  return v[std::min(k, v.size()) - 1];
}

class Scheduler {
 public:
  Scheduler(size_t budget_bytes, size_t resident_bytes, int max_batch, int queue_depth, bool merge = true)
      : budget_(budget_bytes), resident_(resident_bytes), max_batch_(max_batch), queue_depth_(queue_depth),
        merge_(merge) {}

  // Queue a request.  Returns 0, -1 (queue full) or -2 (can never fit the budget).
  int submit(const Request& r) {
    std::lock_guard<std::mutex> g(mu_);
    if (budget_ && resident_ + r.bytes > budget_) { ++rejected_; return -2; }
    if ((int)pending_.size() >= queue_depth_) { ++rejected_; return -1; }
    pending_.push_back(r);
    ++submitted_;
    return 0;
  }

  // Take the next launch for a free worker: the oldest pending request that
  // fits the remaining budget, merged with later campaigns on the same view.
  bool next(Batch* b) {
    std::lock_guard<std::mutex> g(mu_);
    for (size_t i = 0; i < pending_.size(); ++i) {
      const Request& r = pending_[i];
      if (budget_ && resident_ + running_bytes_ + r.bytes > budget_) {
        if (running_bytes_ == 0) {           // resident state grew after submit: it can never fit
          b->view = r.view;
          b->kind = r.kind;
          b->rejected = true;
          b->reqs.assign(1, r);
          b->n_variants = 0;
          b->bytes = 0;
          pending_.erase(pending_.begin() + (long)i);
          ++rejected_;
          return true;
        }
        return false;                        // wait for memory, in arrival order
      }
      b->rejected = false;
      b->view = r.view;
      b->kind = r.kind;
      b->reqs.assign(1, r);
      b->n_variants = r.n_variants;
      b->bytes = r.bytes;
      pending_.erase(pending_.begin() + (long)i);
      if (b->kind == kCampaign && merge_) {
        for (size_t j = 0; j < pending_.size();) {
          const Request& q = pending_[j];
          const bool fits = b->n_variants + q.n_variants <= max_batch_ &&
                            (!budget_ || resident_ + running_bytes_ + b->bytes + q.bytes <= budget_);
          if (q.kind == kCampaign && q.view == b->view && fits) {
            b->reqs.push_back(q);
            b->n_variants += q.n_variants;
            b->bytes += q.bytes;
            pending_.erase(pending_.begin() + (long)j);
          } else {
            ++j;
          }
        }
      }
      running_bytes_ += b->bytes;
      ++launches_;
      variants_launched_ += (uint64_t)b->n_variants;
      return true;
    }
    return false;
  }

  // A launch finished: release its memory and record each request's latency.
  void finish(const Batch& b, int64_t done_ns) {
    std::lock_guard<std::mutex> g(mu_);
    running_bytes_ -= b.bytes;
    if (b.rejected) return;
    for (const Request& r : b.reqs) {
      lat_us_[r.kind].push_back((double)(done_ns - r.arrival_ns) / 1e3);
      ++completed_;
      variants_done_ += (uint64_t)r.n_variants;
    }
    if (first_arrival_ns_ == 0 || (b.reqs.size() && b.reqs[0].arrival_ns < first_arrival_ns_))
      first_arrival_ns_ = b.reqs.empty() ? first_arrival_ns_ : b.reqs[0].arrival_ns;
    last_done_ns_ = std::max(last_done_ns_, done_ns);
  }

  void add_resident(size_t bytes) {
    std::lock_guard<std::mutex> g(mu_);
    resident_ += bytes;
  }

  size_t pending() {
    std::lock_guard<std::mutex> g(mu_);
    return pending_.size();
  }
  size_t running_bytes() {
    std::lock_guard<std::mutex> g(mu_);
    return running_bytes_;
  }
  size_t resident_bytes() {
    std::lock_guard<std::mutex> g(mu_);
    return resident_;
  }

  Percentiles latency(int kind) {
    std::lock_guard<std::mutex> g(mu_);
    Percentiles p;
    const std::vector<double>& v = lat_us_[kind];
    p.n = v.size();
    if (v.empty()) return p;
    p.p50 = percentile(v, 0.50);
    p.p99 = percentile(v, 0.99);
    double s = 0.0;
    for (double x : v) s += x;
    p.mean = s / (double)v.size();
    return p;
  }

  struct Counters {
    uint64_t submitted, completed, rejected, launches, variants_launched, variants_done;
    int64_t first_arrival_ns, last_done_ns;
  };
  Counters counters() {
    std::lock_guard<std::mutex> g(mu_);
    return {submitted_, completed_, rejected_, launches_, variants_launched_, variants_done_, first_arrival_ns_,
            last_done_ns_};
  }

 private:
  std::mutex mu_;
  std::deque<Request> pending_;
  size_t budget_, resident_, running_bytes_ = 0;
  int max_batch_, queue_depth_;
  bool merge_;
  std::vector<double> lat_us_[2];
  uint64_t submitted_ = 0, completed_ = 0, rejected_ = 0, launches_ = 0, variants_launched_ = 0, variants_done_ = 0;
  int64_t first_arrival_ns_ = 0, last_done_ns_ = 0;
};

}  // namespace sgserve
