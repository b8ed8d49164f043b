// Serving: continuous batching of scan requests against resident two-class
// models (the classifier of section 4 behind a request queue).
//
// One host thread replays the trace in real time and runs the scheduler:
//   - requests become visible at their arrival time and queue in arrival
//     order;
//   - while a stream slot is free, the queue's head requests are admitted as
//     long as their device footprint fits the arena (first-fit allocator
//     with coalescing; no overtaking, so no request starves) and form one
//     batch of at most max_batch_requests;
//   - a batch is enqueued on its slot's stream: inputs host->device (unless
//     device resident), then per (feature count, kind) one grouped launch
//     (the persistent kernel of nb_score_groups, each request one group),
//     then outputs device->host, then an event;
//   - completed batches (event query) stamp their requests' completion time
//     and free their arena space.
// Batches in flight overlap one another's copies and kernels (one stream
// per slot, all at the default priority).  The work list of a grouped launch
// lives in the arena with the batch.  In simulation mode the same scheduler
// runs with a modelled completion time per batch and no device calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "nb_internal.hpp"

namespace nb {
namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) with coalescing of freed ranges.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) {
    if (size_) free_[0] = size_;
  }
  // offset of a range of `bytes` (a multiple of kAlign), or SIZE_MAX
  size_t alloc(size_t bytes) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return off;
      }
    }
    return SIZE_MAX;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t peak() const { return peak_; }

 private:
  size_t size_, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

struct Range {
  size_t off = 0, bytes = 0;
};

struct Batch {
  std::vector<int64_t> reqs;
  std::vector<Range> ranges;                 // arena ranges to free on completion (one per request)
  Range wl;                                  // the batch's work-list space (also in ranges)
  std::vector<std::vector<uint8_t>> blobs;   // host images of the work lists (kept until done)
  double sim_done = 0.0;                     // simulation: completion time
  bool busy = false;
};

struct ReqPlan {
  size_t x_bytes = 0, lab_bytes = 0, lp_bytes = 0;
  size_t wl_bytes = 0;       // this request's share of its batch's work-list space
  size_t total() const { return x_bytes + lab_bytes + lp_bytes; }
};

// Upper bound of the work-list bytes one request adds to a grouped launch:
// its descriptor, its items (a tile holds >= 4 blocks of >= 8 files, so at
// most n/32 + 2 items) and, should it open a launch of its own, that
// launch's counters and alignment padding.
size_t work_list_bound(int64_t n) {
  return kGroupDescBound + 16 * (size_t)(n / 32 + 2) + 4 * kAlign;
}

double quantile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - (double)i;
  return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

class Server {
 public:
  Server(const nb_model* models, int32_t n_models, nb_request* reqs, int64_t n, const nb_serve_cfg& cfg)
      : models_(models), n_models_(n_models), reqs_(reqs), n_(n), cfg_(cfg), arena_(cfg.arena_bytes),
        sim_((cfg.flags & NB_SERVE_SIMULATE) != 0), dev_in_((cfg.flags & NB_SERVE_DEVICE_INPUTS) != 0) {}

  int validate() {
    if (cfg_.max_batch_requests < 1) return fail(NB_EINVAL, "max_batch_requests must be >= 1");
    if (cfg_.n_streams < 1 || cfg_.n_streams > 16) return fail(NB_EINVAL, "n_streams must be in [1, 16]");
    if (cfg_.reserved != 0) return fail(NB_EINVAL, "nb_serve_cfg.reserved must be 0");
    if (cfg_.flags & ~(NB_SERVE_DEVICE_INPUTS | NB_SERVE_SIMULATE)) return fail(NB_EINVAL, "unknown serve flags");
    if (elem_bytes(cfg_.xtype) == 0) return fail(NB_EINVAL, "unknown feature type");
    if (cfg_.wtype != NB_W_F32 && cfg_.wtype != NB_W_BF16) return fail(NB_EINVAL, "unknown table type");
    if (!sim_ && (!cfg_.arena || (reinterpret_cast<uintptr_t>(cfg_.arena) & (kAlign - 1))))
      return fail(NB_EINVAL, "arena must be a 256-byte aligned device pointer");
    if (sim_ && !(cfg_.sim_bytes_per_s > 0.0 && cfg_.sim_batch_s >= 0.0))
      return fail(NB_EINVAL, "simulation needs sim_bytes_per_s > 0 and sim_batch_s >= 0");
    if (!models_ || n_models_ < 1) return fail(NB_EINVAL, "models: need at least one");
    for (int32_t m = 0; m < n_models_; ++m) {
      const nb_model& M = models_[m];
      if (M.n_classes != 2) return fail(NB_EINVAL, "serving takes two-class models");
      if (!sim_) {
        nb_layout L;
        if (int rc = check_model(&M, &L)) return rc;
      } else if (M.n_features < 1 || M.n_features > kMaxFeatures) {
        return fail(NB_EINVAL, "model feature count out of range");
      }
    }
    if (!reqs_ || n_ < 0) return fail(NB_EINVAL, "requests: NULL or negative count");
    const int eb = elem_bytes(cfg_.xtype);
    plan_.resize(n_);
    for (int64_t i = 0; i < n_; ++i) {
      nb_request& r = reqs_[i];
      const std::string at = "request " + std::to_string(i) + ": ";
      if (r.model < 0 || r.model >= n_models_) return fail(NB_EINVAL, at + "model index out of range");
      if (r.n < 1) return fail(NB_EINVAL, at + "n must be >= 1");
      if (!r.x && !sim_) return fail(NB_EINVAL, at + "x is NULL");
      if (!r.labels_host && !r.log_post_host) return fail(NB_EINVAL, at + "no output requested");
      if (!(r.arrival_s >= 0.0) || !std::isfinite(r.arrival_s)) return fail(NB_EINVAL, at + "arrival_s must be >= 0");
      const int F = models_[r.model].n_features;
      if (((int64_t)F * eb) % 4 != 0) return fail(NB_EINVAL, at + "row bytes must be a multiple of 4");
      ReqPlan& p = plan_[i];
      p.x_bytes = dev_in_ ? 0 : align_up((size_t)r.n * F * eb, kAlign);
      p.lab_bytes = r.labels_host ? align_up((size_t)r.n * 4, kAlign) : 0;
      p.lp_bytes = r.log_post_host ? align_up((size_t)r.n * 8, kAlign) : 0;
      p.wl_bytes = work_list_bound(r.n);
      r.status = NB_OK;
      r.done_s = -1.0;
    }
    order_.resize(n_);
    for (int64_t i = 0; i < n_; ++i) order_[i] = i;
    std::stable_sort(order_.begin(), order_.end(),
                     [&](int64_t a, int64_t b) { return reqs_[a].arrival_s < reqs_[b].arrival_s; });
    return NB_OK;
  }

  int run(nb_serve_stats* st) {
    int rc = NB_OK;
    slots_.resize(cfg_.n_streams);
    if (!sim_) {
      streams_.assign(cfg_.n_streams, nullptr);
      events_.assign(cfg_.n_streams, nullptr);
      for (int s = 0; s < cfg_.n_streams && !rc; ++s) {
        if (hipStreamCreateWithFlags(&streams_[s], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&events_[s], hipEventDisableTiming) != hipSuccess)
          rc = fail(NB_EHIP, "stream/event creation failed");
      }
    }
    if (!rc) rc = loop();
    if (!sim_) {
      // drain and release; a failure here is reported unless an earlier
      // error already is
      for (auto s : streams_)
        if (s && hipStreamSynchronize(s) != hipSuccess && !rc) rc = fail(NB_EHIP, "hipStreamSynchronize");
      for (auto e : events_)
        if (e) (void)hipEventDestroy(e);
      for (auto s : streams_)
        if (s) (void)hipStreamDestroy(s);
    }
    if (rc) return rc;
    fill_stats(st);
    return NB_OK;
  }

 private:
  bool fits_alone(int64_t i) const {
    return plan_[i].total() + align_up(plan_[i].wl_bytes, kAlign) <= cfg_.arena_bytes;
  }

  double now() const {
    if (sim_) return sim_now_;
    return std::chrono::duration<double>(Clock::now() - t0_).count();
  }

  int loop() {
    t0_ = Clock::now();
    size_t next = 0;                 // next request (arrival order) not yet queued
    std::deque<int64_t> queue;
    int64_t finished = 0;
    int in_flight = 0;
    while (finished < n_) {
      // arrivals
      const double t = now();
      while (next < order_.size() && reqs_[order_[next]].arrival_s <= t) queue.push_back(order_[next++]);
      // completions
      for (int s = 0; s < (int)slots_.size(); ++s) {
        Batch& b = slots_[s];
        if (!b.busy) continue;
        bool done;
        if (sim_) {
          done = b.sim_done <= t;
        } else {
          const hipError_t q = hipEventQuery(events_[s]);
          if (q != hipSuccess && q != hipErrorNotReady) return hip_fail(q, "batch completion");
          done = q == hipSuccess;
        }
        if (!done) continue;
        for (int64_t i : b.reqs) reqs_[i].done_s = sim_ ? b.sim_done : t;
        for (const Range& r : b.ranges) arena_.release(r.off, r.bytes);
        finished += (int64_t)b.reqs.size();
        served_ += (int64_t)b.reqs.size();
        b = Batch();
        --in_flight;
      }
      // rejections: a request that can never fit, even alone in an empty arena
      while (!queue.empty() && !fits_alone(queue.front())) {
        nb_request& r = reqs_[queue.front()];
        r.status = NB_EREJECTED;
        r.done_s = t;
        ++rejected_;
        ++finished;
        queue.pop_front();
      }
      // admission into free slots
      bool issued = false;
      for (int s = 0; s < (int)slots_.size() && !queue.empty(); ++s) {
        if (slots_[s].busy) continue;
        Batch b;
        while (!queue.empty() && (int)b.reqs.size() < cfg_.max_batch_requests) {
          const int64_t i = queue.front();
          if (!fits_alone(i)) break;                             // rejected next iteration
          const size_t off = plan_[i].total() ? arena_.alloc(plan_[i].total()) : 0;
          if (off == SIZE_MAX) break;                            // wait for space: no overtaking
          b.ranges.push_back(Range{off, plan_[i].total()});
          b.reqs.push_back(i);
          queue.pop_front();
        }
        // the batch's work lists: one range; give back the last requests
        // until it fits (the head alone always fits an empty arena)
        while (!b.reqs.empty()) {
          size_t wl = 0;
          for (int64_t i : b.reqs) wl += plan_[i].wl_bytes;
          wl = align_up(wl, kAlign);
          const size_t off = arena_.alloc(wl);
          if (off != SIZE_MAX) {
            b.wl = Range{off, wl};
            break;
          }
          const Range last = b.ranges.back();
          if (last.bytes) arena_.release(last.off, last.bytes);
          b.ranges.pop_back();
          queue.push_front(b.reqs.back());
          b.reqs.pop_back();
        }
        if (b.reqs.empty()) break;
        b.ranges.push_back(b.wl);
        int rc = issue(s, b, t);
        if (rc) return rc;
        slots_[s] = std::move(b);
        slots_[s].busy = true;
        ++batches_;
        ++in_flight;
        max_in_flight_ = std::max(max_in_flight_, in_flight);
        issued = true;
      }
      if (finished >= n_) break;
      if (sim_) {
        // advance the modelled clock to the next event
        double tn = 1e300;
        if (next < order_.size()) tn = std::min(tn, reqs_[order_[next]].arrival_s);
        for (const Batch& b : slots_)
          if (b.busy) tn = std::min(tn, b.sim_done);
        if (!issued) {
          if (tn >= 1e300) return fail(NB_EINVAL, "scheduler stalled (arena smaller than the head request?)");
          sim_now_ = std::max(sim_now_, tn);
        }
      } else if (!issued) {
        std::this_thread::yield();
      }
    }
    return NB_OK;
  }

  // Device offsets of request i's buffers inside its arena range.
  struct Bufs {
    uint8_t* x;
    int32_t* lab;
    float* lp;
  };

  int issue(int s, Batch& b, double t) {
    const int eb = elem_bytes(cfg_.xtype);
    if (sim_) {
      double bytes = 0.0;
      for (int64_t i : b.reqs) bytes += (double)reqs_[i].n * models_[reqs_[i].model].n_features * eb;
      b.sim_done = t + cfg_.sim_batch_s + bytes / cfg_.sim_bytes_per_s;
      return NB_OK;
    }
    hipStream_t st = streams_[s];
    uint8_t* base = static_cast<uint8_t*>(cfg_.arena);
    std::vector<Bufs> bufs(b.reqs.size());
    for (size_t k = 0; k < b.reqs.size(); ++k) {
      const int64_t i = b.reqs[k];
      const ReqPlan& p = plan_[i];
      uint8_t* at = base + b.ranges[k].off;
      const nb_request& r = reqs_[i];
      Bufs& q = bufs[k];
      q.x = dev_in_ ? static_cast<uint8_t*>(const_cast<void*>(r.x)) : at;
      q.lab = r.labels_host ? reinterpret_cast<int32_t*>(at + p.x_bytes) : nullptr;
      q.lp = r.log_post_host ? reinterpret_cast<float*>(at + p.x_bytes + p.lab_bytes) : nullptr;
      if (!dev_in_) {
        const size_t nb = (size_t)r.n * models_[r.model].n_features * eb;
        NB_HIP_CHECK(hipMemcpyAsync(q.x, r.x, nb, hipMemcpyHostToDevice, st));
      }
    }
    // one grouped launch per (feature count, kind)
    size_t wl_used = 0;
    std::map<std::pair<int, int>, std::vector<size_t>> shapes;
    for (size_t k = 0; k < b.reqs.size(); ++k) {
      const nb_model& M = models_[reqs_[b.reqs[k]].model];
      shapes[{M.n_features, M.kind}].push_back(k);
    }
    for (auto& kv : shapes) {
      std::vector<nb_group> groups;
      for (size_t k : kv.second) {
        const nb_request& r = reqs_[b.reqs[k]];
        nb_group g{};
        g.model = r.model;
        g.x = bufs[k].x;
        g.n = r.n;
        g.ld = models_[r.model].n_features;
        g.labels = bufs[k].lab;
        g.log_post = bufs[k].lp;
        groups.push_back(g);
      }
      std::vector<uint8_t> blob;
      GroupLaunch L;
      int rc = prepare_group_launch(models_, n_models_, groups.data(), (int32_t)groups.size(), cfg_.xtype,
                                    cfg_.wtype, 0, &blob, &L);
      if (rc) return rc;
      const size_t off = b.wl.off + wl_used;
      wl_used += align_up(blob.size(), kAlign);
      if (wl_used > b.wl.bytes) return fail(NB_EHIP, "internal: work list exceeds its bound");
      NB_HIP_CHECK(hipMemcpyAsync(base + off, blob.data(), blob.size(), hipMemcpyHostToDevice, st));
      if ((rc = enqueue_group_launch(L, base + off, st))) return rc;
      b.blobs.push_back(std::move(blob));
    }
    for (size_t k = 0; k < b.reqs.size(); ++k) {
      const nb_request& r = reqs_[b.reqs[k]];
      if (r.labels_host)
        NB_HIP_CHECK(hipMemcpyAsync(r.labels_host, bufs[k].lab, (size_t)r.n * 4, hipMemcpyDeviceToHost, st));
      if (r.log_post_host)
        NB_HIP_CHECK(hipMemcpyAsync(r.log_post_host, bufs[k].lp, (size_t)r.n * 8, hipMemcpyDeviceToHost, st));
    }
    NB_HIP_CHECK(hipEventRecord(events_[s], st));
    return NB_OK;
  }

  void fill_stats(nb_serve_stats* st) {
    std::vector<double> lat;
    double first = 1e300, last = 0.0, files = 0.0, bytes = 0.0;
    const int eb = elem_bytes(cfg_.xtype);
    for (int64_t i = 0; i < n_; ++i) {
      const nb_request& r = reqs_[i];
      first = std::min(first, r.arrival_s);
      if (r.status != NB_OK) continue;
      lat.push_back(r.done_s - r.arrival_s);
      last = std::max(last, r.done_s);
      files += (double)r.n;
      bytes += (double)r.n * models_[r.model].n_features * eb;
    }
    std::memset(st, 0, sizeof(*st));
    st->p50_s = quantile(lat, 0.50);
    st->p99_s = quantile(lat, 0.99);
    double sum = 0.0, mx = 0.0;
    for (double v : lat) {
      sum += v;
      mx = std::max(mx, v);
    }
    st->mean_s = lat.empty() ? 0.0 : sum / (double)lat.size();
    st->max_s = mx;
    st->makespan_s = lat.empty() ? 0.0 : last - first;
    st->files_per_s = st->makespan_s > 0 ? files / st->makespan_s : 0.0;
    st->bytes_per_s = st->makespan_s > 0 ? bytes / st->makespan_s : 0.0;
    st->served = served_;
    st->rejected = rejected_;
    st->batches = batches_;
    st->peak_arena_bytes = (int64_t)arena_.peak();
    st->max_in_flight = max_in_flight_;
  }

  const nb_model* models_;
  int32_t n_models_;
  nb_request* reqs_;
  int64_t n_;
  nb_serve_cfg cfg_;
  Arena arena_;
  bool sim_, dev_in_;
  double sim_now_ = 0.0;
  Clock::time_point t0_;
  std::vector<ReqPlan> plan_;
  std::vector<int64_t> order_;
  std::vector<Batch> slots_;
  std::vector<hipStream_t> streams_;
  std::vector<hipEvent_t> events_;
  int64_t served_ = 0, rejected_ = 0, batches_ = 0;
  int max_in_flight_ = 0;
};

}  // namespace
}  // namespace nb

extern "C" int nb_serve(const nb_model* models, int32_t n_models, nb_request* requests, int64_t n_requests,
                        const nb_serve_cfg* cfg, nb_serve_stats* stats) {
  if (!cfg || !stats) return nb::fail(NB_EINVAL, "cfg and stats must not be NULL");
  nb::Server srv(models, n_models, requests, n_requests, *cfg);
  int rc = srv.validate();
  if (rc) return rc;
  return srv.run(stats);
}
