// Continuous-batching personalised PageRank server.
//
// Requests (a seed set, d, tol) are queued per graph.  Every graph has an
// engine thread and a HIP stream of its own; the thread repeats one engine
// step: admit queued requests into free slots of the graph's slot pool
// (device state sized from the HBM budget), run a few D-iteration rounds for
// every active slot (slots admitted at different times sit at different rounds
// of their own solves and share each launch), detect the slots whose solve
// stopped, flush them, take their top-k on the device and complete the
// requests.  Work of requests that arrive while others run overlaps with
// theirs from the next step on, and the graphs' launches overlap on the
// device, so a small graph's requests never wait for a large graph's rounds.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

#include "internal.h"

namespace di {

namespace {

// Rounds an engine step launches before it reads the slots' control blocks:
// one host round trip per four rounds instead of per round; a request that
// stops inside a step waits at most three rounds (launches that return at
// once) for its result.
constexpr int kStepRounds = 4;

struct Request {
  uint64_t id = 0;
  int graph = 0;
  std::vector<int32_t> seeds;
  std::vector<double> w;
  double d = 0.85, tol = 1e-6;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int slot = -1;
  bool cancel = false;
  bool done = false;
  di_result res;
};

struct GraphEntry {
  Graph* g = nullptr;
  hipStream_t stream = nullptr;
  std::thread th;
  std::unique_ptr<SlotPool> pool;
  std::deque<Request*> queue;
  std::vector<Request*> slot_req;  // per slot: the request it runs (or NULL)
  std::vector<int> free_slots;
};

}  // namespace

struct Server {
  di_server_opts opts;
  di_tune tune;
  bool has_tune = false;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<GraphEntry> graphs;
  std::unordered_map<uint64_t, Request*> reqs;
  uint64_t next_id = 1;
  bool stop = false;
  bool started = false;  // engine threads run (no graphs may be added)
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  int64_t submitted = 0, admitted = 0, completed = 0, cancelled = 0;
  int64_t hbm_in_use = 0;
  std::vector<double> latencies;
  double t_first = -1, t_last = 0;
  std::string thread_error;
  bool log = false;  // DI_LOG=1: one line per engine step on stderr

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void loop(int gi);
};

// Engine thread of graph gi.
void Server::loop(int gi) {
  if (hipSetDevice(device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(mu);
    thread_error = "scheduler could not select the device";
    stop = true;
    cv_done.notify_all();
    return;
  }
  GraphEntry& ge = graphs[gi];
  int64_t step_no = 0;
  for (;;) {
    std::vector<SlotInit> inits;
    std::vector<int> active;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] {
        return stop || !ge.queue.empty() || (int)ge.free_slots.size() < ge.pool->capacity();
      });
      if (stop) return;
      const double t = now();
      // cancelled running requests release their slots
      for (int q = 0; q < (int)ge.slot_req.size(); ++q) {
        Request* r = ge.slot_req[q];
        if (r && r->cancel) {
          r->res.status = DI_ECANCELED;
          r->t_done = t;
          r->done = true;
          ++cancelled;
          ge.slot_req[q] = nullptr;
          ge.free_slots.push_back(q);
        }
      }
      // admission: FIFO into free slots
      while (!ge.queue.empty() && !ge.free_slots.empty()) {
        Request* r = ge.queue.front();
        ge.queue.pop_front();
        if (r->cancel) {
          r->res.status = DI_ECANCELED;
          r->t_done = t;
          r->done = true;
          ++cancelled;
          continue;
        }
        const int slot = ge.free_slots.back();
        ge.free_slots.pop_back();
        r->slot = slot;
        r->t_admit = t;
        ge.slot_req[slot] = r;
        ++admitted;
        SlotInit in;
        in.slot = slot;
        in.d = r->d;
        in.tol = r->tol;
        in.seeds = r->seeds;
        in.w = r->w;
        inits.push_back(std::move(in));
      }
      for (int q = 0; q < (int)ge.slot_req.size(); ++q)
        if (ge.slot_req[q]) active.push_back(q);
      cv_done.notify_all();
    }
    std::vector<SlotResult> results;
    if (log) {
      fprintf(stderr, "[di server] graph %d step %lld t=%.4f admit %zu active %zu\n", gi,
              (long long)step_no, now(), inits.size(), active.size());
      fflush(stderr);
    }
    ++step_no;
    di_status rc = guarded([&] {
      ge.pool->admit(inits, ge.stream);
      ge.pool->step(active, kStepRounds, ge.stream);
      if (!active.empty()) {
        const std::vector<int> fin = ge.pool->stopped(active, ge.stream);
        ge.pool->finish(fin, opts.topk, results, ge.stream);
      }
    });
    std::lock_guard<std::mutex> lk(mu);
    if (rc != DI_OK) {
      thread_error = last_error_ref();
      // fail every running request of this graph; its queue stays
      const double t = now();
      for (int q = 0; q < (int)ge.slot_req.size(); ++q)
        if (Request* r = ge.slot_req[q]) {
          r->res.status = DI_EDEVICE;
          r->t_done = t;
          r->done = true;
          ge.slot_req[q] = nullptr;
          ge.free_slots.push_back(q);
        }
      cv_done.notify_all();
      continue;
    }
    const double t = now();
    for (const SlotResult& sr : results) {
      Request* r = ge.slot_req[sr.slot];
      ge.slot_req[sr.slot] = nullptr;
      ge.free_slots.push_back(sr.slot);
      if (!r) continue;
      di_result& o = r->res;
      o.req_id = r->id;
      o.status = r->cancel ? DI_ECANCELED : sr.status;
      o.k = (int32_t)std::min<size_t>(sr.ids.size(), 1024);
      for (int k = 0; k < o.k; ++k) {
        o.top_ids[k] = sr.ids[k];
        o.top_x[k] = sr.x[k];
      }
      o.residual_l1 = sr.residual;
      o.err_bound_l1 = sr.bound;
      o.rounds = sr.rounds;
      o.edges_diffused = sr.edges;
      r->t_done = t;
      o.t_submit = r->t_submit;
      o.t_admit = r->t_admit;
      o.t_done = t;
      r->done = true;
      if (r->cancel) {
        ++cancelled;
      } else {
        ++completed;
        latencies.push_back(t - r->t_submit);
        t_last = std::max(t_last, t);
      }
    }
    cv_done.notify_all();
  }
}

}  // namespace di

struct di_server : di::Server {};

using namespace di;

namespace {

di_result finished_result(Request* r) {
  di_result out = r->res;
  out.req_id = r->id;
  out.t_submit = r->t_submit;
  out.t_admit = r->t_admit;
  out.t_done = r->t_done;
  return out;
}

}  // namespace

extern "C" {

di_status di_server_create(const di_server_opts* opts, di_server** out) {
  return guarded([&] {
    DI_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    auto* s = new di_server();
    try {
      if (opts) s->opts = *opts;
      else memset(&s->opts, 0, sizeof(s->opts));
      if (s->opts.hbm_budget_bytes <= 0) s->opts.hbm_budget_bytes = 32ll << 30;
      if (s->opts.max_slots <= 0) s->opts.max_slots = 256;
      if (s->opts.topk <= 0) s->opts.topk = 100;
      DI_REQUIRE(s->opts.topk <= 1024, "topk must be <= 1024");
      DI_REQUIRE(s->opts.precision == DI_FP32_FLUID || s->opts.precision == DI_FP64,
                 "unknown precision");
      if (s->opts.tune) {
        s->tune = *s->opts.tune;
        s->has_tune = true;
      }
      s->opts.tune = nullptr;
      DI_HIP(hipGetDevice(&s->device));
      const char* lg = getenv("DI_LOG");
      s->log = lg && lg[0] == '1';
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
  });
}

di_status di_server_add_graph(di_server* s, const di_graph* g, int32_t* graph_id) {
  return guarded([&] {
    DI_REQUIRE(s && g && graph_id, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    DI_REQUIRE(!s->started, "graphs must be added before the first submit");
    Graph* gg = const_cast<di_graph*>(g);
    // Slots per graph: an equal share of the budget among up to 4 graphs.
    const int64_t per = slot_bytes(gg, s->opts.precision);
    const int64_t share = s->opts.hbm_budget_bytes / 4;
    const int64_t left = s->opts.hbm_budget_bytes - s->hbm_in_use;
    int cap = (int)std::min<int64_t>(s->opts.max_slots, std::min(share, left) / per);
    if (cap < 1) {
      set_error("HBM budget too small for one request on this graph");
      throw Fail{DI_ENOMEM};
    }
    GraphEntry ge;
    ge.g = gg;
    ge.pool.reset(make_slot_pool(gg, s->opts.precision, cap, s->has_tune ? &s->tune : nullptr));
    DI_HIP(hipStreamCreateWithFlags(&ge.stream, hipStreamNonBlocking));
    ge.slot_req.assign(cap, nullptr);
    for (int q = cap - 1; q >= 0; --q) ge.free_slots.push_back(q);
    s->hbm_in_use += ge.pool->bytes();
    gg->servers += 1;
    s->graphs.push_back(std::move(ge));
    *graph_id = (int32_t)s->graphs.size() - 1;
  });
}

di_status di_server_submit(di_server* s, int32_t graph_id, int32_t n_seeds, const int32_t* seeds,
                           const double* w, double d, double tol, uint64_t* req_id) {
  return guarded([&] {
    DI_REQUIRE(s && seeds && req_id, "NULL argument");
    DI_REQUIRE(std::isfinite(d) && d >= 0.0 && d < 1.0, "d must satisfy 0 <= d < 1");
    DI_REQUIRE(std::isfinite(tol) && tol > 0.0, "tol must be > 0");
    DI_REQUIRE(n_seeds >= 1, "empty seed set");
    std::unique_lock<std::mutex> lk(s->mu);
    DI_REQUIRE(graph_id >= 0 && graph_id < (int32_t)s->graphs.size(), "unknown graph id");
    const int64_t n = s->graphs[graph_id].g->n;
    auto* r = new Request();
    r->seeds.assign(seeds, seeds + n_seeds);
    std::vector<int32_t> sorted = r->seeds;
    std::sort(sorted.begin(), sorted.end());
    double ws = 0.0;
    for (int k = 0; k < n_seeds; ++k) {
      if (seeds[k] < 0 || seeds[k] >= n || (k > 0 && sorted[k] == sorted[k - 1]) ||
          (w && !(std::isfinite(w[k]) && w[k] >= 0.0))) {
        delete r;
        set_error("seed out of range or repeated, or weight negative / not finite");
        throw Fail{DI_EINVAL};
      }
      if (w) ws += w[k];
    }
    if (w && std::fabs(ws - 1.0) > 1e-9) {
      delete r;
      set_error("seed weights must sum to 1");
      throw Fail{DI_EINVAL};
    }
    if (w) r->w.assign(w, w + n_seeds);
    r->id = s->next_id++;
    r->graph = graph_id;
    r->d = d;
    r->tol = tol;
    r->t_submit = s->now();
    memset(&r->res, 0, sizeof(r->res));
    if (s->t_first < 0) s->t_first = r->t_submit;
    s->reqs[r->id] = r;
    s->graphs[graph_id].queue.push_back(r);
    ++s->submitted;
    *req_id = r->id;
    if (!s->started) {
      s->started = true;
      for (int gi = 0; gi < (int)s->graphs.size(); ++gi)
        s->graphs[gi].th = std::thread([s, gi] { s->loop(gi); });
    }
    s->cv_work.notify_all();
  });
}

static di_status take_result(di_server* s, uint64_t req_id, di_result* out, bool block,
                             double timeout_s) {
  DI_REQUIRE(s && out, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  DI_REQUIRE(it != s->reqs.end(), "unknown request id");
  Request* r = it->second;
  if (!r->done && block) {
    auto pred = [&] { return r->done || (s->stop && !s->thread_error.empty()); };
    if (timeout_s < 0) s->cv_done.wait(lk, pred);
    else s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred);
  }
  if (!r->done) {
    if (!s->thread_error.empty()) set_error(s->thread_error);
    return DI_EAGAIN;
  }
  *out = finished_result(r);
  const int32_t st = r->res.status;
  s->reqs.erase(it);
  delete r;
  return st == DI_ECANCELED ? DI_ECANCELED : DI_OK;
}

di_status di_server_poll(di_server* s, uint64_t req_id, di_result* out) {
  di_status rc = DI_OK;
  di_status g = guarded([&] { rc = take_result(s, req_id, out, false, 0.0); });
  return g != DI_OK ? g : rc;
}

di_status di_server_wait(di_server* s, uint64_t req_id, double timeout_s, di_result* out) {
  di_status rc = DI_OK;
  di_status g = guarded([&] { rc = take_result(s, req_id, out, true, timeout_s); });
  return g != DI_OK ? g : rc;
}

di_status di_server_cancel(di_server* s, uint64_t req_id) {
  return guarded([&] {
    DI_REQUIRE(s, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    DI_REQUIRE(it != s->reqs.end(), "unknown request id");
    it->second->cancel = true;
    s->cv_work.notify_all();
  });
}

di_status di_server_stats(di_server* s, di_server_metrics* out) {
  return guarded([&] {
    DI_REQUIRE(s && out, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->admitted = s->admitted;
    out->completed = s->completed;
    out->cancelled = s->cancelled;
    for (auto& ge : s->graphs) {
      out->queued += (int64_t)ge.queue.size();
      for (Request* r : ge.slot_req) out->active += r != nullptr;
    }
    out->hbm_in_use = s->hbm_in_use;
    out->hbm_budget = s->opts.hbm_budget_bytes;
    if (!s->latencies.empty()) {
      std::vector<double> l = s->latencies;
      std::sort(l.begin(), l.end());
      auto pct = [&](double p) {
        const size_t i = (size_t)std::min<double>(l.size() - 1, std::floor(p * (l.size() - 1) + 0.5));
        return l[i];
      };
      out->p50_latency_s = pct(0.50);
      out->p99_latency_s = pct(0.99);
      const double span = s->t_last - s->t_first;
      out->qps = span > 0 ? (double)s->completed / span : 0.0;
    }
  });
}

di_status di_server_destroy(di_server* s) {
  return guarded([&] {
    if (!s) return;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
      s->cv_work.notify_all();
    }
    for (auto& ge : s->graphs)
      if (ge.th.joinable()) ge.th.join();
    for (auto& ge : s->graphs) (void)hipStreamSynchronize(ge.stream);
    for (auto& kv : s->reqs) delete kv.second;
    for (auto& ge : s->graphs) {
      ge.g->servers -= 1;
      ge.pool.reset();
      (void)hipStreamDestroy(ge.stream);
    }
    s->graphs.clear();
    delete s;
  });
}

}  // extern "C"
