// Autotuner of the threshold schedule, threshold factor and window size.
//
// The D-iteration converges to the same limit whatever set of nodes each
// round diffuses (any sequence I works, Section 2.2; Theorem 2 and the Lemma of
// Section 3.1), so the knobs of the
// threshold variant (Section 4.2, and the OP / OP2 scores of Section 4.3)
// trade only speed: a low threshold diffuses more links per round and needs
// fewer rounds, a high one wastes fewer links on small fluid.  Which side
// wins depends on the graph and on the device's per-round latency, so the
// tuner measures: trial solves through the public entry points, timed by the
// library's own device events (di_stats.seconds).

#include <algorithm>
#include <cmath>
#include <limits>
#include <mutex>
#include <vector>

#include "internal.h"

using namespace di;

namespace {

struct Trial {
  di_tune tune;
  double seconds;
  di_status status;
  int64_t rounds;  // most rounds any vector took
};

// Seconds per solve (per vector for batches) of one candidate: one untimed
// run (builds the window tables of a new window size), then the faster of two.
Trial run_candidate(const di_graph* g, int mode, const di_opts& base, int32_t B,
                    const int64_t* seed_ptr, const int32_t* seeds, const di_tune& t,
                    hipStream_t s) {
  Trial out{t, std::numeric_limits<double>::infinity(), DI_OK, 0};
  di_opts o = base;
  o.tune = &t;
  o.flags = 0;
  o.normalize = 1;
  std::vector<di_stats> st(mode == DI_TUNE_BATCH ? B : 1);
  for (int rep = 0; rep < 3; ++rep) {
    const di_status rc =
        mode == DI_TUNE_BATCH
            ? di_solve_batch(g, B, seed_ptr, seeds, nullptr, &o, nullptr, st.data(), s)
            : di_solve(g, nullptr, &o, nullptr, st.data(), s);
    if (rc != DI_OK) {
      out.status = rc;
      return out;
    }
    for (const di_stats& x : st) out.rounds = std::max(out.rounds, x.rounds);
    if (rep == 0) continue;
    // a batch reports the time of its whole group on every vector
    const double secs = mode == DI_TUNE_BATCH ? st[0].seconds / B : st[0].seconds;
    out.seconds = std::min(out.seconds, secs);
  }
  return out;
}

}  // namespace

extern "C" di_status di_autotune(di_graph* g, int32_t mode, const di_opts* opts, int32_t B,
                                 const int64_t* seed_ptr, const int32_t* seeds, di_tune* best,
                                 di_tune_trial* trials, int32_t max_trials, int32_t* n_trials,
                                 void* stream) {
  di_status result = DI_OK;
  const di_status rc = guarded([&] {
    DI_REQUIRE(g != nullptr, "graph is NULL");
    DI_REQUIRE(mode == DI_TUNE_SOLVE || mode == DI_TUNE_BATCH, "unknown tuning mode");
    validate_d_tol(opts);
    DI_REQUIRE(best != nullptr, "best is NULL");
    DI_REQUIRE(max_trials >= 0 && (max_trials == 0 || trials != nullptr),
               "trials is NULL but max_trials > 0");
    if (mode == DI_TUNE_BATCH)
      DI_REQUIRE(B >= 1 && seed_ptr != nullptr && seeds != nullptr,
                 "DI_TUNE_BATCH needs B >= 1 seed sets");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int w0 = window_log2_for(g->n, 0, 0, nullptr);
    DI_REQUIRE(w0 > 0, "graph has too many nodes for the window tables");

    std::vector<Trial> done;
    di_opts cand_opts = *opts;
    auto run = [&](int sched, float c, int wlog, int threads = 0, int persist = 0) {
      di_tune t{};
      t.schedule = sched;
      t.c = c;
      t.window_log2 = wlog;
      t.check_every = 0;
      t.threads = threads;
      t.persist = persist;
      done.push_back(run_candidate(g, mode, cand_opts, B, seed_ptr, seeds, t, s));
      return done.back();
    };
    auto better = [](const Trial& a, const Trial& b) {
      if ((a.status == DI_OK) != (b.status == DI_OK)) return a.status == DI_OK;
      return a.seconds < b.seconds;
    };
    // 0. the default knobs set the round budget of the other candidates: a
    //    threshold too high for the graph takes few nodes per round and may
    //    need orders of magnitude more rounds; such a candidate is cut off
    //    at four times the default's rounds and discarded.
    Trial win = run(DI_SCHED_MEAN, 1.0f, w0);
    if (win.status == DI_OK) {
      const int64_t cap = std::max<int64_t>(64, 4 * win.rounds);
      cand_opts.max_rounds = opts->max_rounds > 0 ? std::min(opts->max_rounds, cap) : cap;
    }
    // 1. schedule x threshold factor at the default window
    const int scheds[] = {DI_SCHED_MEAN, DI_SCHED_OP2, DI_SCHED_OP};
    const float cs[] = {0.03125f, 0.0625f, 0.125f, 0.25f, 0.5f, 1.0f, 2.0f};
    std::vector<Trial> step1{win};
    for (int sc : scheds)
      for (float c : cs) {
        if (sc == DI_SCHED_MEAN && c == 1.0f) continue;  // step 0
        const Trial t = run(sc, c, w0);
        step1.push_back(t);
        if (better(t, win)) win = t;
      }
    // 2. window size for the best pair: walk from the default in each
    //    direction while the time improves (sizes that the LDS budget or the
    //    window-count limit clamp to an already tried size end the walk)
    if (win.status == DI_OK) {
      std::vector<int> tried{w0};
      for (int dir : {-1, 1}) {
        for (int wl = w0 + dir;; wl += dir) {
          const int eff = window_log2_for(g->n, wl, 0, nullptr);
          if (eff <= 0 || std::find(tried.begin(), tried.end(), eff) != tried.end()) break;
          tried.push_back(eff);
          const Trial t = run(win.tune.schedule, win.tune.c, eff);
          if (!better(t, win)) break;
          win = t;
        }
      }
    }
    // 3. 1024-thread workgroups at the chosen window, for the three fastest
    //    (schedule, c) pairs of step 1: with more threads per window the best
    //    threshold factor can differ
    if (win.status == DI_OK) {
      std::stable_sort(step1.begin(), step1.end(), better);
      const int wl = win.tune.window_log2;
      for (size_t k = 0; k < step1.size() && k < 3 && step1[k].status == DI_OK; ++k) {
        const Trial t = run(step1[k].tune.schedule, step1[k].tune.c, wl, 1024);
        if (better(t, win)) win = t;
      }
    }
    // 4. single solves on graphs that one workgroup's LDS holds: the
    //    whole-graph window at every schedule x threshold factor
    if (mode == DI_TUNE_SOLVE && g->n <= DI_SMALL_MAX_NODES && g->m < (1ll << 31)) {
      for (int sc : scheds)
        for (float c : cs) {
          const Trial t = run(sc, c, DI_WINDOW_WHOLE);
          if (better(t, win)) win = t;
        }
    }
    // 5. single solves on graphs of at most DI_PERSIST_MAX_WINDOWS windows:
    //    one launch for every round, at every schedule x threshold factor at
    //    the smallest window that allows it, then larger windows for the
    //    best pair while the time improves
    if (mode == DI_TUNE_SOLVE) {
      int wp = w0;
      while (wp <= 11 && !persist_fits(g->n, g->m, wp)) ++wp;
      if (wp <= 11) {
        Trial pbest{};
        pbest.status = DI_EINVAL;
        for (int sc : scheds)
          for (float c : cs) {
            const Trial t = run(sc, c, wp, 0, 1);
            if (better(t, pbest)) pbest = t;
          }
        for (int wl = wp + 1; pbest.status == DI_OK && wl <= 11 && persist_fits(g->n, g->m, wl);
             ++wl) {
          const Trial t = run(pbest.tune.schedule, pbest.tune.c, wl, 0, 1);
          if (!better(t, pbest)) break;
          pbest = t;
        }
        if (better(pbest, win)) win = pbest;
      }
    }
    const int nt = (int)done.size();
    for (int k = 0; k < nt && k < max_trials; ++k) {
      trials[k].tune = done[k].tune;
      trials[k].seconds = done[k].seconds;
      trials[k].status = done[k].status;
      trials[k].pad = 0;
    }
    if (n_trials) *n_trials = nt;
    if (win.status != DI_OK) {
      set_error("no candidate converged within max_rounds");
      result = DI_ENOTCONV;
      return;
    }
    *best = win.tune;
    std::lock_guard<std::mutex> lk(g->ws_mu);
    const int pi = opts->precision == DI_FP64 ? 1 : 0;
    g->tuned[mode][pi] = win.tune;
    g->has_tuned[mode][pi] = true;
  });
  return rc != DI_OK ? rc : result;
}
