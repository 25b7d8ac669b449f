// sislice_solve_batched: many independent pencils of uneven order on one GPU.
//
// The paper's probes are independent (Section 4.1); so are whole pencils.  One
// pencil of order 512..3072 leaves most of the 256 compute units idle: its
// panel chains, sweeps and small eigenproblems are latency-bound and its host
// steps (convergence checks, validation) leave the device waiting.  The batch
// scheduler therefore runs `workers` pencils at a time, each on a worker handle
// with its own stream and workspaces, driven by its own host thread; the
// largest pencils are taken first (longest-processing-time order) so the tail
// is short.  Within a pencil the shifts are factored and iterated in lock step
// as in the plain path.
//
// Autotuning: the factorization's parameters are chosen per order n (the
// bucket of the cache): the panel width nb, the width of a pivoting panel after
// a rejected pivot-free prefix, and the trailing order from which the update
// takes 128x128 instead of 64x64 MFMA tiles.  For the first pencil of each order
// not yet in the handle's cache, the shifts are planned and the lock-step
// factorization of all points is timed per candidate (coordinate descent: the
// width, then the pivoting width, then the tile switch; best of two runs each),
// one pencil at a time on an otherwise idle device; the fastest is cached in
// the handle and used by every later pencil of that order.
//
// Graphs: with opts.graphs the workers' factorizations replay captured step
// sequences (one per order, shift count and parameters on each worker), so a
// factorization costs one graph launch instead of hundreds of launches and a
// progress readback every few steps.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "driver_util.hpp"
#include "factor_api.hpp"
#include "handle.hpp"

namespace sislice {
namespace {

constexpr int kNbCandidates[] = {32, 48, 64};
constexpr int kNbpivCandidates[] = {16, 32};
constexpr int kWideCandidates[] = {512, 1024, 2048};
constexpr int kMaxWorkers = 16;

void ensure_workers(sislice_handle* h, int nw) {
  while ((int)h->workers.size() < nw) {
    hipStream_t s = nullptr;
    SL_HIP(hipSetDevice(h->device));
    SL_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    sislice_handle* w = nullptr;
    const sislice_status st = sislice_create(&w, h->device, s);
    if (st != SISLICE_OK) {
      hipStreamDestroy(s);
      throw Error(st, "worker handle creation failed");
    }
    w->wait_limit = h->wait_limit;
    h->workers.push_back(w);
    h->worker_streams.push_back(s);
  }
}

// Fastest factorization parameters for order p.n: plan the shifts of p, then
// time the lock-step factorization of the shifts and the top boundary per
// candidate.
sislice_handle::FactorTune tune_factor(sislice_handle* w, const sislice_problem& p,
                                       const sislice_opts& o) {
  sislice_handle::FactorTune best;
  best.nb = default_nb((int)p.n);
  best.nbpiv = 32;
  best.wide_min = 1024;
  std::vector<double> sig(p.n_s);
  double top = 0.0;
  sislice_status st = plan_impl(w, p.n, p.A, p.lda, p.B, p.ldb, p.n_e, p.n_s, o, sig.data(), &top,
                                nullptr, nullptr);
  if (st != SISLICE_OK) return best;
  std::vector<double> pts(sig);
  pts.push_back(top);
  w->use_graphs = o.graphs != 0;
  double tbest = 1e300;
  bool singular = false;
  auto time_cfg = [&](const sislice_handle::FactorTune& t) {
    w->cur_nbpiv = t.nbpiv;
    w->cur_wide_min = t.wide_min;
    double tb = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
      Ring ring(w);
      const auto t0 = Clock::now();
      driver_factor(w, ring, (int)p.n, p.A, p.lda, p.B, p.ldb, pts, t.nb);
      tb = std::min(tb, ms_since(t0));
      if (w->fc.id == 0) singular = true;
    }
    w->cur_nbpiv = 0;
    w->cur_wide_min = 0;
    if (tb < tbest) {
      tbest = tb;
      best = t;
    }
  };
  for (int nb : kNbCandidates) {
    if (nb > kMaxNb || nb >= p.n) continue;
    sislice_handle::FactorTune t = best;
    t.nb = nb;
    time_cfg(t);
    if (singular) break;
  }
  for (int nbpiv : kNbpivCandidates) {
    if (singular || nbpiv == best.nbpiv) continue;
    sislice_handle::FactorTune t = best;
    t.nbpiv = nbpiv;
    time_cfg(t);
  }
  for (int wide : kWideCandidates) {
    if (singular || wide == best.wide_min || wide >= p.n) continue;
    sislice_handle::FactorTune t = best;
    t.wide_min = wide;
    time_cfg(t);
  }
  w->fc.id = 0;  // the timing factorizations are not a solve's
  if (singular) {  // a singular point: keep the defaults
    best.nb = default_nb((int)p.n);
    best.nbpiv = 32;
    best.wide_min = 1024;
  }
  return best;
}

// Runs fn(worker, item) over items with one host thread per worker handle.
template <class F>
void run_workers(sislice_handle* h, int nw, int count, F fn) {
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (int q = 0; q < nw; ++q)
    th.emplace_back([&, q] {
      sislice_handle* w = h->workers[q];
      for (;;) {
        const int i = next.fetch_add(1);
        if (i >= count) break;
        fn(w, i);
      }
    });
  for (auto& t : th) t.join();
}

}  // namespace
}  // namespace sislice

using namespace sislice;

extern "C" sislice_status sislice_solve_batched(sislice_handle* h, int64_t count,
                                                const sislice_problem* problems,
                                                const sislice_opts* opts, int32_t workers,
                                                int32_t* status, sislice_batch_report* report) {
  try {
    check_handle(h);
    SL_CHECK_ARG(count >= 0 && count <= (int64_t)1 << 20, "count out of range");
    SL_CHECK_ARG(count == 0 || (problems && status), "null problems or status array");
    sislice_opts o;
    sislice_default_opts(&o);
    if (opts) o = *opts;
    check_opts(o);
    for (int64_t i = 0; i < count; ++i) {
      const sislice_problem& p = problems[i];
      SL_CHECK_ARG(p.n >= 32 && p.n <= 20000, "problem order must be in [32, 20000]");
      SL_CHECK_ARG(p.n_s >= 1 && p.n_s <= 1024 && p.n_e >= 1 && p.n_e < p.n, "bad n_e / n_s");
      SL_CHECK_ARG(p.A && p.B && p.lda >= p.n && p.ldb >= p.n, "bad matrix argument");
      SL_CHECK_ARG(p.evals && p.evecs && p.resid && p.ldx >= p.n, "bad output argument");
    }
    const auto t_start = Clock::now();
    const int nw = (int)std::max<int64_t>(
        1, std::min<int64_t>({workers > 0 ? workers : 4, kMaxWorkers, std::max<int64_t>(count, 1)}));
    ensure_workers(h, nw);
    SL_HIP(hipStreamSynchronize(h->stream));  // inputs written on the caller's stream
    // ---- autotuning of the panel width per order (skipped when opts fixes it)
    double t_tune = 0.0;
    int tuned_now = 0;
    if (o.nb <= 0) {
      std::vector<int> todo;  // first problem of each order without a cached width
      for (int64_t i = 0; i < count; ++i) {
        const int n = (int)problems[i].n;
        if (h->tuned.count(n)) continue;
        bool seen = false;
        for (int j : todo) seen |= problems[j].n == n;
        if (!seen) todo.push_back((int)i);
      }
      if (!todo.empty()) {
        const auto t0 = Clock::now();
        std::vector<sislice_handle::FactorTune> pick(todo.size());
        std::vector<Error> errs;
        std::mutex mu;
        // one pencil at a time, so that the timings are not disturbed by other work
        run_workers(h, 1, (int)todo.size(), [&](sislice_handle* w, int k) {
          try {
            check_handle(w);
            pick[k] = tune_factor(w, problems[todo[k]], o);
          } catch (const Error& e) {
            std::lock_guard<std::mutex> lk(mu);
            errs.push_back(e);
          }
        });
        set_current_handle(h);
        if (!errs.empty()) throw errs.front();
        for (size_t k = 0; k < todo.size(); ++k) h->tuned[(int)problems[todo[k]].n] = pick[k];
        t_tune = ms_since(t0);
        tuned_now = (int)todo.size();
      }
    }
    // ---- the pencils, largest first
    std::vector<int> order((size_t)count);
    for (int64_t i = 0; i < count; ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return problems[a].n > problems[b].n; });
    std::vector<int64_t> conv((size_t)count, 0);
    int64_t replays0 = 0, built0 = 0;
    for (auto* w : h->workers) {
      replays0 += w->graph_replays;
      built0 += w->graphs_built;
    }
    run_workers(h, nw, (int)count, [&](sislice_handle* w, int k) {
      const int i = order[k];
      const sislice_problem& p = problems[i];
      try {
        check_handle(w);
        sislice_opts oi = o;
        const auto tu = h->tuned.find((int)p.n);
        if (oi.nb <= 0 && tu != h->tuned.end()) {
          oi.nb = tu->second.nb;
          w->cur_nbpiv = tu->second.nbpiv;
          w->cur_wide_min = tu->second.wide_min;
        }
        sislice_report rep;
        std::memset(&rep, 0, sizeof(rep));
        double top = 0.0;
        status[i] = solve_impl(w, p.n, p.A, p.lda, p.B, p.ldb, p.n_e, p.n_s, nullptr, &top, oi,
                               p.evals, p.evecs, p.ldx, p.resid, &rep);
        w->cur_nbpiv = 0;
        w->cur_wide_min = 0;
        check_waits(w);
        conv[i] = (status[i] == SISLICE_OK || status[i] == SISLICE_NOT_CONVERGED) ? rep.n_converged : 0;
      } catch (const Error& e) {
        std::fprintf(stderr, "sislice: problem %d: %s\n", i, e.what());
        status[i] = e.status;
        w->cur_nbpiv = 0;
        w->cur_wide_min = 0;
      }
    });
    set_current_handle(h);
    for (auto s : h->worker_streams) SL_HIP(hipStreamSynchronize(s));
    sislice_status worst = SISLICE_OK;
    int n_ok = 0;
    int64_t nconv = 0;
    for (int64_t i = 0; i < count; ++i) {
      n_ok += status[i] == SISLICE_OK;
      nconv += conv[i];
      if (status[i] < 0 && (worst >= 0 || status[i] < worst)) worst = (sislice_status)status[i];
      if (status[i] > 0 && worst == SISLICE_OK) worst = (sislice_status)status[i];
    }
    int64_t replays1 = 0, built1 = 0;
    for (auto* w : h->workers) {
      replays1 += w->graph_replays;
      built1 += w->graphs_built;
    }
    if (report) {
      report->graph_replays = replays1 - replays0;
      report->graphs_built = built1 - built0;
      report->workers = nw;
      report->n_ok = n_ok;
      report->n_tuned = tuned_now;
      report->n_converged = nconv;
      report->t_total_ms = ms_since(t_start);
      report->t_tune_ms = t_tune;
    }
    return worst;
  } catch (const Error& e) {
    set_current_handle(h);
    std::fprintf(stderr, "sislice: %s\n", e.what());
    return e.status;
  }
}

extern "C" int32_t sislice_tuned_nb(sislice_handle* h, int64_t n) {
  if (!h) return 0;
  auto it = h->tuned.find((int)n);
  return it == h->tuned.end() ? 0 : it->second.nb;
}

extern "C" int32_t sislice_tuned_factor(sislice_handle* h, int64_t n, int32_t* nb, int32_t* nbpiv,
                                        int32_t* wide_min) {
  if (!h) return 0;
  auto it = h->tuned.find((int)n);
  if (it == h->tuned.end()) return 0;
  if (nb) *nb = it->second.nb;
  if (nbpiv) *nbpiv = it->second.nbpiv;
  if (wide_min) *wide_min = it->second.wide_min;
  return 1;
}
