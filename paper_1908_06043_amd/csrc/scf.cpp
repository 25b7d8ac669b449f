// SCF sequence driver (Algorithm 1 over a sequence of pencils; the warm start of
// Section 2.1, shift migration of Section 3.2, missing eigenvalues and the
// partial-trace monitor of Section 3.3): the state that carries shifts and
// eigenvectors from one pencil to the next.
//
//  * First step, or a step whose spectrum moved too far: shifts from the KPM DOS
//    planner and Gaussian Lanczos starts.
//  * Otherwise the shifts migrate (sislice_scf_migrate: k-means of the previous
//    validated values seeded with the previous shifts, k-means++ after a DOS step;
//    clusters mapped to probes by overlap; merge, delete, insert), and every probe
//    starts from the previous eigenvectors of the values that seed it (a random
//    combination of them, or the vectors themselves padded with Gaussian columns
//    when there are fewer than the block size): the warm start that makes the
//    iteration converge in a few steps once the pencils change little.
//  * The monitor: eta = tr(X^T A X) of the previous eigenvectors under the
//    previous pencil (the sum of the previous eigenvalues) and under the new one;
//    a relative change above eta_tol sends the step to the DOS planner.
//  * Missing eigenvalues after a migrated step: the step is repeated with DOS
//    shifts and cold starts.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "blas.hpp"
#include "driver_util.hpp"
#include "handle.hpp"
#include "lanczos.hpp"
#include "eig.hpp"
#include "planner.hpp"
#include "sisubit.hpp"

struct sislice_scf {
  sislice_handle* h = nullptr;
  int n = 0, n_e = 0, n_s = 0;
  sislice_opts o{};
  double eta_tol = 0.05;
  int step = 0;
  bool last_dos = true;
  bool have_prev = false;
  std::vector<double> shifts;
  double top = 0.0;
  std::vector<double> prev_vals;
  std::vector<int32_t> prev_probe;
  double* prev_X = nullptr;  // device n x n_e, owned
  double* Afull = nullptr;   // device n x n, owned (the monitor's full copy of A)
  double* AX = nullptr;      // device n x n_e, owned
  double* start = nullptr;   // device n x 8 n_s, owned
  double* Xg = nullptr;      // device n x 3 n_e, owned (gathered previous vectors)
  double* dots = nullptr;    // device n_e, owned
};

namespace sislice {
namespace {

constexpr uint64_t kTagScf = 0x534346ull;

double host_gauss(uint64_t s, uint64_t k) {
  const double u1 = rng_uniform(s, 2 * k), u2 = rng_uniform(s, 2 * k + 1);
  return std::sqrt(-2.0 * std::log(1.0 - u1)) * std::cos(6.283185307179586 * u2);
}

// tr(Xp^T A Xp) with A read from its lower triangle.
double partial_trace(sislice_scf* s, Ctx& c, const double* A, long lda) {
  const int n = s->n, m = s->n_e;
  sym_full_launch(n, A, lda, s->Afull, n, c.st);
  gemm(c, false, false, {n}, {m}, {n}, {s->Afull}, n, {s->prev_X}, n, {s->AX}, n, 1.0, 0.0);
  ColDotArgs d;
  d.n = n;
  d.ncol0 = m;
  d.X = c.ring->cptrs(std::vector<double*>{s->prev_X});
  d.ldx = n;
  d.Y = c.ring->cptrs(std::vector<double*>{s->AX});
  d.ldy = n;
  d.out = c.ring->ptrs(std::vector<double*>{s->dots});
  d.mode = 0;
  d.partial = static_cast<double*>(ws_get(c.h, kBufMisc, sizeof(double) * coldot_partial_size(n, 1, m)));
  coldot_launch(d, 1, m, c.st);
  std::vector<double> v(m);
  SL_HIP(hipMemcpyAsync(v.data(), s->dots, sizeof(double) * m, hipMemcpyDeviceToHost, c.st));
  SL_HIP(hipStreamSynchronize(c.st));
  c.ring->synced();
  double t = 0.0;
  for (double x : v) t += x;
  return t;
}

// Warm-start blocks of the migrated probes (ascending shift order), `b` columns
// each (the Lanczos block, or the subspace iteration's basis).  A probe must
// lock every eigenvalue of its window (sigma_{j-1}, sigma_{j+1}) (the lower probe
// of each slice takes its values up to tau), so it starts from the previous
// eigenvectors of all the previous values inside that window, not only those of
// the cluster that moved it.  Returns the largest number of such values.
int build_starts(sislice_scf* s, Ctx& c, const ScfMigration& mg, int b) {
  const int n = s->n, P = (int)mg.shifts.size();
  std::vector<std::vector<int>> mem(P);
  for (int r = 0; r < P; ++r) {
    const double lo = r > 0 ? mg.shifts[r - 1] : -1e300;
    const double hi = r + 1 < P ? mg.shifts[r + 1] : s->top;
    for (int i = 0; i < s->n_e; ++i)
      if ((s->prev_vals[i] > lo && s->prev_vals[i] < hi) || mg.value_probe[i] == r) mem[r].push_back(i);
  }
  // Gaussian blocks for every probe first (probes with no members keep them)
  std::vector<unsigned long long> seeds(P);
  std::vector<double*> wp(P);
  for (int r = 0; r < P; ++r) {
    seeds[r] = rng_derive(s->o.seed, kTagScf ^ ((uint64_t)s->step << 20) ^ ((uint64_t)r << 40));
    wp[r] = s->start + (size_t)r * n * b;
  }
  gauss_launch(n, b, P, c.ring->vec(seeds), c.ring->ptrs(wp), n, c.st);
  // the previous vectors of each probe's values, gathered
  std::vector<int> cnt(P), rows(P, n), off(P);
  std::vector<double*> gout(P);
  std::vector<const int*> gidx(P);
  int acc = 0;
  for (int r = 0; r < P; ++r) {
    cnt[r] = (int)mem[r].size();
    off[r] = acc;
    acc += cnt[r];
    // few vectors: they become the leading columns of the start block itself
    gout[r] = cnt[r] < b ? s->start + (size_t)r * n * b : s->Xg + (size_t)off[r] * n;
    gidx[r] = c.ring->vec(mem[r].empty() ? std::vector<int>{0} : mem[r]);
  }
  SL_CHECK_ARG(acc <= 3 * s->n_e, "warm-start windows overlap more than expected");
  SelectArgs sa;
  sa.count = c.ring->vec(cnt);
  sa.rows = c.ring->vec(rows);
  sa.in = c.ring->cptrs(std::vector<double*>(P, s->prev_X));
  sa.ldi = n;
  sa.out = c.ring->ptrs(gout);
  sa.ldo = n;
  sa.idx = reinterpret_cast<const int* const*>(c.ring->cptrs(gidx));
  select_launch(sa, P, (long)n * std::max(1, *std::max_element(cnt.begin(), cnt.end())), c.st);
  // many vectors: a random combination of them (Gaussian coefficients)
  std::vector<int> gm, gn, gk;
  std::vector<const double*> ga;
  std::vector<double*> gc;
  std::vector<double> coef;
  std::vector<size_t> coff;
  for (int r = 0; r < P; ++r) {
    if (cnt[r] < b) continue;
    coff.push_back(coef.size());
    const uint64_t sd = rng_derive(s->o.seed, kTagScf ^ 0x47ull ^ ((uint64_t)s->step << 20) ^ ((uint64_t)r << 40));
    for (int e = 0; e < cnt[r] * b; ++e) coef.push_back(host_gauss(sd, (uint64_t)e));
    gm.push_back(n);
    gn.push_back(b);
    gk.push_back(cnt[r]);
    ga.push_back(s->Xg + (size_t)off[r] * n);
    gc.push_back(s->start + (size_t)r * n * b);
  }
  if (!gm.empty()) {
    const double* G = c.ring->vec(coef);  // staged with the launches' tables
    // per-probe coefficient blocks (cnt x 8) are packed with leading dimension cnt;
    // the batched GEMM takes one leading dimension, so run them one by one
    for (size_t q = 0; q < gm.size(); ++q)
      gemm(c, false, false, {gm[q]}, {gn[q]}, {gk[q]}, {ga[q]}, n, {G + coff[q]}, gk[q], {gc[q]}, n,
           1.0, 0.0);
  }
  int most = 0;
  for (int r = 0; r < P; ++r) most = std::max(most, cnt[r]);
  return most;
}

}  // namespace
}  // namespace sislice

using namespace sislice;

extern "C" {

sislice_status sislice_scf_create(sislice_handle* h, int64_t n, int64_t n_e, int64_t n_s,
                                  const sislice_opts* opts, double eta_tol, sislice_scf** out) {
  try {
    check_handle(h);
    SL_CHECK_ARG(out != nullptr, "null output pointer");
    *out = nullptr;
    SL_CHECK_ARG(n >= 32 && n <= 20000, "n must be in [32, 20000]");
    SL_CHECK_ARG(n_s >= 1 && n_s <= 1024 && n_e >= 1 && n_e < n && n_s <= n_e, "bad n_e / n_s");
    auto* s = new sislice_scf();
    s->h = h;
    s->n = (int)n;
    s->n_e = (int)n_e;
    s->n_s = (int)n_s;
    sislice_default_opts(&s->o);
    if (opts) s->o = *opts;
    try {
      check_opts(s->o);
    } catch (...) {
      delete s;
      throw;
    }
    s->eta_tol = eta_tol > 0 ? eta_tol : 0.05;
    const size_t nn = (size_t)n;
    auto alloc = [&](double** p, size_t cnt) {
      if (hipMalloc(p, sizeof(double) * std::max<size_t>(cnt, 1)) != hipSuccess) {
        *p = nullptr;
        throw Error(SISLICE_ERR_ALLOC, "SCF state allocation failed");
      }
    };
    try {
      alloc(&s->prev_X, nn * n_e);
      alloc(&s->Afull, nn * nn);
      alloc(&s->AX, nn * n_e);
      // start blocks: the Lanczos block, or up to kEigMax columns of a subspace basis
      alloc(&s->start, nn * (s->o.driver == 1 ? kEigMax : kLanczosBlock) * n_s);
      alloc(&s->Xg, nn * 3 * n_e);
      alloc(&s->dots, (size_t)n_e);
    } catch (...) {
      sislice_scf_destroy(s);
      throw;
    }
    *out = s;
    return SISLICE_OK;
  } catch (const Error& e) {
    std::fprintf(stderr, "sislice: %s\n", e.what());
    return e.status;
  }
}

sislice_status sislice_scf_destroy(sislice_scf* s) {
  if (!s) return SISLICE_OK;
  hipSetDevice(s->h->device);
  hipStreamSynchronize(s->h->stream);
  for (double* p : {s->prev_X, s->Afull, s->AX, s->start, s->Xg, s->dots})
    if (p) hipFree(p);
  delete s;
  return SISLICE_OK;
}

sislice_status sislice_scf_step(sislice_scf* s, const double* A, int64_t lda, const double* B,
                                int64_t ldb, double* evals, double* evecs, int64_t ldx,
                                double* resid, double* sigmas, double* omega_top,
                                sislice_scf_report* rep) {
  try {
    SL_CHECK_ARG(s != nullptr, "null SCF state");
    sislice_handle* h = s->h;
    check_handle(h);
    const int n = s->n, n_e = s->n_e, n_s = s->n_s;
    SL_CHECK_ARG(A && B && lda >= n && ldb >= n, "bad matrix argument");
    SL_CHECK_ARG(evals && evecs && resid && ldx >= n, "bad output argument");
    const auto t0 = Clock::now();
    sislice_scf_report r;
    std::memset(&r, 0, sizeof(r));
    r.step = s->step;
    bool dos = !s->have_prev;
    const double* start = nullptr;
    int start_cols = kLanczosBlock;
    {
      Ring ring(h);
      Ctx c{h, h->stream, &ring};
      if (s->have_prev) {
        double eta_prev = 0.0, scale = 0.0;
        for (double v : s->prev_vals) {
          eta_prev += v;
          scale += std::fabs(v);
        }
        const double eta_new = partial_trace(s, c, A, lda);
        r.eta_prev = eta_prev;
        r.eta_new = eta_new;
        if (std::fabs(eta_new - eta_prev) > s->eta_tol * std::max(scale, 1e-300)) {
          dos = true;
          r.replanned = 1;
        }
      } else {
        r.replanned = 1;
      }
      if (!dos) {
        const ScfMigration mg = scf_migrate(s->prev_vals.data(), s->prev_probe.data(), n_e,
                                            s->shifts.data(), n_s, s->last_dos, s->o.seed ^ (uint64_t)s->step);
        if ((int)mg.shifts.size() < n_s) {
          dos = true;  // no probe could be split: fall back to the DOS planner
          r.replanned = 1;
        } else {
          r.merged = mg.merged;
          r.deleted = mg.deleted;
          r.inserted = mg.inserted;
          s->shifts = mg.shifts;
          // Algorithm 2 is seeded with the previous eigenvectors themselves
          // (Sec. 2.1): up to kEigMax leading columns of each probe's basis
          start_cols = s->o.driver == 1 ? kEigMax : kLanczosBlock;
          build_starts(s, c, mg, start_cols);
          start = s->start;
          // The top boundary of a warm step sits two local spacings above the
          // previous n_e-th value: the planner's boundary holds a margin of values
          // beyond lambda_{n_e} that the kept eigenvectors do not span, and the top
          // probe would spend most of the step on them.  Should the perturbation
          // lift lambda_{n_e} past it, the solve moves the boundary up (top-boundary
          // recovery).
          const int m = std::min(n_e - 1, std::max(8, n_e / n_s));
          const double lam_ne = s->prev_vals[n_e - 1];
          const double spacing = m > 0 ? (lam_ne - s->prev_vals[n_e - 1 - m]) / m : 0.0;
          s->top = lam_ne + 2.0 * spacing + 1e-12 * std::max(1.0, std::fabs(lam_ne));
          if (!(s->top > s->shifts.back()))
            s->top = s->shifts.back() + (s->shifts.back() - s->shifts.front()) / n_s + 1e-12;
        }
      }
      // the next ring reuses the pinned staging memory: let the stream pass it first
      SL_HIP(hipStreamSynchronize(h->stream));
      ring.synced();
    }
    std::vector<int32_t> probe_of(n_e, 0);
    sislice_report sr;
    sislice_status st = SISLICE_OK;
    for (int attempt = 0; attempt < 2; ++attempt) {
      if (dos) {
        s->shifts.assign(n_s, 0.0);
        st = plan_impl(h, n, A, lda, B, ldb, n_e, n_s, s->o, s->shifts.data(), &s->top, nullptr, nullptr);
        if (st != SISLICE_OK) break;
        start = nullptr;
      }
      std::memset(&sr, 0, sizeof(sr));
      const auto ts = Clock::now();
      st = solve_impl(h, n, A, lda, B, ldb, n_e, n_s, s->shifts.data(), &s->top, s->o, evals, evecs,
                      ldx, resid, &sr, start, probe_of.data(), start_cols);
      r.t_solve_ms += ms_since(ts);
      r.block_steps += sr.block_steps;
      r.cycles_max = std::max(r.cycles_max, sr.cycles_max);
      r.probes_inserted += sr.probes_inserted;
      r.t_factor_ms += sr.t_factor_ms;
      r.flops_factor += sr.flops_factor;
      if ((st == SISLICE_MISSING_EIGS || st == SISLICE_SINGULAR_SHIFT) && !dos) {
        dos = true;  // the migrated shifts missed eigenvalues: repeat with DOS shifts
        r.replanned = 2;
        continue;
      }
      break;
    }
    r.status_solve = st;
    r.factor_id = sr.factor_id;
    if (st == SISLICE_OK || st == SISLICE_NOT_CONVERGED) {
      s->prev_vals.resize(n_e);
      SL_HIP(hipMemcpyAsync(s->prev_vals.data(), evals, sizeof(double) * n_e, hipMemcpyDeviceToHost,
                            h->stream));
      SL_HIP(hipMemcpy2DAsync(s->prev_X, sizeof(double) * n, evecs, sizeof(double) * ldx,
                              sizeof(double) * n, n_e, hipMemcpyDeviceToDevice, h->stream));
      SL_HIP(hipStreamSynchronize(h->stream));
      s->prev_probe = probe_of;
      s->have_prev = true;
      s->last_dos = dos;
    }
    if (sigmas)
      for (int j = 0; j < n_s; ++j) sigmas[j] = s->shifts[j];
    if (omega_top) *omega_top = s->top;
    ++s->step;
    r.t_total_ms = ms_since(t0);
    if (rep) *rep = r;
    check_waits(h);
    return st;
  } catch (const Error& e) {
    std::fprintf(stderr, "sislice: %s\n", e.what());
    return e.status;
  }
}

}  // extern "C"
