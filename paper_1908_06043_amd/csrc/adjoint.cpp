// sislice_adjoint: gradients of a loss of the lowest n_e eigenpairs with
// respect to A and B (first-order perturbation theory of the pencil of
// Section 1), reusing the shift factorizations of the solve.
//
//  1. The factorizations of the shifts and the top boundary: the ones the last
//     sislice_solve left in the driver workspace when factor_id matches, else
//     factored again.  A point with inertia <= n_e lies below lambda_{n_e+1}:
//     then (A - sigma B)^{-1} is positive definite on the B-orthogonal
//     complement of X, which makes it a valid preconditioner there.  Points
//     above (the top boundary usually is) are not used.
//  2. Occupied-occupied part: K = X^T g_X, the m x m middle matrices M_A, M_B,
//     Ua = X M_A / 2, Ub = X M_B / 2 (so that G = U X^T + X U^T).
//  3. Unoccupied part: z_i solves (A - lambda_i B) z_i = -(I - B X X^T) g_i with
//     X^T B z_i = 0.  Columns are grouped by their nearest point (at most 8 per
//     group); every group is one "shift" of the multi-shift sweeps, so one
//     launch pair preconditions all columns.  Conjugate gradients per column on
//     the complement, the preconditioned residual projected with
//     I - X (B X)^T each iteration; all scalars stay on the device and the host
//     checks convergence every few iterations.
//  4. Ua += Z / 2, Ub -= Z Lam / 2 and the fused rank-2m outputs.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "adjoint.hpp"
#include "blas.hpp"
#include "driver_util.hpp"
#include "factor_api.hpp"
#include "handle.hpp"
#include "solve.hpp"

namespace sislice {
namespace {

constexpr int kAdjGroup = 8;  // columns per preconditioner group (the sweeps' narrow width)
constexpr int kAdjCheck = 4;  // iterations between host convergence checks

sislice_status adjoint_impl(sislice_handle* h, int n, const double* A, long lda, const double* B,
                            long ldb, int m, const double* evals, const double* X, long ldx,
                            const double* glam, const double* gX, long ldg, int ns,
                            const double* sig, double top, uint64_t fid, double tol, int max_iter,
                            double* GA, long ldga, double* GB, long ldgb,
                            sislice_adjoint_report* rep) {
  const auto t_start = Clock::now();
  set_current_handle(h);
  hipStream_t st = h->stream;
  Ring ring(h);
  Ctx c{h, st, &ring};
  std::vector<double> pts(sig, sig + ns);
  pts.push_back(top);
  const int S1 = ns + 1;
  for (int j = 1; j < ns; ++j) SL_CHECK_ARG(pts[j] > pts[j - 1], "shifts must be ascending");
  SL_CHECK_ARG(top > pts[ns - 1], "omega_top must exceed every shift");
  // ---- 1. factorizations
  double t_factor = 0.0;
  auto& f = h->fc;
  const bool reuse = fid != 0 && f.id == fid && f.n == n && f.A == A && f.B == B && f.lda == lda &&
                     f.ldb == ldb && f.pts == pts;
  if (!reuse) {
    const auto t0 = Clock::now();
    driver_factor(h, ring, n, A, lda, B, ldb, pts, default_nb(n));
    t_factor = ms_since(t0);
    if (f.id == 0) return SISLICE_SINGULAR_SHIFT;
  }
  // usable preconditioners: points below lambda_{n_e+1}, i.e. with inertia <= n_e
  std::vector<char> usable(S1);
  bool any = false;
  for (int s = 0; s < S1; ++s) {
    usable[s] = f.inertia[3 * s] <= m;
    any |= usable[s] != 0;
  }
  SL_CHECK_ARG(any, "every shift lies above lambda_{n_e+1}: no positive definite preconditioner");
  // eigenvalues on the host: grouping and the degeneracy threshold
  std::vector<double> lam(m);
  SL_HIP(hipMemcpyAsync(lam.data(), evals, sizeof(double) * m, hipMemcpyDeviceToHost, st));
  SL_HIP(hipStreamSynchronize(st));
  double lmax = 0.0;
  for (double v : lam) lmax = std::max(lmax, std::fabs(v));
  const double degtol = 64.0 * std::numeric_limits<double>::epsilon() * lmax;
  // groups: columns by nearest point, at most kAdjGroup per group
  std::vector<std::vector<int>> by_pt(S1);
  for (int i = 0; i < m; ++i) {
    int best = -1;
    for (int s = 0; s < S1; ++s)
      if (usable[s] && (best < 0 || std::fabs(lam[i] - pts[s]) < std::fabs(lam[i] - pts[best])))
        best = s;
    by_pt[best].push_back(i);
  }
  std::vector<int> gpt;  // point of each group
  std::vector<int> col_of, slot(m, -1);
  for (int s = 0; s < S1; ++s)
    for (size_t q0 = 0; q0 < by_pt[s].size(); q0 += kAdjGroup) {
      const int g = (int)gpt.size();
      gpt.push_back(s);
      for (int q = 0; q < kAdjGroup; ++q) {
        const size_t k = q0 + q;
        const int i = k < by_pt[s].size() ? by_pt[s][k] : -1;
        col_of.push_back(i);
        if (i >= 0) slot[i] = g * kAdjGroup + q;
      }
    }
  const int G = (int)gpt.size();
  const int NP = G * kAdjGroup;
  // solve preparation of the points that groups use and the solve has not prepared
  {
    std::vector<int> need;
    for (int s : gpt)
      if (!f.prepped[s] && std::find(need.begin(), need.end(), s) == need.end()) need.push_back(s);
    if (!need.empty()) {
      std::vector<int32_t*> ip;
      std::vector<int*> pe, bl;
      std::vector<double*> ld, li;
      for (int s : need) {
        ip.push_back(f.ipv[s]);
        pe.push_back(f.perm[s]);
        bl.push_back(f.blk[s]);
        ld.push_back(f.LD[s]);
        li.push_back(f.Linv[s]);
        f.prepped[s] = 1;
      }
      solve_prep_launch(n, (int)need.size(), reinterpret_cast<const int* const*>(ring.ptrs(ip)),
                        ring.ptrs(pe), ring.ptrs(bl), ring.cptrs(ld), n, ring.ptrs(li), st);
    }
  }
  // ---- workspace
  Sizer z;
  z.take<double>((size_t)m * m);  // K
  z.take<double>((size_t)m * m);  // MA
  z.take<double>((size_t)m * m);  // MB
  z.take<double>((size_t)n * m);  // Ua
  z.take<double>((size_t)n * m);  // Ub
  z.take<double>((size_t)n * m);  // BX
  z.take<double>((size_t)n * m);  // E = BX K
  for (int q = 0; q < 4; ++q) z.take<double>((size_t)n * NP);  // R, Y, Z, Q
  z.take<double>((size_t)2 * n * NP);                          // Pst
  z.take<double>((size_t)m * NP);                              // projection coefficients
  for (int q = 0; q < 5; ++q) z.take<double>(NP);              // lamc, rho, bn2, rrel, ryo
  z.take<int>(NP);                                             // act
  z.take<int>(NP);                                             // restarts
  z.take<int>(NP);                                             // col_of
  z.take<int>(m);                                              // slot
  z.take<double>((size_t)G * n * kAdjGroup);                   // sweep scratch Z
  z.take<double>((size_t)G * n * kAdjGroup);                   // sweep scratch V
  Carver cv(ws_get(h, kBufAdjoint, z.off));
  double* Km = cv.take<double>((size_t)m * m);
  double* MA = cv.take<double>((size_t)m * m);
  double* MB = cv.take<double>((size_t)m * m);
  double* Ua = cv.take<double>((size_t)n * m);
  double* Ub = cv.take<double>((size_t)n * m);
  double* BX = cv.take<double>((size_t)n * m);
  double* E = cv.take<double>((size_t)n * m);
  double* Rc = cv.take<double>((size_t)n * NP);
  double* Yc = cv.take<double>((size_t)n * NP);
  double* Zc = cv.take<double>((size_t)n * NP);
  double* Qc = cv.take<double>((size_t)n * NP);
  double* Pst = cv.take<double>((size_t)2 * n * NP);
  double* Cp = cv.take<double>((size_t)m * NP);
  double* lamc = cv.take<double>(NP);
  double* rho = cv.take<double>(NP);
  double* bn2 = cv.take<double>(NP);
  double* rrel = cv.take<double>(NP);
  double* ryo = cv.take<double>(NP);
  int* act = cv.take<int>(NP);
  int* nrest = cv.take<int>(NP);
  int* d_col = cv.take<int>(NP);
  int* d_slot = cv.take<int>(m);
  double* Zs = cv.take<double>((size_t)G * n * kAdjGroup);
  double* Vs = cv.take<double>((size_t)G * n * kAdjGroup);
  double* Af = f.Af;  // [A B] full, n x 2n
  double* Bf = Af + (size_t)n * n;
  SL_HIP(hipMemcpyAsync(d_col, col_of.data(), sizeof(int) * NP, hipMemcpyHostToDevice, st));
  SL_HIP(hipMemcpyAsync(d_slot, slot.data(), sizeof(int) * m, hipMemcpyHostToDevice, st));
  // ---- 2. occupied-occupied part
  if (gX) gemm(c, true, false, {m}, {m}, {n}, {X}, ldx, {gX}, ldg, {Km}, m, 1.0, 0.0);
  adj_mid_launch(m, evals, glam, gX ? Km : nullptr, m, degtol, MA, MB, m, st);
  gemm(c, false, false, {n}, {m}, {m}, {X}, ldx, {MA}, m, {Ua}, n, 0.5, 0.0);
  gemm(c, false, false, {n}, {m}, {m}, {X}, ldx, {MB}, m, {Ub}, n, 0.5, 0.0);
  // ---- 3. projected solves
  int iters = 0, breakdowns = 0, still = 0;
  double maxrel = 0.0, t_solve = 0.0;
  if (gX) {
    const auto t0 = Clock::now();
    gemm(c, false, false, {n}, {m}, {n}, {Bf}, n, {X}, ldx, {BX}, n, 1.0, 0.0);
    gemm(c, false, false, {n}, {m}, {m}, {BX}, n, {Km}, m, {E}, n, 1.0, 0.0);
    adj_rhs_launch(n, NP, d_col, E, n, gX, ldg, evals, Rc, n, lamc, st);
    unsigned* sync = sync_words(h, (size_t)G + 64);
    // Y = Pi (A - sigma B)^{-1} R, Pi = I - X (B X)^T
    auto precondition = [&]() {
      SolveArgs sa;
      sa.n = n;
      sa.nshift = G;
      sa.nrhs = kAdjGroup;
      sa.epoch = next_epoch(h);
      std::vector<double*> ld(G), li(G), yy(G), xx(G), zz(G), vv(G);
      std::vector<int*> pe(G), bl(G);
      for (int g = 0; g < G; ++g) {
        ld[g] = f.LD[gpt[g]];
        pe[g] = f.perm[gpt[g]];
        bl[g] = f.blk[gpt[g]];
        li[g] = f.Linv[gpt[g]];
        yy[g] = Rc + (size_t)g * kAdjGroup * n;
        xx[g] = Yc + (size_t)g * kAdjGroup * n;
        zz[g] = Zs + (size_t)g * kAdjGroup * n;
        vv[g] = Vs + (size_t)g * kAdjGroup * n;
      }
      sa.LD = ring.cptrs(ld);
      sa.ldld = n;
      sa.perm = ring.cptrs(pe);
      sa.blk = ring.cptrs(bl);
      sa.Linv = ring.cptrs(li);
      sa.Y = ring.cptrs(yy);
      sa.ldy = n;
      sa.X = ring.ptrs(xx);
      sa.ldx = n;
      sa.Z = ring.ptrs(zz);
      sa.V = ring.ptrs(vv);
      sa.ldz = n;
      sa.ctr = sync;
      solve_launch(sa, st, 0);
      gemm(c, true, false, {m}, {NP}, {n}, {BX}, n, {Yc}, n, {Cp}, m, 1.0, 0.0);
      gemm(c, false, false, {n}, {NP}, {m}, {X}, ldx, {Cp}, m, {Yc}, n, -1.0, 1.0);
    };
    PcgArgs pa;
    pa.n = n;
    pa.np = NP;
    pa.Pst = Pst;
    pa.ldp = 2L * n;
    pa.Q = Qc;
    pa.ldq = n;
    pa.Z = Zc;
    pa.R = Rc;
    pa.Y = Yc;
    pa.ld = n;
    pa.lamc = lamc;
    pa.rho = rho;
    pa.bn2 = bn2;
    pa.rrel = rrel;
    pa.ryo = ryo;
    pa.nrest = nrest;
    pa.act = act;
    pa.tol2 = tol * tol;
    precondition();
    pcg_init_launch(pa, st);
    std::vector<int> hact(NP);
    for (int it = 1; it <= max_iter; ++it) {
      gemm(c, false, false, {n}, {NP}, {2 * n}, {Af}, n, {Pst}, 2L * n, {Qc}, n, 1.0, 0.0);
      pcg_alpha_launch(pa, st);
      precondition();
      pcg_beta_launch(pa, st);
      iters = it;
      if (it % kAdjCheck == 0 || it == max_iter) {
        SL_HIP(hipMemcpyAsync(hact.data(), act, sizeof(int) * NP, hipMemcpyDeviceToHost, st));
        SL_HIP(hipStreamSynchronize(st));
        if (std::none_of(hact.begin(), hact.end(), [](int v) { return v == 1 || v == 3; })) break;
      }
    }
    // Z on the complement (removes the rounding drift along X)
    gemm(c, true, false, {m}, {NP}, {n}, {BX}, n, {Zc}, n, {Cp}, m, 1.0, 0.0);
    gemm(c, false, false, {n}, {NP}, {m}, {X}, ldx, {Cp}, m, {Zc}, n, -1.0, 1.0);
    adj_combine_launch(n, m, Zc, n, d_slot, evals, Ua, Ub, n, st);
    std::vector<double> hrel(NP);
    SL_HIP(hipMemcpyAsync(hact.data(), act, sizeof(int) * NP, hipMemcpyDeviceToHost, st));
    SL_HIP(hipMemcpyAsync(hrel.data(), rrel, sizeof(double) * NP, hipMemcpyDeviceToHost, st));
    SL_HIP(hipStreamSynchronize(st));
    for (int t = 0; t < NP; ++t) {
      if (col_of[t] < 0) continue;
      breakdowns += hact[t] == 2;
      still += hact[t] == 1 || hact[t] == 3;
      maxrel = std::max(maxrel, std::sqrt(std::max(hrel[t], 0.0)));
    }
    t_solve = ms_since(t0);
  }
  // ---- 4. outputs
  hipEvent_t e0 = h->ev[0], e1 = h->ev[1];
  SL_HIP(hipEventRecord(e0, st));
  adj_syr2k_launch(n, m, X, ldx, Ua, Ub, n, GA, ldga, GB, ldgb, st);
  SL_HIP(hipEventRecord(e1, st));
  SL_HIP(hipStreamSynchronize(st));
  ring.synced();
  float t_outer = 0.f;
  SL_HIP(hipEventElapsedTime(&t_outer, e0, e1));
  if (rep) {
    rep->iterations = iters;
    rep->reused_factors = reuse ? 1 : 0;
    rep->n_groups = G;
    rep->breakdowns = breakdowns;
    rep->max_rel_residual = maxrel;
    rep->t_factor_ms = t_factor;
    rep->t_solve_ms = t_solve;
    rep->t_total_ms = ms_since(t_start);
    rep->flops_outer = 4.0 * (double)n * n * m;
    rep->t_outer_ms = t_outer;
  }
  if (still > 0 || breakdowns > 0) return SISLICE_NOT_CONVERGED;
  return SISLICE_OK;
}

}  // namespace
}  // namespace sislice

using namespace sislice;

extern "C" sislice_status sislice_adjoint(sislice_handle* h, int64_t n, const double* A,
                                          int64_t lda, const double* B, int64_t ldb, int64_t n_e,
                                          const double* evals, const double* evecs, int64_t ldx,
                                          const double* g_evals, const double* g_evecs,
                                          int64_t ldg, int64_t n_s, const double* sigmas,
                                          double omega_top, uint64_t factor_id, double tol,
                                          int32_t max_iter, double* GA, int64_t ldga, double* GB,
                                          int64_t ldgb, sislice_adjoint_report* report) {
  try {
    check_handle(h);
    SL_CHECK_ARG(n >= 32 && n <= 20000, "n must be in [32, 20000]");
    SL_CHECK_ARG(n_e >= 1 && n_e < n, "n_e must be in [1, n)");
    SL_CHECK_ARG(n_s >= 1 && n_s <= 1024, "n_s must be in [1, 1024]");
    SL_CHECK_ARG(A && B && lda >= n && ldb >= n, "bad matrix argument");
    SL_CHECK_ARG(evals && evecs && ldx >= n && sigmas, "bad eigenpair argument");
    SL_CHECK_ARG(!g_evecs || ldg >= n, "ldg must be >= n");
    SL_CHECK_ARG(GA && GB && ldga >= n && ldgb >= n, "bad gradient argument");
    SL_CHECK_ARG(std::isfinite(omega_top), "omega_top must be finite");
    if (!(tol > 0.0)) tol = 1e-10;
    if (max_iter <= 0) max_iter = 500;
    const sislice_status st =
        adjoint_impl(h, (int)n, A, lda, B, ldb, (int)n_e, evals, evecs, ldx, g_evals, g_evecs, ldg,
                     (int)n_s, sigmas, omega_top, factor_id, tol, max_iter, GA, ldga, GB, ldgb,
                     report);
    check_waits(h);
    return st;
  } catch (const Error& e) {
    std::fprintf(stderr, "sislice: %s\n", e.what());
    return e.status;
  }
}
