// The plain per-pencil path (Algorithm 1, one pass on a fixed pencil) and the
// KPM shift planner (Section 3.1), orchestrating the device kernels.
//
//  1. Factor A - sigma_j B for every shift and the top boundary together and read
//     the inertias (Section 2.2) -- all counts are known before any iteration.
//  2. Per shift, block shift-invert Lanczos in the B inner product (block 8):
//     W = (A - sigma B)^{-1} U_last, full B-reorthogonalisation against the
//     locked and active bases (twice), Z = B W for all shifts in one GEMM,
//     CholeskyQR2, projected matrix T from the projections.  Probes advance in
//     lock step; when the active basis is full, eig(T) gives Ritz pairs and
//     residual estimates; converged pairs inside the probe's window
//     (sigma_{j-1}, sigma_{j+1}) are locked, the best unconverged ones are kept
//     (thick restart).  A probe stops once both of its slices hold as many
//     locked values as their exact counts.
//  3. Explicit Rayleigh-Ritz with A on the locked vectors (Section 2.1),
//     residuals, slice validation (Section 2.2), lowest n_e out.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <vector>

#include "blas.hpp"
#include "eig.hpp"
#include "factor_api.hpp"
#include "handle.hpp"
#include "lanczos.hpp"
#include "planner.hpp"
#include "driver_util.hpp"
#include "sisubit.hpp"
#include "solve.hpp"

namespace sislice {
namespace {

struct ProbeHost {
  double sigma = 0, lo = 0, hi = 0;
  int64_t need = 0;
  int mq = 0;        // active basis columns incl. the newest block
  int nl = 0;        // locked columns
  int64_t nin = 0;   // locked columns with values inside the probe's window
  bool active = true;
  bool broke = false;
  int cycles = 0;
  int steps = 0;
  std::vector<double> lock_lam;
};


// ||M||_2 of a symmetric full matrix by block power iteration with a final
// Rayleigh-Ritz on 8 vectors (a lower bound that converges quickly; only a
// tolerance scale is needed).
double sym_norm2(Ctx& c, int n, const double* M, double* X, double* Y, double* G, double* R,
                 double* H, double* Wv, double* Vv, int* flag, int* active1, uint64_t seed) {
  const int b = kLanczosBlock;
  std::vector<unsigned long long> sd{rng_derive(seed, 0x4E524Dull)};
  gauss_launch(n, b, 1, c.ring->vec(sd), c.ring->ptrs(std::vector<double*>{X}), n, c.st);
  for (int it = 0; it < 12; ++it) {
    gemm(c, false, false, {n}, {b}, {n}, {M}, n, {X}, n, {Y}, n, 1.0, 0.0);
    gemm(c, true, false, {b}, {b}, {n}, {Y}, n, {Y}, n, {G}, b, 1.0, 0.0);
    CholQrArgs q;
    q.n = n;
    q.active = active1;
    q.G = c.ring->cptrs(std::vector<double*>{G});
    q.Vin = c.ring->cptrs(std::vector<double*>{Y});
    q.Uin = q.Vin;
    q.ldin = n;
    q.Vout = c.ring->ptrs(std::vector<double*>{X});
    q.Uout = c.ring->ptrs(std::vector<double*>{Y});
    q.ldout = n;
    q.R = c.ring->ptrs(std::vector<double*>{R});
    q.flag = flag;
    cholqr_launch(q, 1, c.st);
  }
  gemm(c, false, false, {n}, {b}, {n}, {M}, n, {X}, n, {Y}, n, 1.0, 0.0);
  gemm(c, true, false, {b}, {b}, {n}, {X}, n, {Y}, n, {H}, b, 1.0, 0.0);
  EigArgs e;
  e.m = c.ring->vec(std::vector<int>{b});
  e.A = c.ring->cptrs(std::vector<double*>{H});
  e.lda = b;
  e.W = c.ring->ptrs(std::vector<double*>{Wv});
  e.V = c.ring->ptrs(std::vector<double*>{Vv});
  e.ldv = b;
  eig_launch(e, 1, b, c.st);
  double w[kLanczosBlock];
  SL_HIP(hipMemcpyAsync(w, Wv, sizeof(w), hipMemcpyDeviceToHost, c.st));
  SL_HIP(hipStreamSynchronize(c.st));
  c.ring->synced();
  double mx = 0.0;
  for (double v : w) mx = std::max(mx, std::fabs(v));
  return mx;
}

}  // namespace

void check_opts(const sislice_opts& o) {
  SL_CHECK_ARG(o.block == kLanczosBlock, "only block size 8 is built");
  SL_CHECK_ARG(o.max_basis >= 32 && o.max_basis <= kEigMax && o.max_basis % kLanczosBlock == 0,
               "max_basis must be a multiple of 8 in [32, 112]");
  SL_CHECK_ARG(o.max_cycles >= 1, "max_cycles must be positive");
  SL_CHECK_ARG(o.kpm_moments >= 4 && o.kpm_moments <= 4096, "kpm_moments out of range");
  SL_CHECK_ARG(o.kpm_vectors >= 1 && o.kpm_vectors <= kSolveMaxRhs, "kpm_vectors in [1, 32]");
  SL_CHECK_ARG(o.bounds_steps >= 2 && o.bounds_steps <= 100, "bounds_steps in [2, 100]");
  SL_CHECK_ARG(o.tol > 0 && o.tol < 1, "tol in (0, 1)");
  SL_CHECK_ARG(o.driver == 0 || o.driver == 1, "driver must be 0 (Lanczos) or 1 (subspace iteration)");
  SL_CHECK_ARG(o.subspace_iters >= 1 && o.subspace_iters <= 64, "subspace_iters in [1, 64]");
  SL_CHECK_ARG(o.max_recovery >= 0 && o.max_recovery <= 8, "max_recovery in [0, 8]");
}

// ---------------------------------------------------------------- planner

sislice_status plan_impl(sislice_handle* h, int64_t n64, const double* A, int64_t lda,
                         const double* B, int64_t ldb, int64_t n_e, int64_t n_s,
                         const sislice_opts& o, double* sig, double* top, double* mom_out,
                         double* bounds_out, int dos_mode, int dos_k, int dos_nv) {
  const int n = (int)n64;
  const int nv = dos_mode >= 0 ? std::max(o.kpm_vectors, dos_nv) : o.kpm_vectors;
  const int M = o.kpm_moments, bs = o.bounds_steps;
  hipStream_t st = h->stream;
  Ring ring(h);
  Ctx c{h, st, &ring};
  const int m_b = std::min(bs, n);  // Lanczos steps for the bounds
  // workspace
  Sizer z;
  z.take<double>((size_t)n * n);      // Af: A with both triangles
  z.take<double>((size_t)n * n);      // LD of B
  z.take<double>((size_t)n * n);      // M = D^{-1/2} L^{-1} (lower)
  z.take<double>((size_t)n * n);      // M^T (upper); scratch of the inversion before that
  z.take<int32_t>(n);                 // ipiv
  z.take<int>(n);                     // perm
  z.take<int>(n);                     // blk
  z.take<double>(solve_linv_size(n));
  z.take<double>(n);                  // D^{-1/2}
  for (int q = 0; q < 6; ++q) z.take<double>((size_t)n * nv);  // t_prev, t_cur, t_next, X1..X3
  z.take<double>((size_t)n * (m_b + 1));  // Lanczos basis
  z.take<double>((size_t)n * 4);          // w
  z.take<double>(8192);                   // small scalars
  z.take<double>(skinny_partial_size(n, std::max(nv, 1)));
  z.take<int>(64);
  const int dk = dos_mode >= 0 ? std::min(dos_k, n) : 0;  // Lanczos DOS steps
  if (dos_mode >= 0) {
    z.take<double>((size_t)n * dos_nv * (dk + 1));  // the runs' bases, block j = n x nv
    z.take<double>((size_t)(dk + 1) * dos_nv * 4);  // alpha, s2, beta, coefficients
  }
  Carver cv(ws_get(h, kBufKpm, z.off));
  double* Af = cv.take<double>((size_t)n * n);
  double* LDB = cv.take<double>((size_t)n * n);
  double* Mi = cv.take<double>((size_t)n * n);
  double* MT = cv.take<double>((size_t)n * n);
  int32_t* ipB = cv.take<int32_t>(n);
  int* permB = cv.take<int>(n);
  int* blkB = cv.take<int>(n);
  double* LinvB = cv.take<double>(solve_linv_size(n));
  double* dsc = cv.take<double>(n);
  double* T0 = cv.take<double>((size_t)n * nv);
  double* T1 = cv.take<double>((size_t)n * nv);
  double* T2 = cv.take<double>((size_t)n * nv);
  double* X1 = cv.take<double>((size_t)n * nv);
  double* X2 = cv.take<double>((size_t)n * nv);
  double* X3 = cv.take<double>((size_t)n * nv);
  double* Vb = cv.take<double>((size_t)n * (m_b + 1));
  double* wv = cv.take<double>((size_t)n * 4);
  double* small = cv.take<double>(8192);
  double* spart = cv.take<double>(skinny_partial_size(n, std::max(nv, 1)));
  int* iflag = cv.take<int>(64);
  double* Vd = dos_mode >= 0 ? cv.take<double>((size_t)n * dos_nv * (dk + 1)) : nullptr;
  double* dsc2 = dos_mode >= 0 ? cv.take<double>((size_t)(dk + 1) * dos_nv * 4) : nullptr;
  SL_CHECK_ARG(nv >= 1 && nv <= kSkinnyMaxCol, "kpm_vectors must be in [1, 32]");
  SL_HIP(hipMemsetAsync(iflag, 0, 64 * sizeof(int), st));
  sym_full_launch(n, A, lda, Af, n, st);
  // B = L D L^T without interchanges (B is SPD), so L_B = L D^{1/2}
  {
    double* lds[1] = {LDB};
    int32_t* ips[1] = {ipB};
    double zero = 0.0;
    FactorPlan fp = build_factor(h, kBufFactor, n, B, ldb, B, ldb, 1, &zero, lds, n, ips,
                                 default_nb(n), false);
    factor_launch(fp, st);
    int64_t inert[3];
    SL_HIP(hipMemcpyAsync(inert, fp.d_inertia, sizeof(inert), hipMemcpyDeviceToHost, st));
    SL_HIP(hipStreamSynchronize(st));
    ring.synced();
    if (inert[0] != 0 || inert[1] != 0) throw Error(SISLICE_ERR_ARG, "B is not positive definite");
  }
  {
    auto tLD = ring.cptrs(std::vector<double*>{LDB});
    auto tip = ring.cptrs(std::vector<int32_t*>{ipB});
    auto tperm = ring.ptrs(std::vector<int*>{permB});
    auto tblk = ring.ptrs(std::vector<int*>{blkB});
    auto tLinv = ring.ptrs(std::vector<double*>{LinvB});
    solve_prep_launch(n, 1, reinterpret_cast<const int* const*>(tip), tperm, tblk, tLD, n, tLinv, st);
  }
  inv_sqrt_diag_launch(n, LDB, n, dsc, iflag, st);
  // Explicit L^{-1} by doubling: starting from the inverted 64x64 diagonal blocks,
  // each level joins neighbouring groups of h rows,
  //   inv([X11 0; L21 X22]) has lower-left block -X22 (L21 X11),
  // with the groups of one level as one batched MFMA GEMM (MT is the scratch).
  SL_HIP(hipMemsetAsync(Mi, 0, sizeof(double) * (size_t)n * n, st));
  diag_inv_scatter_launch(n, LinvB, Mi, n, st);
  for (int hh = kSolveBlock; hh < n; hh *= 2) {
    std::vector<int> gm, gn, gk2;
    std::vector<const double*> aL, aX11, aX22, aT;
    std::vector<double*> oT, oX21;
    for (int r0 = 0; r0 + hh < n; r0 += 2 * hh) {
      const int r1 = std::min(r0 + 2 * hh, n), m2 = r1 - r0 - hh;
      gm.push_back(m2);
      gn.push_back(hh);
      gk2.push_back(m2);
      aL.push_back(LDB + (r0 + hh) + (size_t)r0 * n);
      aX11.push_back(Mi + r0 + (size_t)r0 * n);
      aX22.push_back(Mi + (r0 + hh) + (size_t)(r0 + hh) * n);
      oT.push_back(MT + (r0 + hh) + (size_t)r0 * n);
      aT.push_back(MT + (r0 + hh) + (size_t)r0 * n);
      oX21.push_back(Mi + (r0 + hh) + (size_t)r0 * n);
    }
    std::vector<int> gk1(gm.size(), hh);
    gemm(c, false, false, gm, gn, gk1, aL, n, aX11, n, oT, n, 1.0, 0.0);
    gemm(c, false, false, gm, gn, gk2, aX22, n, aT, n, oX21, n, -1.0, 0.0);
  }
  row_scale_launch(n, n, dsc, Mi, n, st);  // M = D^{-1/2} L^{-1}
  transpose_launch(n, Mi, n, MT, n, st);
  // H Y = M A M^T Y for k <= 32 columns: three HBM-bound skinny products
  auto apply_H = [&](const double* Yin, double* out, int k) {
    skinny_launch(n, k, MT, n, 2, Yin, n, 1.0, 0.0, X1, n, spart, st);
    skinny_launch(n, k, Af, n, 0, X1, n, 1.0, 0.0, X3, n, spart, st);
    skinny_launch(n, k, Mi, n, 1, X3, n, 1.0, 0.0, out, n, spart, st);
  };
  if (dos_mode >= 0) {
    // ---- the paper's DOS estimate (Section 3.1): dos_nv runs of dk-step Lanczos on
    // H, advanced together (one application of H serves every run), each with full
    // reorthogonalisation against its own basis; alpha, beta read at the end
    const int R = dos_nv;
    double* d_alpha = dsc2;                              // [dk][R]
    double* d_s2 = dsc2 + (size_t)(dk + 1) * R;          // [dk + 1][R]
    double* d_beta = dsc2 + (size_t)2 * (dk + 1) * R;    // [dk][R]
    double* d_coef = dsc2 + (size_t)3 * (dk + 1) * R;    // [R][dk + 1]
    const long ldv = (long)n * R;  // run r's j-th vector at Vd + j * ldv + r * n
    std::vector<unsigned long long> sd{rng_derive(o.seed, kTagDos)};
    gauss_launch(n, R, 1, ring.vec(sd), ring.ptrs(std::vector<double*>{Vd}), n, st);
    ColDotArgs cr;
    cr.n = n;
    cr.ncol0 = R;
    cr.mode = 0;
    cr.partial = static_cast<double*>(ws_get(h, kBufEig, sizeof(double) * coldot_partial_size(n, 1, R)));
    auto dotR = [&](const double* x, const double* y, double* out) {
      ColDotArgs d = cr;
      d.x1 = x;
      d.ldx = n;
      d.y1 = y;
      d.ldy = n;
      d.out1 = out;
      coldot_launch(d, 1, R, st);
    };
    dotR(Vd, Vd, d_s2 + (size_t)dk * R);
    scale_cols_launch(n, R, d_s2 + (size_t)dk * R, Vd, n, Vd, n, nullptr, st);
    for (int j = 0; j < dk; ++j) {
      double* vj = Vd + (size_t)j * ldv;
      apply_H(vj, X2, R);
      dotR(vj, X2, d_alpha + (size_t)j * R);
      std::vector<int> mj(R, j + 1), one(R, 1), nn(R, n);
      std::vector<const double*> bas(R), wc(R), cc(R);
      std::vector<double*> co(R), wo(R);
      for (int r = 0; r < R; ++r) {
        bas[r] = Vd + (size_t)r * n;
        wc[r] = X2 + (size_t)r * n;
        wo[r] = X2 + (size_t)r * n;
        co[r] = d_coef + (size_t)r * (dk + 1);
        cc[r] = d_coef + (size_t)r * (dk + 1);
      }
      for (int pass = 0; pass < 2; ++pass) {  // w_r -= V_r (V_r^T w_r)
        gemm(c, true, false, mj, one, nn, bas, ldv, wc, n, co, dk + 1, 1.0, 0.0);
        gemm(c, false, false, nn, one, mj, bas, ldv, cc, dk + 1, wo, n, -1.0, 1.0);
      }
      dotR(X2, X2, d_s2 + (size_t)j * R);
      scale_cols_launch(n, R, d_s2 + (size_t)j * R, X2, n, Vd + (size_t)(j + 1) * ldv, n,
                        d_beta + (size_t)j * R, st);
    }
    std::vector<double> al((size_t)dk * R), be((size_t)dk * R);
    SL_HIP(hipMemcpyAsync(al.data(), d_alpha, sizeof(double) * al.size(), hipMemcpyDeviceToHost, st));
    SL_HIP(hipMemcpyAsync(be.data(), d_beta, sizeof(double) * be.size(), hipMemcpyDeviceToHost, st));
    SL_HIP(hipStreamSynchronize(st));
    ring.synced();
    // Ritz pairs of the R tridiagonals on the device eigensolver
    SL_CHECK_ARG(dk <= kEigMax, "Lanczos DOS steps must be <= 112");
    std::vector<double> Th((size_t)R * dk * dk, 0.0);
    for (int r = 0; r < R; ++r)
      for (int j = 0; j < dk; ++j) {
        double* T = Th.data() + (size_t)r * dk * dk;
        T[j + (size_t)j * dk] = al[(size_t)j * R + r];
        if (j + 1 < dk) T[(j + 1) + (size_t)j * dk] = T[j + (size_t)(j + 1) * dk] = be[(size_t)j * R + r];
      }
    double* dT = static_cast<double*>(ws_get(h, kBufMisc, sizeof(double) * ((size_t)2 * R * dk * dk + (size_t)R * dk)));
    double* dS = dT + (size_t)R * dk * dk;
    double* dW = dS + (size_t)R * dk * dk;
    SL_HIP(hipMemcpyAsync(dT, Th.data(), sizeof(double) * Th.size(), hipMemcpyHostToDevice, st));
    std::vector<double*> pT(R), pS(R), pW(R);
    for (int r = 0; r < R; ++r) {
      pT[r] = dT + (size_t)r * dk * dk;
      pS[r] = dS + (size_t)r * dk * dk;
      pW[r] = dW + (size_t)r * dk;
    }
    EigArgs e;
    e.m = ring.vec(std::vector<int>(R, dk));
    e.A = ring.cptrs(pT);
    e.lda = dk;
    e.W = ring.ptrs(pW);
    e.V = ring.ptrs(pS);
    e.ldv = dk;
    eig_launch(e, R, dk, st);
    std::vector<double> thv((size_t)R * dk), Sv((size_t)R * dk * dk);
    SL_HIP(hipMemcpyAsync(thv.data(), dW, sizeof(double) * thv.size(), hipMemcpyDeviceToHost, st));
    SL_HIP(hipMemcpyAsync(Sv.data(), dS, sizeof(double) * Sv.size(), hipMemcpyDeviceToHost, st));
    SL_HIP(hipStreamSynchronize(st));
    ring.synced();
    std::vector<double> z2((size_t)R * dk);
    for (int r = 0; r < R; ++r)
      for (int j = 0; j < dk; ++j) {
        const double g = Sv[(size_t)r * dk * dk + (size_t)j * dk];  // first component of vector j
        z2[(size_t)r * dk + j] = g * g;
      }
    const LanczosDos d(thv.data(), z2.data(), dk, R, n);
    dos_plan(d, n_e, n_s, dos_mode, o.top_margin, sig, top);
    if (bounds_out) {
      bounds_out[0] = d.a;
      bounds_out[1] = d.b;
    }
    return SISLICE_OK;
  }
  // ---- spectral bounds: m_b-step Lanczos on H with full reorthogonalisation; the
  // normalisations stay on the device, alpha and beta are read once at the end
  std::vector<unsigned long long> sdb{rng_derive(o.seed, kTagBounds)};
  gauss_launch(n, 1, 1, ring.vec(sdb), ring.ptrs(std::vector<double*>{Vb}), n, st);
  ColDotArgs cd;
  cd.n = n;
  cd.ncol0 = 1;
  cd.mode = 0;
  cd.partial = static_cast<double*>(ws_get(h, kBufEig, sizeof(double) * coldot_partial_size(n, 1, nv)));
  auto dot1 = [&](const double* x, const double* y, double* out) {
    ColDotArgs d = cd;
    d.x1 = x;
    d.ldx = n;
    d.y1 = y;
    d.ldy = n;
    d.out1 = out;
    coldot_launch(d, 1, 1, st);
  };
  double* d_alpha = small + 128;  // [m_b]
  double* d_s2 = small + 192;     // [m_b + 1] squared norms
  double* d_beta = small + 256;   // [m_b]
  SL_CHECK_ARG(m_b <= 60, "bounds_steps too large");
  dot1(Vb, Vb, d_s2 + m_b);
  scale_by_norm_launch(n, d_s2 + m_b, Vb, Vb, nullptr, st);
  for (int j = 0; j < m_b; ++j) {
    double* vj = Vb + (size_t)j * n;
    apply_H(vj, wv, 1);
    if (n <= kLanczosTailMaxN) {
      // alpha, the two Gram-Schmidt passes, beta and the next vector in one workgroup
      lanczos_tail_launch(n, j, Vb, wv, d_alpha, d_s2, d_beta, st);
      continue;
    }
    dot1(vj, wv, d_alpha + j);
    for (int pass = 0; pass < 2; ++pass) {
      // coef = V^T w ; w -= V coef
      gemm(c, true, false, {j + 1}, {1}, {n}, {Vb}, n, {wv}, n, {small + 512}, j + 1, 1.0, 0.0);
      gemm(c, false, false, {n}, {1}, {j + 1}, {Vb}, n, {small + 512}, j + 1, {wv}, n, -1.0, 1.0);
    }
    dot1(wv, wv, d_s2 + j);
    scale_by_norm_launch(n, d_s2 + j, wv, Vb + (size_t)(j + 1) * n, d_beta + j, st);
  }
  std::vector<double> alpha(m_b, 0.0), beta(m_b, 0.0);
  SL_HIP(hipMemcpyAsync(alpha.data(), d_alpha, sizeof(double) * m_b, hipMemcpyDeviceToHost, st));
  SL_HIP(hipMemcpyAsync(beta.data(), d_beta, sizeof(double) * m_b, hipMemcpyDeviceToHost, st));
  SL_HIP(hipStreamSynchronize(st));
  ring.synced();
  int m = m_b;
  for (int j = 0; j < m_b; ++j)
    if (beta[j] == 0.0) {
      m = j + 1;
      break;
    }
  // Ritz values of the tridiagonal T_m on the device eigensolver
  double* Tm = small + 1024;  // m*m, then m Ritz values
  double* Sv = small + 2048;  // m*m
  SL_CHECK_ARG((size_t)m * m + m <= 1024, "bounds_steps too large");
  std::vector<double> Th((size_t)m * m, 0.0);
  for (int j = 0; j < m; ++j) {
    Th[j + (size_t)j * m] = alpha[j];
    if (j + 1 < m) Th[(j + 1) + (size_t)j * m] = Th[j + (size_t)(j + 1) * m] = beta[j];
  }
  SL_HIP(hipMemcpyAsync(Tm, Th.data(), sizeof(double) * m * m, hipMemcpyHostToDevice, st));
  double* thv = Tm + (size_t)m * m;
  {
    EigArgs e;
    e.m = ring.vec(std::vector<int>{m});
    e.A = ring.cptrs(std::vector<double*>{Tm});
    e.lda = m;
    e.W = ring.ptrs(std::vector<double*>{thv});
    e.V = ring.ptrs(std::vector<double*>{Sv});
    e.ldv = m;
    eig_launch(e, 1, m, st);
  }
  std::vector<double> th(m), S((size_t)m * m);
  SL_HIP(hipMemcpyAsync(th.data(), thv, sizeof(double) * m, hipMemcpyDeviceToHost, st));
  SL_HIP(hipMemcpyAsync(S.data(), Sv, sizeof(double) * m * m, hipMemcpyDeviceToHost, st));
  SL_HIP(hipStreamSynchronize(st));
  ring.synced();
  const double rlo = std::fabs(beta[m - 1] * S[(m - 1) + 0 * (size_t)m]);
  const double rhi = std::fabs(beta[m - 1] * S[(m - 1) + (size_t)(m - 1) * m]);
  const double pad = 0.01 * (th[m - 1] - th[0]);
  const double a = th[0] - rlo - pad, bb = th[m - 1] + rhi + pad;
  // ---- Chebyshev moments: doubling identities mu_{2k} = 2<t_k,t_k> - mu_0,
  // mu_{2k+1} = 2<t_{k+1},t_k> - mu_1 with t_k = T_k(H~) v
  const double cc = 0.5 * (a + bb), dd = 0.5 * (bb - a);
  rademacher_launch(n, nv, rng_derive(o.seed, kTagKpm), T0, n, st);
  const int K = M / 2 + 1;  // t_0 .. t_K
  double* dots = small + 4096;  // [2K+2][nv]
  SL_CHECK_ARG((size_t)(2 * K + 2) * nv + 4096 <= 8192, "too many moments for the scratch area");
  ColDotArgs cdv = cd;
  cdv.ncol0 = nv;
  auto dotv = [&](const double* x, const double* y, double* out) {
    ColDotArgs d = cdv;
    d.x1 = x;
    d.ldx = n;
    d.y1 = y;
    d.ldy = n;
    d.out1 = out;
    coldot_launch(d, 1, nv, st);
  };
  // t_next = 2 H~ t_cur - t_prev = (2/d) H t_cur - (2c/d) t_cur - t_prev  (t_1 = H~ t_0)
  auto scaled_step = [&](const double* tcur, const double* tprev, double* tnext, bool first) {
    apply_H(tcur, X2, nv);
    const double f1 = first ? 1.0 / dd : 2.0 / dd;
    const double f2 = first ? -cc / dd : -2.0 * cc / dd;
    lincomb3_launch((long)n * nv, f1, X2, f2, tcur, -1.0, first ? nullptr : tprev, tnext, st);
  };
  double* tp = T0;
  double* tc = T1;
  double* tn = T2;
  dotv(tp, tp, dots + 0 * nv);            // <t0,t0>
  scaled_step(tp, nullptr, tc, true);     // t1
  dotv(tc, tp, dots + 1 * nv);            // <t1,t0>
  for (int k = 1; k < K; ++k) {
    dotv(tc, tc, dots + (2 * k) * nv);    // <t_k,t_k>
    scaled_step(tc, tp, tn, false);       // t_{k+1}
    dotv(tn, tc, dots + (2 * k + 1) * nv);  // <t_{k+1},t_k>
    double* t = tp;
    tp = tc;
    tc = tn;
    tn = t;
  }
  std::vector<double> hd((size_t)(2 * K) * nv);
  SL_HIP(hipMemcpyAsync(hd.data(), dots, sizeof(double) * hd.size(), hipMemcpyDeviceToHost, st));
  int bad = 0;
  SL_HIP(hipMemcpyAsync(&bad, iflag, sizeof(int), hipMemcpyDeviceToHost, st));
  SL_HIP(hipStreamSynchronize(st));
  ring.synced();
  if (bad) throw Error(SISLICE_ERR_ARG, "B is not positive definite");
  auto total = [&](int q) {
    double s = 0.0;
    for (int v = 0; v < nv; ++v) s += hd[(size_t)q * nv + v];
    return s / ((double)n * nv);
  };
  std::vector<double> mu(M, 0.0);
  const double mu0 = total(0), mu1 = total(1);
  mu[0] = mu0;
  if (M > 1) mu[1] = mu1;
  for (int k = 1; 2 * k < M; ++k) {
    mu[2 * k] = 2.0 * total(2 * k) - mu0;
    if (2 * k + 1 < M) mu[2 * k + 1] = 2.0 * total(2 * k + 1) - mu1;
  }
  kpm_place(mu.data(), M, a, bb, n, n_e, n_s, o.top_margin, sig, top);
  if (mom_out)
    for (int k = 0; k < M; ++k) mom_out[k] = mu[k];
  if (bounds_out) {
    bounds_out[0] = a;
    bounds_out[1] = bb;
  }
  return SISLICE_OK;
}

// ---------------------------------------------------------------- solve

DriverWs driver_factor(sislice_handle* h, Ring& ring, int n, const double* A, long lda,
                       const double* B, long ldb, const std::vector<double>& pts, int nb) {
  hipStream_t st = h->stream;
  const int S1 = (int)pts.size();
  Sizer z;
  z.take<double>((size_t)2 * n * n);  // [Af Bf], n x 2n
  for (int s = 0; s < S1; ++s) z.take<double>((size_t)n * n);
  for (int s = 0; s < S1; ++s) z.take<int32_t>(n);
  for (int s = 0; s < S1; ++s) {
    z.take<int>(n);
    z.take<int>(n);
    z.take<double>(solve_linv_size(n));
  }
  z.take<double>(64 * 8);  // norm estimation scratch
  z.take<double>((size_t)n * 8 * 2);
  z.take<int>(64);
  h->fc.id = 0;  // the driver workspace is about to be overwritten
  Carver cv(ws_get(h, kBufDriver, z.off));
  DriverWs w;
  w.Af = cv.take<double>((size_t)2 * n * n);
  w.Bf = w.Af + (size_t)n * n;
  w.LD.resize(S1);
  w.ipv.resize(S1);
  for (int s = 0; s < S1; ++s) w.LD[s] = cv.take<double>((size_t)n * n);
  for (int s = 0; s < S1; ++s) w.ipv[s] = cv.take<int32_t>(n);
  w.perm.resize(S1);
  w.blk.resize(S1);
  w.Linv.resize(S1);
  for (int s = 0; s < S1; ++s) {
    w.perm[s] = cv.take<int>(n);
    w.blk[s] = cv.take<int>(n);
    w.Linv[s] = cv.take<double>(solve_linv_size(n));
  }
  w.nsmall = cv.take<double>(64 * 8);
  w.nX = cv.take<double>((size_t)n * 8 * 2);
  w.nflag = cv.take<int>(64);
  sym_full_launch(n, A, lda, w.Af, n, st);
  sym_full_launch(n, B, ldb, w.Bf, n, st);
  w.fp = build_factor(h, kBufFactor, n, A, lda, B, ldb, S1, pts.data(), w.LD.data(), n, w.ipv.data(),
                      nb, true);
  factor_run(h, w.fp, st);
  w.inert.assign(3 * S1, 0);
  SL_HIP(hipMemcpyAsync(w.inert.data(), w.fp.d_inertia, sizeof(int64_t) * 3 * S1,
                        hipMemcpyDeviceToHost, st));
  SL_HIP(hipStreamSynchronize(st));
  ring.synced();
  for (int s = 0; s < S1; ++s)
    if (w.inert[3 * s + 1] != 0) return w;  // singular: nothing is cached
  // the factorizations stay in the driver workspace for sislice_adjoint
  auto& f = h->fc;
  f.id = ++h->fc_counter;
  f.n = n;
  f.A = A;
  f.B = B;
  f.lda = lda;
  f.ldb = ldb;
  f.Af = w.Af;
  f.pts = pts;
  f.LD = w.LD;
  f.ipv = w.ipv;
  f.perm = w.perm;
  f.blk = w.blk;
  f.Linv = w.Linv;
  f.inertia = w.inert;
  f.prepped.assign(S1, 0);
  return w;
}


sislice_status solve_impl(sislice_handle* h, int64_t n64, const double* A, int64_t lda,
                          const double* B, int64_t ldb, int64_t n_e, int64_t n_s,
                          const double* sigmas_in, double* omega_top_io, const sislice_opts& o,
                          double* evals, double* evecs, int64_t ldx, double* resid_out,
                          sislice_report* rep, const double* start, int32_t* probe_of,
                          int start_cols) {
  const auto t_start = Clock::now();
  const int n = (int)n64;
  const int P = (int)n_s;
  set_current_handle(h);
  prof_reset(h);
  h->prof = o.profile != 0;
  h->prof_mask = (o.profile & 0x100) ? (unsigned)(o.profile & 0x3F) : 0x3Fu;
  h->use_graphs = o.graphs != 0;
  const int b = kLanczosBlock;
  hipStream_t st = h->stream;
  std::vector<double> sig(P);
  double top = 0;
  double t_plan = 0;
  if (!sigmas_in) {
    const auto t0 = Clock::now();
    plan_impl(h, n64, A, lda, B, ldb, n_e, n_s, o, sig.data(), &top, nullptr, nullptr);
    t_plan = ms_since(t0);
  } else {
    for (int j = 0; j < P; ++j) sig[j] = sigmas_in[j];
    top = *omega_top_io;
    for (int j = 1; j < P; ++j) SL_CHECK_ARG(sig[j] > sig[j - 1], "shifts must be ascending");
    SL_CHECK_ARG(top > sig[P - 1], "omega_top must exceed every shift");
  }
  Ring ring(h);
  Ctx c{h, st, &ring};
  const int S1 = P + 1;  // shifts + top boundary
  // ---- 1. factorizations and inertia
  const auto t_f0 = Clock::now();
  std::vector<double> pts(sig);
  pts.push_back(top);
  const int nb = o.nb > 0 ? std::min(o.nb, kMaxNb) : default_nb(n);
  DriverWs dw = driver_factor(h, ring, n, A, lda, B, ldb, pts, nb);
  std::vector<int64_t> inert = dw.inert;
  // Top boundary recovery: fewer than n_e eigenvalues below omega_top (the planner's
  // estimate fell short).  Move the boundary up in doubling steps, refactoring only
  // that point, until the count reaches n_e; the last probe's slice grows with it.
  if (h->fc.id != 0 && inert[3 * P] < n_e) {
    double step = std::max(top - sig[P - 1], 1e-6 * (std::fabs(top) + 1.0));
    for (int tries = 0; tries < 40 && inert[3 * P] < n_e; ++tries) {
      top += step;
      step *= 2.0;
      double* ldp = dw.LD[P];
      int32_t* ipp = dw.ipv[P];
      FactorPlan f1 = build_factor(h, kBufFactor, n, A, lda, B, ldb, 1, &top, &ldp, n, &ipp, nb, true);
      factor_launch(f1, st);
      SL_HIP(hipMemcpyAsync(&inert[3 * P], f1.d_inertia, sizeof(int64_t) * 3, hipMemcpyDeviceToHost, st));
      SL_HIP(hipStreamSynchronize(st));
      ring.synced();
      if (inert[3 * P + 1] != 0) inert[3 * P] = -1;  // exactly singular: step on
    }
    SL_CHECK_ARG(inert[3 * P] >= n_e, "no top boundary with n_e eigenvalues below it");
    pts[P] = top;
    h->fc.pts[P] = top;
    for (int q = 0; q < 3; ++q) h->fc.inertia[3 * P + q] = inert[3 * P + q];
    h->fc.prepped[P] = 0;
  }
  const double t_factor = ms_since(t_f0);
  if (h->fc.id == 0) {  // an exact zero pivot
    if (rep) {
      rep->n_shifts = P;
      rep->t_factor_ms = t_factor;
    }
    return SISLICE_SINGULAR_SHIFT;
  }
  double* Af = dw.Af;
  double* Bf = dw.Bf;
  const std::vector<double*>& LD = dw.LD;
  const std::vector<int32_t*>& ipv = dw.ipv;
  const std::vector<int*>& perm = dw.perm;
  const std::vector<int*>& blk = dw.blk;
  const std::vector<double*>& Linv = dw.Linv;
  double* nsmall = dw.nsmall;
  double* nX = dw.nX;
  int* nflag = dw.nflag;
  const FactorPlan& fp = dw.fp;
  std::vector<int64_t> nu(P);
  for (int s = 0; s < P; ++s) nu[s] = inert[3 * s];
  const int64_t nu_top = inert[3 * P];
  for (int s = 1; s < P; ++s) SL_CHECK_ARG(nu[s] >= nu[s - 1], "inertia not monotone");
  if (rep) {
    rep->n_shifts = P;
    rep->nu_top = nu_top;
    rep->omega_top = top;
    rep->flops_factor = (double)S1 * (double)n * n * n / 3.0;
    if (rep->nu)
      for (int s = 0; s < P; ++s) rep->nu[s] = nu[s];
  }
  *omega_top_io = top;
  // solve preparation for the probe shifts
  solve_prep_launch(n, P, reinterpret_cast<const int* const*>(ring.ptrs(std::vector<int32_t*>(ipv.begin(), ipv.begin() + P))),
                    ring.ptrs(std::vector<int*>(perm.begin(), perm.begin() + P)),
                    ring.ptrs(std::vector<int*>(blk.begin(), blk.begin() + P)),
                    ring.cptrs(std::vector<double*>(LD.begin(), LD.begin() + P)), n,
                    ring.ptrs(std::vector<double*>(Linv.begin(), Linv.begin() + P)), st);
  for (int s = 0; s < P; ++s) h->fc.prepped[s] = 1;
  if (rep) rep->factor_id = h->fc.id;
  // ||A||_2 and ||B||_2 estimates
  std::vector<int> one{1};
  int* active1 = ring.vec(one);
  const double anorm = sym_norm2(c, n, Af, nX, nX + (size_t)n * 8, nsmall, nsmall + 64, nsmall + 128,
                                 nsmall + 192, nsmall + 256, nflag, active1, o.seed);
  active1 = ring.vec(one);
  const double bnorm = sym_norm2(c, n, Bf, nX, nX + (size_t)n * 8, nsmall, nsmall + 64, nsmall + 128,
                                 nsmall + 192, nsmall + 256, nflag, active1, o.seed ^ 0x5A5Aull);
  if (rep) rep->anorm = anorm;
  // ---- 2. the probes: block shift-invert Lanczos (reading R1), or the paper's
  // subspace iteration (Algorithm 2); both hand their Ritz pairs, in chunks of
  // at most kEigMax per probe, to the validation
  struct Chunk {
    int probe, off, cnt;
    std::vector<int> cols;
  };
  std::vector<Chunk> chunks;
  int NL = 0;
  std::vector<double> vals, ress;
  double* Xf = nullptr;
  int block_steps = 0, cycles_max = 0;
  double bytes_solve = 0.0;
  double t_lanczos = 0.0, t_rr = 0.0;
  if (o.driver == 1) {
    const auto t_s0 = Clock::now();
    std::vector<SubspaceProbe> sp(P);
    int64_t max_need = 0;
    for (int j = 0; j < P; ++j) {
      auto& q = sp[j];
      q.sigma = sig[j];
      q.lo = j > 0 ? sig[j - 1] : -std::numeric_limits<double>::infinity();
      q.hi = j + 1 < P ? sig[j + 1] : top;
      const int64_t nlo = j > 0 ? nu[j - 1] : 0;
      const int64_t nhi = j + 1 < P ? nu[j + 1] : nu_top;
      q.need = nhi - nlo;
      max_need = std::max(max_need, q.need);
      q.LD = LD[j];
      q.perm = perm[j];
      q.blk = blk[j];
      q.Linv = Linv[j];
    }
    const int k = std::min(subspace_dim(max_need), n);
    SubspaceOut so = subspace_probes(c, n, Af, Bf, sp, anorm, o, k, o.subspace_iters, start,
                                     start_cols, 0, n);
    for (int j = 0; j < P; ++j) {
      Chunk ch;
      ch.probe = j;
      ch.off = NL;
      ch.cnt = k;
      for (int i = 0; i < k; ++i) ch.cols.push_back(i);
      NL += k;
      chunks.push_back(std::move(ch));
    }
    vals = so.vals;
    ress = so.ress;
    Xf = so.X;
    block_steps = so.applications;
    cycles_max = so.rounds_max;
    bytes_solve = so.bytes_solve;
    t_lanczos = ms_since(t_s0);
  } else {
    // ---- 2. block Lanczos per probe
    const auto t_l0 = Clock::now();
    std::vector<ProbeHost> pr(P);
    int64_t max_need = 0;
    for (int j = 0; j < P; ++j) {
      pr[j].sigma = sig[j];
      pr[j].lo = j > 0 ? sig[j - 1] : -std::numeric_limits<double>::infinity();
      pr[j].hi = j + 1 < P ? sig[j + 1] : top;
      const int64_t nlo = j > 0 ? nu[j - 1] : 0;
      const int64_t nhi = j + 1 < P ? nu[j + 1] : nu_top;
      pr[j].need = nhi - nlo;
      max_need = std::max(max_need, pr[j].need);
    }
    // locked capacity: the values a probe needs plus room for deflated pairs
    const int LC = (int)std::min<int64_t>(n, 2 * max_need + 16);
    int MB = o.max_basis;
    while (MB > 16 && MB + 2 * b + LC > n) MB -= b;
    const int QC = MB + 2 * b;
    // thick restart: keep the Ritz vectors nearest the shift and add four blocks per
    // cycle (measured against six and two: fewer Lanczos steps without more cycles)
    const int kkeep_max = std::max(b, MB - 4 * b);
    Sizer zl;
    zl.take<double>((size_t)n * b * P);  // W_all
    zl.take<double>((size_t)n * b * P);  // Z_all
    for (int j = 0; j < P; ++j) {
      zl.take<double>((size_t)n * QC);  // Q
      zl.take<double>((size_t)n * QC);  // UQ
      zl.take<double>((size_t)n * LC);  // L
      zl.take<double>((size_t)n * LC);  // UL
      zl.take<double>((size_t)n * MB);  // Xt
      zl.take<double>((size_t)n * MB);  // Ut
      zl.take<double>((size_t)n * b);   // solve scratch Z
      zl.take<double>((size_t)n * b);   // solve scratch V
      zl.take<double>((size_t)QC * QC);  // T
      zl.take<double>((size_t)QC * QC);  // S (eigvecs)
      zl.take<double>((size_t)QC * QC);  // S lock sel
      zl.take<double>((size_t)QC * QC);  // S keep sel
      zl.take<double>((size_t)QC * b);   // CQ
      zl.take<double>((size_t)LC * b);   // CL
      zl.take<double>(4 * b * b);        // G, R1, R2, Rt
      zl.take<int>(2 * QC);              // idx lock / keep
    }
    zl.take<double>((size_t)2 * QC * P);  // theta, est of every probe (one readback)
    zl.take<int>(P);  // flags
    const int ts_mmax = std::max(LC, QC);
    zl.take<double>(tsmt_partial_size(n, 2 * P, ts_mmax));  // tall-skinny partials
    Carver cl(ws_get(h, kBufLanczos, zl.off));
    double* Wall = cl.take<double>((size_t)n * b * P);
    double* Zall = cl.take<double>((size_t)n * b * P);
    struct ProbeDev {
      double *Q, *UQ, *L, *UL, *Xt, *Ut, *Zs, *Vs, *T, *S, *SL, *SK, *th, *est, *CQ, *CL, *G, *R1, *R2, *Rt;
      int *il, *ik;
    };
    std::vector<ProbeDev> pd(P);
    for (int j = 0; j < P; ++j) {
      auto& d = pd[j];
      d.Q = cl.take<double>((size_t)n * QC);
      d.UQ = cl.take<double>((size_t)n * QC);
      d.L = cl.take<double>((size_t)n * LC);
      d.UL = cl.take<double>((size_t)n * LC);
      d.Xt = cl.take<double>((size_t)n * MB);
      d.Ut = cl.take<double>((size_t)n * MB);
      d.Zs = cl.take<double>((size_t)n * b);
      d.Vs = cl.take<double>((size_t)n * b);
      d.T = cl.take<double>((size_t)QC * QC);
      d.S = cl.take<double>((size_t)QC * QC);
      d.SL = cl.take<double>((size_t)QC * QC);
      d.SK = cl.take<double>((size_t)QC * QC);
      d.CQ = cl.take<double>((size_t)QC * b);
      d.CL = cl.take<double>((size_t)LC * b);
      double* g4 = cl.take<double>(4 * b * b);
      d.G = g4;
      d.R1 = g4 + b * b;
      d.R2 = g4 + 2 * b * b;
      d.Rt = g4 + 3 * b * b;
      int* ii = cl.take<int>(2 * QC);
      d.il = ii;
      d.ik = ii + QC;
    }
    // the Ritz values and estimates of all probes side by side, read back in one copy
    double* thest = cl.take<double>((size_t)2 * QC * P);
    for (int j = 0; j < P; ++j) {
      pd[j].th = thest + (size_t)2 * QC * j;
      pd[j].est = pd[j].th + QC;
    }
    int* dflags = cl.take<int>(P);
    double* tspart = cl.take<double>(tsmt_partial_size(n, 2 * P, ts_mmax));
    for (int j = 0; j < P; ++j) SL_HIP(hipMemsetAsync(pd[j].T, 0, sizeof(double) * QC * QC, st));
    unsigned* sync = sync_words(h, (size_t)P + 64);  // one ticket counter per probe
    auto Wj = [&](int j) { return Wall + (size_t)j * n * b; };
    auto Zj = [&](int j) { return Zall + (size_t)j * n * b; };
    // start blocks: Gaussian from the shared stream, or the caller's (warm start),
    // B-orthonormalised (CholeskyQR2)
    if (start) {
      SL_HIP(hipMemcpyAsync(Wall, start, sizeof(double) * (size_t)n * b * P, hipMemcpyDeviceToDevice, st));
    } else {
      std::vector<unsigned long long> seeds(P);
      std::vector<double*> wp(P);
      for (int j = 0; j < P; ++j) {
        seeds[j] = rng_derive(o.seed, kTagLanczos ^ ((uint64_t)j << 32));
        wp[j] = Wj(j);
      }
      gauss_launch(n, b, P, ring.vec(seeds), ring.ptrs(wp), n, st);
    }
    std::vector<int> all(P);
    std::iota(all.begin(), all.end(), 0);
    auto act_vec = [&](const auto& js, auto f) {
      using T = decltype(f(js[0]));
      std::vector<T> v;
      v.reserve(js.size());
      for (const auto& j : js) v.push_back(f(j));
      return v;
    };
    auto cholqr2 = [&](const std::vector<int>& js, const std::vector<double*>& Vin,
                       const std::vector<double*>& Uin, long ldin, const std::vector<double*>& Vout,
                       const std::vector<double*>& Uout, bool coupling) {
      const int na = (int)js.size();
      std::vector<int> ones(na, 1), bs(na, b), ns(na, n);
      std::vector<const double*> cV(Vin.begin(), Vin.end()), cU(Uin.begin(), Uin.end());
      auto gram = [&](const std::vector<const double*>& Vv, const std::vector<const double*>& Uv, long ld) {
        TsArgs ta;
        ta.n = n;
        ta.m = ring.vec(bs);
        ta.V = ring.cptrs(Vv);
        ta.ldv = ld;
        ta.X = ring.cptrs(Uv);
        ta.ldx = ld;
        ta.C = ring.ptrs(act_vec(js, [&](int j) { return pd[j].G; }));
        ta.ldc = b;
        ta.partial = tspart;
        tsmt_launch(ta, na, b, st);
      };
      gram(cV, cU, ldin);
      CholQrArgs q;
      q.n = n;
      q.active = ring.vec(ones);
      q.G = ring.cptrs(act_vec(js, [&](int j) { return pd[j].G; }));
      q.Vin = ring.cptrs(Vin);
      q.Uin = ring.cptrs(Uin);
      q.ldin = ldin;
      q.Vout = ring.ptrs(Vout);
      q.Uout = ring.ptrs(Uout);
      q.ldout = n;
      q.R = ring.ptrs(act_vec(js, [&](int j) { return pd[j].R1; }));
      q.flag = dflags;  // indexed by position; only read when all probes are active
      cholqr_launch(q, na, st);
      std::vector<const double*> cVo(Vout.begin(), Vout.end()), cUo(Uout.begin(), Uout.end());
      gram(cVo, cUo, n);
      q.Vin = ring.cptrs(Vout);
      q.Uin = ring.cptrs(Uout);
      q.ldin = n;
      q.R = ring.ptrs(act_vec(js, [&](int j) { return pd[j].R2; }));
      cholqr_launch(q, na, st);
      if (coupling) {
        CouplingArgs ca;
        ca.active = ring.vec(ones);
        ca.R1 = ring.cptrs(act_vec(js, [&](int j) { return pd[j].R1; }));
        ca.R2 = ring.cptrs(act_vec(js, [&](int j) { return pd[j].R2; }));
        ca.Rt = ring.ptrs(act_vec(js, [&](int j) { return pd[j].Rt; }));
        ca.T = ring.ptrs(act_vec(js, [&](int j) { return pd[j].T; }));
        ca.ldt = QC;
        ca.row0 = ring.vec(act_vec(js, [&](int j) { return pr[j].mq; }));
        coupling_launch(ca, na, st);
      }
    };
    // Z = B W, then B-orthonormalise into Q[:, 0:8]
    gemm(c, false, false, {n}, {b * P}, {n}, {Bf}, n, {Wall}, n, {Zall}, n, 1.0, 0.0);
    cholqr2(all, act_vec(all, Wj), act_vec(all, Zj), n, act_vec(all, [&](int j) { return pd[j].Q; }),
            act_vec(all, [&](int j) { return pd[j].UQ; }), false);
    for (int j = 0; j < P; ++j) pr[j].mq = b;
    // slice bookkeeping
    std::vector<int64_t> n_exact(P + 1);
    for (int s = 0; s <= P; ++s) {
      const int64_t lo = s == 0 ? 0 : nu[s - 1];
      const int64_t hi = s == P ? nu_top : nu[s];
      n_exact[s] = hi - lo;
    }
    auto slice_done = [&](int s) {
      int64_t cnt = 0;
      if (s == 0) {
        for (double v : pr[0].lock_lam) cnt += v < sig[0];
      } else if (s == P) {
        for (double v : pr[P - 1].lock_lam) cnt += v >= sig[P - 1] && v < top;
      } else {
        const double lo = sig[s - 1], hi = sig[s], tau = 0.5 * (lo + hi);
        for (double v : pr[s - 1].lock_lam) cnt += v >= lo && v <= tau;
        for (double v : pr[s].lock_lam) cnt += v > tau && v < hi;
      }
      return cnt >= n_exact[s];
    };
    const double lock_tol = o.tol / 100.0;
    for (int cyc = 0; cyc < o.max_cycles; ++cyc) {
      std::vector<int> act;
      for (int j = 0; j < P; ++j)
        if (pr[j].active) act.push_back(j);
      if (act.empty()) break;
      // ---- steps until every active probe's basis is full
      while (true) {
        std::vector<int> js;
        for (int j : act)
          if (pr[j].mq <= MB) js.push_back(j);  // the projected order mq - b stays <= MB
        if (js.empty()) break;
        const int na = (int)js.size();
        block_steps += na;
        for (int j : js) pr[j].steps++;
        // a. W_j = (A - sigma_j B)^{-1} U_j[:, last block]
        SolveArgs sa;
        sa.n = n;
        sa.nshift = na;
        sa.nrhs = b;
        sa.epoch = next_epoch(h);
        sa.LD = ring.cptrs(act_vec(js, [&](int j) { return LD[j]; }));
        sa.ldld = n;
        sa.perm = ring.cptrs(act_vec(js, [&](int j) { return perm[j]; }));
        sa.blk = ring.cptrs(act_vec(js, [&](int j) { return blk[j]; }));
        sa.Linv = ring.cptrs(act_vec(js, [&](int j) { return Linv[j]; }));
        sa.Y = ring.cptrs(act_vec(js, [&](int j) { return pd[j].UQ + (size_t)(pr[j].mq - b) * n; }));
        sa.ldy = n;
        sa.X = ring.ptrs(act_vec(js, Wj));
        sa.ldx = n;
        sa.Z = ring.ptrs(act_vec(js, [&](int j) { return pd[j].Zs; }));
        sa.V = ring.ptrs(act_vec(js, [&](int j) { return pd[j].Vs; }));
        sa.ldz = n;
        sa.ctr = sync;
        solve_launch(sa, st, 0);
        bytes_solve += 8.0 * (double)n * (double)n * na;
        // b. full B-reorthogonalisation, twice; T's new column block from the projections
        const auto vb = std::vector<int>(na, b);
        const auto vn = std::vector<int>(na, n);
        const auto vmq = act_vec(js, [&](int j) { return pr[j].mq; });
        const auto vnl = act_vec(js, [&](int j) { return pr[j].nl; });
        const auto pW = act_vec(js, [&](int j) { return (const double*)Wj(j); });
        const auto pWm = act_vec(js, Wj);
        // one tall-skinny launch computes both projections (locked basis: CL = UL^T W,
        // active basis: CQ = UQ^T W) and one applies W -= L CL + Q CQ
        std::vector<int> m_lq(vnl);
        m_lq.insert(m_lq.end(), vmq.begin(), vmq.end());
        std::vector<int> ld_lq(na, LC);
        ld_lq.insert(ld_lq.end(), na, QC);
        std::vector<const double*> v_lq = act_vec(js, [&](int j) { return (const double*)pd[j].UL; });
        for (int j : js) v_lq.push_back(pd[j].UQ);
        std::vector<const double*> x_lq(pW);
        x_lq.insert(x_lq.end(), pW.begin(), pW.end());
        std::vector<double*> c_lq = act_vec(js, [&](int j) { return pd[j].CL; });
        for (int j : js) c_lq.push_back(pd[j].CQ);
        int mtot = 0;
        for (int q = 0; q < na; ++q) mtot = std::max(mtot, vnl[q] + vmq[q]);
        for (int pass = 0; pass < 2; ++pass) {
          TsArgs ta;
          ta.n = n;
          ta.m = ring.vec(m_lq);
          ta.V = ring.cptrs(v_lq);
          ta.ldv = n;
          ta.X = ring.cptrs(x_lq);
          ta.ldx = n;
          ta.C = ring.ptrs(c_lq);
          ta.ldcb = ring.vec(ld_lq);
          ta.partial = tspart;
          tsmt_launch(ta, 2 * na, ts_mmax, st);
          TsArgs tm;
          tm.n = n;
          tm.m = ring.vec(vnl);
          tm.V = ring.cptrs(act_vec(js, [&](int j) { return (const double*)pd[j].L; }));
          tm.ldv = n;
          tm.C = ring.ptrs(act_vec(js, [&](int j) { return pd[j].CL; }));
          tm.ldc = LC;
          tm.m2 = ring.vec(vmq);
          tm.V2 = ring.cptrs(act_vec(js, [&](int j) { return (const double*)pd[j].Q; }));
          tm.ldv2 = n;
          tm.C2 = ring.cptrs(act_vec(js, [&](int j) { return (const double*)pd[j].CQ; }));
          tm.ldc2 = QC;
          tm.Y = ring.ptrs(pWm);
          tm.ldy = n;
          tm.alpha = -1.0;
          tm.beta = 1.0;
          tsmm_launch(tm, na, mtot, st);
          TWriteArgs tw;
          tw.T = ring.ptrs(act_vec(js, [&](int j) { return pd[j].T; }));
          tw.ldt = QC;
          tw.S = ring.cptrs(act_vec(js, [&](int j) { return pd[j].CQ; }));
          tw.lds = QC;
          tw.rows = ring.vec(vmq);
          tw.r0 = ring.vec(std::vector<int>(na, 0));
          tw.c0 = ring.vec(act_vec(js, [&](int j) { return pr[j].mq - b; }));
          tw.cols = b;
          tw.add = pass;
          twrite_launch(tw, na, st);
        }
        // c. Z = B W for every probe in one GEMM (inactive blocks are recomputed harmlessly)
        gemm(c, false, false, {n}, {b * P}, {n}, {Bf}, n, {Wall}, n, {Zall}, n, 1.0, 0.0);
        // d. CholeskyQR2 into the next block; coupling block of T
        cholqr2(js, pWm, act_vec(js, Zj), n, act_vec(js, [&](int j) { return pd[j].Q + (size_t)pr[j].mq * n; }),
                act_vec(js, [&](int j) { return pd[j].UQ + (size_t)pr[j].mq * n; }), true);
        for (int j : js) pr[j].mq += b;
      }
      // ---- cycle end: Ritz pairs of T, estimates, locking and thick restart
      const int na = (int)act.size();
      const auto vmt = act_vec(act, [&](int j) { return pr[j].mq - b; });
      int mtmax = 0;
      for (int v : vmt) mtmax = std::max(mtmax, v);
      EigArgs e;
      e.m = ring.vec(vmt);
      e.A = ring.cptrs(act_vec(act, [&](int j) { return pd[j].T; }));
      e.lda = QC;
      e.W = ring.ptrs(act_vec(act, [&](int j) { return pd[j].th; }));
      e.V = ring.ptrs(act_vec(act, [&](int j) { return pd[j].S; }));
      e.ldv = QC;
      eig_launch(e, na, mtmax, st);
      RitzEstArgs re;
      re.mt = ring.vec(vmt);
      re.S = ring.cptrs(act_vec(act, [&](int j) { return pd[j].S; }));
      re.lds = QC;
      re.Rt = ring.cptrs(act_vec(act, [&](int j) { return pd[j].Rt; }));
      re.est = ring.ptrs(act_vec(act, [&](int j) { return pd[j].est; }));
      ritz_est_launch(re, na, st);
      // one copy into pinned staging (every probe's theta and est) instead of two
      // pageable copies per probe, each of which waits for the device
      double* hte = static_cast<double*>(host_stage(h, sizeof(double) * 2 * QC * P));
      SL_HIP(hipMemcpyAsync(hte, thest, sizeof(double) * 2 * QC * P, hipMemcpyDeviceToHost, st));
      SL_HIP(hipStreamSynchronize(st));
      std::vector<std::vector<double>> th(na), es(na);
      for (int q = 0; q < na; ++q) {
        const double* src = hte + (size_t)2 * QC * act[q];
        th[q].assign(src, src + QC);
        es[q].assign(src + QC, src + 2 * QC);
      }
      ring.synced();
      std::vector<std::vector<int>> lk(na), kp(na);
      std::vector<std::vector<double>> thk(na);
      for (int q = 0; q < na; ++q) {
        const int j = act[q];
        auto& p = pr[j];
        p.cycles++;
        const int mt = vmt[q];
        const double scale = (anorm + std::fabs(p.sigma) * bnorm) / anorm;
        std::vector<int> rest;
        for (int i = 0; i < mt; ++i) {
          const double t = th[q][i];
          if (t == 0.0 || !std::isfinite(t)) continue;
          const double lam = p.sigma + 1.0 / t;
          const double r = es[q][i] / std::fabs(t) * scale;
          // Converged pairs are locked.  Inside the window they count toward the
          // probe's slices.  Outside it they deflate: they are the pairs nearest to
          // the shift and would otherwise fill the kept restart vectors for good,
          // crowding out farther values the window still needs.  Room stays reserved
          // for the values still missing from the window.
          const bool inwin = lam > p.lo && lam < p.hi;
          const int used = p.nl + (int)lk[q].size();
          const int64_t missing = std::max<int64_t>(0, p.need - p.nin);
          if (r <= lock_tol && inwin && used < LC) {
            lk[q].push_back(i);
            p.lock_lam.push_back(lam);
            ++p.nin;
          } else if (r <= lock_tol && !inwin && used + missing < LC) {
            lk[q].push_back(i);
            p.lock_lam.push_back(lam);
          } else {
            rest.push_back(i);
          }
        }
        std::stable_sort(rest.begin(), rest.end(),
                         [&](int x, int y) { return std::fabs(th[q][x]) > std::fabs(th[q][y]); });
        const int kk = std::min<int>((int)rest.size(), kkeep_max);
        kp[q].assign(rest.begin(), rest.begin() + kk);
        for (int i : kp[q]) thk[q].push_back(th[q][i]);
      }
      // device: select columns, lock GEMMs, keep GEMMs, move newest block, reset T
      std::vector<int> nlk(na), nkp(na), rows(na);
      for (int q = 0; q < na; ++q) {
        nlk[q] = (int)lk[q].size();
        nkp[q] = (int)kp[q].size();
        rows[q] = vmt[q];
      }
      std::vector<int*> il_ptr(na), ik_ptr(na);
      for (int q = 0; q < na; ++q) {
        il_ptr[q] = ring.vec(lk[q]);
        ik_ptr[q] = ring.vec(kp[q]);
      }
      SelectArgs sl;
      sl.count = ring.vec(nlk);
      sl.rows = ring.vec(rows);
      sl.in = ring.cptrs(act_vec(act, [&](int j) { return pd[j].S; }));
      sl.ldi = QC;
      sl.out = ring.ptrs(act_vec(act, [&](int j) { return pd[j].SL; }));
      sl.ldo = QC;
      sl.idx = ring.cptrs(il_ptr);
      select_launch(sl, na, (long)QC * QC, st);
      SelectArgs sk = sl;
      sk.count = ring.vec(nkp);
      sk.out = ring.ptrs(act_vec(act, [&](int j) { return pd[j].SK; }));
      sk.idx = ring.cptrs(ik_ptr);
      select_launch(sk, na, (long)QC * QC, st);
      const auto vn = std::vector<int>(na, n);
      gemm(c, false, false, vn, nlk, vmt, act_vec(act, [&](int j) { return (const double*)pd[j].Q; }), n,
           act_vec(act, [&](int j) { return (const double*)pd[j].SL; }), QC,
           act_vec(act, [&](int j) { return pd[j].L + (size_t)pr[j].nl * n; }), n, 1.0, 0.0);
      gemm(c, false, false, vn, nlk, vmt, act_vec(act, [&](int j) { return (const double*)pd[j].UQ; }), n,
           act_vec(act, [&](int j) { return (const double*)pd[j].SL; }), QC,
           act_vec(act, [&](int j) { return pd[j].UL + (size_t)pr[j].nl * n; }), n, 1.0, 0.0);
      gemm(c, false, false, vn, nkp, vmt, act_vec(act, [&](int j) { return (const double*)pd[j].Q; }), n,
           act_vec(act, [&](int j) { return (const double*)pd[j].SK; }), QC,
           act_vec(act, [&](int j) { return pd[j].Xt; }), n, 1.0, 0.0);
      gemm(c, false, false, vn, nkp, vmt, act_vec(act, [&](int j) { return (const double*)pd[j].UQ; }), n,
           act_vec(act, [&](int j) { return (const double*)pd[j].SK; }), QC,
           act_vec(act, [&](int j) { return pd[j].Ut; }), n, 1.0, 0.0);
      CopyArgs cp;
      cp.n = n;
      cp.ncol = ring.vec(std::vector<int>(na, b));
      cp.lds = n;
      cp.ldd = n;
      cp.src = ring.cptrs(act_vec(act, [&](int j) { return pd[j].Q + (size_t)(pr[j].mq - b) * n; }));
      cp.dst = ring.ptrs([&] {
        std::vector<double*> v;
        for (int q = 0; q < na; ++q) v.push_back(pd[act[q]].Q + (size_t)nkp[q] * n);
        return v;
      }());
      copy_launch(cp, na, b, st);
      cp.src = ring.cptrs(act_vec(act, [&](int j) { return pd[j].UQ + (size_t)(pr[j].mq - b) * n; }));
      cp.dst = ring.ptrs([&] {
        std::vector<double*> v;
        for (int q = 0; q < na; ++q) v.push_back(pd[act[q]].UQ + (size_t)nkp[q] * n);
        return v;
      }());
      copy_launch(cp, na, b, st);
      cp.ncol = ring.vec(nkp);
      cp.src = ring.cptrs(act_vec(act, [&](int j) { return pd[j].Xt; }));
      cp.dst = ring.ptrs(act_vec(act, [&](int j) { return pd[j].Q; }));
      copy_launch(cp, na, kkeep_max, st);
      cp.src = ring.cptrs(act_vec(act, [&](int j) { return pd[j].Ut; }));
      cp.dst = ring.ptrs(act_vec(act, [&](int j) { return pd[j].UQ; }));
      copy_launch(cp, na, kkeep_max, st);
      std::vector<double*> thp(na);
      for (int q = 0; q < na; ++q) thp[q] = ring.vec(thk[q]);
      TResetArgs tr;
      tr.active = ring.vec(std::vector<int>(na, 1));
      tr.T = ring.ptrs(act_vec(act, [&](int j) { return pd[j].T; }));
      tr.ldt = QC;
      tr.dim = QC;
      tr.k = ring.vec(nkp);
      tr.theta = ring.cptrs(thp);
      treset_launch(tr, na, st);
      for (int q = 0; q < na; ++q) {
        auto& p = pr[act[q]];
        p.nl += nlk[q];
        p.mq = nkp[q] + b;
      }
      // probe activity from slice completion
      std::vector<bool> done(P + 1);
      for (int s = 0; s <= P; ++s) done[s] = slice_done(s);
      for (int j = 0; j < P; ++j) {
        pr[j].active = !(done[j] && done[j + 1]) && pr[j].nl < LC;
        cycles_max = std::max(cycles_max, pr[j].cycles);
      }
    }
    SL_HIP(hipStreamSynchronize(st));
    ring.synced();
    t_lanczos = ms_since(t_l0);
    // ---- 3. explicit Rayleigh-Ritz with A on the locked vectors, residuals
    const auto t_r0 = Clock::now();
    for (int j = 0; j < P; ++j) {
      std::vector<int> ord(pr[j].nl);
      std::iota(ord.begin(), ord.end(), 0);
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return pr[j].lock_lam[x] < pr[j].lock_lam[y]; });
      for (int s0 = 0; s0 < (int)ord.size(); s0 += kEigMax) {
        Chunk ch;
        ch.probe = j;
        ch.off = NL;
        ch.cnt = std::min<int>(kEigMax, (int)ord.size() - s0);
        ch.cols.assign(ord.begin() + s0, ord.begin() + s0 + ch.cnt);
        NL += ch.cnt;
        chunks.push_back(std::move(ch));
      }
    }
    const int NC = (int)chunks.size();
    vals.assign(NL, 0.0);
    ress.assign(NL, 0.0);
    double *Xa = nullptr, *AXa = nullptr, *BXa = nullptr, *AXf = nullptr, *BXf = nullptr,
           *Hm = nullptr, *Om = nullptr, *Ym = nullptr, *rr = nullptr, *xn = nullptr;
    constexpr int kRrMats = 6;  // G, its eigenvectors U, U w^{-1/2}, S = G^{-1/2}, S H, S H S
    const size_t e2 = (size_t)kEigMax * kEigMax;
    if (NL > 0) {
      Sizer zr;
      for (int q = 0; q < 6; ++q) zr.take<double>((size_t)n * NL);
      zr.take<double>((size_t)NC * kEigMax * kEigMax);
      zr.take<double>((size_t)NC * kEigMax);
      zr.take<double>((size_t)NC * kEigMax * kEigMax);
      zr.take<double>(NL);
      zr.take<double>(NL);
      zr.take<double>((size_t)NC * kRrMats * e2);
      zr.take<double>((size_t)NC * kEigMax);
      zr.take<double>((size_t)NC * e2);
      Carver cr(ws_get(h, kBufEig, zr.off));
      Xa = cr.take<double>((size_t)n * NL);
      AXa = cr.take<double>((size_t)n * NL);
      BXa = cr.take<double>((size_t)n * NL);
      Xf = cr.take<double>((size_t)n * NL);
      AXf = cr.take<double>((size_t)n * NL);
      BXf = cr.take<double>((size_t)n * NL);
      Hm = cr.take<double>((size_t)NC * kEigMax * kEigMax);
      Om = cr.take<double>((size_t)NC * kEigMax);
      Ym = cr.take<double>((size_t)NC * kEigMax * kEigMax);
      rr = cr.take<double>(NL);
      xn = cr.take<double>(NL);
      double* Gm = cr.take<double>((size_t)NC * kRrMats * e2);
      double* Gw = cr.take<double>((size_t)NC * kEigMax);
      double* Y2 = cr.take<double>((size_t)NC * e2);
      std::vector<int> cnts(NC), rowsn(NC, n);
      std::vector<int*> idxp(NC);
      for (int q = 0; q < NC; ++q) {
        cnts[q] = chunks[q].cnt;
        idxp[q] = ring.vec(chunks[q].cols);
      }
      SelectArgs sx;
      sx.count = ring.vec(cnts);
      sx.rows = ring.vec(rowsn);
      sx.in = ring.cptrs(act_vec(chunks, [&](const Chunk& ch) { return pd[ch.probe].L; }));
      sx.ldi = n;
      sx.out = ring.ptrs(act_vec(chunks, [&](const Chunk& ch) { return Xa + (size_t)ch.off * n; }));
      sx.ldo = n;
      sx.idx = ring.cptrs(idxp);
      select_launch(sx, NC, (long)n * kEigMax, st);
      gemm(c, false, false, {n}, {NL}, {n}, {Af}, n, {Xa}, n, {AXa}, n, 1.0, 0.0);
      gemm(c, false, false, {n}, {NL}, {n}, {Bf}, n, {Xa}, n, {BXa}, n, 1.0, 0.0);
      auto cX = act_vec(chunks, [&](const Chunk& ch) { return (const double*)(Xa + (size_t)ch.off * n); });
      auto cAX = act_vec(chunks, [&](const Chunk& ch) { return (const double*)(AXa + (size_t)ch.off * n); });
      auto cBX = act_vec(chunks, [&](const Chunk& ch) { return (const double*)(BXa + (size_t)ch.off * n); });
      std::vector<double*> pH(NC), pO(NC), pY(NC);
      for (int q = 0; q < NC; ++q) {
        pH[q] = Hm + (size_t)q * kEigMax * kEigMax;
        pO[q] = Om + (size_t)q * kEigMax;
        pY[q] = Ym + (size_t)q * kEigMax * kEigMax;
      }
      gemm(c, true, false, cnts, cnts, rowsn, cX, n, cAX, n, pH, kEigMax, 1.0, 0.0);
      int cmax = 0;
      for (int v : cnts) cmax = std::max(cmax, v);
      // The locked vectors are B-orthonormal only up to the drift of many restart
      // cycles (the deflation-locked ones in particular), and a standard
      // Rayleigh-Ritz step would carry that drift into the residuals.  The
      // symmetric orthonormalisation S = G^{-1/2} of G = X^T B X (from the
      // eigenpairs of G, which is close to the identity) makes the step the exact
      // generalized one: eig(S H S) = (Omega, Y), Ritz vectors X S Y.
      std::vector<double*> pG(NC), pU(NC), pUs(NC), pS(NC), pT(NC), pH2(NC), pGw(NC), pY2(NC);
      for (int q = 0; q < NC; ++q) {
        double* g0 = Gm + (size_t)q * kRrMats * e2;
        pG[q] = g0;
        pU[q] = g0 + e2;
        pUs[q] = g0 + 2 * e2;
        pS[q] = g0 + 3 * e2;
        pT[q] = g0 + 4 * e2;
        pH2[q] = g0 + 5 * e2;
        pGw[q] = Gw + (size_t)q * kEigMax;
        pY2[q] = Y2 + (size_t)q * e2;
      }
      auto cc = [](const std::vector<double*>& v) { return std::vector<const double*>(v.begin(), v.end()); };
      gemm(c, true, false, cnts, cnts, rowsn, cX, n, cBX, n, pG, kEigMax, 1.0, 0.0);
      EigArgs eg;
      eg.m = ring.vec(cnts);
      eg.A = ring.cptrs(pG);
      eg.lda = kEigMax;
      eg.W = ring.ptrs(pGw);
      eg.V = ring.ptrs(pU);
      eg.ldv = kEigMax;
      eig_launch(eg, NC, cmax, st);
      for (int q = 0; q < NC; ++q)
        scale_cols_launch(cnts[q], cnts[q], pGw[q], pU[q], kEigMax, pUs[q], kEigMax, nullptr, st);
      gemm(c, false, true, cnts, cnts, cnts, cc(pUs), kEigMax, cc(pU), kEigMax, pS, kEigMax, 1.0, 0.0);
      gemm(c, false, false, cnts, cnts, cnts, cc(pS), kEigMax, cc(pH), kEigMax, pT, kEigMax, 1.0, 0.0);
      gemm(c, false, false, cnts, cnts, cnts, cc(pT), kEigMax, cc(pS), kEigMax, pH2, kEigMax, 1.0, 0.0);
      EigArgs e;
      e.m = ring.vec(cnts);
      e.A = ring.cptrs(pH2);
      e.lda = kEigMax;
      e.W = ring.ptrs(pO);
      e.V = ring.ptrs(pY);
      e.ldv = kEigMax;
      eig_launch(e, NC, cmax, st);
      gemm(c, false, false, cnts, cnts, cnts, cc(pS), kEigMax, cc(pY), kEigMax, pY2, kEigMax, 1.0, 0.0);
      std::vector<const double*> cY(pY2.begin(), pY2.end());
      gemm(c, false, false, rowsn, cnts, cnts, cX, n, cY, kEigMax,
           act_vec(chunks, [&](const Chunk& ch) { return Xf + (size_t)ch.off * n; }), n, 1.0, 0.0);
      gemm(c, false, false, rowsn, cnts, cnts, cAX, n, cY, kEigMax,
           act_vec(chunks, [&](const Chunk& ch) { return AXf + (size_t)ch.off * n; }), n, 1.0, 0.0);
      gemm(c, false, false, rowsn, cnts, cnts, cBX, n, cY, kEigMax,
           act_vec(chunks, [&](const Chunk& ch) { return BXf + (size_t)ch.off * n; }), n, 1.0, 0.0);
      ColDotArgs r1;
      r1.n = n;
      r1.ncol = ring.vec(cnts);
      r1.X = ring.cptrs(act_vec(chunks, [&](const Chunk& ch) { return AXf + (size_t)ch.off * n; }));
      r1.ldx = n;
      r1.Y = ring.cptrs(act_vec(chunks, [&](const Chunk& ch) { return BXf + (size_t)ch.off * n; }));
      r1.ldy = n;
      r1.w = ring.cptrs(pO);
      r1.out = ring.ptrs(act_vec(chunks, [&](const Chunk& ch) { return rr + ch.off; }));
      r1.mode = 1;
      r1.partial = static_cast<double*>(ws_get(h, kBufMisc, sizeof(double) * coldot_partial_size(n, NC, kEigMax)));
      coldot_launch(r1, NC, cmax, st);
      ColDotArgs r2 = r1;
      r2.X = ring.cptrs(act_vec(chunks, [&](const Chunk& ch) { return Xf + (size_t)ch.off * n; }));
      r2.Y = r2.X;
      r2.ldy = n;
      r2.out = ring.ptrs(act_vec(chunks, [&](const Chunk& ch) { return xn + ch.off; }));
      r2.mode = 0;
      coldot_launch(r2, NC, cmax, st);
      std::vector<double> hr(NL), hx(NL), ho((size_t)NC * kEigMax);
      SL_HIP(hipMemcpyAsync(hr.data(), rr, sizeof(double) * NL, hipMemcpyDeviceToHost, st));
      SL_HIP(hipMemcpyAsync(hx.data(), xn, sizeof(double) * NL, hipMemcpyDeviceToHost, st));
      SL_HIP(hipMemcpyAsync(ho.data(), Om, sizeof(double) * NC * kEigMax, hipMemcpyDeviceToHost, st));
      SL_HIP(hipStreamSynchronize(st));
      ring.synced();
      for (int q = 0; q < NC; ++q)
        for (int i = 0; i < chunks[q].cnt; ++i) {
          const int t = chunks[q].off + i;
          vals[t] = ho[(size_t)q * kEigMax + i];
          ress[t] = hr[t] / (anorm * std::sqrt(std::max(hx[t], 1e-300)));
        }
    }
    t_rr = ms_since(t_r0);
  }
  double flops_update = 0.0, bytes_panel = 0.0;
  if (rep && o.profile) {
    // algorithmic flops of the trailing updates and bytes of the panels, from the
    // panel starts of every shift
    std::vector<int> ps((size_t)S1 * fp.npmax);
    std::vector<FactorState> fs(S1);
    SL_HIP(hipMemcpy(ps.data(), fp.pstart_base, sizeof(int) * ps.size(), hipMemcpyDeviceToHost));
    SL_HIP(hipMemcpy(fs.data(), fp.d_state, sizeof(FactorState) * S1, hipMemcpyDeviceToHost));
    for (int s = 0; s < S1; ++s) {
      const int np = fs[s].npanel;
      for (int q = 0; q < np; ++q) {
        const int k0 = ps[(size_t)s * fp.npmax + q];
        const int k1 = q + 1 < np ? ps[(size_t)s * fp.npmax + q + 1] : n;
        const double m = (double)(n - k1);
        flops_update += m * (m + 1.0) * (double)(k1 - k0);
        bytes_panel += 2.0 * 8.0 * (double)(n - k0) * (double)(k1 - k0);
      }
    }
  }
  // ---- 3b. missing eigenvalues (Sec. 3.3).  When a slice holds more eigenvalues
  // than validated candidates, a density-of-states estimate (KPM) places new
  // shifts at equal-count points inside that slice, about one per n_e / n_s
  // eigenvalues; only the new probes run (the paper's subspace iteration, each
  // on the window between its neighbours in the merged shift set), their Ritz
  // pairs join the others and every slice is validated again.
  // psig/pnu: the shifts of all probes (inserted ones included) and their
  // inertias; origin: the original probe toward which a probe's values count
  // (an inserted probe: the nearer of the two shifts bounding its slice).
  std::vector<double> psig(sig);
  std::vector<int64_t> pnu(nu);
  std::vector<int> origin(P);
  std::iota(origin.begin(), origin.end(), 0);
  int n_inserted = 0, n_rounds = 0;
  DevBuf merged_x, merged_tmp;
  // probe m's values as one contiguous range [offs[m], offs[m] + cnts[m])
  auto probe_ranges = [&](int PP, std::vector<int64_t>& offs, std::vector<int64_t>& cnts) {
    offs.assign(PP, 0);
    cnts.assign(PP, 0);
    for (const auto& ch : chunks) cnts[ch.probe] += ch.cnt;
    int64_t acc = 0;
    for (int j = 0; j < PP; ++j) {
      offs[j] = acc;
      acc += cnts[j];
    }
  };
  {
    std::vector<double> kmu;
    double ka = 0.0, kb = 0.0;
    std::vector<double> kg;
    for (int round = 0; round < o.max_recovery; ++round) {
      const int PP = (int)psig.size();
      std::vector<int64_t> offs, cnts;
      probe_ranges(PP, offs, cnts);
      std::vector<int32_t> sc(PP + 1), se(PP + 1), sd(PP + 1), ch0(std::max(NL, 1), 0);
      validate(PP, psig.data(), pnu.data(), top, nu_top, offs.data(), cnts.data(), vals.data(),
               ress.data(), sc.data(), se.data(), sd.data(), ch0.data());
      std::vector<int> miss;
      for (int s = 0; s <= PP; ++s)
        if (sc[s] == 1) miss.push_back(s);
      if (miss.empty()) break;
      // the probes' Ritz vectors leave the workspaces that the next steps reuse
      merged_tmp.alloc(sizeof(double) * (size_t)n * std::max(NL, 1));
      double* xold = static_cast<double*>(merged_tmp.p);
      SL_HIP(hipMemcpyAsync(xold, Xf, sizeof(double) * (size_t)n * NL, hipMemcpyDeviceToDevice, st));
      if (kmu.empty()) {
        kmu.assign(o.kpm_moments, 0.0);
        std::vector<double> s_tmp(n_s);
        double t_tmp = 0.0, bnd[2];
        const sislice_status ps = plan_impl(h, n, A, lda, B, ldb, n_e, n_s, o, s_tmp.data(), &t_tmp,
                                            kmu.data(), bnd);
        SL_CHECK_ARG(ps == SISLICE_OK, "density-of-states estimate for probe insertion failed");
        ka = bnd[0];
        kb = bnd[1];
        kg.assign(o.kpm_moments, 0.0);
        jackson(o.kpm_moments, kg.data());
      }
      auto Phi = [&](double w) { return kpm_cdos(kmu.data(), kg.data(), o.kpm_moments, ka, kb, n, w); };
      const double K = std::max(1.0, (double)n_e / (double)n_s);
      std::vector<double> newpts;
      for (int s : miss) {
        const double l = s == 0 ? std::min(ka, psig[0] - (psig.size() > 1 ? psig[1] - psig[0] : 1.0))
                                : psig[s - 1];
        const double u = s == PP ? top : psig[s];
        const int q = std::max(1, (int)std::ceil((double)se[s] / K));
        const double fl = Phi(l), fu = Phi(u);
        for (int t = 1; t <= q; ++t) {
          double w;
          if (fu - fl > 1e-8) {
            const double target = fl + t * (fu - fl) / (q + 1);
            double lo = l, hi = u;
            for (int it = 0; it < 100; ++it) {
              const double mid = 0.5 * (lo + hi);
              (Phi(mid) < target ? lo : hi) = mid;
            }
            w = 0.5 * (lo + hi);
          } else {
            w = l + t * (u - l) / (q + 1);  // the estimate sees nothing here: equal spacing
          }
          const double gap = 1e-9 * (std::fabs(u) + std::fabs(l) + 1.0);
          if (w > l + gap && w < u - gap) newpts.push_back(w);
        }
      }
      std::sort(newpts.begin(), newpts.end());
      newpts.erase(std::unique(newpts.begin(), newpts.end()), newpts.end());
      if (newpts.empty()) break;
      const int Pn = (int)newpts.size();
      // factor the new shifts (storage for LD, ipiv and the solve preparation)
      const size_t per = Carver::round(sizeof(double) * (size_t)n * n) + Carver::round(sizeof(int32_t) * n) +
                         2 * Carver::round(sizeof(int) * n) + Carver::round(sizeof(double) * solve_linv_size(n));
      DevBuf fac;
      fac.alloc(per * Pn + 256);
      Carver cf(fac.p);
      std::vector<double*> nLD(Pn), nLinv(Pn);
      std::vector<int32_t*> nip(Pn);
      std::vector<int*> nperm(Pn), nblk(Pn);
      for (int i = 0; i < Pn; ++i) {
        nLD[i] = cf.take<double>((size_t)n * n);
        nip[i] = cf.take<int32_t>(n);
        nperm[i] = cf.take<int>(n);
        nblk[i] = cf.take<int>(n);
        nLinv[i] = cf.take<double>(solve_linv_size(n));
      }
      const int nbf = o.nb > 0 ? std::min(o.nb, kMaxNb) : default_nb(n);
      FactorPlan f = build_factor(h, kBufFactor, n, A, lda, B, ldb, Pn, newpts.data(), nLD.data(), n,
                                  nip.data(), nbf, true);
      factor_launch(f, st);
      std::vector<int64_t> ni(3 * Pn);
      SL_HIP(hipMemcpyAsync(ni.data(), f.d_inertia, sizeof(int64_t) * 3 * Pn, hipMemcpyDeviceToHost, st));
      SL_HIP(hipStreamSynchronize(st));
      ring.synced();
      solve_prep_launch(n, Pn, reinterpret_cast<const int* const*>(ring.ptrs(nip)), ring.ptrs(nperm),
                        ring.ptrs(nblk), ring.cptrs(nLD), n, ring.ptrs(nLinv), st);
      // the merged shift set and the windows of the new probes in it
      std::vector<std::pair<double, int>> all;  // (shift, index: < PP old probe, else PP + new)
      for (int m = 0; m < PP; ++m) all.push_back({psig[m], m});
      for (int i = 0; i < Pn; ++i)
        if (ni[3 * i + 1] == 0) all.push_back({newpts[i], PP + i});  // an exact zero pivot: dropped
      std::sort(all.begin(), all.end());
      const int PM = (int)all.size();
      std::vector<int64_t> mnu(PM);
      std::vector<double> msig(PM);
      for (int m = 0; m < PM; ++m) {
        msig[m] = all[m].first;
        mnu[m] = all[m].second < PP ? pnu[all[m].second] : ni[3 * (all[m].second - PP)];
      }
      std::vector<SubspaceProbe> sp;
      std::vector<int> sp_at;  // merged index of each new probe
      int64_t max_need = 0;
      for (int m = 0; m < PM; ++m) {
        if (all[m].second < PP) continue;
        const int i = all[m].second - PP;
        SubspaceProbe q;
        q.sigma = msig[m];
        q.lo = m > 0 ? msig[m - 1] : -std::numeric_limits<double>::infinity();
        q.hi = m + 1 < PM ? msig[m + 1] : top;
        q.need = (m + 1 < PM ? mnu[m + 1] : nu_top) - (m > 0 ? mnu[m - 1] : 0);
        q.LD = nLD[i];
        q.perm = nperm[i];
        q.blk = nblk[i];
        q.Linv = nLinv[i];
        max_need = std::max(max_need, q.need);
        sp.push_back(q);
        sp_at.push_back(m);
      }
      if (sp.empty()) break;
      const int kr = std::min(subspace_dim(max_need), n);
      const auto t_i0 = Clock::now();
      SubspaceOut so = subspace_probes(c, n, Af, Bf, sp, anorm, o, kr, o.subspace_iters, nullptr, 0, 0, n);
      t_lanczos += ms_since(t_i0);
      block_steps += so.applications;
      cycles_max = std::max(cycles_max, so.rounds_max);
      bytes_solve += so.bytes_solve;
      // merge: every probe's values contiguous, in merged shift order
      std::vector<int> src_new(PM, -1);  // new probe -> its position in sp
      for (size_t q = 0; q < sp_at.size(); ++q) src_new[sp_at[q]] = (int)q;
      std::vector<Chunk> mchunks;
      std::vector<double> mvals, mress;
      std::vector<const double*> csrc;
      std::vector<int> ccnt;
      std::vector<int64_t> coff;
      int mNL = 0;
      std::vector<int> morigin(PM);
      for (int m = 0; m < PM; ++m) {
        const int id = all[m].second;
        int cnt;
        if (id < PP) {
          cnt = (int)cnts[id];
          csrc.push_back(xold + (size_t)offs[id] * n);
          for (int t = 0; t < cnt; ++t) {
            mvals.push_back(vals[offs[id] + t]);
            mress.push_back(ress[offs[id] + t]);
          }
          morigin[m] = origin[id];
        } else {
          const int q = src_new[m];
          cnt = kr;
          csrc.push_back(so.X + (size_t)q * n * kr);
          for (int t = 0; t < kr; ++t) {
            mvals.push_back(so.vals[(size_t)q * kr + t]);
            mress.push_back(so.ress[(size_t)q * kr + t]);
          }
          // the original probe nearer to this shift among those bounding its slice
          int lo_o = -1, hi_o = -1;
          for (int mm = m - 1; mm >= 0; --mm)
            if (all[mm].second < PP) {
              lo_o = origin[all[mm].second];
              break;
            }
          for (int mm = m + 1; mm < PM; ++mm)
            if (all[mm].second < PP) {
              hi_o = origin[all[mm].second];
              break;
            }
          if (lo_o < 0) morigin[m] = hi_o;
          else if (hi_o < 0) morigin[m] = lo_o;
          else morigin[m] = std::fabs(msig[m] - sig[lo_o]) <= std::fabs(sig[hi_o] - msig[m]) ? lo_o : hi_o;
        }
        Chunk chm;
        chm.probe = m;
        chm.off = mNL;
        chm.cnt = cnt;
        mchunks.push_back(chm);
        ccnt.push_back(cnt);
        coff.push_back(mNL);
        mNL += cnt;
      }
      merged_x.alloc(sizeof(double) * (size_t)n * std::max(mNL, 1));
      double* xm = static_cast<double*>(merged_x.p);
      {
        std::vector<double*> dst(PM);
        int cmax = 0;
        for (int m = 0; m < PM; ++m) {
          dst[m] = xm + (size_t)coff[m] * n;
          cmax = std::max(cmax, ccnt[m]);
        }
        CopyArgs cp;
        cp.n = n;
        cp.ncol = ring.vec(ccnt);
        cp.src = ring.cptrs(csrc);
        cp.lds = n;
        cp.dst = ring.ptrs(dst);
        cp.ldd = n;
        if (cmax > 0) copy_launch(cp, PM, cmax, st);
      }
      SL_HIP(hipStreamSynchronize(st));
      ring.synced();
      merged_tmp.release();
      chunks = std::move(mchunks);
      vals = std::move(mvals);
      ress = std::move(mress);
      NL = mNL;
      Xf = xm;
      psig = msig;
      pnu = mnu;
      origin = morigin;
      n_inserted += (int)sp.size();
      ++n_rounds;
      if (rep) rep->factor_id = 0;  // the cached factorizations no longer match the probes
    }
  }
  // ---- 4. validation (host) and output
  const auto t_h0 = Clock::now();
  const int PP = (int)psig.size();
  std::vector<int64_t> offs, cnts;
  probe_ranges(PP, offs, cnts);
  std::vector<int32_t> scase(PP + 1), sexact(PP + 1), scand(PP + 1), chosen(std::max(NL, 1), 0);
  const int64_t nval = validate(PP, psig.data(), pnu.data(), top, nu_top, offs.data(), cnts.data(),
                                vals.data(), ress.data(), scase.data(), sexact.data(), scand.data(),
                                chosen.data());
  // A value is taken from the probe whose shift is nearer, but both probes of a
  // slice usually lock it.  When the chosen copy misses the tolerance (a vector
  // of a dense cluster that one probe resolved less well) and the other probe's
  // copy of the same value meets it, the better copy is reported.  Copies match
  // when they agree to 1e-9 relative to the spectral scale, and the exchange is
  // refused when any other chosen value lies that close (a near-degenerate pair
  // must keep two distinct vectors).
  {
    const double dmatch = 1e-9 * std::max(1.0, std::fabs(top) + std::fabs(psig[0]));
    std::vector<int> cidx;
    for (int t = 0; t < NL; ++t)
      if (chosen[t]) cidx.push_back(t);
    std::sort(cidx.begin(), cidx.end(), [&](int x, int y) { return vals[x] < vals[y]; });
    auto chosen_near = [&](double v, int self) {
      auto it = std::lower_bound(cidx.begin(), cidx.end(), v - dmatch,
                                 [&](int x, double w) { return vals[x] < w; });
      for (; it != cidx.end() && vals[*it] <= v + dmatch; ++it)
        if (*it != self) return true;
      return false;
    };
    for (int t : cidx) {
      if (!(ress[t] > o.tol)) continue;
      int best = -1;
      for (int u = 0; u < NL; ++u) {
        if (chosen[u] || !(ress[u] <= o.tol) || std::fabs(vals[u] - vals[t]) > dmatch) continue;
        if (best < 0 || ress[u] < ress[best]) best = u;
      }
      if (best >= 0 && !chosen_near(vals[t], t)) {
        chosen[t] = 0;
        chosen[best] = 1;
      }
    }
  }
  std::vector<int> pick;
  for (int t = 0; t < NL; ++t)
    if (chosen[t]) pick.push_back(t);
  std::stable_sort(pick.begin(), pick.end(), [&](int x, int y) { return vals[x] < vals[y]; });
  const int nout = (int)std::min<int64_t>(n_e, (int64_t)pick.size());
  int64_t nconv = 0;
  bool missing = nval < n_e || (int64_t)pick.size() < n_e;
  for (int s = 0; s <= PP; ++s) missing |= scase[s] == 1;
  if (nout > 0) {
    std::vector<const double*> src(nout);
    std::vector<int> scol(nout);
    std::vector<double> v(nout), r(nout);
    std::vector<int> val_probe(std::max(NL, 1), -1);
    for (const auto& ch : chunks)
      for (int i = 0; i < ch.cnt; ++i) val_probe[ch.off + i] = ch.probe;
    for (int q = 0; q < nout; ++q) {
      src[q] = Xf;
      scol[q] = pick[q];
      v[q] = vals[pick[q]];
      r[q] = ress[pick[q]];
      nconv += r[q] <= o.tol;
      if (probe_of) probe_of[q] = origin[val_probe[pick[q]]];
    }
    GatherArgs g;
    g.n = n;
    g.src = ring.cptrs(std::vector<double*>(src.size(), Xf));
    g.src_col = ring.vec(scol);
    g.lds = n;
    g.dst = evecs;
    g.ldd = ldx;
    g.val = ring.vec(v);
    g.res = ring.vec(r);
    g.evals = evals;
    g.resid = resid_out;
    gather_launch(g, nout, st);
  }
  SL_HIP(hipStreamSynchronize(st));
  ring.synced();
  const double t_host = ms_since(t_h0);
  if (rep && o.profile) {
    for (int q = 0; q < 6; ++q) {
      rep->t_kern_ms[q] = 0.0;
      rep->n_kern[q] = 0;
    }
    prof_collect(h, rep->t_kern_ms, rep->n_kern);
    rep->flops_update = flops_update;
    rep->bytes_panel = bytes_panel;
    rep->bytes_solve = bytes_solve;
  }
  prof_reset(h);
  h->prof = false;
  if (rep) {
    rep->n_validated = nval;
    rep->n_converged = nconv;
    rep->cycles_max = cycles_max;
    rep->block_steps = block_steps;
    rep->t_factor_ms = t_factor;
    rep->t_lanczos_ms = t_lanczos;
    rep->t_rr_ms = t_rr;
    rep->t_host_ms = t_host;
    rep->t_total_ms = ms_since(t_start);
    (void)t_plan;
    rep->probes_inserted = n_inserted;
    rep->recovery_rounds = n_rounds;
    // slices of the caller's shifts: a slice split by inserted probes reports the
    // sums of its parts, and case 1 (missing) or else 2 (trimmed) if any part has it
    std::vector<int32_t> oc(P + 1, 0), oe(P + 1, 0), od(P + 1, 0);
    for (int t = 0; t <= PP; ++t) {
      int s = 0;
      if (t > 0)
        while (s < P && sig[s] <= psig[t - 1]) ++s;
      oe[s] += sexact[t];
      od[s] += scand[t];
      if (scase[t] == 1) oc[s] = 1;
      else if (scase[t] == 2 && oc[s] == 0) oc[s] = 2;
    }
    if (rep->slice_case)
      for (int s = 0; s <= P; ++s) rep->slice_case[s] = oc[s];
    if (rep->slice_exact)
      for (int s = 0; s <= P; ++s) rep->slice_exact[s] = oe[s];
    if (rep->slice_cand)
      for (int s = 0; s <= P; ++s) rep->slice_cand[s] = od[s];
  }
  if (missing) return SISLICE_MISSING_EIGS;
  if (nconv < n_e) return SISLICE_NOT_CONVERGED;
  return SISLICE_OK;
}

}  // namespace sislice

using namespace sislice;

extern "C" {

sislice_status sislice_plan_shifts_kpm(sislice_handle* h, int64_t n, const double* A, int64_t lda,
                                       const double* B, int64_t ldb, int64_t n_e, int64_t n_s,
                                       const sislice_opts* opts, double* sigmas, double* omega_top,
                                       double* moments, double* bounds) {
  try {
    check_handle(h);
    sislice_opts o;
    sislice_default_opts(&o);
    if (opts) o = *opts;
    check_opts(o);
    SL_CHECK_ARG(n >= 16 && n <= 20000, "n must be in [16, 20000]");
    SL_CHECK_ARG(n_s >= 1 && n_e >= 1 && n_e < n, "bad n_e / n_s");
    SL_CHECK_ARG(A && B && lda >= n && ldb >= n && sigmas && omega_top, "bad argument");
    return plan_impl(h, n, A, lda, B, ldb, n_e, n_s, o, sigmas, omega_top, moments, bounds);
  } catch (const Error& e) {
    std::fprintf(stderr, "sislice: %s\n", e.what());
    return e.status;
  }
}

sislice_status sislice_plan_shifts_lanczos(sislice_handle* h, int64_t n, const double* A,
                                           int64_t lda, const double* B, int64_t ldb, int64_t n_e,
                                           int64_t n_s, const sislice_opts* opts, int32_t mode,
                                           int32_t k, int32_t nv, double* sigmas, double* omega_top,
                                           double* bounds) {
  try {
    check_handle(h);
    sislice_opts o;
    sislice_default_opts(&o);
    if (opts) o = *opts;
    check_opts(o);
    SL_CHECK_ARG(n >= 16 && n <= 20000, "n must be in [16, 20000]");
    SL_CHECK_ARG(n_s >= 1 && n_e >= 1 && n_e < n, "bad n_e / n_s");
    SL_CHECK_ARG(mode == 0 || mode == 1, "mode must be 0 (equal counts) or 1 (DOSCluster)");
    SL_CHECK_ARG(k >= 2 && k <= kEigMax && nv >= 1 && nv <= kSkinnyMaxCol, "k in [2, 112], nv in [1, 32]");
    SL_CHECK_ARG(A && B && lda >= n && ldb >= n && sigmas && omega_top, "bad argument");
    return plan_impl(h, n, A, lda, B, ldb, n_e, n_s, o, sigmas, omega_top, nullptr, bounds, mode, k,
                     nv);
  } catch (const Error& e) {
    std::fprintf(stderr, "sislice: %s\n", e.what());
    return e.status;
  }
}

sislice_status sislice_solve(sislice_handle* h, int64_t n, const double* A, int64_t lda,
                             const double* B, int64_t ldb, int64_t n_e, int64_t n_s,
                             const double* sigmas, double* omega_top, const sislice_opts* opts,
                             double* evals, double* evecs, int64_t ldx, double* resid,
                             sislice_report* report) {
  try {
    check_handle(h);
    sislice_opts o;
    sislice_default_opts(&o);
    if (opts) o = *opts;
    check_opts(o);
    SL_CHECK_ARG(n >= 32 && n <= 20000, "n must be in [32, 20000]");
    SL_CHECK_ARG(n_s >= 1 && n_s <= 1024, "n_s must be in [1, 1024]");
    SL_CHECK_ARG(n_e >= 1 && n_e < n, "n_e must be in [1, n)");
    SL_CHECK_ARG(A && B && lda >= n && ldb >= n && omega_top, "bad matrix argument");
    SL_CHECK_ARG(evals && evecs && resid && ldx >= n, "bad output argument");
    const sislice_status st = solve_impl(h, n, A, lda, B, ldb, n_e, n_s, sigmas, omega_top, o,
                                         evals, evecs, ldx, resid, report, nullptr, nullptr);
    check_waits(h);
    return st;
  } catch (const Error& e) {
    std::fprintf(stderr, "sislice: %s\n", e.what());
    return e.status;
  }
}

sislice_status sislice_sisubit(sislice_handle* h, int64_t n, const double* A, int64_t lda,
                               const double* B, int64_t ldb, double sigma, int64_t k,
                               const double* V0, int64_t ldv, int32_t M, double* evals, double* X,
                               int64_t ldx, double* resid) {
  try {
    check_handle(h);
    SL_CHECK_ARG(n >= 32 && n <= 20000, "n must be in [32, 20000]");
    SL_CHECK_ARG(k >= 1 && k <= kEigMax && k <= n, "k must be in [1, min(112, n)]");
    SL_CHECK_ARG(M >= 1 && M <= 64, "M must be in [1, 64]");
    SL_CHECK_ARG(A && B && lda >= n && ldb >= n, "bad matrix argument");
    SL_CHECK_ARG(V0 && ldv >= n && evals && X && ldx >= n && resid, "bad vector argument");
    const int nn = (int)n, kk = (int)k;
    hipStream_t st = h->stream;
    set_current_handle(h);
    Ring ring(h);
    Ctx c{h, st, &ring};
    // the algorithm's second step: the LDL^T of A - sigma B (kept in the handle's
    // factor cache like the solve's)
    DriverWs dw = driver_factor(h, ring, nn, A, lda, B, ldb, {sigma}, default_nb(nn));
    if (dw.inert[1] != 0) return SISLICE_SINGULAR_SHIFT;
    solve_prep_launch(nn, 1, reinterpret_cast<const int* const*>(ring.ptrs(std::vector<int32_t*>{dw.ipv[0]})),
                      ring.ptrs(std::vector<int*>{dw.perm[0]}), ring.ptrs(std::vector<int*>{dw.blk[0]}),
                      ring.cptrs(std::vector<double*>{dw.LD[0]}), nn,
                      ring.ptrs(std::vector<double*>{dw.Linv[0]}), st);
    h->fc.prepped[0] = 1;
    std::vector<int> one{1};
    const double anorm = sym_norm2(c, nn, dw.Af, dw.nX, dw.nX + (size_t)nn * 8, dw.nsmall,
                                   dw.nsmall + 64, dw.nsmall + 128, dw.nsmall + 192,
                                   dw.nsmall + 256, dw.nflag, ring.vec(one), 0);
    SubspaceProbe p;
    p.sigma = sigma;
    p.lo = -std::numeric_limits<double>::infinity();
    p.hi = std::numeric_limits<double>::infinity();
    p.LD = dw.LD[0];
    p.perm = dw.perm[0];
    p.blk = dw.blk[0];
    p.Linv = dw.Linv[0];
    sislice_opts o;
    sislice_default_opts(&o);
    SubspaceOut so = subspace_probes(c, nn, dw.Af, dw.Bf, {p}, anorm, o, kk, M, V0, kk, 1, ldv);
    SL_HIP(hipMemcpyAsync(evals, so.vals.data(), sizeof(double) * kk, hipMemcpyHostToDevice, st));
    SL_HIP(hipMemcpyAsync(resid, so.ress.data(), sizeof(double) * kk, hipMemcpyHostToDevice, st));
    SL_HIP(hipMemcpy2DAsync(X, sizeof(double) * ldx, so.X, sizeof(double) * nn, sizeof(double) * nn,
                            kk, hipMemcpyDeviceToDevice, st));
    SL_HIP(hipStreamSynchronize(st));
    ring.synced();
    check_waits(h);
    return SISLICE_OK;
  } catch (const Error& e) {
    std::fprintf(stderr, "sislice: %s\n", e.what());
    return e.status;
  }
}

}  // extern "C"
