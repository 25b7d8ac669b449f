// Host driver of the paper's shift-invert subspace iteration (Algorithm 2) on
// the device, for every probe of a pencil in lock step: one launch per step
// serves all active probes (the sweeps, the B-apply, the Gram matrices, the
// Cholesky factors, the Rayleigh-Ritz products).
#include <algorithm>
#include <cmath>
#include <vector>

#include "blas.hpp"
#include "driver_util.hpp"
#include "eig.hpp"
#include "handle.hpp"
#include "lanczos.hpp"
#include "planner.hpp"
#include "sisubit.hpp"
#include "solve.hpp"

namespace sislice {

int subspace_dim(int64_t max_need) {
  const int64_t k = std::max<int64_t>(2 * max_need, 16);
  const int64_t r = ceil_div(k, kLanczosBlock) * kLanczosBlock;
  return (int)std::min<int64_t>(r, kEigMax);
}

SubspaceOut subspace_probes(Ctx& c, int n, const double* Af, const double* Bf,
                            const std::vector<SubspaceProbe>& pr, double anorm,
                            const sislice_opts& o, int k, int M, const double* start,
                            int start_cols, int rounds, long start_ld) {
  sislice_handle* h = c.h;
  hipStream_t st = c.st;
  Ring& ring = *c.ring;
  const int P = (int)pr.size();
  SL_CHECK_ARG(k >= 1 && k <= kEigMax && k <= n, "subspace dimension out of range");
  SL_CHECK_ARG(M >= 1, "subspace iterations per round must be >= 1");
  SubspaceOut out;
  out.k = k;
  const size_t nk = (size_t)n * k;
  const size_t kk = (size_t)k * k;
  Sizer z;
  for (int q = 0; q < 7; ++q) z.take<double>(nk * P);  // V Z W V2 Z2 AV Xr
  z.take<double>((size_t)n * kSolveMaxRhs * P);       // sweep scratch
  z.take<double>((size_t)n * kSolveMaxRhs * P);
  for (int q = 0; q < 4; ++q) z.take<double>(kk * P);  // G Li H Y
  for (int q = 0; q < 3; ++q) z.take<double>((size_t)k * P);  // omega, ||r||, ||x||^2
  z.take<int>(P);
  Carver cw(ws_get(h, kBufLanczos, z.off));
  double* V = cw.take<double>(nk * P);
  double* Z = cw.take<double>(nk * P);
  double* W = cw.take<double>(nk * P);
  double* V2 = cw.take<double>(nk * P);
  double* Z2 = cw.take<double>(nk * P);
  double* AV = cw.take<double>(nk * P);
  double* Xr = cw.take<double>(nk * P);
  double* Ss = cw.take<double>((size_t)n * kSolveMaxRhs * P);
  double* Sv = cw.take<double>((size_t)n * kSolveMaxRhs * P);
  double* G = cw.take<double>(kk * P);
  double* Li = cw.take<double>(kk * P);
  double* H = cw.take<double>(kk * P);
  double* Y = cw.take<double>(kk * P);
  double* om = cw.take<double>((size_t)k * P);
  double* rn = cw.take<double>((size_t)k * P);
  double* xn = cw.take<double>((size_t)k * P);
  int* flags = cw.take<int>(P);
  unsigned* sync = sync_words(h, (size_t)P + 64);
  out.X = Xr;
  auto blk = [&](double* base, int j) { return base + (size_t)j * nk; };
  auto small = [&](double* base, int j) { return base + (size_t)j * kk; };
  auto pick = [](const std::vector<int>& js, auto f) {
    using T = decltype(f(0));
    std::vector<T> v;
    v.reserve(js.size());
    for (int j : js) v.push_back(f(j));
    return v;
  };
  // start blocks: Gaussian from the probe's SplitMix64 stream (the stream of
  // the Lanczos start blocks), leading columns replaced by the caller's
  {
    std::vector<unsigned long long> seeds(P);
    std::vector<double*> vp(P);
    for (int j = 0; j < P; ++j) {
      seeds[j] = rng_derive(o.seed, kTagLanczos ^ ((uint64_t)j << 32));
      vp[j] = blk(V, j);
    }
    gauss_launch(n, k, P, ring.vec(seeds), ring.ptrs(vp), n, st);
    if (start && start_cols > 0) {
      const int sc = std::min(start_cols, k);
      CopyArgs cp;
      cp.n = n;
      cp.ncol = ring.vec(std::vector<int>(P, sc));
      cp.src = ring.cptrs([&] {
        std::vector<const double*> v(P);
        for (int j = 0; j < P; ++j) v[j] = start + (size_t)j * start_ld * start_cols;
        return v;
      }());
      cp.lds = start_ld;
      cp.dst = ring.ptrs(vp);
      cp.ldd = n;
      copy_launch(cp, P, sc, st);
    }
  }
  const std::vector<int> vn(P, n), vk(P, k);
  auto subset = [](const std::vector<int>& v, size_t m) { return std::vector<int>(v.begin(), v.begin() + m); };
  // Z = B V for every probe in one product (the blocks are adjacent)
  gemm(c, false, false, {n}, {k * P}, {n}, {Bf}, n, {V}, n, {Z}, n, 1.0, 0.0);
  // one CholeskyQR pass: (Vi, Zi = B Vi) -> (Vo, Zo) with Vo^T B Vo = I
  auto cholqr_pass = [&](const std::vector<int>& js, double* Vi, double* Zi, double* Vo, double* Zo) {
    const size_t na = js.size();
    const auto mk = subset(vk, na), mn = subset(vn, na);
    gemm(c, true, false, mk, mk, mn, pick(js, [&](int j) { return (const double*)blk(Vi, j); }), n,
         pick(js, [&](int j) { return (const double*)blk(Zi, j); }), n,
         pick(js, [&](int j) { return small(G, j); }), k, 1.0, 0.0);
    chol_inv_launch(ring.vec(mk), ring.cptrs(pick(js, [&](int j) { return small(G, j); })), k,
                    ring.ptrs(pick(js, [&](int j) { return small(Li, j); })), k,
                    flags, (int)na, st);
    const auto cLi = pick(js, [&](int j) { return (const double*)small(Li, j); });
    gemm(c, false, true, mn, mk, mk, pick(js, [&](int j) { return (const double*)blk(Vi, j); }), n,
         cLi, k, pick(js, [&](int j) { return blk(Vo, j); }), n, 1.0, 0.0);
    gemm(c, false, true, mn, mk, mk, pick(js, [&](int j) { return (const double*)blk(Zi, j); }), n,
         cLi, k, pick(js, [&](int j) { return blk(Zo, j); }), n, 1.0, 0.0);
  };
  auto cholqr2 = [&](const std::vector<int>& js, double* Vi, double* Zi, double* Vo, double* Zo) {
    cholqr_pass(js, Vi, Zi, V2, Z2);
    cholqr_pass(js, V2, Z2, Vo, Zo);
  };
  std::vector<int> act(P);
  for (int j = 0; j < P; ++j) act[j] = j;
  std::vector<int> nround(P, 0);
  out.vals.assign((size_t)k * P, 0.0);
  out.ress.assign((size_t)k * P, 0.0);
  std::vector<char> done(P, 0);
  const int cap = rounds > 0 ? rounds : std::max(1, o.max_cycles);
  for (int round = 0; round < cap && !act.empty(); ++round) {
    const size_t na = act.size();
    const auto mk = subset(vk, na), mn = subset(vn, na);
    for (int j : act) nround[j]++;
    // Algorithm 2, first step: CholeskyQR of the start basis
    cholqr2(act, V, Z, V, Z);
    for (int it = 0; it < M; ++it) {
      // third step: W = L^{-T} D^{-1} L^{-1} (B V) for every probe, 32 columns per sweep
      for (int c0 = 0; c0 < k; c0 += kSolveMaxRhs) {
        SolveArgs sa;
        sa.n = n;
        sa.nshift = (int)na;
        sa.nrhs = std::min(kSolveMaxRhs, k - c0);
        sa.LD = ring.cptrs(pick(act, [&](int j) { return pr[j].LD; }));
        sa.ldld = n;
        sa.perm = ring.cptrs(pick(act, [&](int j) { return pr[j].perm; }));
        sa.blk = ring.cptrs(pick(act, [&](int j) { return pr[j].blk; }));
        sa.Linv = ring.cptrs(pick(act, [&](int j) { return pr[j].Linv; }));
        sa.Y = ring.cptrs(pick(act, [&](int j) { return (const double*)(blk(Z, j) + (size_t)c0 * n); }));
        sa.ldy = n;
        sa.X = ring.ptrs(pick(act, [&](int j) { return blk(W, j) + (size_t)c0 * n; }));
        sa.ldx = n;
        sa.Z = ring.ptrs(pick(act, [&](int j) { return Ss + (size_t)j * n * kSolveMaxRhs; }));
        sa.V = ring.ptrs(pick(act, [&](int j) { return Sv + (size_t)j * n * kSolveMaxRhs; }));
        sa.ldz = n;
        sa.ctr = sync;
        solve_launch(sa, st, 0);
        out.bytes_solve += 8.0 * (double)n * (double)n * (double)na;
      }
      out.applications += (int)na;
      // fourth step: CholeskyQR of W in the B inner product (B W in AV's place)
      if (na == (size_t)P)
        gemm(c, false, false, {n}, {k * P}, {n}, {Bf}, n, {W}, n, {AV}, n, 1.0, 0.0);
      else
        gemm(c, false, false, mn, mk, mn, std::vector<const double*>(na, Bf), n,
             pick(act, [&](int j) { return (const double*)blk(W, j); }), n,
             pick(act, [&](int j) { return blk(AV, j); }), n, 1.0, 0.0);
      cholqr2(act, W, AV, V, Z);
    }
    // fifth step: Rayleigh-Ritz with A and B on the B-orthonormal basis
    const auto cV = pick(act, [&](int j) { return (const double*)blk(V, j); });
    const auto cAV = pick(act, [&](int j) { return (const double*)blk(AV, j); });
    const auto cZ = pick(act, [&](int j) { return (const double*)blk(Z, j); });
    gemm(c, false, false, mn, mk, mn, std::vector<const double*>(na, Af), n, cV, n,
         pick(act, [&](int j) { return blk(AV, j); }), n, 1.0, 0.0);
    gemm(c, true, false, mk, mk, mn, cV, n, cAV, n, pick(act, [&](int j) { return small(H, j); }), k,
         1.0, 0.0);
    EigArgs e;
    e.m = ring.vec(mk);
    e.A = ring.cptrs(pick(act, [&](int j) { return small(H, j); }));
    e.lda = k;
    e.W = ring.ptrs(pick(act, [&](int j) { return om + (size_t)j * k; }));
    e.V = ring.ptrs(pick(act, [&](int j) { return small(Y, j); }));
    e.ldv = k;
    eig_launch(e, (int)na, k, st);
    const auto cY = pick(act, [&](int j) { return (const double*)small(Y, j); });
    gemm(c, false, false, mn, mk, mk, cV, n, cY, k, pick(act, [&](int j) { return blk(W, j); }), n,
         1.0, 0.0);  // X = V Y
    gemm(c, false, false, mn, mk, mk, cAV, n, cY, k, pick(act, [&](int j) { return blk(V2, j); }), n,
         1.0, 0.0);  // A X
    gemm(c, false, false, mn, mk, mk, cZ, n, cY, k, pick(act, [&](int j) { return blk(Z2, j); }), n,
         1.0, 0.0);  // B X
    ColDotArgs r1;
    r1.n = n;
    r1.ncol = ring.vec(mk);
    r1.X = ring.cptrs(pick(act, [&](int j) { return blk(V2, j); }));
    r1.ldx = n;
    r1.Y = ring.cptrs(pick(act, [&](int j) { return blk(Z2, j); }));
    r1.ldy = n;
    r1.w = ring.cptrs(pick(act, [&](int j) { return om + (size_t)j * k; }));
    r1.out = ring.ptrs(pick(act, [&](int j) { return rn + (size_t)j * k; }));
    r1.mode = 1;
    r1.partial = static_cast<double*>(ws_get(h, kBufMisc, sizeof(double) * coldot_partial_size(n, (int)na, k)));
    coldot_launch(r1, (int)na, k, st);
    ColDotArgs r2 = r1;
    r2.X = ring.cptrs(pick(act, [&](int j) { return blk(W, j); }));
    r2.Y = r2.X;
    r2.out = ring.ptrs(pick(act, [&](int j) { return xn + (size_t)j * k; }));
    r2.mode = 0;
    coldot_launch(r2, (int)na, k, st);
    std::vector<double> ho((size_t)k * P), hr((size_t)k * P), hx((size_t)k * P);
    SL_HIP(hipMemcpyAsync(ho.data(), om, sizeof(double) * k * P, hipMemcpyDeviceToHost, st));
    SL_HIP(hipMemcpyAsync(hr.data(), rn, sizeof(double) * k * P, hipMemcpyDeviceToHost, st));
    SL_HIP(hipMemcpyAsync(hx.data(), xn, sizeof(double) * k * P, hipMemcpyDeviceToHost, st));
    SL_HIP(hipStreamSynchronize(st));
    ring.synced();
    std::vector<int> next, fin;
    for (int j : act) {
      int64_t ok = 0;
      for (int i = 0; i < k; ++i) {
        const size_t t = (size_t)j * k + i;
        out.vals[t] = ho[t];
        out.ress[t] = hr[t] / (anorm * std::sqrt(std::max(hx[t], 1e-300)));
        ok += ho[t] > pr[j].lo && ho[t] < pr[j].hi && out.ress[t] <= o.tol;
      }
      if (rounds <= 0 && ok >= pr[j].need) {
        done[j] = 1;
        fin.push_back(j);
      } else {
        next.push_back(j);
      }
    }
    const bool last = round + 1 == cap;
    // finished probes keep their Ritz vectors; the others restart from them
    std::vector<int> keep(fin);
    if (last) keep.insert(keep.end(), next.begin(), next.end());
    if (!keep.empty()) {
      CopyArgs cp;
      cp.n = n;
      cp.ncol = ring.vec(std::vector<int>(keep.size(), k));
      cp.src = ring.cptrs(pick(keep, [&](int j) { return (const double*)blk(W, j); }));
      cp.lds = n;
      cp.dst = ring.ptrs(pick(keep, [&](int j) { return blk(Xr, j); }));
      cp.ldd = n;
      copy_launch(cp, (int)keep.size(), k, st);
    }
    if (!last && !next.empty()) {
      CopyArgs cp;
      cp.n = n;
      cp.ncol = ring.vec(std::vector<int>(next.size(), k));
      cp.src = ring.cptrs(pick(next, [&](int j) { return (const double*)blk(W, j); }));
      cp.lds = n;
      cp.dst = ring.ptrs(pick(next, [&](int j) { return blk(V, j); }));
      cp.ldd = n;
      copy_launch(cp, (int)next.size(), k, st);
      cp.src = ring.cptrs(pick(next, [&](int j) { return (const double*)blk(Z2, j); }));
      cp.dst = ring.ptrs(pick(next, [&](int j) { return blk(Z, j); }));
      copy_launch(cp, (int)next.size(), k, st);
    }
    act = last ? std::vector<int>{} : next;
  }
  SL_HIP(hipStreamSynchronize(st));
  ring.synced();
  for (int j = 0; j < P; ++j) {
    out.rounds_max = std::max(out.rounds_max, nround[j]);
    if (rounds <= 0 && !done[j]) out.converged = false;
  }
  return out;
}

}  // namespace sislice
