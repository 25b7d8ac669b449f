// sislice_ldlt_solve: X <- C^{-1} X through the documented factor format.
#include "handle.hpp"
#include "solve.hpp"

using namespace sislice;

extern "C" sislice_status sislice_ldlt_solve(sislice_handle* h, int64_t n, const double* LD,
                                             int64_t ldld, const int32_t* ipiv, int64_t nrhs,
                                             double* X, int64_t ldx) {
  try {
    check_handle(h);
    SL_CHECK_ARG(n >= 0 && n <= (int64_t)1 << 24, "n out of range");
    SL_CHECK_ARG(nrhs >= 0 && nrhs <= 64, "nrhs must be in [0, 64]");
    if (n == 0 || nrhs == 0) return SISLICE_OK;
    SL_CHECK_ARG(LD && ipiv && X && ldld >= n && ldx >= n, "bad argument");
    Sizer z;
    z.take<int>(n);
    z.take<int>(n);
    z.take<double>(solve_linv_size(n));
    z.take<double>((size_t)n * kSolveMaxRhs);
    z.take<double>((size_t)n * kSolveMaxRhs);
    z.take<void*>(16);
    Carver c(ws_get(h, kBufSolve, z.off));
    int* perm = c.take<int>(n);
    int* blk = c.take<int>(n);
    double* Linv = c.take<double>(solve_linv_size(n));
    double* Zs = c.take<double>((size_t)n * kSolveMaxRhs);
    double* Vs = c.take<double>((size_t)n * kSolveMaxRhs);
    void** tab = c.take<void*>(16);
    unsigned* sync = sync_words(h, 64);
    // tables: LD, ipiv, perm, blk, Linv, Z, V, Y/X (filled per chunk)
    void** ht = static_cast<void**>(host_stage(h, sizeof(void*) * 16));
    ht[0] = const_cast<double*>(LD);
    ht[1] = const_cast<int32_t*>(ipiv);
    ht[2] = perm;
    ht[3] = blk;
    ht[4] = Linv;
    ht[5] = Zs;
    ht[6] = Vs;
    SL_HIP(hipMemcpyAsync(tab, ht, sizeof(void*) * 7, hipMemcpyHostToDevice, h->stream));
    solve_prep_launch((int)n, 1, reinterpret_cast<const int* const*>(tab + 1),
                      reinterpret_cast<int* const*>(tab + 2), reinterpret_cast<int* const*>(tab + 3),
                      reinterpret_cast<const double* const*>(tab + 0), ldld,
                      reinterpret_cast<double* const*>(tab + 4), h->stream);
    for (int64_t c0 = 0; c0 < nrhs; c0 += kSolveMaxRhs) {
      const int nr = (int)std::min<int64_t>(kSolveMaxRhs, nrhs - c0);
      // one device table slot per chunk so earlier launches keep their pointers
      double** dx = reinterpret_cast<double**>(tab + 8 + (c0 / kSolveMaxRhs) % 2);
      double* xp = X + c0 * ldx;
      SL_HIP(hipMemcpyAsync(dx, &xp, sizeof(void*), hipMemcpyHostToDevice, h->stream));
      SL_HIP(hipStreamSynchronize(h->stream));
      SolveArgs a;
      a.n = (int)n;
      a.nshift = 1;
      a.nrhs = nr;
      a.epoch = next_epoch(h);
      a.LD = reinterpret_cast<const double* const*>(tab + 0);
      a.ldld = ldld;
      a.perm = reinterpret_cast<const int* const*>(tab + 2);
      a.blk = reinterpret_cast<const int* const*>(tab + 3);
      a.Linv = reinterpret_cast<const double* const*>(tab + 4);
      a.Y = dx;
      a.ldy = ldx;
      a.X = dx;
      a.ldx = ldx;
      a.Z = reinterpret_cast<double* const*>(tab + 5);
      a.V = reinterpret_cast<double* const*>(tab + 6);
      a.ldz = n;
      a.ctr = sync;
      solve_launch(a, h->stream);
    }
    return SISLICE_OK;
  } catch (const Error& e) {
    std::fprintf(stderr, "sislice: %s\n", e.what());
    return e.status;
  }
}
