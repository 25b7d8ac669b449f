// Multi-shift LDL^T solve kernels (launch interface).
#pragma once

#include "common.hpp"

namespace sislice {

constexpr int kSolveBlock = 64;    // rows per dependency block
constexpr int kSolveMaxRhs = 32;   // right-hand sides per launch

struct SolveArgs {
  int n = 0, nshift = 0, nrhs = 0;
  unsigned epoch = 0;            // strictly increasing per launch pair
  const double* const* LD = nullptr;
  long ldld = 0;
  const int* const* perm = nullptr;
  const int* const* blk = nullptr;
  const double* const* Linv = nullptr;  // solve_linv_size(n) doubles per shift (solve_prep_launch)
  const double* const* Y = nullptr;     // input  n x nrhs (ldy)
  long ldy = 0;
  double* const* X = nullptr;           // output n x nrhs (ldx); may alias Y
  long ldx = 0;
  double* const* Z = nullptr;           // scratch n x nrhs (ldz); the forward result
  double* const* V = nullptr;           // scratch n x nrhs (ldz); the backward result
  long ldz = 0;
  unsigned* ctr = nullptr;              // nshift ticket counters, zero-initialised once
  int applyD = 1;                       // backward sweep applies D^{-1} first (0: identity)
  unsigned* wait_err = nullptr;         // raised when a hand-off wait exceeds wait_limit polls
  unsigned wait_limit = 0;              // (both set by solve_launch from the handle)
};

// mode 0: X = P^T L^{-T} D^{-1} L^{-1} P Y (both sweeps, Z/V scratch)
// mode 1: Z = L^{-1} P Y only (forward sweep; the result is left in Z)
// mode 2: X = P^T L^{-T} [D^{-1}] Z only (backward sweep reading Z)

void solve_prep_launch(int n, int S, const int* const* d_ipiv, int* const* d_perm,
                       int* const* d_blk, const double* const* d_LD, long ldld,
                       double* const* d_Linv, hipStream_t st);
void solve_launch(SolveArgs a, hipStream_t st, int mode = 0);
// Scatter the 64x64 diagonal-block inverses (layout of solve_prep_launch's Linv)
// onto the block diagonal of an n x n matrix.
void diag_inv_scatter_launch(int n, const double* Linv, double* Li, long ldli, hipStream_t st);

inline long solve_nblk(long n) { return ceil_div(n, kSolveBlock); }
// Depth of the sweeps' look-ahead: the nearest kSolveLook blocks enter a block's
// result through precomputed products, the rest through P_b.
constexpr int kSolveLook = 2;
// per shift: the 64x64 diagonal-block inverses of L, then the forward and the
// backward look-ahead blocks of each depth ((1 + 2 kSolveLook) * nblk column-major
// 64x64 blocks)
inline size_t solve_linv_size(long n) {
  return (1 + 2 * (size_t)kSolveLook) * (size_t)solve_nblk(n) * kSolveBlock * kSolveBlock;
}


}  // namespace sislice
