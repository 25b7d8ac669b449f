// The paper's per-probe iteration (Algorithm 2, shift-invert subspace iteration)
// on the device: launch interface of its small kernels and its host driver.
#pragma once

#include <vector>

#include "common.hpp"

namespace sislice {

struct Ctx;

// Li_b = L_b^{-1} (lower, zeros above) with G_b = L_b L_b^T for the k_b x k_b
// (k_b <= kEigMax) matrices G_b (lower triangle read); flag[b] = 1 when a pivot
// was not positive.
void chol_inv_launch(const int* d_k, const double* const* G, long ldg, double* const* Li, long ldl,
                     int* flag, int batch, hipStream_t st);

// One probe: its shift, its window (sigma_{j-1}, sigma_{j+1}) and the number of
// eigenvalues in it (from the inertias), and the prepared factorization of
// A - sigma B.
struct SubspaceProbe {
  double sigma = 0, lo = 0, hi = 0;
  int64_t need = 0;
  const double* LD = nullptr;
  const int* perm = nullptr;
  const int* blk = nullptr;
  const double* Linv = nullptr;
};

struct SubspaceOut {
  int k = 0;                     // basis columns per probe
  std::vector<double> vals;      // k Ritz values per probe (probe-major, ascending)
  std::vector<double> ress;      // their residuals ||A x - lambda B x|| / (||A||_2 ||x||)
  double* X = nullptr;           // device n x (k P): Ritz vectors, probe j at column j k
  int rounds_max = 0;            // rounds of M iterations of the slowest probe
  int applications = 0;          // k-column shift-invert applications over all probes
  double bytes_solve = 0.0;      // algorithmic bytes of the triangular sweeps
  bool converged = true;         // every probe met its window's count
};

// Basis size of the probes: max(2 need, 16) for the largest need, a multiple of
// the Lanczos block, at most kEigMax (the projected eigensolver's order).
int subspace_dim(int64_t max_need);

// Algorithm 2 for every probe in lock step.  Each round is one call of the
// algorithm: CholeskyQR of the start basis in the B inner product, M times the
// shift-invert application followed by CholeskyQR, then Rayleigh-Ritz with A and
// B and the residuals; a probe whose window holds `need` Ritz values meeting the
// tolerance is done, the others start their next round from their Ritz vectors.
// `rounds` > 0 runs exactly that many rounds with no convergence test.  `start`
// (device, n x start_cols per probe, probe j at column j start_cols, leading
// dimension start_ld) replaces the leading columns of the Gaussian start blocks.
// CholeskyQR is applied twice per step (the second pass restores
// B-orthonormality to working precision).
SubspaceOut subspace_probes(Ctx& c, int n, const double* Af, const double* Bf,
                            const std::vector<SubspaceProbe>& pr, double anorm,
                            const sislice_opts& o, int k, int M, const double* start,
                            int start_cols, int rounds, long start_ld);

}  // namespace sislice
