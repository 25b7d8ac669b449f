// Batched small symmetric eigensolver (launch interface).
#pragma once

#include "common.hpp"

namespace sislice {

constexpr int kEigMax = 112;  // largest order of the one-workgroup Jacobi solver (A in LDS)

struct EigArgs {
  const int* m = nullptr;              // device [batch] orders (<= kEigMax; 0 = skip)
  const double* const* A = nullptr;    // device table: column-major, lower triangle read
  long lda = 0;
  double* const* W = nullptr;          // eigenvalues ascending
  double* const* V = nullptr;          // eigenvectors, column j for W[j]
  long ldv = 0;
  int max_sweeps = 40;
};

size_t eig_lds_bytes(int mmax);
void eig_launch(const EigArgs& a, int batch, int mmax, hipStream_t st);

}  // namespace sislice
