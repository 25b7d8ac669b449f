// Launch plans of the device kernels (internal to the library).
#pragma once

#include "common.hpp"

namespace sislice {

// One lock-step factorization of `nshift` shifted matrices of order n.
struct FactorPlan {
  int n = 0, nshift = 0, nb = 32;
  bool pivot = true;  // false: LDL^T without interchanges (B is SPD)
  const double* A = nullptr;
  const double* B = nullptr;
  long lda = 0, ldb = 0;
  const double* d_sigmas = nullptr;  // device [nshift]
  double* const* d_LD = nullptr;     // device table of nshift device pointers
  long ldld = 0;
  double* const* d_W = nullptr;  // panel buffers n x (nb + 2)
  long ldw = 0;
  int* const* d_perm = nullptr;
  int* const* d_sw = nullptr;
  int* const* d_blk = nullptr;
  int* const* d_colpanel = nullptr;
  int* const* d_pstart = nullptr;
  int* const* d_snap = nullptr;
  int* const* d_ipiv = nullptr;
  FactorState* d_state = nullptr;
  int64_t* d_inertia = nullptr;  // device [3 * nshift]
};

void factor_launch(const FactorPlan& fp, hipStream_t st);

inline int factor_npanel_max(int n, int nb) { return (int)ceil_div(n, nb - 1) + 1; }

}  // namespace sislice
