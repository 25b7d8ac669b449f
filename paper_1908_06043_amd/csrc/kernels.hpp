// Launch plans of the device kernels (internal to the library).
#pragma once

#include <algorithm>

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
  int* pstart_base = nullptr;    // device [nshift * npmax] panel starts
  int npmax = 0;
  // pivot-free speculative panel path (per shift): staged L of the panel (n x nb),
  // D of the panel, inverse of the diagonal block (nb x nb), column maxima
  double* const* d_aux = nullptr;  // [nb] D | [nb] max|w| in block | [nb] max|w| below (uint64 bits) | nb*nb Linv
  int fast = 1;                    // use the pivot-free path
  int nbpiv = 32;                  // columns a pivoting panel handles after a rejection
  int wide_min = 1024;             // trailing order from which the update takes 128x128 tiles
  int update_pipe = 1;             // 128x128 updates by the persistent pipelined kernel
  int stream_c = 0;                // the 128-tile update streams C (shift groups on two streams)
  int cus = 256;                   // compute units of the device (its persistent grid)
  int groups = 1;                  // shift groups run on separate streams (with readback)
};

// The whole factorization: shift-form, then the panel/update steps with the
// per-shift progress read back every few steps, the deferred interchanges and
// the inertia.
void factor_launch(const FactorPlan& fp, hipStream_t st);
// The two parts on their own.  With readback == false every step up to the bound
// factor_npanel_max is launched and nothing synchronises (a sequence that a HIP
// graph can capture: its kernels read the shifted matrices through the plan's
// device tables only).
void factor_shift_form_launch(const FactorPlan& fp, hipStream_t st);
void factor_steps_launch(const FactorPlan& fp, hipStream_t st, bool readback);
// One-time kernel attributes of the factorization (outside any capture).
void factor_prepare();

// Narrowest panel that is not the last one: a pivoting panel stops at nb - 1
// columns (room for a closing 2x2 pivot) and, behind the pivot-free path, after
// nbpiv columns from the first rejected one.
inline int factor_min_panel(int nb, int nbpiv, bool fast) {
  const int w = fast ? std::min(nbpiv, nb - 1) : nb - 1;
  return w < 1 ? 1 : w;
}

// Upper bound on the number of panel steps (and so on the panels) of one
// factorization; sizes the panel-start and interchange-snapshot arrays.
inline int factor_npanel_max(int n, int nb, int nbpiv, bool fast) {
  return (int)ceil_div(n, factor_min_panel(nb, nbpiv, fast)) + 2;
}

}  // namespace sislice
