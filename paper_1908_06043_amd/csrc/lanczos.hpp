// Small per-probe Lanczos kernels (launch interface).
#pragma once

#include "common.hpp"

namespace sislice {

constexpr int kLanczosBlock = 8;

struct CholQrArgs {
  int n = 0;
  const int* active = nullptr;
  const double* const* G = nullptr;     // 8x8 Gram, column-major
  const double* const* Vin = nullptr;
  const double* const* Uin = nullptr;
  long ldin = 0;
  double* const* Vout = nullptr;        // may alias Vin
  double* const* Uout = nullptr;
  long ldout = 0;
  double* const* R = nullptr;           // 8x8 upper factor out
  int* flag = nullptr;                  // breakdown flags
};
void cholqr_launch(const CholQrArgs& a, int batch, hipStream_t st);

struct TWriteArgs {
  double* const* T = nullptr;
  long ldt = 0;
  const double* const* S = nullptr;
  long lds = 0;
  const int* rows = nullptr;
  const int* r0 = nullptr;
  const int* c0 = nullptr;
  int cols = 0;
  int add = 0;
};
void twrite_launch(const TWriteArgs& a, int batch, hipStream_t st);

struct CouplingArgs {
  const int* active = nullptr;
  const double* const* R1 = nullptr;
  const double* const* R2 = nullptr;
  double* const* Rt = nullptr;
  double* const* T = nullptr;
  long ldt = 0;
  const int* row0 = nullptr;            // first row of the newest block in T
};
void coupling_launch(const CouplingArgs& a, int batch, hipStream_t st);

struct RitzEstArgs {
  const int* mt = nullptr;
  const double* const* S = nullptr;
  long lds = 0;
  const double* const* Rt = nullptr;
  double* const* est = nullptr;
};
void ritz_est_launch(const RitzEstArgs& a, int batch, hipStream_t st);

struct SelectArgs {
  const int* count = nullptr;
  const int* rows = nullptr;
  const double* const* in = nullptr;
  long ldi = 0;
  double* const* out = nullptr;
  long ldo = 0;
  const int* const* idx = nullptr;
};
void select_launch(const SelectArgs& a, int batch, long maxelems, hipStream_t st);

struct CopyArgs {
  int n = 0;
  const int* ncol = nullptr;
  const double* const* src = nullptr;
  long lds = 0;
  double* const* dst = nullptr;
  long ldd = 0;
};
void copy_launch(const CopyArgs& a, int batch, int maxcol, hipStream_t st);

struct TResetArgs {
  const int* active = nullptr;
  double* const* T = nullptr;
  long ldt = 0;
  int dim = 0;
  const int* k = nullptr;
  const double* const* theta = nullptr;
};
void treset_launch(const TResetArgs& a, int batch, hipStream_t st);

void row_scale_launch(int n, int ncol, const double* scale, double* X, long ldx, hipStream_t st);
void inv_sqrt_diag_launch(int n, const double* LD, long ldld, double* scale, int* bad,
                          hipStream_t st);

struct GatherArgs {
  int n = 0;
  const double* const* src = nullptr;
  const int* src_col = nullptr;
  long lds = 0;
  double* dst = nullptr;
  long ldd = 0;
  const double* val = nullptr;
  const double* res = nullptr;
  double* evals = nullptr;
  double* resid = nullptr;
};
void gather_launch(const GatherArgs& a, int count, hipStream_t st);

}  // namespace sislice
