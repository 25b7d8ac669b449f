// Dense FP64 building blocks (launch interface).
#pragma once

#include "common.hpp"

namespace sislice {

// C_b = alpha op(A_b) op(B_b) + beta C_b for b < batch; op(A) is m x k, op(B) k x n.
// Per-batch sizes come from the device arrays m/n/k when non-null, else from
// m0/n0/k0.  beta == 0 never reads C.  splits > 1 reduces K in `splits` ordered
// partial products (deterministic), which needs `partial` with room for
// batch * splits * mmax * nmax doubles.
struct GemmArgs {
  const int* m = nullptr;
  const int* n = nullptr;
  const int* k = nullptr;
  int m0 = 0, n0 = 0, k0 = 0;
  const double* const* A = nullptr;
  long lda = 0;
  const double* const* B = nullptr;
  long ldb = 0;
  double* const* C = nullptr;
  long ldc = 0;
  // a batch of one may pass its operands directly (no device tables to upload)
  const double* A1 = nullptr;
  const double* B1 = nullptr;
  double* C1 = nullptr;
  double alpha = 1.0, beta = 0.0;
  int splits = 1;
  double* partial = nullptr;
  long pld = 0, pstride = 0;
};

void gemm_launch(GemmArgs g, int batch, int mmax, int nmax, bool ta, bool tb, hipStream_t st);
void sym_full_launch(int n, const double* S, long lds, double* F, long ldf, hipStream_t st);

// C = alpha M X + beta C, M n x n (tri: 0 full, 1 lower, 2 upper with zeros stored
// in the other half), X n x ncol, ncol <= kSkinnyMaxCol; `partial` holds
// ceil(n / kSkinnyKc) * n * ncol doubles.
constexpr int kSkinnyMaxCol = 32;
constexpr int kSkinnyKc = 256;
inline size_t skinny_partial_size(int n, int ncol) {
  return (size_t)ceil_div(n, kSkinnyKc) * n * ncol;
}
void skinny_launch(int n, int ncol, const double* M, long ldm, int tri, const double* X, long ldx,
                   double alpha, double beta, double* C, long ldc, double* partial, hipStream_t st);
void lincomb3_launch(long tot, double f1, const double* X, double f2, const double* Y, double f3,
                     const double* Z, double* out, hipStream_t st);
void scale_by_norm_launch(int n, const double* s2, const double* x, double* y, double* rec,
                          hipStream_t st);
// One step tail of the single-vector Lanczos on H after w = H v_j (V: n x (j + 2), columns
// contiguous): alpha[j] = v_j^T w; w orthogonalised twice against V[:, 0..j] (classical
// Gram-Schmidt); s2[j] = ||w||^2, beta[j] = ||w||, V[:, j + 1] = w / beta[j] (zero when
// beta[j] == 0).  One workgroup; n <= kLanczosTailMaxN, j + 1 <= kLanczosTailMaxCols.
constexpr int kLanczosTailMaxN = 16384;
constexpr int kLanczosTailMaxCols = 64;
void lanczos_tail_launch(int n, int j, double* V, double* w, double* alpha, double* s2,
                         double* beta, hipStream_t st);
void transpose_launch(int n, const double* S, long lds, double* T, long ldt, hipStream_t st);
// Y[:, c] = X[:, c] / sqrt(s2[c]) (ncol columns), rec[c] = sqrt(s2[c]) (may be null).
void scale_cols_launch(int n, int ncol, const double* s2, const double* X, long ldx, double* Y,
                       long ldy, double* rec, hipStream_t st);

// Batched tall-skinny products with 8 columns (the Lanczos block):
//   tsmt: C_b (m_b x 8, ldc) = alpha V_b^T X_b          (V_b n x m_b, X_b n x 8)
//   tsmm: Y_b (n x 8, ldy) = beta Y_b + alpha (V_b C_b + V2_b C2_b)
//         (V2/C2/m2 optional; C_b m_b x 8 with ldc, C2_b m2_b x 8 with ldc2)
// tsmt needs `partial` with batch * ceil(n / kTsRows) * mmax * 8 doubles.
constexpr int kTsRows = 256;
constexpr size_t kTsmmMaxLds = 160 * 1024;
struct TsArgs {
  int n = 0;
  const int* m = nullptr;
  const double* const* V = nullptr;
  long ldv = 0;
  const double* const* X = nullptr;
  long ldx = 0;
  double* const* C = nullptr;
  long ldc = 0;
  const int* ldcb = nullptr;  // tsmt: per-entry output leading dimension (overrides ldc)
  const int* m2 = nullptr;
  const double* const* V2 = nullptr;
  long ldv2 = 0;
  const double* const* C2 = nullptr;
  long ldc2 = 0;
  double* const* Y = nullptr;
  long ldy = 0;
  double alpha = 1.0, beta = 0.0;
  double* partial = nullptr;
  int nchunk = 0, mmax = 0;
};
inline size_t tsmt_partial_size(int n, int batch, int mmax) {
  return (size_t)batch * ceil_div(n, kTsRows) * mmax * 8;
}
void tsmt_launch(TsArgs a, int batch, int mmax, hipStream_t st);
void tsmm_launch(TsArgs a, int batch, int mtot_max, hipStream_t st);

constexpr int kDotChunk = 2048;

// mode 0: out[b][c] = X[:,c] . Y[:,c];  mode 1: out[b][c] = ||X[:,c] - w[b][c] Y[:,c]||_2
struct ColDotArgs {
  int n = 0;
  const int* ncol = nullptr;
  int ncol0 = 0;
  const double* const* X = nullptr;
  long ldx = 0;
  const double* const* Y = nullptr;
  long ldy = 0;
  const double* const* w = nullptr;
  double* const* out = nullptr;
  // a batch of one may pass its columns directly (no device tables to upload)
  const double* x1 = nullptr;
  const double* y1 = nullptr;
  const double* w1 = nullptr;
  double* out1 = nullptr;
  int mode = 0;
  double* partial = nullptr;  // batch * maxcol * ceil(n / kDotChunk)
  int maxcol = 0, nchunk = 0;
};

void coldot_launch(ColDotArgs a, int batch, int maxcol, hipStream_t st);
inline size_t coldot_partial_size(int n, int batch, int maxcol) {
  return (size_t)batch * maxcol * ceil_div(n, kDotChunk);
}

void gauss_launch(int n, int ncol, int batch, const unsigned long long* d_seeds, double* const* X,
                  long ldx, hipStream_t st);
void rademacher_launch(int n, int ncol, unsigned long long seed, double* X, long ldx,
                       hipStream_t st);

}  // namespace sislice
