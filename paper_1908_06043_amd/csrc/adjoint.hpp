// Eigenpair adjoint kernels (launch interface).
#pragma once

#include "common.hpp"

namespace sislice {

// Middle matrices of the occupied-occupied part (m x m, column-major, ldm):
//   MA = diag(g) + T o F,  MB = -diag(lam g) - S/2 - (lam_i + lam_j)(T o F)/2
// with K = X^T g_X (S, T its symmetric / antisymmetric parts) and
// F_ji = 1/(lam_i - lam_j) when |lam_i - lam_j| > degtol, else 0.
// glam or K may be null (zero).
void adj_mid_launch(int m, const double* lam, const double* glam, const double* K, long ldk,
                    double degtol, double* MA, double* MB, long ldm, hipStream_t st);

// Right-hand sides in the grouped column layout: R[:, t] = E[:, c] - G[:, c] and
// lamc[t] = lam[c] for c = col_of[t] >= 0; zero columns (and lamc 0) for c < 0.
void adj_rhs_launch(int n, int np, const int* col_of, const double* E, long lde, const double* G,
                    long ldg, const double* lam, double* R, long ldr, double* lamc, hipStream_t st);

// Column-wise flexible preconditioned conjugate gradients (Polak-Ribiere beta,
// which tolerates the rounding of the shift-invert preconditioner), one
// workgroup per column.  Pst (2n x np, ldp) holds the search directions P on rows
// [0, n) and -lam_t P on rows [n, 2n), so that Q = [A B] Pst is (A - lam_t B) P
// in one product.  act[t]: 1 iterating, 0 converged (or zero right-hand side),
// 3 restart requested (a non-positive curvature p^T Q: the direction restarts
// from the preconditioned residual), 2 stopped after kPcgMaxRestarts restarts.
constexpr int kPcgMaxRestarts = 8;
struct PcgArgs {
  int n = 0, np = 0;
  double* Pst = nullptr;
  long ldp = 0;
  const double* Q = nullptr;
  long ldq = 0;
  double* Z = nullptr;  // solution
  double* R = nullptr;  // residual
  double* Y = nullptr;  // preconditioned residual
  long ld = 0;          // leading dimension of Z, R, Y
  const double* lamc = nullptr;
  double* rho = nullptr;   // r^T y
  double* bn2 = nullptr;   // ||b||^2
  double* rrel = nullptr;  // ||r||^2 / ||b||^2
  double* ryo = nullptr;   // r_{k+1}^T y_k (the Polak-Ribiere correction)
  int* nrest = nullptr;    // restarts taken
  int* act = nullptr;
  double tol2 = 0.0;       // converged when ||r||^2 <= tol2 ||b||^2
};
void pcg_init_launch(const PcgArgs& a, hipStream_t st);   // Z = 0, P = Y, rho, ||b||
void pcg_alpha_launch(const PcgArgs& a, hipStream_t st);  // Z += alpha P, R -= alpha Q
void pcg_beta_launch(const PcgArgs& a, hipStream_t st);   // P = Y + beta P, convergence

// Ua[:, i] += Z[:, slot[i]] / 2,  Ub[:, i] -= lam_i Z[:, slot[i]] / 2.
void adj_combine_launch(int n, int m, const double* Z, long ldz, const int* slot, const double* lam,
                        double* Ua, double* Ub, long ldu, hipStream_t st);

// The two symmetric rank-2m outputs in one launch:
//   GA = Ua X^T + X Ua^T,  GB = Ub X^T + X Ub^T   (n x n, both triangles written)
// FP64 MFMA on the lower 64x64 tiles, mirrored through LDS.
void adj_syr2k_launch(int n, int m, const double* X, long ldx, const double* Ua, const double* Ub,
                      long ldu, double* GA, long ldga, double* GB, long ldgb, hipStream_t st);

}  // namespace sislice
