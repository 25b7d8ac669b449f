// Small dense kernels of the shift-invert subspace iteration (Algorithm 2):
// the Cholesky factor of the B-Gram matrix of a probe's basis and its inverse,
// for CholeskyQR (V <- V L^{-T} with V^T B V = L L^T).
#include "common.hpp"
#include "eig.hpp"
#include "handle.hpp"
#include "sisubit.hpp"

namespace sislice {

// One 1024-thread workgroup per matrix, k <= kEigMax, the matrix in LDS.
// Cholesky G = L L^T right-looking (a pivot, its column, the trailing update:
// three barriers per column), then L^{-1} in place from the last column back
// (column j of the inverse is -L^{-1}_{jj} times the already inverted trailing
// block applied to column j of L).  Writes L^{-1} (lower, zeros above) to Li and
// flag[b] = 1 when a pivot is not positive (G not numerically definite: the
// factor is then of the matrix with that pivot replaced by one).
__global__ __launch_bounds__(1024) void k_chol_inv(const int* ks, const double* const* G, long ldg,
                                                  double* const* Li, long ldl, int* flag) {
  __shared__ double A[kEigMax][kEigMax + 1];
  __shared__ double x[kEigMax];
  __shared__ int bad;
  const int b = blockIdx.x, tid = threadIdx.x;
  const int k = ks[b];
  const double* g = G[b];
  for (int e = tid; e < k * k; e += 1024) {
    const int i = e % k, j = e / k;
    if (i >= j) A[i][j] = g[i + (long)j * ldg];
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      double d = A[j][j];
      if (!(d > 0.0)) {
        bad = 1;
        d = 1.0;
      }
      A[j][j] = sqrt(d);
    }
    __syncthreads();
    const double djj = A[j][j];
    for (int i = j + 1 + tid; i < k; i += 1024) A[i][j] /= djj;
    __syncthreads();
    const int m = k - j - 1;
    for (int e = tid; e < m * m; e += 1024) {
      const int i = j + 1 + e / m, l = j + 1 + e % m;
      if (l <= i) A[i][l] -= A[i][j] * A[l][j];
    }
    __syncthreads();
  }
  // in-place inverse of the lower factor
  for (int j = k - 1; j >= 0; --j) {
    for (int i = j + 1 + tid; i < k; i += 1024) x[i] = A[i][j];
    __syncthreads();
    const double inv = 1.0 / A[j][j];
    for (int i = j + 1 + tid; i < k; i += 1024) {
      double s = 0.0;
      for (int l = j + 1; l <= i; ++l) s += A[i][l] * x[l];
      A[i][j] = -inv * s;
    }
    if (tid == 0) A[j][j] = inv;
    __syncthreads();
  }
  double* li = Li[b];
  for (int e = tid; e < k * k; e += 1024) {
    const int i = e % k, j = e / k;
    li[i + (long)j * ldl] = (i >= j) ? A[i][j] : 0.0;
  }
  if (tid == 0 && flag) flag[b] = bad;
}

void chol_inv_launch(const int* d_k, const double* const* G, long ldg, double* const* Li, long ldl,
                     int* flag, int batch, hipStream_t st) {
  if (batch <= 0) return;
  SL_LAUNCH(k_chol_inv, dim3(batch), dim3(1024), 0, st, d_k, G, ldg, Li, ldl, flag);
  SL_LAUNCH_CHECK();
}

}  // namespace sislice
