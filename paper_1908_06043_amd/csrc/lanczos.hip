// Small per-probe kernels of block shift-invert Lanczos in the B inner product:
// CholeskyQR of an 8-column block (Section 2.1: G = V^T B V = R^T R,
// V <- V R^{-1}), writes into the projected matrix T, Ritz residual estimates,
// column selection and copies for locking / thick restart, row scaling and the
// final gather of validated eigenpairs.  All are batched over probes through
// pointer tables; a probe with a zero size is skipped.
#include "common.hpp"
#include "handle.hpp"
#include "lanczos.hpp"

namespace sislice {

constexpr int LB = kLanczosBlock;  // 8

// Cholesky G = R^T R (R upper) of the 8x8 Gram matrix, computed redundantly by
// every thread, then Vout = Vin R^{-1}, Uout = Uin R^{-1} on this workgroup's rows.
// Breakdown (a pivot <= 1e-26 * max diag, or not finite) zeroes the outputs and
// raises the probe's flag.
__global__ __launch_bounds__(256) void k_cholqr_apply(CholQrArgs a) {
  const int b = blockIdx.y;
  if (!a.active[b]) return;
  __shared__ double R[LB][LB];
  __shared__ double Ri[LB][LB];
  __shared__ int bad;
  if (threadIdx.x == 0) {
    const double* G = a.G[b];
    double dmax = 0.0;
    for (int i = 0; i < LB; ++i) dmax = fmax(dmax, fabs(G[i + i * LB]));
    bad = 0;
    for (int i = 0; i < LB; ++i)
      for (int j = 0; j < LB; ++j) R[i][j] = 0.0;
    for (int j = 0; j < LB; ++j) {
      double s = G[j + j * LB];
      for (int k = 0; k < j; ++k) s -= R[k][j] * R[k][j];
      if (!(s > 1e-26 * dmax) || !isfinite(s)) {
        bad = 1;
        s = 1.0;
      }
      const double rjj = sqrt(s);
      R[j][j] = rjj;
      for (int i = j + 1; i < LB; ++i) {
        double t = 0.5 * (G[j + i * LB] + G[i + j * LB]);
        for (int k = 0; k < j; ++k) t -= R[k][j] * R[k][i];
        R[j][i] = t / rjj;
      }
    }
    for (int j = 0; j < LB; ++j) {
      for (int i = 0; i < LB; ++i) Ri[i][j] = 0.0;
      Ri[j][j] = 1.0 / R[j][j];
      for (int i = j - 1; i >= 0; --i) {
        double t = 0.0;
        for (int k = i + 1; k <= j; ++k) t += R[i][k] * Ri[k][j];
        Ri[i][j] = -t / R[i][i];
      }
    }
    if (bad)
      for (int i = 0; i < LB; ++i)
        for (int j = 0; j < LB; ++j) Ri[i][j] = 0.0;
    if (blockIdx.x == 0) {
      double* Rout = a.R[b];
      for (int i = 0; i < LB; ++i)
        for (int j = 0; j < LB; ++j) Rout[i + j * LB] = R[i][j];
      a.flag[b] = bad;
    }
  }
  __syncthreads();
  const double* Vin = a.Vin[b];
  const double* Uin = a.Uin[b];
  double* Vout = a.Vout[b];
  double* Uout = a.Uout[b];
  for (int r = blockIdx.x * 256 + threadIdx.x; r < a.n; r += gridDim.x * 256) {
    double v[LB], u[LB];
#pragma unroll
    for (int c = 0; c < LB; ++c) {
      v[c] = Vin[r + (long)c * a.ldin];
      u[c] = Uin[r + (long)c * a.ldin];
    }
#pragma unroll
    for (int j = 0; j < LB; ++j) {
      double sv = 0.0, su = 0.0;
#pragma unroll
      for (int k = 0; k <= j; ++k) {
        sv += v[k] * Ri[k][j];
        su += u[k] * Ri[k][j];
      }
      Vout[r + (long)j * a.ldout] = sv;
      Uout[r + (long)j * a.ldout] = su;
    }
  }
}

void cholqr_launch(const CholQrArgs& a, int batch, hipStream_t st) {
  const unsigned nchunk = (unsigned)std::min<long>(ceil_div(a.n, 256), 64);
  SL_LAUNCH(k_cholqr_apply, dim3(nchunk, batch), dim3(256), 0, st, a);
  SL_LAUNCH_CHECK();
}

// T[r0 + i, c0 + c] (+)= S[i, c] and the mirrored entry, for i < rows, c < cols.
// Inside the diagonal block (rows c0 .. c0+cols) the two mirrored entries of S
// are averaged and written by one thread (symmetric result, no write race).
__global__ __launch_bounds__(256) void k_t_write(TWriteArgs a) {
  const int b = blockIdx.x;
  const int rows = a.rows[b];
  if (rows <= 0) return;
  const int r0 = a.r0[b], c0 = a.c0[b];
  double* T = a.T[b];
  const double* S = a.S[b];
  for (int e = threadIdx.x; e < rows * a.cols; e += 256) {
    const int i = e % rows, c = e / rows;
    const int gr = r0 + i, gc = c0 + c;
    double v = S[i + (long)c * a.lds];
    if (gr >= c0 && gr < c0 + a.cols) {
      const int ii = gr - c0;
      if (ii < c) continue;
      v = 0.5 * (v + S[(gc - r0) + (long)ii * a.lds]);
    }
    const long p = (long)gr + (long)gc * a.ldt;
    const long q = (long)gc + (long)gr * a.ldt;
    if (a.add) v += T[p];
    T[p] = v;
    T[q] = v;
  }
}

void twrite_launch(const TWriteArgs& a, int batch, hipStream_t st) {
  SL_LAUNCH(k_t_write, dim3(batch), dim3(256), 0, st, a);
  SL_LAUNCH_CHECK();
}

// Coupling block of the newest Lanczos block: Rt = R2 * R1 (both 8x8 upper),
// written into T below the last block and mirrored.
__global__ __launch_bounds__(64) void k_t_coupling(CouplingArgs a) {
  const int b = blockIdx.x;
  if (!a.active[b]) return;
  const int t = threadIdx.x, i = t / LB, j = t % LB;
  const double* R1 = a.R1[b];
  const double* R2 = a.R2[b];
  double s = 0.0;
  for (int k = 0; k < LB; ++k) s += R2[i + k * LB] * R1[k + j * LB];
  double* T = a.T[b];
  const int r0 = a.row0[b], c0 = r0 - LB;
  T[(r0 + i) + (long)(c0 + j) * a.ldt] = s;
  T[(c0 + j) + (long)(r0 + i) * a.ldt] = s;
  a.Rt[b][i + j * LB] = s;
}

void coupling_launch(const CouplingArgs& a, int batch, hipStream_t st) {
  SL_LAUNCH(k_t_coupling, dim3(batch), dim3(64), 0, st, a);
  SL_LAUNCH_CHECK();
}

// est[i] = || Rt * S[mt-8 : mt, i] ||_2  (the B-norm of Op x_i - theta_i x_i)
__global__ __launch_bounds__(128) void k_ritz_est(RitzEstArgs a) {
  const int b = blockIdx.x;
  const int mt = a.mt[b];
  if (mt <= 0) return;
  const double* S = a.S[b];
  const double* Rt = a.Rt[b];
  for (int i = threadIdx.x; i < mt; i += blockDim.x) {
    double y[LB];
#pragma unroll
    for (int k = 0; k < LB; ++k) y[k] = S[(mt - LB + k) + (long)i * a.lds];
    double nrm = 0.0;
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < LB; ++k) s += Rt[r + k * LB] * y[k];
      nrm += s * s;
    }
    a.est[b][i] = sqrt(nrm);
  }
}

void ritz_est_launch(const RitzEstArgs& a, int batch, hipStream_t st) {
  SL_LAUNCH(k_ritz_est, dim3(batch), dim3(128), 0, st, a);
  SL_LAUNCH_CHECK();
}

// out[:, c] = in[:, idx[c]] for c < count (column gather, small matrices)
__global__ __launch_bounds__(256) void k_select_cols(SelectArgs a) {
  const int b = blockIdx.y;
  const int cnt = a.count[b];
  const int rows = a.rows[b];
  const double* in = a.in[b];
  double* out = a.out[b];
  const int* idx = a.idx[b];
  for (long e = blockIdx.x * 256L + threadIdx.x; e < (long)rows * cnt; e += (long)gridDim.x * 256) {
    const int r = (int)(e % rows), c = (int)(e / rows);
    out[r + (long)c * a.ldo] = in[r + (long)idx[c] * a.ldi];
  }
}

void select_launch(const SelectArgs& a, int batch, long maxelems, hipStream_t st) {
  SL_LAUNCH(k_select_cols, dim3((unsigned)std::max<long>(1, std::min<long>(ceil_div(maxelems, 256), 1024)), batch),
                     dim3(256), 0, st, a);
  SL_LAUNCH_CHECK();
}

// dst[:, 0:ncol] = src[:, 0:ncol] (n rows), batched; ncol may be zero.
__global__ __launch_bounds__(256) void k_copy_cols(CopyArgs a) {
  const int b = blockIdx.y;
  const int nc = a.ncol[b];
  const double* src = a.src[b];
  double* dst = a.dst[b];
  for (long e = blockIdx.x * 256L + threadIdx.x; e < (long)a.n * nc; e += (long)gridDim.x * 256) {
    const int r = (int)(e % a.n), c = (int)(e / a.n);
    dst[r + (long)c * a.ldd] = src[r + (long)c * a.lds];
  }
}

void copy_launch(const CopyArgs& a, int batch, int maxcol, hipStream_t st) {
  const long tot = (long)a.n * maxcol;
  SL_LAUNCH(k_copy_cols, dim3((unsigned)std::max<long>(1, std::min<long>(ceil_div(tot, 256), 4096)), batch),
                     dim3(256), 0, st, a);
  SL_LAUNCH_CHECK();
}

// T = 0 except diag(T)[0:k] = theta_keep (thick restart)
__global__ __launch_bounds__(256) void k_t_reset(TResetArgs a) {
  const int b = blockIdx.y;
  if (!a.active[b]) return;
  double* T = a.T[b];
  const int k = a.k[b];
  const double* th = a.theta[b];
  for (long e = blockIdx.x * 256L + threadIdx.x; e < (long)a.dim * a.dim; e += (long)gridDim.x * 256) {
    const int r = (int)(e % a.dim), c = (int)(e / a.dim);
    T[r + (long)c * a.ldt] = (r == c && r < k) ? th[r] : 0.0;
  }
}

void treset_launch(const TResetArgs& a, int batch, hipStream_t st) {
  const long tot = (long)a.dim * a.dim;
  SL_LAUNCH(k_t_reset, dim3((unsigned)std::max<long>(1, std::min<long>(ceil_div(tot, 256), 256)), batch),
                     dim3(256), 0, st, a);
  SL_LAUNCH_CHECK();
}

// Row scaling: X[i, c] *= scale[i] (D^{-1/2} of the KPM operator), single matrix.
__global__ __launch_bounds__(256) void k_row_scale(int n, int ncol, const double* scale, double* X,
                                                   long ldx) {
  for (long e = blockIdx.x * 256L + threadIdx.x; e < (long)n * ncol; e += (long)gridDim.x * 256) {
    const int r = (int)(e % n), c = (int)(e / n);
    X[r + (long)c * ldx] *= scale[r];
  }
}

// scale[i] = 1 / sqrt(D[i]) from the diagonal of an LD factor (pivot-free LDL^T of SPD B)
__global__ __launch_bounds__(256) void k_inv_sqrt_diag(int n, const double* LD, long ldld,
                                                       double* scale, int* bad) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const double d = LD[i + (long)i * ldld];
    if (!(d > 0.0)) *bad = 1;
    scale[i] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  }
}

void row_scale_launch(int n, int ncol, const double* scale, double* X, long ldx, hipStream_t st) {
  const long tot = (long)n * ncol;
  SL_LAUNCH(k_row_scale, dim3((unsigned)std::max<long>(1, std::min<long>(ceil_div(tot, 256), 4096))),
                     dim3(256), 0, st, n, ncol, scale, X, ldx);
  SL_LAUNCH_CHECK();
}

void inv_sqrt_diag_launch(int n, const double* LD, long ldld, double* scale, int* bad,
                          hipStream_t st) {
  SL_LAUNCH(k_inv_sqrt_diag, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n, LD,
                     ldld, scale, bad);
  SL_LAUNCH_CHECK();
}

// Final gather: column c of the output gets column src_col[c] of matrix src[c].
__global__ __launch_bounds__(256) void k_gather_out(GatherArgs a) {
  const int c = blockIdx.y;
  const double* src = a.src[c] + (long)a.src_col[c] * a.lds;
  double* dst = a.dst + (long)c * a.ldd;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < a.n; r += gridDim.x * 256) dst[r] = src[r];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.evals[c] = a.val[c];
    a.resid[c] = a.res[c];
  }
}

void gather_launch(const GatherArgs& a, int count, hipStream_t st) {
  if (count <= 0) return;
  SL_LAUNCH(k_gather_out, dim3((unsigned)std::min<long>(ceil_div(a.n, 256), 64), count),
                     dim3(256), 0, st, a);
  SL_LAUNCH_CHECK();
}

}  // namespace sislice
