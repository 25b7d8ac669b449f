// Eigenpair adjoint kernels: the occupied-occupied middle matrices, the
// column-wise preconditioned conjugate gradients of the projected solves, and
// the fused symmetric rank-2m outputs G_A, G_B (first-order perturbation theory
// of the symmetric-definite pencil of Section 1).
//
// Design (gfx950): the projected solves are n_e independent SPD systems, one
// per eigenvalue, solved together.  Every conjugate-gradient scalar stays on
// the device: one workgroup owns a column, reduces its dot products in a fixed
// order (deterministic) and applies the update in the same launch, so an
// iteration is one GEMM (A and B applied at once), the grouped shift-invert
// sweeps, two projection GEMMs and two column kernels, with no host round trip.
// The outputs are two symmetric rank-2m products with the same X: one launch
// computes the lower 64x64 tiles of both on FP64 MFMA (operand loads shared)
// and mirrors them through LDS, so G_A and G_B are exactly symmetric.
#include "adjoint.hpp"
#include "handle.hpp"

namespace sislice {

// ------------------------------------------------------------ middle matrices

__global__ __launch_bounds__(256) void k_adj_mid(int m, const double* __restrict__ lam,
                                                 const double* __restrict__ glam,
                                                 const double* __restrict__ K, long ldk,
                                                 double degtol, double* __restrict__ MA,
                                                 double* __restrict__ MB, long ldm) {
  const long e = blockIdx.x * 256L + threadIdx.x;
  if (e >= (long)m * m) return;
  const int j = (int)(e % m), i = (int)(e / m);  // entry (j, i): row j, column i
  const double li = lam[i], lj = lam[j];
  double ma, mb;
  if (i == j) {
    const double g = glam ? glam[i] : 0.0;
    const double kii = K ? K[i + (long)i * ldk] : 0.0;
    ma = g;
    mb = -li * g - 0.5 * kii;
  } else {
    const double kji = K ? K[j + (long)i * ldk] : 0.0;
    const double kij = K ? K[i + (long)j * ldk] : 0.0;
    const double s = 0.5 * (kji + kij), t = 0.5 * (kji - kij);
    const double d = li - lj;
    const double tf = fabs(d) > degtol ? t / d : 0.0;
    ma = tf;
    mb = -0.5 * s - 0.5 * (li + lj) * tf;
  }
  MA[j + (long)i * ldm] = ma;
  MB[j + (long)i * ldm] = mb;
}

void adj_mid_launch(int m, const double* lam, const double* glam, const double* K, long ldk,
                    double degtol, double* MA, double* MB, long ldm, hipStream_t st) {
  if (m <= 0) return;
  const long tot = (long)m * m;
  SL_LAUNCH(k_adj_mid, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, st, m, lam, glam, K, ldk,
            degtol, MA, MB, ldm);
  SL_LAUNCH_CHECK();
}

// ------------------------------------------------------------ right-hand sides

__global__ __launch_bounds__(256) void k_adj_rhs(int n, const int* __restrict__ col_of,
                                                 const double* __restrict__ E, long lde,
                                                 const double* __restrict__ G, long ldg,
                                                 const double* __restrict__ lam,
                                                 double* __restrict__ R, long ldr,
                                                 double* __restrict__ lamc) {
  const int t = blockIdx.y;
  const int c = col_of[t];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) R[i + (long)t * ldr] = c >= 0 ? E[i + (long)c * lde] - G[i + (long)c * ldg] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) lamc[t] = c >= 0 ? lam[c] : 0.0;
}

void adj_rhs_launch(int n, int np, const int* col_of, const double* E, long lde, const double* G,
                    long ldg, const double* lam, double* R, long ldr, double* lamc, hipStream_t st) {
  if (n <= 0 || np <= 0) return;
  SL_LAUNCH(k_adj_rhs, dim3((unsigned)ceil_div(n, 256), np), dim3(256), 0, st, n, col_of, E, lde, G,
            ldg, lam, R, ldr, lamc);
  SL_LAUNCH_CHECK();
}

// ------------------------------------------------------------ conjugate gradients

// Sum of v over the 256-thread workgroup in a fixed order; every thread gets it.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_pcg_init(PcgArgs a) {
  __shared__ double red[4];
  const int t = blockIdx.x;
  const long n = a.n;
  double* P = a.Pst + t * a.ldp;
  const double* R = a.R + t * a.ld;
  const double* Y = a.Y + t * a.ld;
  double* Z = a.Z + t * a.ld;
  const double lm = a.lamc[t];
  double ry = 0.0, rr = 0.0;
  for (long i = threadIdx.x; i < n; i += 256) {
    const double r = R[i], y = Y[i];
    ry += r * y;
    rr += r * r;
    P[i] = y;
    P[n + i] = -lm * y;
    Z[i] = 0.0;
  }
  ry = block_sum(ry, red);
  rr = block_sum(rr, red);
  if (threadIdx.x == 0) {
    a.rho[t] = ry;
    a.bn2[t] = rr;
    a.rrel[t] = rr > 0.0 ? 1.0 : 0.0;
    a.act[t] = rr > 0.0 ? 1 : 0;
    a.nrest[t] = 0;
  }
}

void pcg_init_launch(const PcgArgs& a, hipStream_t st) {
  if (a.np <= 0) return;
  SL_LAUNCH(k_pcg_init, dim3(a.np), dim3(256), 0, st, a);
  SL_LAUNCH_CHECK();
}

__global__ __launch_bounds__(256) void k_pcg_alpha(PcgArgs a) {
  __shared__ double red[4];
  const int t = blockIdx.x;
  if (a.act[t] != 1) return;
  const long n = a.n;
  const double* P = a.Pst + t * a.ldp;
  const double* Q = a.Q + t * a.ldq;
  double* Z = a.Z + t * a.ld;
  double* R = a.R + t * a.ld;
  const double* Y = a.Y + t * a.ld;
  double pq = 0.0;
  for (long i = threadIdx.x; i < n; i += 256) pq += P[i] * Q[i];
  pq = block_sum(pq, red);
  if (!(pq > 0.0)) {  // positive definite in exact arithmetic: restart the direction
    if (threadIdx.x == 0) a.act[t] = 3;
    return;
  }
  const double al = a.rho[t] / pq;
  double ryo = 0.0;
  for (long i = threadIdx.x; i < n; i += 256) {
    Z[i] += al * P[i];
    const double r = R[i] - al * Q[i];
    R[i] = r;
    ryo += r * Y[i];
  }
  ryo = block_sum(ryo, red);
  if (threadIdx.x == 0) a.ryo[t] = ryo;
}

void pcg_alpha_launch(const PcgArgs& a, hipStream_t st) {
  if (a.np <= 0) return;
  SL_LAUNCH(k_pcg_alpha, dim3(a.np), dim3(256), 0, st, a);
  SL_LAUNCH_CHECK();
}

__global__ __launch_bounds__(256) void k_pcg_beta(PcgArgs a) {
  __shared__ double red[4];
  const int t = blockIdx.x;
  const int st = a.act[t];
  if (st != 1 && st != 3) return;
  const long n = a.n;
  double* P = a.Pst + t * a.ldp;
  const double* R = a.R + t * a.ld;
  const double* Y = a.Y + t * a.ld;
  const double lm = a.lamc[t];
  double ry = 0.0, rr = 0.0;
  for (long i = threadIdx.x; i < n; i += 256) {
    const double r = R[i];
    ry += r * Y[i];
    rr += r * r;
  }
  ry = block_sum(ry, red);
  rr = block_sum(rr, red);
  const double b2 = a.bn2[t];
  if (rr <= a.tol2 * b2) {
    if (threadIdx.x == 0) {
      a.act[t] = 0;
      a.rrel[t] = rr / b2;
    }
    return;
  }
  double be = 0.0;
  if (st == 1) {
    be = (ry - a.ryo[t]) / a.rho[t];  // Polak-Ribiere
    if (!(be > 0.0)) be = 0.0;
  } else if (a.nrest[t] >= kPcgMaxRestarts) {
    if (threadIdx.x == 0) {
      a.act[t] = 2;
      a.rrel[t] = rr / b2;
    }
    return;
  }
  for (long i = threadIdx.x; i < n; i += 256) {
    const double p = Y[i] + be * P[i];
    P[i] = p;
    P[n + i] = -lm * p;
  }
  if (threadIdx.x == 0) {
    a.rho[t] = ry;
    a.rrel[t] = rr / b2;
    if (st == 3) {
      a.act[t] = 1;
      ++a.nrest[t];
    }
  }
}

void pcg_beta_launch(const PcgArgs& a, hipStream_t st) {
  if (a.np <= 0) return;
  SL_LAUNCH(k_pcg_beta, dim3(a.np), dim3(256), 0, st, a);
  SL_LAUNCH_CHECK();
}

// ------------------------------------------------------------ outputs

__global__ __launch_bounds__(256) void k_adj_combine(int n, const double* __restrict__ Z, long ldz,
                                                     const int* __restrict__ slot,
                                                     const double* __restrict__ lam,
                                                     double* __restrict__ Ua, double* __restrict__ Ub,
                                                     long ldu) {
  const int c = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double z = 0.5 * Z[i + (long)slot[c] * ldz];
  Ua[i + (long)c * ldu] += z;
  Ub[i + (long)c * ldu] -= lam[c] * z;
}

void adj_combine_launch(int n, int m, const double* Z, long ldz, const int* slot, const double* lam,
                        double* Ua, double* Ub, long ldu, hipStream_t st) {
  if (n <= 0 || m <= 0) return;
  SL_LAUNCH(k_adj_combine, dim3((unsigned)ceil_div(n, 256), m), dim3(256), 0, st, n, Z, ldz, slot,
            lam, Ua, Ub, ldu);
  SL_LAUNCH_CHECK();
}

// G = U X^T + X U^T for U in {Ua, Ub}: workgroup = one lower 64x64 tile of both
// outputs, wavefront = a 32x32 quarter built from 2x2 MFMA 16x16x4 blocks.  The
// accumulator element r of lane l holds G(i0 + l % 16, j0 + l / 16 + 4 r).  The
// k loop runs over the m columns once, feeding both products of both outputs;
// the operands of step k + 1 are loaded while step k's MFMAs issue.  Tiles below
// the diagonal are stored directly and, transposed through LDS, to the mirror
// tile; diagonal tiles store their lower triangle and its mirror.
__global__ __launch_bounds__(256) void k_adj_syr2k(int n, int m, const double* __restrict__ X,
                                                   long ldx, const double* __restrict__ Ua,
                                                   const double* __restrict__ Ub, long ldu,
                                                   double* __restrict__ GA, long ldga,
                                                   double* __restrict__ GB, long ldgb) {
  __shared__ double sT[64][65];
  const int lin = blockIdx.x;
  int ti = (int)((sqrt(8.0 * lin + 1.0) - 1.0) * 0.5);
  while (ti * (ti + 1) / 2 > lin) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= lin) ++ti;
  const int tj = lin - ti * (ti + 1) / 2;
  const int row0 = ti * 64, col0 = tj * 64;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
  const int lr = l & 15, lk = l >> 4;
  int ri[2], cj[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) ri[x] = min(row0 + wi + 16 * x + lr, n - 1);
#pragma unroll
  for (int y = 0; y < 2; ++y) cj[y] = min(col0 + wj + 16 * y + lr, n - 1);
  d4 accA[2][2], accB[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      accA[x][y] = d4{0.0, 0.0, 0.0, 0.0};
      accB[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    }
  // operands of one k-step: rows (X, Ua, Ub at ri) and columns (X, Ua, Ub at cj)
  struct Ops {
    double xr[2], ar[2], br[2], xc[2], ac[2], bc[2];
  };
  auto load = [&](int ks, Ops& o) {
    const int k = 4 * ks + lk;
    const bool kv = k < m;
    const long kx = (long)(kv ? k : 0) * ldx, ku = (long)(kv ? k : 0) * ldu;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const double vx = X[ri[x] + kx], va = Ua[ri[x] + ku], vb = Ub[ri[x] + ku];
      o.xr[x] = kv ? vx : 0.0;
      o.ar[x] = kv ? va : 0.0;
      o.br[x] = kv ? vb : 0.0;
    }
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const double vx = X[cj[y] + kx], va = Ua[cj[y] + ku], vb = Ub[cj[y] + ku];
      o.xc[y] = kv ? vx : 0.0;
      o.ac[y] = kv ? va : 0.0;
      o.bc[y] = kv ? vb : 0.0;
    }
  };
  auto step = [&](const Ops& o) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        accA[x][y] = mfma16x16x4(o.xc[y], o.ar[x], accA[x][y]);
        accA[x][y] = mfma16x16x4(o.ac[y], o.xr[x], accA[x][y]);
        accB[x][y] = mfma16x16x4(o.xc[y], o.br[x], accB[x][y]);
        accB[x][y] = mfma16x16x4(o.bc[y], o.xr[x], accB[x][y]);
      }
  };
  const int nks = (m + 3) >> 2;
  Ops o0, o1;
  load(0, o0);
  for (int ks = 0; ks < nks; ks += 2) {
    if (ks + 1 < nks) load(ks + 1, o1);
    step(o0);
    if (ks + 1 < nks) {
      if (ks + 2 < nks) load(ks + 2, o0);
      step(o1);
    }
  }
  const bool diag = ti == tj;
  auto store = [&](const d4 (&acc)[2][2], double* G, long ldg) {
    __syncthreads();  // sT is free (the previous output is stored)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int li = wi + 16 * x + lr, lj = wj + 16 * y + lk + 4 * r;
          sT[li][lj] = acc[x][y][r];
          const int i = row0 + li, j = col0 + lj;
          if (!diag && i < n && j < n) G[i + (long)j * ldg] = acc[x][y][r];
        }
    __syncthreads();
    // coalesced stores: the mirror tile (and, on the diagonal, the whole tile)
    const int a = tid & 63;
    for (int b = tid >> 6; b < 64; b += 4) {
      if (diag) {
        const int i = row0 + a, j = col0 + b;  // element (i, j) of the diagonal tile
        if (i < n && j < n) G[i + (long)j * ldg] = a >= b ? sT[a][b] : sT[b][a];
      } else {
        const int i = col0 + a, j = row0 + b;  // mirror element (i, j) = (j, i) of the tile
        if (i < n && j < n) G[i + (long)j * ldg] = sT[b][a];
      }
    }
  };
  store(accA, GA, ldga);
  store(accB, GB, ldgb);
}

void adj_syr2k_launch(int n, int m, const double* X, long ldx, const double* Ua, const double* Ub,
                      long ldu, double* GA, long ldga, double* GB, long ldgb, hipStream_t st) {
  if (n <= 0) return;
  const long T = ceil_div(n, 64);
  SL_LAUNCH(k_adj_syr2k, dim3((unsigned)(T * (T + 1) / 2)), dim3(256), 0, st, n, m, X, ldx, Ua, Ub,
            ldu, GA, ldga, GB, ldgb);
  SL_LAUNCH_CHECK();
}

}  // namespace sislice
