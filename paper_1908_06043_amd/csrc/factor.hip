// Blocked Bunch-Kaufman LDL^T of C = A - sigma B for several shifts at once,
// and the Sylvester inertia read from D.
//
// The paper (Section 2.1) identifies this factorization as the major cost of a
// spectral probe and (Section 2.2) reads the exact eigenvalue count below sigma
// from D.  The pivoting rule is Bunch-Kaufman's (alpha = (1+sqrt 17)/8).
//
// Design (gfx950): every shift of the GPU's share advances in lock step.
//   * k_bk_panel: one 1024-thread workgroup per shift factors a panel of up to nb
//     columns in the "lazy" form S = A_trail - L_panel W_panel^T: each column of
//     S (and the pivot-candidate column when Bunch-Kaufman needs it) is formed by
//     a GEMV against the panel so far, pivots are chosen by block-wide argmax
//     reductions, symmetric interchanges are applied to the not-yet-updated
//     trailing matrix (lower storage) and to the panel rows.
//   * k_trailing_update: the lower triangle of the trailing matrix is updated
//     with C22 -= L21 W21^T on FP64 MFMA (v_mfma_f64_16x16x4), 64x64 tiles, all
//     shifts in one launch.
//   * Interchanges found in later panels are applied to earlier L columns once at
//     the end (k_perm_suffix builds the suffix permutations, k_left_gather moves
//     the rows), so that P C P^T = L D L^T with a single permutation P.
// Panel widths depend on the pivots (nb-1 or nb columns), so the per-shift
// progress lives in device memory (FactorState) and the host launches an upper
// bound of panel/update pairs; launches past the end return at once.
#include <algorithm>
#include <climits>

#include "common.hpp"
#include "handle.hpp"
#include "kernels.hpp"

namespace sislice {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ void wave_argmax(double& v, int& i) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(i, off);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
}

// Block-wide (max |value|, smallest index) reduction; every thread gets the result.
template <int NW>
__device__ __forceinline__ void block_argmax(double& v, int& i, double* rv, int* ri) {
  wave_argmax(v, i);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    rv[w] = v;
    ri[w] = i;
  }
  __syncthreads();
  v = rv[0];
  i = ri[0];
#pragma unroll
  for (int q = 1; q < NW; ++q) {
    const double ov = rv[q];
    const int oi = ri[q];
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------------ kernels

// LD[i, j] = A[i, j] - sigma_s B[i, j] on the lower triangle (Algorithm 2, step 2).
__global__ __launch_bounds__(256) void k_shift_form(int n, const double* __restrict__ A, long lda,
                                                    const double* __restrict__ B, long ldb,
                                                    const double* __restrict__ sigmas,
                                                    double* const* LDs, long ldld) {
  const int j = blockIdx.x;
  const int s = blockIdx.y;
  const double sg = sigmas[s];
  double* LD = LDs[s];
  for (int i = j + threadIdx.x; i < n; i += blockDim.x)
    LD[i + (long)j * ldld] = A[i + (long)j * lda] - sg * B[i + (long)j * ldb];
}

__global__ __launch_bounds__(256) void k_factor_init(int n, FactorState* states, int* const* perms,
                                                     int* const* swps) {
  const int s = blockIdx.y;
  int* perm = perms[s];
  int* sw = swps[s];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    perm[i] = i;
    sw[i] = i;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    FactorState z;
    z.k0 = 0;
    z.kb = 0;
    z.done = (n == 0);
    z.npanel = 0;
    z.neg = z.zero = z.pos = 0;
    z.jstart = 0;
    z.pad = 0;
    states[s] = z;
  }
}


// ---------------------------------------------------------------- pivot-free path
//
// Bunch-Kaufman takes a 1x1 pivot without interchange at column k exactly when
// |d_k| >= alpha * max_{i>k} |s_ik| for the Schur-complement column s at step k.
// As long as that holds for every column, the factorization is the pivot-free
// LDL^T, which parallelises like Cholesky: the panel's diagonal block is factored
// in LDS (k_fast_diag), the rows below follow from one triangular solve with the
// block (k_fast_trsm: W21 = C21 L11^{-T}, L21 = W21 D1^{-1}) together with the
// column maxima of |W|, and k_fast_commit accepts the longest prefix of columns
// that pass the test.  The pivoting panel kernel then continues from the first
// rejected column, so the result is the Bunch-Kaufman factorization itself.

__device__ __forceinline__ double u64_to_f64(unsigned long long v) { return __longlong_as_double((long long)v); }

__global__ __launch_bounds__(256) void k_fast_diag(int n, const double* const* LDs, long ldld,
                                                   double* const* Wps, long ldw,
                                                   double* const* Lps, double* const* auxs,
                                                   const FactorState* states, int nb) {
  // A: the diagonal block, eliminated in place (column k holds the unscaled W
  // column of step k once step k - 1 is done); X: L11^{-1}, built alongside by
  // applying every elimination step to the identity.
  __shared__ double A[kMaxNb][kMaxNb + 1];
  __shared__ double X[kMaxNb][kMaxNb + 1];
  const int s = blockIdx.x, tid = threadIdx.x;
  const FactorState st = states[s];
  const int k0 = st.k0 + st.kb;
  if (st.done || k0 >= n) return;
  const int nbe = min(nb, n - k0);
  const double* LD = LDs[s];
  double* Wp = Wps[s];
  double* Lp = Lps[s];
  double* aux = auxs[s];
  double* Dv = aux;
  double* cin = aux + nb;
  unsigned long long* cout = reinterpret_cast<unsigned long long*>(aux + 2 * nb);
  double* Linv = aux + 3 * nb;
  const int cl = tid & (kMaxNb - 1), rg = tid >> 6;  // column of this lane, row phase 0..3
  for (int i = rg; i < kMaxNb; i += 4) {
    A[i][cl] = (i < nbe && cl < nbe && i >= cl) ? LD[(k0 + i) + (long)(k0 + cl) * ldld] : 0.0;
    X[i][cl] = (i == cl) ? 1.0 : 0.0;
  }
  for (int c = tid; c < nb; c += 256) cout[c] = 0ull;
  __syncthreads();
  for (int k = 0; k + 1 < nbe; ++k) {
    const double d = A[k][k];
    // trailing lower part of the block: A[i][j] -= A[i][k] A[j][k] / d, i >= j > k
    if (cl > k && cl < nbe) {
      const double ljk = A[cl][k] / d;
      for (int i = cl + rg; i < nbe; i += 4) A[i][cl] -= A[i][k] * ljk;
    }
    // rows below k of L^{-1}: X[i][c] -= (A[i][k] / d) X[k][c], c <= k < i
    if (cl <= k) {
      const double xkc = X[k][cl];
      for (int i = k + 1 + rg; i < nbe; i += 4) X[i][cl] -= (A[i][k] / d) * xkc;
    }
    __syncthreads();
  }
  // outputs: D, unscaled W and scaled L of the block, column maxima inside the
  // block, L11^{-1} column-major
  for (int i = rg; i < nbe; i += 4) {
    if (cl < nbe && i >= cl) {
      const double w = A[i][cl];
      Wp[(k0 + i) + (long)cl * ldw] = w;
      if (i > cl) Lp[(k0 + i) + (long)cl * ldw] = w / A[cl][cl];
    }
    if (cl < nbe) Linv[i + (long)cl * nb] = (i >= cl) ? X[i][cl] : 0.0;
  }
  if (tid < nbe) {
    const int k = tid;
    double mx = 0.0;
    for (int i = k + 1; i < nbe; ++i) {
      const double a = fabs(A[i][k]);
      mx = (a > mx || a != a) ? a : mx;
    }
    cin[k] = mx;
    Dv[k] = A[k][k];
  }
}

__global__ __launch_bounds__(256) void k_fast_trsm(int n, const double* const* LDs, long ldld,
                                                   double* const* Wps, long ldw,
                                                   double* const* Lps, double* const* auxs,
                                                   const FactorState* states, int nb) {
  __shared__ double C[64][kMaxNb + 1];
  __shared__ double Li[kMaxNb][kMaxNb + 1];
  __shared__ double Dsh[kMaxNb];
  const int s = blockIdx.y, tid = threadIdx.x;
  const FactorState st = states[s];
  const int k0 = st.k0 + st.kb;
  if (st.done || k0 >= n) return;
  const int nbe = min(nb, n - k0);
  const int r0 = k0 + nbe + 64 * blockIdx.x;
  if (r0 >= n) return;
  const double* LD = LDs[s];
  double* Wp = Wps[s];
  double* Lp = Lps[s];
  const double* aux = auxs[s];
  unsigned long long* cout = reinterpret_cast<unsigned long long*>(const_cast<double*>(aux) + 2 * nb);
  const double* Linv = aux + 3 * nb;
  for (int e = tid; e < 64 * nbe; e += 256) {
    const int r = e & 63, k = e >> 6;
    C[r][k] = (r0 + r < n) ? LD[(r0 + r) + (long)(k0 + k) * ldld] : 0.0;
  }
  for (int e = tid; e < nbe * nbe; e += 256) {
    const int i = e % nbe, k = e / nbe;
    Li[i][k] = Linv[i + (long)k * nb];
  }
  if (tid < nbe) Dsh[tid] = aux[tid];
  __syncthreads();
  // wavefront cg handles columns cg, cg+4, ...; lane r handles row r0 + r
  const int r = tid & 63, cg = tid >> 6;
  for (int c = cg; c < nbe; c += 4) {
    double w = 0.0;
    for (int k = 0; k <= c; ++k) w += C[r][k] * Li[c][k];
    if (r0 + r < n) {
      Wp[(r0 + r) + (long)c * ldw] = w;
      Lp[(r0 + r) + (long)c * ldw] = w / Dsh[c];
    }
    double mx = (r0 + r < n) ? fabs(w) : 0.0;
    if (mx != mx) mx = __longlong_as_double(0x7FF0000000000000ll);  // NaN ranks as +inf
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if (r == 0) atomicMax(cout + c, (unsigned long long)__double_as_longlong(mx));
  }
}

template <bool PIVOT>
__global__ __launch_bounds__(256) void k_fast_commit(int n, double* const* LDs, long ldld,
                                                     const double* const* Lps, long ldw,
                                                     const double* const* auxs, int* const* blks,
                                                     int* const* colpanels, FactorState* states,
                                                     int nb) {
  __shared__ int js;
  const int s = blockIdx.y, c = blockIdx.x, tid = threadIdx.x;
  const FactorState st = states[s];
  const int k0 = st.k0 + st.kb;
  if (st.done || k0 >= n) return;
  const int nbe = min(nb, n - k0);
  if (c >= nbe) return;
  const double* aux = auxs[s];
  const double* Dv = aux;
  const double* cin = aux + nb;
  const unsigned long long* cout = reinterpret_cast<const unsigned long long*>(aux + 2 * nb);
  if (tid == 0) {
    int j = 0;
    for (; j < nbe; ++j) {
      const double d = Dv[j];
      const double cm = fmax(cin[j], u64_to_f64(cout[j]));
      bool ok = isfinite(d) && d != 0.0 && isfinite(cm) && cin[j] == cin[j];
      if (PIVOT) ok = ok && fabs(d) >= kBkAlpha * cm;
      if (!ok) break;
    }
    js = j;
  }
  __syncthreads();
  const int jst = js;
  if (c < jst) {
    double* LD = LDs[s];
    const double* Lp = Lps[s];
    const int col = k0 + c;
    for (int i = col + 1 + tid; i < n; i += 256) LD[i + (long)col * ldld] = Lp[i + (long)c * ldw];
    if (tid == 0) {
      LD[col + (long)col * ldld] = Dv[c];
      blks[s][col] = 1;
      colpanels[s][col] = st.npanel;
    }
  }
  if (c == 0 && tid == 0) {
    long neg = 0, pos = 0;
    for (int q = 0; q < jst; ++q) {
      if (Dv[q] < 0.0)
        ++neg;
      else
        ++pos;
    }
    states[s].jstart = jst;
    states[s].neg += neg;
    states[s].pos += pos;
  }
}

template <bool PIVOT>
__global__ __launch_bounds__(1024) void k_bk_panel(int n, double* const* LDs, long ldld,
                                                   double* const* Wps, long ldw, int* const* perms,
                                                   int* const* swps, int* const* blks,
                                                   int* const* colpanels, int* const* pstarts,
                                                   FactorState* states, int nb, int nbpiv) {
  constexpr int NT = 1024, NW = NT / 64;
  const int s = blockIdx.x, tid = threadIdx.x;
  FactorState* st = states + s;
  double* __restrict__ LD = LDs[s];
  double* __restrict__ Wp = Wps[s];
  int* perm = perms[s];
  int* sw = swps[s];
  int* blk = blks[s];
  int* colpanel = colpanels[s];
  int* pstart = pstarts[s];

  __shared__ double wk[kMaxNb + 2];
  __shared__ double red_v[NW];
  __shared__ int red_i[NW];
  __shared__ double sh_absakk, sh_arr;
  __shared__ int sh_k0, sh_done, sh_panel, sh_jstart;

  if (tid == 0) {
    const int k0 = st->k0 + st->kb;
    sh_k0 = k0;
    sh_done = (k0 >= n) || st->done;
    sh_panel = st->npanel;
    sh_jstart = st->jstart;
  }
  __syncthreads();
  if (sh_done) {
    if (tid == 0) {
      st->k0 = sh_k0 < n ? sh_k0 : n;
      st->kb = 0;
      st->done = 1;
    }
    return;
  }
  const int k0 = sh_k0, P = sh_panel;
  const int rem = n - k0;
  const int jstart = sh_jstart;
  const int jmax0 = (rem <= nb) ? rem : nb - 1;
  const int jmax = min(jmax0, jstart + nbpiv);
  long neg = 0, zer = 0, pos = 0;

  int j = jstart;
  while (j < jmax) {
    const int k = k0 + j;
    // row k of the panel's W
    for (int p = tid; p < j; p += NT) wk[p] = Wp[k + (long)p * ldw];
    __syncthreads();
    // column k of the Schur complement -> W(:, j); argmax below the diagonal
    double bv = -1.0;
    int bi = INT_MAX;
    for (int i0 = k + tid; i0 < n; i0 += 2 * NT) {
      const int i1 = i0 + NT;
      const bool two = i1 < n;
      double a0 = LD[i0 + (long)k * ldld], a1 = two ? LD[i1 + (long)k * ldld] : 0.0;
      double b0 = 0.0, b1 = 0.0;
      const double* L0 = LD + i0 + (long)k0 * ldld;
      const double* L1 = LD + (two ? i1 : i0) + (long)k0 * ldld;
      int p = 0;
      for (; p + 1 < j; p += 2) {
        const double w0 = wk[p], w1 = wk[p + 1];
        const double x00 = L0[(long)p * ldld], x01 = L0[(long)(p + 1) * ldld];
        const double x10 = L1[(long)p * ldld], x11 = L1[(long)(p + 1) * ldld];
        a0 -= x00 * w0;
        b0 -= x01 * w1;
        a1 -= x10 * w0;
        b1 -= x11 * w1;
      }
      if (p < j) {
        a0 -= L0[(long)p * ldld] * wk[p];
        a1 -= L1[(long)p * ldld] * wk[p];
      }
      a0 += b0;
      a1 += b1;
      Wp[i0 + (long)j * ldw] = a0;
      if (two) Wp[i1 + (long)j * ldw] = a1;
      if (i0 == k) {
        sh_absakk = fabs(a0);
      } else {
        const double a = fabs(a0);
        if (a > bv) {
          bv = a;
          bi = i0;
        }
      }
      if (two) {
        const double a = fabs(a1);
        if (a > bv) {
          bv = a;
          bi = i1;
        }
      }
    }
    block_argmax<NW>(bv, bi, red_v, red_i);
    const double absakk = sh_absakk;
    const double colmax = bv > 0.0 ? bv : 0.0;
    const int imax = bi;

    int kstep = 1, kp = k;
    if (PIVOT && absakk < kBkAlpha * colmax) {
      // candidate column imax of the Schur complement -> W(:, j+1)
      for (int p = tid; p < j; p += NT) wk[p] = Wp[imax + (long)p * ldw];
      __syncthreads();
      double rv = -1.0;
      int ri = INT_MAX;
      for (int i = k + tid; i < n; i += NT) {
        double acc = (i < imax) ? LD[imax + (long)i * ldld] : LD[i + (long)imax * ldld];
        const double* Lr = LD + i + (long)k0 * ldld;
        for (int p = 0; p < j; ++p) acc -= Lr[(long)p * ldld] * wk[p];
        Wp[i + (long)(j + 1) * ldw] = acc;
        if (i == imax) {
          sh_arr = fabs(acc);
        } else {
          const double a = fabs(acc);
          if (a > rv) {
            rv = a;
            ri = i;
          }
        }
      }
      block_argmax<NW>(rv, ri, red_v, red_i);
      const double rowmax = rv;
      const double arr = sh_arr;
      if (absakk * rowmax >= kBkAlpha * colmax * colmax) {
        kstep = 1;
        kp = k;
      } else if (arr >= kBkAlpha * rowmax) {
        kstep = 1;
        kp = imax;
      } else {
        kstep = 2;
        kp = imax;
      }
    }
    const int kk = k + kstep - 1;
    if (kp != kk) {
      // symmetric interchange kk <-> kp of the not-yet-updated trailing matrix:
      // kk becomes a pivot column, so only position kp needs column kk's entries
      for (int i = kk + 1 + tid; i < n; i += NT) {
        if (i == kp) continue;
        const double v = LD[i + (long)kk * ldld];
        if (i > kp)
          LD[i + (long)kp * ldld] = v;
        else
          LD[kp + (long)i * ldld] = v;
      }
      // rows kk, kp of the panel's L columns and of W
      for (int c = tid; c < j; c += NT) {
        double* a = LD + kk + (long)(k0 + c) * ldld;
        double* b = LD + kp + (long)(k0 + c) * ldld;
        const double t = *a;
        *a = *b;
        *b = t;
        double* wa = Wp + kk + (long)c * ldw;
        double* wb = Wp + kp + (long)c * ldw;
        const double tw = *wa;
        *wa = *wb;
        *wb = tw;
      }
      if (tid == 0) {
        LD[kp + (long)kp * ldld] = LD[kk + (long)kk * ldld];
        for (int q = j; q <= j + 1; ++q) {
          double* wa = Wp + kk + (long)q * ldw;
          double* wb = Wp + kp + (long)q * ldw;
          const double tw = *wa;
          *wa = *wb;
          *wb = tw;
        }
        const int tp = perm[kk];
        perm[kk] = perm[kp];
        perm[kp] = tp;
      }
    }
    if (tid == 0) {
      sw[k] = (kstep == 1) ? kp : k;
      if (kstep == 2) sw[k + 1] = kp;
    }
    __syncthreads();
    if (kstep == 1 && kp != k) {
      // the pivot column is the candidate column
      for (int i = k + tid; i < n; i += NT) Wp[i + (long)j * ldw] = Wp[i + (long)(j + 1) * ldw];
      __syncthreads();
    }
    if (kstep == 1) {
      const double d = Wp[k + (long)j * ldw];
      const double dinv = (d != 0.0) ? 1.0 / d : 0.0;
      for (int i = k + 1 + tid; i < n; i += NT)
        LD[i + (long)k * ldld] = Wp[i + (long)j * ldw] * dinv;
      if (tid == 0) {
        LD[k + (long)k * ldld] = d;
        blk[k] = 1;
        colpanel[k] = P;
        if (d < 0.0)
          ++neg;
        else if (d > 0.0)
          ++pos;
        else
          ++zer;
      }
    } else {
      const double d11 = Wp[k + (long)j * ldw];
      const double d21 = Wp[k + 1 + (long)j * ldw];
      const double d22 = Wp[k + 1 + (long)(j + 1) * ldw];
      // [l1 l2] = [w1 w2] D^{-1}, scaled by the off-diagonal d21 (never 0 here)
      const double a = d11 / d21, g = d22 / d21;
      const double t = 1.0 / (d21 * (a * g - 1.0));
      for (int i = k + 2 + tid; i < n; i += NT) {
        const double w1 = Wp[i + (long)j * ldw];
        const double w2 = Wp[i + (long)(j + 1) * ldw];
        LD[i + (long)k * ldld] = t * (g * w1 - w2);
        LD[i + (long)(k + 1) * ldld] = t * (a * w2 - w1);
      }
      if (tid == 0) {
        LD[k + (long)k * ldld] = d11;
        LD[k + 1 + (long)k * ldld] = d21;
        LD[k + 1 + (long)(k + 1) * ldld] = d22;
        blk[k] = 2;
        blk[k + 1] = 0;
        colpanel[k] = P;
        colpanel[k + 1] = P;
        const double det = d11 * d22 - d21 * d21;
        const double tr = d11 + d22;
        if (det < 0.0) {
          ++neg;
          ++pos;
        } else if (det > 0.0) {
          if (tr < 0.0)
            neg += 2;
          else
            pos += 2;
        } else {
          ++zer;
          if (tr < 0.0)
            ++neg;
          else if (tr > 0.0)
            ++pos;
          else
            ++zer;
        }
      }
    }
    __syncthreads();
    j += kstep;
  }
  if (tid == 0) {
    st->k0 = k0;
    st->kb = j;
    st->npanel = P + 1;
    st->done = (k0 + j >= n);
    st->neg += neg;
    st->zero += zer;
    st->pos += pos;
    st->jstart = 0;
    pstart[P] = k0;
  }
}

// C22 -= L21 W21^T on the lower triangle of the trailing matrix of every shift.
// 64x64 tile per 256-thread workgroup; each wavefront owns a 32x32 quarter as
// 2x2 MFMA 16x16 blocks.  The A operand is W (tile columns), the B operand is L
// (tile rows), so that accumulator element r of lane l is C(i0 + l%16,
// j0 + l/16 + 4r): sixteen consecutive rows of one column per register,
// i.e. coalesced column-major reads and writes.
__global__ __launch_bounds__(256) void k_trailing_update(int n, double* const* LDs, long ldld,
                                                         double* const* Wps, long ldw,
                                                         const FactorState* states) {
  extern __shared__ double smem[];
  const int s = blockIdx.y;
  const int k0 = states[s].k0, kb = states[s].kb;
  const int k1 = k0 + kb;
  if (kb <= 0 || k1 >= n) return;
  const int T = (n - k1 + 63) / 64;
  const int lin = blockIdx.x;
  if (lin >= T * (T + 1) / 2) return;
  int ti = (int)((sqrt(8.0 * lin + 1.0) - 1.0) * 0.5);
  while (ti * (ti + 1) / 2 > lin) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= lin) ++ti;
  const int tj = lin - ti * (ti + 1) / 2;
  const int row0 = k1 + ti * 64, col0 = k1 + tj * 64;
  const double* LD0 = LDs[s];
  double* LD = LDs[s];
  const double* Wp = Wps[s];
  const int Kp = (kb + 3) & ~3;
  double* sL = smem;            // [Kp][64]: L(row0 + i, k0 + k)
  double* sW = smem + Kp * 64;  // [Kp][64]: W(col0 + j, k)
  const int tid = threadIdx.x;
  for (int e = tid; e < Kp * 64; e += 256) {
    const int i = e & 63, k = e >> 6;
    const bool okk = k < kb;
    sL[e] = (okk && row0 + i < n) ? LD0[row0 + i + (long)(k0 + k) * ldld] : 0.0;
    sW[e] = (okk && col0 + i < n) ? Wp[col0 + i + (long)k * ldw] : 0.0;
  }
  __syncthreads();
  const int w = tid >> 6, l = tid & 63;
  const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  const int lr = l & 15, lk = l >> 4;
  for (int kk = 0; kk < Kp; kk += 4) {
    const double* pl = sL + (kk + lk) * 64;
    const double* pw = sW + (kk + lk) * 64;
    const double b0 = pl[wi + lr], b1 = pl[wi + 16 + lr];
    const double a0 = pw[wj + lr], a1 = pw[wj + 16 + lr];
    acc[0][0] = mfma16x16x4(a0, b0, acc[0][0]);
    acc[0][1] = mfma16x16x4(a1, b0, acc[0][1]);
    acc[1][0] = mfma16x16x4(a0, b1, acc[1][0]);
    acc[1][1] = mfma16x16x4(a1, b1, acc[1][1]);
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) {
    const int i = row0 + wi + 16 * bi + lr;
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jc = col0 + wj + 16 * bj + lk + 4 * r;
        if (i < n && jc < n && i >= jc) LD[i + (long)jc * ldld] -= acc[bi][bj][r];
      }
    }
  }
}

// Suffix compositions of the interchanges: for the panel ending at e, Q_e[v] is
// the final row of the entry found at row v (v >= e) when that panel finished.
__global__ __launch_bounds__(256) void k_perm_suffix(int n, const int* const* swps,
                                                     const int* const* pstarts,
                                                     const FactorState* states, int* const* snaps) {
  extern __shared__ int q[];
  const int s = blockIdx.x;
  const int* sw = swps[s];
  const int* pstart = pstarts[s];
  int* snap = snaps[s];
  const int np = states[s].npanel;
  for (int v = threadIdx.x; v < n; v += blockDim.x) q[v] = v;
  __syncthreads();
  int cur = n - 1;
  for (int P = np - 1; P >= 1; --P) {
    const int e = pstart[P];
    if (threadIdx.x == 0) {
      for (int t = cur; t >= e; --t) {
        const int p = sw[t];
        if (p != t) {
          const int x = q[t];
          q[t] = q[p];
          q[p] = x;
        }
      }
    }
    cur = e - 1;
    __syncthreads();
    for (int v = e + threadIdx.x; v < n; v += blockDim.x) snap[(long)(P - 1) * n + v] = q[v];
    __syncthreads();
  }
}

// Apply the later panels' interchanges to the rows of each finished L column.
__global__ __launch_bounds__(256) void k_left_gather(int n, double* const* LDs, long ldld,
                                                     const int* const* colpanels,
                                                     const int* const* pstarts,
                                                     const FactorState* states,
                                                     const int* const* snaps) {
  extern __shared__ double col[];
  const int c = blockIdx.x, s = blockIdx.y;
  const int P = colpanels[s][c];
  const int np = states[s].npanel;
  if (P + 1 >= np) return;
  const int e = pstarts[s][P + 1];
  if (e >= n) return;
  double* LD = LDs[s] + (long)c * ldld;
  const int* q = snaps[s] + (long)P * n;
  for (int v = e + threadIdx.x; v < n; v += blockDim.x) col[q[v] - e] = LD[v];
  __syncthreads();
  for (int i = e + threadIdx.x; i < n; i += blockDim.x) LD[i] = col[i - e];
}

// ipiv in the documented format and the inertia triple of every shift.
__global__ __launch_bounds__(256) void k_factor_finalize(int n, const int* const* perms,
                                                         const int* const* blks, int* const* ipivs,
                                                         const FactorState* states,
                                                         int64_t* inertia) {
  const int s = blockIdx.y;
  const int* perm = perms[s];
  const int* blk = blks[s];
  int* ipiv = ipivs[s];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const bool two = (blk[i] == 2) || (blk[i] == 0);
    ipiv[i] = two ? -(perm[i] + 1) : perm[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    inertia[3 * s + 0] = states[s].neg;
    inertia[3 * s + 1] = states[s].zero;
    inertia[3 * s + 2] = states[s].pos;
  }
}

// ------------------------------------------------------------------ host side

void factor_launch(const FactorPlan& fp, hipStream_t st) {
  const int n = fp.n, S = fp.nshift, nb = fp.nb;
  if (S <= 0 || n <= 0) return;
  SL_LAUNCH(k_shift_form, dim3(n, S), dim3(256), 0, st, n, fp.A, fp.lda, fp.B, fp.ldb,
                     fp.d_sigmas, fp.d_LD, fp.ldld);
  SL_LAUNCH_CHECK();
  SL_LAUNCH(k_factor_init, dim3((unsigned)ceil_div(n, 256), S), dim3(256), 0, st, n,
                     fp.d_state, fp.d_perm, fp.d_sw);
  SL_LAUNCH_CHECK();
  sislice_handle* ph = current_handle();
  const int nbpiv = fp.fast ? fp.nbpiv : nb;
  const int min_kb = factor_min_panel(nb, fp.nbpiv, fp.fast != 0);
  // Panel widths depend on the pivots: launch chunks of panel steps and read the
  // per-shift progress back between chunks (kmin = least factored prefix).
  constexpr int kChunk = 8;
  FactorState* hs = static_cast<FactorState*>(host_stage(ph, sizeof(FactorState) * S));
  long kmin = 0;
  int steps = 0;
  const int step_cap = factor_npanel_max(n, nb, fp.nbpiv, fp.fast != 0);
  SL_CHECK_ARG(step_cap <= fp.npmax, "panel bookkeeping smaller than the step bound");
  while (kmin < n && steps < step_cap) {
    for (int q = 0; q < kChunk && steps < step_cap; ++q, ++steps) {
      // lower bound of this step's first column: kmin + q * min_kb
      const long k0_lb = std::min<long>(n, kmin + (long)q * min_kb);
      if (fp.fast) {
        const int tf = prof_begin(ph, kProfPanel);
        SL_LAUNCH(k_fast_diag, dim3(S), dim3(256), 0, st, n, (const double* const*)fp.d_LD,
                           fp.ldld, fp.d_W, fp.ldw, fp.d_Lp, fp.d_aux, fp.d_state, nb);
        SL_LAUNCH_CHECK();
        const long rows = n - k0_lb - 1;
        if (rows > 0) {
          SL_LAUNCH(k_fast_trsm, dim3((unsigned)ceil_div(rows, 64), S), dim3(256), 0, st, n,
                             (const double* const*)fp.d_LD, fp.ldld, fp.d_W, fp.ldw, fp.d_Lp, fp.d_aux,
                             fp.d_state, nb);
          SL_LAUNCH_CHECK();
        }
        if (fp.pivot)
          SL_LAUNCH(k_fast_commit<true>, dim3(nb, S), dim3(256), 0, st, n, fp.d_LD, fp.ldld,
                             (const double* const*)fp.d_Lp, fp.ldw, (const double* const*)fp.d_aux,
                             fp.d_blk, fp.d_colpanel, fp.d_state, nb);
        else
          SL_LAUNCH(k_fast_commit<false>, dim3(nb, S), dim3(256), 0, st, n, fp.d_LD, fp.ldld,
                             (const double* const*)fp.d_Lp, fp.ldw, (const double* const*)fp.d_aux,
                             fp.d_blk, fp.d_colpanel, fp.d_state, nb);
        SL_LAUNCH_CHECK();
        prof_end(ph, tf);
      }
      const int tp = prof_begin(ph, kProfPanel);
      if (fp.pivot)
        SL_LAUNCH(k_bk_panel<true>, dim3(S), dim3(1024), 0, st, n, fp.d_LD, fp.ldld, fp.d_W,
                           fp.ldw, fp.d_perm, fp.d_sw, fp.d_blk, fp.d_colpanel, fp.d_pstart,
                           fp.d_state, nb, nbpiv);
      else
        SL_LAUNCH(k_bk_panel<false>, dim3(S), dim3(1024), 0, st, n, fp.d_LD, fp.ldld,
                           fp.d_W, fp.ldw, fp.d_perm, fp.d_sw, fp.d_blk, fp.d_colpanel,
                           fp.d_pstart, fp.d_state, nb, nbpiv);
      SL_LAUNCH_CHECK();
      prof_end(ph, tp);
      const long k1_lb = std::min<long>(n, k0_lb + min_kb);
      if (k1_lb >= n) continue;
      const long T = ceil_div(n - k1_lb, 64);
      const size_t lds = (size_t)2 * ((nb + 3) & ~3) * 64 * sizeof(double);
      const int tu = prof_begin(ph, kProfUpdate);
      SL_LAUNCH(k_trailing_update, dim3((unsigned)(T * (T + 1) / 2), S), dim3(256), lds,
                         st, n, fp.d_LD, fp.ldld, fp.d_W, fp.ldw, fp.d_state);
      SL_LAUNCH_CHECK();
      prof_end(ph, tu);
    }
    SL_HIP(hipMemcpyAsync(hs, fp.d_state, sizeof(FactorState) * S, hipMemcpyDeviceToHost, st));
    SL_HIP(hipStreamSynchronize(st));
    kmin = n;
    for (int q = 0; q < S; ++q) kmin = std::min<long>(kmin, hs[q].done ? n : hs[q].k0 + hs[q].kb);
  }
  SL_CHECK_ARG(kmin >= n, "factorization did not complete");
  if (fp.pivot) {
    static bool attr_set = false;
    if (!attr_set) {
      SL_HIP(hipFuncSetAttribute((const void*)k_left_gather,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
      SL_HIP(hipFuncSetAttribute((const void*)k_perm_suffix,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
      attr_set = true;
    }
    SL_LAUNCH(k_perm_suffix, dim3(S), dim3(256), (size_t)n * sizeof(int), st, n, fp.d_sw,
                       fp.d_pstart, fp.d_state, fp.d_snap);
    SL_LAUNCH_CHECK();
    SL_LAUNCH(k_left_gather, dim3(n, S), dim3(256), (size_t)n * sizeof(double), st, n,
                       fp.d_LD, fp.ldld, fp.d_colpanel, fp.d_pstart, fp.d_state, fp.d_snap);
    SL_LAUNCH_CHECK();
  }
  SL_LAUNCH(k_factor_finalize, dim3((unsigned)ceil_div(n, 256), S), dim3(256), 0, st, n,
                     fp.d_perm, fp.d_blk, fp.d_ipiv, fp.d_state, fp.d_inertia);
  SL_LAUNCH_CHECK();
}

}  // namespace sislice
