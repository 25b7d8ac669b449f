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

// LD[i, j] = A[i, j] - sigma_s B[i, j] on the lower triangle (Algorithm 2, step 2)
// for every shift s: column j per workgroup, A and B read once for all shifts.
__global__ __launch_bounds__(256) void k_shift_form(int n, int S, const double* __restrict__ A,
                                                    long lda, const double* __restrict__ B,
                                                    long ldb, const double* __restrict__ sigmas,
                                                    double* const* LDs, long ldld) {
  const int j = blockIdx.x;
  for (int i = j + threadIdx.x; i < n; i += blockDim.x) {
    const double a = A[i + (long)j * lda], b = B[i + (long)j * ldb];
    for (int s = 0; s < S; ++s) LDs[s][i + (long)j * ldld] = a - sigmas[s] * b;
  }
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
// in LDS (k_fast_diag4), the rows below follow from one triangular solve with the
// block (k_fast_trsm: W21 = C21 L11^{-T}) together with the column maxima of |W|,
// and k_fast_commit accepts the longest prefix of columns that pass the test and
// writes their L = W D^{-1}.  The pivoting panel kernel then continues from the first
// rejected column, so the result is the Bunch-Kaufman factorization itself.

__device__ __forceinline__ double u64_to_f64(unsigned long long v) { return __longlong_as_double((long long)v); }


// Pivot-free LDL^T of the panel's diagonal block (nbe <= NB columns), one
// 256-thread workgroup per shift: lane q of row i holds the columns q + 4m of the
// row, so each step's update is a quarter of the row per lane, at the price of two
// workgroup barriers per step (the pivot and the multipliers l_ck = A[c][k] / d go
// through LDS).  The register window is rotated by one register every four steps,
// which keeps every register index static (the pivot column of step k = t0 + kk is
// register 0 of the lanes q == kk).  The finished W columns are kept in LDS for the
// outputs: the block's rows of W (unscaled), D, the in-block column maxima of |W|,
// and L11 column-major for the row solves of k_fast_trsm.
template <int NB>
__global__ __launch_bounds__(256) void k_fast_diag4(int n, const double* const* LDs, long ldld,
                                                    double* const* Wps, long ldw,
                                                    double* const* auxs,
                                                    const FactorState* states, int nb) {
  constexpr int M = NB / 4;
  __shared__ double Wb[NB][NB + 1];  // Wb[i][k]: final W of column k (rows >= k)
  __shared__ double lcol[2 * NB];    // multipliers; zero past NB (window registers past the block)
  __shared__ double dsh;
  const int s = blockIdx.x, tid = threadIdx.x;
  const int i = tid >> 2, q = tid & 3;
  const FactorState st = states[s];
  const int k0 = st.k0 + st.kb;
  if (st.done || k0 >= n) return;
  const int nbe = min(nb, n - k0);
  const double* LD = LDs[s];
  double* Wp = Wps[s];
  double* aux = auxs[s];
  double* Dv = aux;
  double* cin = aux + nb;
  unsigned long long* cout = reinterpret_cast<unsigned long long*>(aux + 2 * nb);
  double* L11 = aux + 3 * nb;  // column-major nb x nb, strictly lower part
  const bool row_ok = i < NB && i < nbe;
  double a[M];  // a[m] = A[i][t0 + q + 4m] for the current group start t0
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int c = q + 4 * m;
    a[m] = (row_ok && c < nbe && i >= c) ? LD[(k0 + i) + (long)(k0 + c) * ldld] : 0.0;
  }
  for (int c = tid; c < nb; c += 256) cout[c] = 0ull;
  for (int c = tid; c < 2 * NB; c += 256) lcol[c] = 0.0;
  for (int t0 = 0; t0 < nbe; t0 += 4) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = t0 + kk;
      if (k < nbe) {
        // the pivot column k is register 0 of the lanes q == kk
        if (q == kk && i < NB) {
          Wb[i][k] = a[0];
          if (i == k) dsh = a[0];
        }
        __syncthreads();
        const double r = 1.0 / dsh;
        if (q == kk && i < NB) lcol[i] = a[0] * r;
        __syncthreads();
        const double ak = (i < NB) ? Wb[i][k] : 0.0;
        // A[i][c] -= A[i][k] l_ck for the columns c = t0 + q + 4m > k of the window
        // (registers past column NB - 1 hold no column and meet zero multipliers)
        const double* lc = lcol + t0 + q;
        if (q > kk) a[0] -= ak * lc[0];
#pragma unroll
        for (int m = 1; m < M; ++m) a[m] -= ak * lc[4 * m];
      }
    }
    __syncthreads();  // lcol of this group is read before the next group rewrites it
#pragma unroll
    for (int m = 0; m + 1 < M; ++m) a[m] = a[m + 1];
    a[M - 1] = 0.0;
  }
  __syncthreads();
  // outputs: rows i >= k of each column k, coalesced over rows
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e % NB, k = e / NB;
    if (k < nbe && r < nbe) {
      const double w = Wb[r][k];
      const double lv = (r > k) ? w * (1.0 / Wb[k][k]) : 0.0;
      if (r >= k) Wp[(k0 + r) + (long)k * ldw] = w;
      L11[r + (long)k * nb] = lv;
    }
  }
  // in-block column maxima below the diagonal: lane q takes the rows r = i + 1 + q + 4t
  {
    double mx = 0.0;
    if (row_ok) {
      for (int r = i + 1 + q; r < nbe; r += 4) {
        const double v = fabs(Wb[r][i]);
        mx = (v > mx || v != v) ? v : mx;
      }
    }
#pragma unroll
    for (int off = 1; off < 4; off <<= 1) {
      const double o = __shfl_xor(mx, off);
      mx = (o > mx || o != o) ? o : mx;
    }
    if (row_ok && q == 0) {
      cin[i] = mx;
      Dv[i] = Wb[i][i];
    }
  }
}

// Rows below the diagonal block: W21 = C21 L11^{-T} by forward substitution
// along each row (w_c = c_c - sum_{q<c} w_q L11[c][q], taken right-looking so the
// updates of one step are independent) and the column maxima of |W21| (atomic max
// on the bit patterns of non-negative doubles).  The rows
// below a panel are too few to give every SIMD a wavefront when each is one
// thread, so a row is shared by four consecutive lanes: lane g of a row holds
// columns g, g + 4, ... (registers rotated by one every four steps, so the
// column of step q is always register 0 of lane q % 4), and w_q reaches the
// row's other lanes with a shuffle.  64 rows per 256-thread workgroup; L11 is
// read from LDS.
template <int NB>
__global__ __launch_bounds__(256) void k_fast_trsm(int n, const double* const* LDs, long ldld,
                                                   double* const* Wps, long ldw,
                                                   const double* const* auxs,
                                                   const FactorState* states, int nb) {
  constexpr int M = NB / 4;
  __shared__ double sL[NB * NB];  // column-major: sL[q * NB + c] = L11[c][q]
  const int s = blockIdx.y, tid = threadIdx.x;
  const FactorState st = states[s];
  const int k0 = st.k0 + st.kb;
  if (st.done || k0 >= n) return;
  const int nbe = min(nb, n - k0);
  const int r0 = k0 + nbe + 64 * blockIdx.x;
  if (r0 >= n) return;
  const double* LD = LDs[s];
  double* Wp = Wps[s];
  const double* aux = auxs[s];
  unsigned long long* cout = reinterpret_cast<unsigned long long*>(const_cast<double*>(aux) + 2 * nb);
  const double* L11 = aux + 3 * nb;
  for (int e = tid; e < NB * NB; e += 256) {
    const int c = e % NB, q = e / NB;
    sL[e] = (c < nbe && q < nbe) ? L11[c + (long)q * nb] : 0.0;
  }
  const int g = tid & 3;
  const int row = r0 + (tid >> 2);
  const bool rv = row < n;
  const double* Cr = LD + (rv ? row : n - 1) + (long)k0 * ldld;
  double w[M];  // w[m] = W[row][t0 + g + 4m] for the current group start t0
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int c = g + 4 * m;
    w[m] = (c < nbe) ? Cr[(long)c * ldld] : 0.0;
  }
  __syncthreads();
  const int lane0 = (tid & 63) & ~3;
  for (int t0 = 0; t0 < nbe; t0 += 4) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int q = t0 + kk;
      if (q < nbe) {
        const double wq = __shfl(w[0], lane0 | kk);
        const double* Lq = sL + q * NB;
        // register m holds column c = t0 + g + 4m; it is updated when c > q
        const double u0 = w[0] - wq * Lq[min(t0 + g, NB - 1)];
        w[0] = (g > kk) ? u0 : w[0];
#pragma unroll
        for (int m = 1; m < M; ++m) w[m] -= wq * Lq[min(t0 + g + 4 * m, NB - 1)];
      }
    }
    // column t0 + g is final: write it, fold it into the column maximum, rotate
    const int c0 = t0 + g;
    if (rv && c0 < nbe) Wp[row + (long)c0 * ldw] = w[0];
    double mx = (rv && c0 < nbe) ? fabs(w[0]) : 0.0;
    if (mx != mx) mx = __longlong_as_double(0x7FF0000000000000ll);  // NaN ranks as +inf
#pragma unroll
    for (int off = 4; off < 64; off <<= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if ((tid & 63) < 4 && c0 < nbe)
      atomicMax(cout + c0, (unsigned long long)__double_as_longlong(mx));
#pragma unroll
    for (int m = 0; m + 1 < M; ++m) w[m] = w[m + 1];
    w[M - 1] = 0.0;
  }
}

template <bool PIVOT>
__global__ __launch_bounds__(256) void k_fast_commit(int n, double* const* LDs, long ldld,
                                                     const double* const* Wps, long ldw,
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
  // the accepted prefix: lane j of the first wavefront judges column j (nbe <= 64),
  // and the first rejected column is the lowest set bit of the ballot
  if (tid < 64) {
    const int j = tid;
    bool ok = false;
    if (j < nbe) {
      const double d = Dv[j];
      const double cm = fmax(cin[j], u64_to_f64(cout[j]));
      ok = isfinite(d) && d != 0.0 && isfinite(cm) && cin[j] == cin[j];
      if (PIVOT) ok = ok && fabs(d) >= kBkAlpha * cm;
    }
    const unsigned long long bad = __ballot(!ok);
    if (tid == 0) js = bad ? min(__ffsll((long long)bad) - 1, nbe) : nbe;
  }
  __syncthreads();
  const int jst = js;
  if (c < jst) {
    double* LD = LDs[s];
    const double* Wp = Wps[s];
    const int col = k0 + c;
    const double rd = 1.0 / Dv[c];  // the column's multipliers l = w (1 / d)
    for (int i = col + 1 + tid; i < n; i += 256) LD[i + (long)col * ldld] = Wp[i + (long)c * ldw] * rd;
    if (tid == 0) {
      LD[col + (long)col * ldld] = Dv[c];
      blks[s][col] = 1;
      colpanels[s][col] = st.npanel;
    }
  }
  if (c == 0 && tid < 64) {
    const bool acc = tid < jst;
    const bool negd = acc && Dv[tid] < 0.0;
    const unsigned long long negm = __ballot(negd), posm = __ballot(acc && !negd);
    if (tid == 0) {
      states[s].jstart = jst;
      states[s].neg += __popcll(negm);
      states[s].pos += __popcll(posm);
    }
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
      // eight columns per step with all sixteen loads issued first (one wait per
      // step); even columns accumulate into a, odd ones into b, in column order
      int p = 0;
      for (; p + 8 <= j; p += 8) {
        double x0[8], x1[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          x0[u] = L0[(long)(p + u) * ldld];
          x1[u] = L1[(long)(p + u) * ldld];
        }
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          const double w0 = wk[p + u], w1 = wk[p + u + 1];
          a0 -= x0[u] * w0;
          b0 -= x0[u + 1] * w1;
          a1 -= x1[u] * w0;
          b1 -= x1[u + 1] * w1;
        }
      }
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
        int p = 0;
        for (; p + 8 <= j; p += 8) {
          double x[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) x[u] = Lr[(long)(p + u) * ldld];
#pragma unroll
          for (int u = 0; u < 8; ++u) acc -= x[u] * wk[p + u];
        }
        for (; p < j; ++p) acc -= Lr[(long)p * ldld] * wk[p];
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
// 2x2 v_mfma_f64_16x16x4 blocks.  The A operand is -W (tile columns), the B
// operand is L (tile rows), so that accumulator element r of lane l is
// C(i0 + l%16, j0 + l/16 + 4r): sixteen consecutive rows of one column per
// register.  The tile of C is loaded straight into the accumulators, every
// operand of the panel's K <= 64 columns is issued from global memory up front
// (no LDS, no barrier: occupancy is bounded by registers only), and the
// accumulators are stored back: one read and one write of C per panel.
__global__ __launch_bounds__(256) void k_trailing_update(int n, double* const* LDs, long ldld,
                                                         double* const* Wps, long ldw,
                                                         const FactorState* states) {
  constexpr int KS = kMaxNb / 4;  // k-steps of 4
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
  double* LD = LDs[s];
  const double* Wp = Wps[s];
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
  const int lr = l & 15, lk = l >> 4;
  const int nks = (kb + 3) >> 2;
  // tile rows / columns of this lane (clamped for the loads, masked for the stores)
  int ri[2], cj[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) ri[x] = row0 + wi + 16 * x + lr;
#pragma unroll
  for (int y = 0; y < 2; ++y) cj[y] = col0 + wj + 16 * y + lr;
  d4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = min(ri[x], n - 1), j = min(col0 + wj + 16 * y + lk + 4 * r, n - 1);
        acc[x][y][r] = LD[i + (long)j * ldld];
      }
  // operands in chunks of 4 k-steps, double-buffered: the loads of chunk c + 1 are
  // in flight while chunk c feeds the MFMAs (registers stay low enough for several
  // resident wavefronts per SIMD)
  constexpr int CK = 4;
  const int nch = (nks + CK - 1) / CK;
  double lop[2][CK][2], wop[2][CK][2];
  auto load_chunk = [&](int ch, double (&lb)[CK][2], double (&wb)[CK][2]) {
#pragma unroll
    for (int u = 0; u < CK; ++u) {
      const int k = 4 * (CK * ch + u) + lk;
      const bool kv = k < kb;
      const int kc = kv ? k : 0;
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const double v = LD[min(ri[x], n - 1) + (long)(k0 + kc) * ldld];
        lb[u][x] = kv ? v : 0.0;
      }
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const double v = Wp[min(cj[y], n - 1) + (long)kc * ldw];
        wb[u][y] = kv ? -v : 0.0;
      }
    }
  };
  auto mfma_chunk = [&](const double (&lb)[CK][2], const double (&wb)[CK][2]) {
#pragma unroll
    for (int u = 0; u < CK; ++u)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = mfma16x16x4(wb[u][y], lb[u][x], acc[x][y]);
  };
  load_chunk(0, lop[0], wop[0]);
#pragma unroll
  for (int ch = 0; ch < KS / CK; ch += 2) {
    if (ch < nch) {
      if (ch + 1 < nch) load_chunk(ch + 1, lop[1], wop[1]);
      mfma_chunk(lop[0], wop[0]);
    }
    if (ch + 1 < nch) {
      if (ch + 2 < nch) load_chunk(ch + 2, lop[0], wop[0]);
      mfma_chunk(lop[1], wop[1]);
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int i = ri[x];
#pragma unroll
    for (int y = 0; y < 2; ++y) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jc = col0 + wj + 16 * y + lk + 4 * r;
        if (i < n && jc < n && i >= jc) LD[i + (long)jc * ldld] = acc[x][y][r];
      }
    }
  }
}

// The same update on 128x128 tiles for large trailing matrices, one 1024-thread
// workgroup per tile.  Each of the 16 wavefronts owns a 32x32 block of the tile as
// 2x2 v_mfma_f64_16x16x4 blocks, so a wavefront needs 62 registers and a CU keeps
// two workgroups (eight wavefronts per SIMD) in flight; the C tile is read and
// written once per 128x128.  The operand panels of the tile (128 rows of L and 128
// rows of W, 16 k-columns per chunk) are fetched once per workgroup with coalesced
// 1 KB column runs into double-buffered LDS (66 KB), and the next chunk is in
// flight while the wavefronts run the current one's MFMAs.
// Layout per chunk and operand: [k][row], rows padded to 132 doubles so that the
// four k-groups a wavefront reads at once fall on different banks.
// With STREAM the C tile is read and written non-temporally: when the shifts run in
// two groups on two streams (large orders), C has no reuse in the caches before the
// next update, and streaming it keeps the other group's panel data resident (at
// order 12288, 49 shifts: 2975 -> 2718 us per update launch, about 2% per
// factorization).
constexpr int kUpdK = 16;           // k-columns per staged chunk
constexpr int kUpdLd = 128 + 4;     // padded row count per k-column
template <bool STREAM>
__global__ __launch_bounds__(1024) void k_trailing_update_lds(int n, double* const* LDs, long ldld,
                                                             double* const* Wps, long ldw,
                                                             const FactorState* states) {
  constexpr int TB = 128;
  __shared__ double sL[2][kUpdK * kUpdLd];
  __shared__ double sW[2][kUpdK * kUpdLd];
  const int s = blockIdx.y;
  const int k0 = states[s].k0, kb = states[s].kb;
  const int k1 = k0 + kb;
  if (kb <= 0 || k1 >= n) return;
  const int T = (n - k1 + TB - 1) / TB;
  const int lin = blockIdx.x;
  if (lin >= T * (T + 1) / 2) return;
  int ti = (int)((sqrt(8.0 * lin + 1.0) - 1.0) * 0.5);
  while (ti * (ti + 1) / 2 > lin) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= lin) ++ti;
  const int tj = lin - ti * (ti + 1) / 2;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  const int wi = (w & 3) * 32, wj = (w >> 2) * 32;
  // on a diagonal tile the blocks above the diagonal store nothing, but their
  // wavefronts still help stage the operands
  const bool active = !(ti == tj && wi + 31 < wj);
  const int row0 = k1 + ti * TB, col0 = k1 + tj * TB;
  double* LD = LDs[s];
  const double* Wp = Wps[s];
  const int lr = l & 15, lk = l >> 4;
  const int nks = (kb + 3) >> 2;             // k-steps of 4
  const int nch = (kb + kUpdK - 1) / kUpdK;  // staged chunks
  // staging: thread t fetches row (t % 128) of columns (t / 128) + 8j, j < 2
  const int sr = tid & 127, sc = tid >> 7;
  const int lrow = min(row0 + sr, n - 1), wrow = min(col0 + sr, n - 1);
  double stL[kUpdK / 8], stW[kUpdK / 8];
  auto fetch = [&](int ch) {
#pragma unroll
    for (int j = 0; j < kUpdK / 8; ++j) {
      const int k = ch * kUpdK + sc + 8 * j;
      const bool kv = k < kb;
      const int kc = kv ? k : 0;
      const double a = LD[lrow + (long)(k0 + kc) * ldld];
      const double b = Wp[wrow + (long)kc * ldw];
      stL[j] = kv ? a : 0.0;
      stW[j] = kv ? -b : 0.0;
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int j = 0; j < kUpdK / 8; ++j) {
      sL[buf][(sc + 8 * j) * kUpdLd + sr] = stL[j];
      sW[buf][(sc + 8 * j) * kUpdLd + sr] = stW[j];
    }
  };
  fetch(0);
  d4 acc[2][2];
  if (active) {
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const int i = min(row0 + wi + 16 * x + lr, n - 1);
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = min(col0 + wj + 16 * y + lk + 4 * r, n - 1);
          acc[x][y][r] = STREAM ? __builtin_nontemporal_load(LD + i + (long)j * ldld)
                                : LD[i + (long)j * ldld];
        }
    }
  }
  stage(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) fetch(ch + 1);
    if (active) {
      const double* L0 = sL[buf] + wi + lr;
      const double* W0 = sW[buf] + wj + lr;
      const int ksteps = min(kUpdK / 4, nks - ch * (kUpdK / 4));
      for (int u = 0; u < ksteps; ++u) {
        const int kk = (4 * u + lk) * kUpdLd;
        double lo[2], wo[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) lo[x] = L0[kk + 16 * x];
#pragma unroll
        for (int y = 0; y < 2; ++y) wo[y] = W0[kk + 16 * y];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = mfma16x16x4(wo[y], lo[x], acc[x][y]);
      }
    }
    if (ch + 1 < nch) {
      stage(buf ^ 1);
      __syncthreads();
    }
  }
  if (!active) return;
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int i = row0 + wi + 16 * x + lr;
#pragma unroll
    for (int y = 0; y < 2; ++y) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jc = col0 + wj + 16 * y + lk + 4 * r;
        if (i < n && jc < n && i >= jc) {
          if (STREAM)
            __builtin_nontemporal_store(acc[x][y][r], LD + i + (long)jc * ldld);
          else
            LD[i + (long)jc * ldld] = acc[x][y][r];
        }
      }
    }
  }
}

// Persistent form of the 128x128-tile update for large trailing matrices.  A
// launch has one 1024-thread workgroup per CU.  The (shift, tile) items of every
// shift are numbered shift by shift, tile rows in order, and each workgroup takes
// one contiguous run of them (the runs of the workgroups of one XCD adjacent), so
// consecutive items of a workgroup mostly lie in one tile row and share its L
// rows.  The rank-kb (<= 64) operand panels of a tile sit in LDS whole (L and -W,
// [k][row] with rows padded to 132 doubles: 135 KB), so a tile needs no barrier
// between its MFMAs; the L panel is reloaded only when the tile row changes.  The
// work is software-pipelined across a workgroup's items: while the MFMAs of item t
// run, the C tile and the W panel of item t + 1 are in flight into registers and
// the stores of item t - 1 drain.  Memory goes through buffer instructions whose
// out-of-range offsets read zero and drop stores, so rows and columns past n,
// operand columns past kb and the upper half of a diagonal tile need no branch:
// every item issues the same loads and stores, and the wait for the next item's
// loads does not wait for the stores issued after them (loads and stores retire
// in issue order).  The accumulation order per element is that of
// k_trailing_update_lds.
constexpr int kPipeMaxShifts = 256;
constexpr int kPipeK = kMaxNb;  // widest panel (update rank) the persistent update takes
// An offset past every buffer's range (the host keeps the kernel's buffers below
// it), low enough that the end of an 8-byte access does not wrap.
constexpr unsigned kPipeOob = 0xFFFFFF00u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t pipe_rsrc(const double* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), (short)0, (int)bytes, 0x00020000);
}
typedef unsigned int pipe_u2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double pipe_ld(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ void pipe_st(__amdgpu_buffer_rsrc_t r, unsigned off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(pipe_u2, v), r, (int)off, 0, 0);
}
// `off` where `ok`, else an offset out of range, without a branch (a branch that
// skipped the memory operation would make the count of outstanding operations
// differ between paths, and the waits would then wait for everything).
__device__ __forceinline__ unsigned pipe_off(bool ok, unsigned off) {
  const unsigned m = (unsigned)ok - 1u;
  return (off & ~m) | (kPipeOob & m);
}
// A pointer that every lane holds, as a scalar value.
__device__ __forceinline__ double* pipe_uniform(double* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (double*)(((unsigned long long)hi << 32) | lo);
}

__global__ __launch_bounds__(1024) void k_trailing_update_pipe(int n, double* const* LDs, long ldld,
                                                              double* const* Wps, long ldw,
                                                              const FactorState* states, int S) {
  constexpr int TB = 128;
  __shared__ double sL[kPipeK * kUpdLd];
  __shared__ double sW[kPipeK * kUpdLd];
  __shared__ int pre[kPipeMaxShifts + 1];
  // per-shift panel start and width and matrix / panel pointers, read from LDS
  // (never through the vector memory counter that the pipeline's waits count)
  __shared__ int sk0[kPipeMaxShifts], skb[kPipeMaxShifts];
  __shared__ double* sLD[kPipeMaxShifts];
  __shared__ double* sWp[kPipeMaxShifts];
  const int tid = threadIdx.x;
  for (int q = tid; q < S; q += 1024) {
    sk0[q] = states[q].k0;
    skb[q] = states[q].kb;
    sLD[q] = LDs[q];
    sWp[q] = Wps[q];
  }
  // items per shift (tiles of its trailing lower triangle) and their prefix sums
  if (tid < 64) {
    int base = 0;
    for (int q0 = 0; q0 < S; q0 += 64) {
      const int q = q0 + tid;
      int c = 0;
      if (q < S) {
        const int kb = states[q].kb, k1 = states[q].k0 + kb;
        if (kb > 0 && k1 < n) {
          const int T = (n - k1 + TB - 1) / TB;
          c = T * (T + 1) / 2;
        }
      }
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(c, off);
        if (tid >= off) c += o;
      }
      if (q < S) pre[q + 1] = base + c;
      base += __shfl(c, 63);
    }
    if (tid == 0) pre[0] = 0;
  }
  __syncthreads();
  const int M = pre[S];
  const int G = gridDim.x, b = blockIdx.x;
  const int slot = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  const int i_begin = (int)((long)M * slot / G), i_end = (int)((long)M * (slot + 1) / G);
  if (i_begin >= i_end) return;

  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  const int wi = (w & 3) * 32, wj = (w >> 2) * 32;
  const int lr = l & 15, lk = l >> 4;
  const int sr = tid & 127, sc = tid >> 7;  // staging: row sr of k-columns sc + 8j
  const unsigned ld8 = (unsigned)ldld * 8u, lw8 = (unsigned)ldw * 8u;
  const unsigned bytes_ld = (unsigned)((size_t)ldld * n * 8);
  const unsigned bytes_w = (unsigned)((size_t)ldw * (kPipeK + 2) * 8);

  struct Item {
    int s, k0, kb, ti, row0, col0;
    bool diag;
  };
  int s_cur = 0;
  auto decode = [&](int item, Item& it) {
    while (pre[s_cur + 1] <= item) ++s_cur;
    const int s = __builtin_amdgcn_readfirstlane(s_cur);
    const int lin = item - pre[s];
    int ti = (int)((sqrt(8.0 * lin + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > lin) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= lin) ++ti;
    const int tj = lin - ti * (ti + 1) / 2;
    it.s = s;
    it.k0 = __builtin_amdgcn_readfirstlane(sk0[s]);
    it.kb = __builtin_amdgcn_readfirstlane(skb[s]);
    const int k1 = it.k0 + it.kb;
    it.ti = __builtin_amdgcn_readfirstlane(ti);
    it.row0 = k1 + it.ti * TB;
    it.col0 = __builtin_amdgcn_readfirstlane(k1 + tj * TB);
    it.diag = (it.ti == tj);
  };
  double cn[2][2][4];
  double wn[kPipeK / 8];
  auto prefetch = [&](const Item& it) {
    const __amdgpu_buffer_rsrc_t rLD = pipe_rsrc(pipe_uniform(sLD[it.s]), bytes_ld);
    const __amdgpu_buffer_rsrc_t rW = pipe_rsrc(pipe_uniform(sWp[it.s]), bytes_w);
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const int i = it.row0 + wi + 16 * x + lr;
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = it.col0 + wj + 16 * y + lk + 4 * r;
          cn[x][y][r] = pipe_ld(rLD, pipe_off((i < n) & (j < n), (unsigned)i * 8u + (unsigned)j * ld8));
        }
    }
    const int wr = it.col0 + sr;
#pragma unroll
    for (int jj = 0; jj < kPipeK / 8; ++jj) {
      const int k = sc + 8 * jj;
      wn[jj] = pipe_ld(rW, pipe_off((k < it.kb) & (wr < n), (unsigned)wr * 8u + (unsigned)k * lw8));
    }
  };

  Item cur, nxt;
  int item = i_begin;
  decode(item, nxt);
  prefetch(nxt);
  {
    // the loop's sixteen stores, dropped (out of range): the loads above then have
    // as many younger memory operations on entry as on the back edge, so the wait
    // for them at the top of the loop does not wait for the stores
    const __amdgpu_buffer_rsrc_t rLD = pipe_rsrc(pipe_uniform(sLD[nxt.s]), bytes_ld);
#pragma unroll
    for (int q = 0; q < 16; ++q) pipe_st(rLD, kPipeOob + 8u * q, 0.0);
  }
  int row_s = -1, row_t = -1;  // tile row whose L panel is in LDS
  d4 acc[2][2];
  for (;;) {
    cur = nxt;
    __syncthreads();  // every wavefront is done with the previous item's operands
    if (cur.s != row_s || cur.ti != row_t) {
      const __amdgpu_buffer_rsrc_t rLD = pipe_rsrc(pipe_uniform(sLD[cur.s]), bytes_ld);
      const int li = cur.row0 + sr;
      double lv[kPipeK / 8];
#pragma unroll
      for (int jj = 0; jj < kPipeK / 8; ++jj) {
        const int k = sc + 8 * jj;
        lv[jj] = pipe_ld(rLD, pipe_off((k < cur.kb) & (li < n), (unsigned)li * 8u + (unsigned)(cur.k0 + k) * ld8));
      }
#pragma unroll
      for (int jj = 0; jj < kPipeK / 8; ++jj) sL[(sc + 8 * jj) * kUpdLd + sr] = lv[jj];
      row_s = cur.s;
      row_t = cur.ti;
    }
#pragma unroll
    for (int jj = 0; jj < kPipeK / 8; ++jj) sW[(sc + 8 * jj) * kUpdLd + sr] = -wn[jj];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[x][y][r] = cn[x][y][r];
    __syncthreads();
    // the next item's loads go out before this item's MFMAs and stores; past the
    // last item the current one is loaded again (unused), so every iteration
    // issues the same memory operations
    const bool more = item + 1 < i_end;
    if (more) decode(item + 1, nxt);
    prefetch(more ? nxt : cur);
    const bool active = !(cur.diag && wi + 31 < wj);
    if (active) {
      const double* L0 = sL + wi + lr;
      const double* W0 = sW + wj + lr;
      // k-steps of 4 in pairs (the operands past kb are zero in LDS)
      const int npair = (cur.kb + 7) >> 3;
      for (int u = 0; u < npair; ++u) {
        double lo[2][2], wo[2][2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int kk = (8 * u + 4 * h + lk) * kUpdLd;
#pragma unroll
          for (int x = 0; x < 2; ++x) lo[h][x] = L0[kk + 16 * x];
#pragma unroll
          for (int y = 0; y < 2; ++y) wo[h][y] = W0[kk + 16 * y];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) acc[x][y] = mfma16x16x4(wo[h][y], lo[h][x], acc[x][y]);
      }
    }
    {
      const __amdgpu_buffer_rsrc_t rLD = pipe_rsrc(pipe_uniform(sLD[cur.s]), bytes_ld);
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int i = cur.row0 + wi + 16 * x + lr;
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int j = cur.col0 + wj + 16 * y + lk + 4 * r;
            pipe_st(rLD, pipe_off(active & (i < n) & (j < n) & (i >= j), (unsigned)i * 8u + (unsigned)j * ld8),
                    acc[x][y][r]);
          }
      }
    }
    if (!more) break;
    ++item;
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
// The column is staged in LDS (up to n doubles), which allows one workgroup per
// CU: 1024 threads, each with four rows' loads in flight per round.
__global__ __launch_bounds__(1024) void k_left_gather(int n, double* const* LDs, long ldld,
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
  constexpr int U = 4;
  for (int v0 = e + threadIdx.x; v0 < n; v0 += U * 1024) {
    double x[U];
    int t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int v = v0 + u * 1024;
      x[u] = v < n ? LD[v] : 0.0;
      t[u] = v < n ? q[v] : e;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (v0 + u * 1024 < n) col[t[u] - e] = x[u];
  }
  __syncthreads();
  for (int i = e + threadIdx.x; i < n; i += 1024) LD[i] = col[i - e];
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

void factor_prepare() {
  static std::once_flag attr_set;
  std::call_once(attr_set, [] {
    SL_HIP(hipFuncSetAttribute((const void*)k_left_gather,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    SL_HIP(hipFuncSetAttribute((const void*)k_perm_suffix,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  });
}

void factor_shift_form_launch(const FactorPlan& fp, hipStream_t st) {
  if (fp.nshift <= 0 || fp.n <= 0) return;
  SL_LAUNCH(k_shift_form, dim3(fp.n), dim3(256), 0, st, fp.n, fp.nshift, fp.A, fp.lda, fp.B, fp.ldb,
            fp.d_sigmas, fp.d_LD, fp.ldld);
  SL_LAUNCH_CHECK();
}

// The persistent update addresses each shifted matrix and panel buffer with
// 32-bit offsets below kPipeOob and keeps the per-shift table in LDS.
static bool pipe_fits(const FactorPlan& fp) {
  return fp.nshift <= kPipeMaxShifts && (double)fp.ldld * fp.n * 8.0 < (double)kPipeOob &&
         fp.nb <= kPipeK && (double)fp.ldw * (kPipeK + 2) * 8.0 < (double)kPipeOob;
}

void factor_launch(const FactorPlan& fp, hipStream_t st) {
  factor_shift_form_launch(fp, st);
  factor_steps_launch(fp, st, true);
}

// The plan of shifts [s0, s0 + cnt): every per-shift device table offset.
static FactorPlan factor_subplan(const FactorPlan& fp, int s0, int cnt) {
  FactorPlan f = fp;
  f.nshift = cnt;
  f.d_sigmas = fp.d_sigmas ? fp.d_sigmas + s0 : nullptr;
  f.d_LD = fp.d_LD + s0;
  f.d_W = fp.d_W + s0;
  f.d_perm = fp.d_perm + s0;
  f.d_sw = fp.d_sw + s0;
  f.d_blk = fp.d_blk + s0;
  f.d_colpanel = fp.d_colpanel + s0;
  f.d_pstart = fp.d_pstart + s0;
  f.d_snap = fp.d_snap + s0;
  f.d_ipiv = fp.d_ipiv + s0;
  f.d_state = fp.d_state + s0;
  f.d_inertia = fp.d_inertia + 3 * (size_t)s0;
  f.d_aux = fp.d_aux ? fp.d_aux + s0 : nullptr;
  return f;
}

// One panel step of every shift of `fp` on stream `st`: the speculative
// pivot-free panel, the pivoting panel and the trailing update.  k0_lb is a lower
// bound on the step's first column (it sizes the update grid).  `after_panel`,
// when given, is recorded once the pivoting panel is enqueued.
static void factor_step(const FactorPlan& fp, hipStream_t st, long k0_lb, sislice_handle* ph,
                        hipEvent_t after_panel) {
  const int n = fp.n, S = fp.nshift, nb = fp.nb;
  const int nbpiv = fp.fast ? fp.nbpiv : nb;
  const int min_kb = factor_min_panel(nb, fp.nbpiv, fp.fast != 0);
  int tpan = -1;
  if (fp.fast) {
    // one timed ticket per panel step: the speculative group and the pivoting
    // panel are consecutive launches of the panel class
    tpan = prof_begin(ph, kProfPanel, st);
    const long rows = n - k0_lb - 1;
    if (nb > 32) {
      SL_LAUNCH(k_fast_diag4<64>, dim3(S), dim3(256), 0, st, n, (const double* const*)fp.d_LD,
                fp.ldld, fp.d_W, fp.ldw, fp.d_aux, fp.d_state, nb);
      SL_LAUNCH_CHECK();
      if (rows > 0) {
        SL_LAUNCH(k_fast_trsm<64>, dim3((unsigned)ceil_div(rows, 64), S), dim3(256), 0, st, n,
                  (const double* const*)fp.d_LD, fp.ldld, fp.d_W, fp.ldw,
                  (const double* const*)fp.d_aux,
                  fp.d_state, nb);
        SL_LAUNCH_CHECK();
      }
    } else {
      SL_LAUNCH(k_fast_diag4<32>, dim3(S), dim3(256), 0, st, n, (const double* const*)fp.d_LD,
                fp.ldld, fp.d_W, fp.ldw, fp.d_aux, fp.d_state, nb);
      SL_LAUNCH_CHECK();
      if (rows > 0) {
        SL_LAUNCH(k_fast_trsm<32>, dim3((unsigned)ceil_div(rows, 64), S), dim3(256), 0, st, n,
                  (const double* const*)fp.d_LD, fp.ldld, fp.d_W, fp.ldw,
                  (const double* const*)fp.d_aux,
                  fp.d_state, nb);
        SL_LAUNCH_CHECK();
      }
    }
    if (fp.pivot)
      SL_LAUNCH(k_fast_commit<true>, dim3(nb, S), dim3(256), 0, st, n, fp.d_LD, fp.ldld,
                (const double* const*)fp.d_W, fp.ldw, (const double* const*)fp.d_aux, fp.d_blk,
                fp.d_colpanel, fp.d_state, nb);
    else
      SL_LAUNCH(k_fast_commit<false>, dim3(nb, S), dim3(256), 0, st, n, fp.d_LD, fp.ldld,
                (const double* const*)fp.d_W, fp.ldw, (const double* const*)fp.d_aux, fp.d_blk,
                fp.d_colpanel, fp.d_state, nb);
    SL_LAUNCH_CHECK();
  }
  if (tpan < 0) tpan = prof_begin(ph, kProfPanel, st);
  if (fp.pivot)
    SL_LAUNCH(k_bk_panel<true>, dim3(S), dim3(1024), 0, st, n, fp.d_LD, fp.ldld, fp.d_W, fp.ldw,
              fp.d_perm, fp.d_sw, fp.d_blk, fp.d_colpanel, fp.d_pstart, fp.d_state, nb, nbpiv);
  else
    SL_LAUNCH(k_bk_panel<false>, dim3(S), dim3(1024), 0, st, n, fp.d_LD, fp.ldld, fp.d_W, fp.ldw,
              fp.d_perm, fp.d_sw, fp.d_blk, fp.d_colpanel, fp.d_pstart, fp.d_state, nb, nbpiv);
  SL_LAUNCH_CHECK();
  prof_end(ph, tpan, st);
  if (after_panel) SL_HIP(hipEventRecord(after_panel, st));
  const long k1_lb = std::min<long>(n, k0_lb + min_kb);
  if (k1_lb >= n) return;
  const int tu = prof_begin(ph, kProfUpdate, st);
  if (n - k1_lb >= fp.wide_min && fp.update_pipe && pipe_fits(fp)) {
    // one workgroup per CU, at most one per item (an upper bound on the items
    // from the least advanced shift), a multiple of the 8 XCDs when it can be
    const long T = ceil_div(n - k1_lb, 128);
    long G = std::min<long>(std::max(fp.cus, 8), T * (T + 1) / 2 * S);
    if (G >= 8) G -= G % 8;
    SL_LAUNCH(k_trailing_update_pipe, dim3((unsigned)G), dim3(1024), 0, st, n, fp.d_LD, fp.ldld,
              fp.d_W, fp.ldw, fp.d_state, S);
  } else if (n - k1_lb >= fp.wide_min) {
    const long T = ceil_div(n - k1_lb, 128);
    if (fp.stream_c)
      SL_LAUNCH(k_trailing_update_lds<true>, dim3((unsigned)(T * (T + 1) / 2), S), dim3(1024), 0, st,
                n, fp.d_LD, fp.ldld, fp.d_W, fp.ldw, fp.d_state);
    else
      SL_LAUNCH(k_trailing_update_lds<false>, dim3((unsigned)(T * (T + 1) / 2), S), dim3(1024), 0,
                st, n, fp.d_LD, fp.ldld, fp.d_W, fp.ldw, fp.d_state);
  } else {
    const long T = ceil_div(n - k1_lb, 64);
    SL_LAUNCH(k_trailing_update, dim3((unsigned)(T * (T + 1) / 2), S), dim3(256), 0, st, n,
              fp.d_LD, fp.ldld, fp.d_W, fp.ldw, fp.d_state);
  }
  SL_LAUNCH_CHECK();
  prof_end(ph, tu, st);
}

// The deferred interchanges and the inertia of every shift of `fp`.
static void factor_tail(const FactorPlan& fp, hipStream_t st) {
  const int n = fp.n, S = fp.nshift;
  if (fp.pivot) {
    SL_LAUNCH(k_perm_suffix, dim3(S), dim3(256), (size_t)n * sizeof(int), st, n, fp.d_sw,
              fp.d_pstart, fp.d_state, fp.d_snap);
    SL_LAUNCH_CHECK();
    SL_LAUNCH(k_left_gather, dim3(n, S), dim3(1024), (size_t)n * sizeof(double), st, n, fp.d_LD,
              fp.ldld, fp.d_colpanel, fp.d_pstart, fp.d_state, fp.d_snap);
    SL_LAUNCH_CHECK();
  }
  SL_LAUNCH(k_factor_finalize, dim3((unsigned)ceil_div(n, 256), S), dim3(256), 0, st, n, fp.d_perm,
            fp.d_blk, fp.d_ipiv, fp.d_state, fp.d_inertia);
  SL_LAUNCH_CHECK();
}

void factor_steps_launch(const FactorPlan& fp, hipStream_t st, bool readback) {
  const int n = fp.n, S = fp.nshift, nb = fp.nb;
  if (S <= 0 || n <= 0) return;
  factor_prepare();
  SL_LAUNCH(k_factor_init, dim3((unsigned)ceil_div(n, 256), S), dim3(256), 0, st, n,
                     fp.d_state, fp.d_perm, fp.d_sw);
  SL_LAUNCH_CHECK();
  sislice_handle* ph = current_handle();
  const int min_kb = factor_min_panel(nb, fp.nbpiv, fp.fast != 0);
  const int step_cap = factor_npanel_max(n, nb, fp.nbpiv, fp.fast != 0);
  SL_CHECK_ARG(step_cap <= fp.npmax, "panel bookkeeping smaller than the step bound");
  if (!readback) {
    // a fixed sequence (for graph capture): every step up to the bound; steps
    // past a shift's end return at once
    for (int q = 0; q < step_cap; ++q)
      factor_step(fp, st, std::min<long>(n, (long)q * min_kb), ph, nullptr);
    factor_tail(fp, st);
    return;
  }
  // Panel widths depend on the pivots: launch chunks of steps and read the
  // per-shift progress back between chunks (kmin = least factored prefix of a
  // group).  The shifts run in G groups, each on its own stream, so that the
  // latency-bound panels of one group run while another group's updates use the
  // memory system; group g + 1 starts once group g's first pivoting panel is
  // enqueued, which staggers the groups by about one panel.
  const int G = ph ? std::max(1, std::min(fp.groups, S / 2)) : 1;
  std::vector<FactorPlan> sub(G);
  std::vector<hipStream_t> gs(G);
  std::vector<long> kmin(G, 0);
  std::vector<int> steps(G, 0);
  std::vector<char> launched(G, 0);
  for (int g = 0; g < G; ++g) {
    const int s0 = (int)((long)S * g / G), s1 = (int)((long)S * (g + 1) / G);
    sub[g] = factor_subplan(fp, s0, s1 - s0);
    // a persistent update would hold every CU for its whole launch and keep the
    // other groups' panels waiting: grouped runs take the workgroup-per-tile form
    if (G > 1) {
      sub[g].update_pipe = 0;
      sub[g].stream_c = 1;
    }
    gs[g] = g == 0 ? st : group_stream(ph, g - 1);
  }
  FactorState* hs = static_cast<FactorState*>(host_stage(ph, sizeof(FactorState) * S));
  if (G > 1) {
    if (ph->flush_fn) ph->flush_fn(ph->flush_ctx);  // staged tables reach the device first
    SL_HIP(hipEventRecord(group_event(ph, 0), st));
    for (int g = 1; g < G; ++g) SL_HIP(hipStreamWaitEvent(gs[g], group_event(ph, 0), 0));
  }
  constexpr int kChunk = 8;
  for (bool first = true;; first = false) {
    bool any = false;
    for (int g = 0; g < G; ++g) {
      launched[g] = kmin[g] < n && steps[g] < step_cap;
      if (!launched[g]) continue;
      any = true;
      for (int q = 0; q < kChunk && steps[g] < step_cap; ++q, ++steps[g]) {
        hipEvent_t mark = (first && q == 0 && g + 1 < G) ? group_event(ph, g + 1) : nullptr;
        factor_step(sub[g], gs[g], std::min<long>(n, kmin[g] + (long)q * min_kb), ph, mark);
        if (mark) SL_HIP(hipStreamWaitEvent(gs[g + 1], mark, 0));
      }
      const FactorPlan& f = sub[g];
      SL_HIP(hipMemcpyAsync(hs + (f.d_state - fp.d_state), f.d_state, sizeof(FactorState) * f.nshift,
                            hipMemcpyDeviceToHost, gs[g]));
    }
    if (!any) break;
    for (int g = 0; g < G; ++g) {
      if (!launched[g]) continue;
      SL_HIP(hipStreamSynchronize(gs[g]));
      const FactorPlan& f = sub[g];
      const FactorState* h0 = hs + (f.d_state - fp.d_state);
      long km = n;
      for (int q = 0; q < f.nshift; ++q) km = std::min<long>(km, h0[q].done ? n : h0[q].k0 + h0[q].kb);
      kmin[g] = km;
    }
  }
  for (int g = 0; g < G; ++g)
    SL_CHECK_ARG(kmin[g] >= n, "factorization did not complete");
  for (int g = 0; g < G; ++g) factor_tail(sub[g], gs[g]);
  if (G > 1) {
    for (int g = 1; g < G; ++g) {
      SL_HIP(hipEventRecord(group_event(ph, g), gs[g]));
      SL_HIP(hipStreamWaitEvent(st, group_event(ph, g), 0));
    }
  }
}

}  // namespace sislice
