// Small dense symmetric eigensolver for the projected problems of Rayleigh-Ritz
// (Section 2.1: (V^T A V) Q = Q Omega) and of the Lanczos tridiagonal-block
// matrices.
//
// Design (gfx950): one 1024-thread workgroup per matrix, everything resident in
// LDS: the lower triangle of A packed (m(m+1)/2 doubles) and the eigenvector
// matrix V (m x m), which for m <= 112 fits the 160 KB of a CU.  Cyclic Jacobi in
// the parallel round-robin order: each round rotates m/2 disjoint (p, q) pairs
// (Golub & Van Loan, symmetric Schur 2x2 rotation), applies all of them to A as
// independent 2x2 blocks J_k^T A_{kl} J_l and to the columns of V, then moves to
// the next pairing.  A rotation is skipped when |a_pq| <= 1e-15 sqrt(|a_pp a_qq|)
// (relative threshold, so tiny and large eigenvalues both converge to full
// relative accuracy); the iteration stops after a sweep without rotations.
#include "common.hpp"
#include "eig.hpp"
#include "handle.hpp"

namespace sislice {

__device__ __forceinline__ int pidx(int i, int j, int m) {
  // column-major packed lower triangle, i >= j
  return j * m - (j * (j - 1)) / 2 + (i - j);
}

__device__ __forceinline__ int sidx(int i, int j, int m) {
  return i >= j ? pidx(i, j, m) : pidx(j, i, m);
}

__device__ __forceinline__ int rr_player(int pos, int r, int M) {
  return pos == 0 ? 0 : 1 + ((pos - 1 + r) % (M - 1));
}

__global__ __launch_bounds__(1024) void k_syevj(EigArgs a) {
  extern __shared__ double sh[];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int m = a.m[b];
  if (m <= 0) return;
  const int M = m + (m & 1);
  const int h = M / 2;
  const int npk = m * (m + 1) / 2;
  double* A = sh;                    // packed lower
  double* V = sh + npk;              // V[j * m + i]
  double* cs = V + m * m;            // [h]
  double* sn = cs + h;               // [h]
  int* pp = reinterpret_cast<int*>(sn + h);  // [h]
  int* qq = pp + h;                          // [h]
  int* flag = qq + h;                        // [2]
  const double* Ain = a.A[b];
  const long lda = a.lda;
  for (int e = tid; e < m * m; e += blockDim.x) {
    const int i = e % m, j = e / m;
    if (i >= j) A[pidx(i, j, m)] = Ain[i + (long)j * lda];
    V[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int ntask_blk = h * (h + 1) / 2;
  // Each thread's tasks are the same in every round: decode them once.
  //   A: 2x2 block tasks t = tid + 1024 j -> pair indices (k >= l)
  //   V: column-pair tasks t = tid + 1024 j -> (row i, pair k)
  constexpr int JA = 2, JV = 7;  // enough for m <= kEigMax (h <= 56)
  int tk[JA], tl[JA], vi[JV], vk[JV];
#pragma unroll
  for (int j = 0; j < JA; ++j) {
    const int t = tid + 1024 * j;
    int k = -1, l = 0;
    if (t < ntask_blk) {
      k = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
      while (k * (k + 1) / 2 > t) --k;
      while ((k + 1) * (k + 2) / 2 <= t) ++k;
      l = t - k * (k + 1) / 2;
    }
    tk[j] = k;
    tl[j] = l;
  }
#pragma unroll
  for (int j = 0; j < JV; ++j) {
    const int t = tid + 1024 * j;
    vi[j] = (t < m * h) ? t % m : -1;
    vk[j] = (t < m * h) ? t / m : 0;
  }
  // flag[0]: a rotation happened in this sweep; rflag[r & 1]: in round r (the slot
  // of the next round is cleared by thread 0 while the current one is being set)
  int* rflag = flag + 2;
  for (int sweep = 0; sweep < a.max_sweeps; ++sweep) {
    if (tid == 0) {
      flag[0] = 0;
      rflag[0] = 0;
      rflag[1] = 0;
    }
    __syncthreads();
    for (int r = 0; r < M - 1; ++r) {
      if (tid == 0) rflag[(r + 1) & 1] = 0;
      if (tid < h) {
        int p = rr_player(tid, r, M), q = rr_player(M - 1 - tid, r, M);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0;
        if (q < m) {
          const double apq = A[pidx(q, p, m)];
          const double app = A[pidx(p, p, m)], aqq = A[pidx(q, q, m)];
          if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > 1e-300) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                          : -1.0 / (-tau + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            flag[0] = 1;
            rflag[r & 1] = 1;
          }
        }
        pp[tid] = p;
        qq[tid] = q;
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      if (rflag[r & 1] == 0) continue;  // no rotation in this round: A and V unchanged
      // A <- J^T A J as independent 2x2 blocks of pair pairs (k >= l)
#pragma unroll
      for (int j = 0; j < JA; ++j) {
        const int k = tk[j], l = tl[j];
        if (k < 0) continue;
        const double ck = cs[k], sk = sn[k], cl = cs[l], sl = sn[l];
        if (sk == 0.0 && sl == 0.0) continue;
        const int pk = pp[k], qk = qq[k], pl = pp[l], ql = qq[l];
        if (k == l) {
          if (qk >= m) continue;
          const int ipq = pidx(qk, pk, m);
          const double apq = A[ipq];
          const double tt = sk / ck;
          A[pidx(pk, pk, m)] -= tt * apq;
          A[pidx(qk, qk, m)] += tt * apq;
          A[ipq] = 0.0;
        } else {
          const bool vq_k = qk < m, vq_l = ql < m;
          const int i00 = sidx(pk, pl, m);
          const int i01 = vq_l ? sidx(pk, ql, m) : -1;
          const int i10 = vq_k ? sidx(qk, pl, m) : -1;
          const int i11 = (vq_k && vq_l) ? sidx(qk, ql, m) : -1;
          const double x00 = A[i00], x01 = vq_l ? A[i01] : 0.0;
          const double x10 = vq_k ? A[i10] : 0.0, x11 = (vq_k && vq_l) ? A[i11] : 0.0;
          // rows: J_k^T
          const double r00 = ck * x00 - sk * x10, r01 = ck * x01 - sk * x11;
          const double r10 = sk * x00 + ck * x10, r11 = sk * x01 + ck * x11;
          // columns: J_l
          A[i00] = cl * r00 - sl * r01;
          if (vq_l) A[i01] = sl * r00 + cl * r01;
          if (vq_k) A[i10] = cl * r10 - sl * r11;
          if (vq_k && vq_l) A[i11] = sl * r10 + cl * r11;
        }
      }
      // V <- V J
#pragma unroll
      for (int j = 0; j < JV; ++j) {
        const int i = vi[j], k = vk[j];
        if (i < 0) continue;
        const double c = cs[k], s = sn[k];
        if (s == 0.0) continue;
        const int p = pp[k], q = qq[k];
        const double vp = V[p * m + i], vq = V[q * m + i];
        V[p * m + i] = c * vp - s * vq;
        V[q * m + i] = s * vp + c * vq;
      }
      __syncthreads();
    }
    if (flag[0] == 0) break;
    __syncthreads();
  }
  __syncthreads();
  // sort ascending: rank of each eigenvalue (ties by index)
  int* rank = flag + 2;
  for (int i = tid; i < m; i += blockDim.x) {
    const double wi = A[pidx(i, i, m)];
    int rk = 0;
    for (int j = 0; j < m; ++j) {
      const double wj = A[pidx(j, j, m)];
      rk += (wj < wi) || (wj == wi && j < i);
    }
    rank[i] = rk;
  }
  __syncthreads();
  double* W = a.W[b];
  double* Vout = a.V[b];
  const long ldv = a.ldv;
  for (int i = tid; i < m; i += blockDim.x) W[rank[i]] = A[pidx(i, i, m)];
  for (int e = tid; e < m * m; e += blockDim.x) {
    const int i = e % m, j = e / m;
    Vout[i + (long)rank[j] * ldv] = V[j * m + i];
  }
}

size_t eig_lds_bytes(int mmax) {
  const int M = mmax + (mmax & 1);
  const int h = M / 2;
  return sizeof(double) * ((size_t)mmax * (mmax + 1) / 2 + (size_t)mmax * mmax + 2 * h) +
         sizeof(int) * (2 * h + 2 + mmax) + 64;
}

void eig_launch(const EigArgs& a, int batch, int mmax, hipStream_t st) {
  static std::once_flag attr;
  std::call_once(attr, [] {
    SL_HIP(hipFuncSetAttribute((const void*)k_syevj, hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024));
  });
  const size_t lds = eig_lds_bytes(mmax);
  SL_CHECK_ARG(lds <= 160 * 1024, "projected problem too large for the LDS eigensolver");
  const int tk = prof_begin(current_handle(), kProfEig);
  SL_LAUNCH(k_syevj, dim3(batch), dim3(1024), lds, st, a);
  SL_LAUNCH_CHECK();
  prof_end(current_handle(), tk);
}

}  // namespace sislice
