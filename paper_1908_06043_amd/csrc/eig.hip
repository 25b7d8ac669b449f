// Small dense symmetric eigensolver for the projected problems of Rayleigh-Ritz
// (Section 2.1: (V^T A V) Q = Q Omega) and of the Lanczos tridiagonal-block
// matrices.
//
// Design (gfx950): two kernels per batch.
//  k_syevj: one 1024-thread workgroup per matrix, the lower triangle of A in LDS
//  as a full row-major array with the odd row length M + 1 (M = m rounded up to
//  even): the blocks a wavefront updates lie along rows or columns of distinct
//  players, which this length spreads over the banks (the packed triangle measured
//  2.45 us per rotation round at m = 112, this layout 1.80).  Cyclic Jacobi in the parallel round-robin order:
//  each round rotates m/2 disjoint (p, q) pairs (Golub & Van Loan, symmetric
//  Schur 2x2 rotation) and applies all of them to A as independent 2x2 blocks
//  J_k^T A_{kl} J_l, then moves to the next pairing.  The (c, s) of every pair of
//  every round are written to a rotation record in device memory; at the end the
//  eigenvalues are sorted ascending and the rank of each diagonal position kept.
//  k_syevj_vecs: forms V = J_1 J_2 ... by replaying the record on rows of the
//  identity.  Rows of V never mix, so one wavefront owns two rows in LDS (lane k
//  applies pair k of each round) and needs no workgroup barrier, and the rows of
//  one matrix spread over many CUs instead of sharing the LDS bandwidth of the one
//  CU that runs the rotations.
// A rotation is skipped when |a_pq| <= 1e-15 sqrt(|a_pp a_qq|) (relative
// threshold, so tiny and large eigenvalues both converge to full relative
// accuracy); the iteration stops after a sweep without rotations.
#include "common.hpp"
#include "eig.hpp"
#include "handle.hpp"

#include <algorithm>

namespace sislice {

__device__ __forceinline__ int pidx(int i, int j, int m) {
  // lower triangle (i >= j) of a row-major array with rows of M + 1 doubles
  return i * (m + (m & 1) + 1) + j;
}

__device__ __forceinline__ int sidx(int i, int j, int m) {
  return i >= j ? pidx(i, j, m) : pidx(j, i, m);
}


// Per-matrix metadata after k_syevj: [0] sweeps that rotated, [1 + i] rank of
// diagonal position i in ascending order.
constexpr int kMetaStride = kEigMax + 16;

// 1 / x and 1 / sqrt(x) for x > 0 from the hardware approximations refined by
// two Newton steps (relative error near the rounding unit).
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx, y * y, 1.5);
  y = y * fma(-hx, y * y, 1.5);
  return y;
}

// The round-robin player of a position, advanced by one round: position 0 holds
// player 0, the others cycle through 1 .. M - 1 (in round r position pos >= 1
// holds 1 + (pos - 1 + r) mod (M - 1)).
__device__ __forceinline__ int rr_next(int v, int M) { return v == 0 ? 0 : (v == M - 1 ? 1 : v + 1); }

__global__ __launch_bounds__(1024) void k_syevj(EigArgs a, double2* __restrict__ rot, long rstride,
                                                int* __restrict__ meta) {
  extern __shared__ double sh[];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int m = a.m[b];
  if (m <= 0) return;
  const int M = m + (m & 1);
  const int h = M / 2;
  const int npk = M * (M + 1);
  double* A = sh;                                                 // lower triangle, rows of M + 1
  double2* csn = reinterpret_cast<double2*>(sh + ((npk + 1) & ~1));  // [h] (c, s)
  int* flag = reinterpret_cast<int*>(csn + h);                      // [4], then rank [m]
  double2* rb = rot + (long)b * rstride;                            // [sweep][round][pair]
  const double* Ain = a.A[b];
  const long lda = a.lda;
  for (int e = tid; e < m * m; e += blockDim.x) {
    const int i = e % m, j = e / m;
    if (i >= j) A[pidx(i, j, m)] = Ain[i + (long)j * lda];
  }
  __syncthreads();
  const int ntask_blk = h * (h + 1) / 2;
  // Each thread's 2x2 block tasks t = tid + 1024 j -> pair indices (k >= l) are
  // the same in every round: decode them once.  The players of the pairs' two
  // positions (k and M - 1 - k) advance by one per round in registers: after
  // M - 1 rounds (one sweep) they are back where they started.
  constexpr int JA = 2;  // enough for m <= kEigMax (h <= 56)
  int tk[JA], tl[JA], uk[JA], vk[JA], ul[JA], vl[JA];
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
    uk[j] = k < 0 ? 0 : k;
    vk[j] = k < 0 ? 0 : M - 1 - k;
    ul[j] = l;
    vl[j] = M - 1 - l;
  }
  int up = tid, vp = M - 1 - tid;  // players of pair `tid` (rotation phase, tid < h)
  // flag[0]: a rotation happened in this sweep; rflag[r & 1]: in round r (the slot
  // of the next round is cleared by thread 0 while the current one is being set)
  int* rflag = flag + 2;
  int nsw = 0;
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
        const int p = min(up, vp), q = max(up, vp);
        double c = 1.0, s = 0.0;
        if (q < m) {
          const double apq = A[pidx(q, p, m)];
          const double app = A[pidx(p, p, m)], aqq = A[pidx(q, q, m)];
          if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > 1e-300) {
            // t = tan of the angle that zeroes a_pq, the root of t^2 + 2 tau t - 1
            // of smaller modulus, tau = (a_qq - a_pp) / (2 a_pq) (Golub & Van Loan,
            // symmetric Schur), written as t = sgn(tau) |e| / (|d| + sqrt(d^2 + e^2))
            // with d = a_qq - a_pp, e = 2 a_pq (one square root, one reciprocal)
            const double d = aqq - app, e = 2.0 * apq;
            const double hyp = sqrt(fma(d, d, e * e));
            double t;
            if (hyp < 1e300) {
              t = fabs(e) * rcp_nr(fabs(d) + hyp);
              if (d != 0.0 && ((d < 0.0) != (e < 0.0))) t = -t;
            } else {  // d^2 + e^2 overflows: the scaled form
              const double tau = d / e;
              t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                               : -1.0 / (-tau + sqrt(1.0 + tau * tau));
            }
            c = rsq_nr(fma(t, t, 1.0));
            s = t * c;
            flag[0] = 1;
            rflag[r & 1] = 1;
          }
        }
        csn[tid] = make_double2(c, s);
        rb[(long)(sweep * (M - 1) + r) * h + tid] = make_double2(c, s);
      }
      __syncthreads();
      // no rotation in this round: A is unchanged and nothing reads (c, s) before
      // the next round's rotation phase rewrites them, so no closing barrier
      const bool rotated = rflag[r & 1] != 0;
      if (rotated) {
        // A <- J^T A J as independent 2x2 blocks of pair pairs (k >= l)
#pragma unroll
        for (int j = 0; j < JA; ++j) {
          const int k = tk[j], l = tl[j];
          if (k < 0) continue;
          const double2 csk = csn[k], csl = csn[l];
          const double ck = csk.x, sk = csk.y, cl = csl.x, sl = csl.y;
          if (sk == 0.0 && sl == 0.0) continue;
          const int pk = min(uk[j], vk[j]), qk = max(uk[j], vk[j]);
          const int pl = min(ul[j], vl[j]), ql = max(ul[j], vl[j]);
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
      }
      // every round, rotated or not, moves the players on
#pragma unroll
      for (int j = 0; j < JA; ++j) {
        uk[j] = rr_next(uk[j], M);
        vk[j] = rr_next(vk[j], M);
        ul[j] = rr_next(ul[j], M);
        vl[j] = rr_next(vl[j], M);
      }
      up = rr_next(up, M);
      vp = rr_next(vp, M);
      if (rotated) __syncthreads();
    }
    if (flag[0] == 0) break;
    ++nsw;
    __syncthreads();
  }
  __syncthreads();
  // sort ascending: rank of each eigenvalue (ties by index)
  int* rank = flag + 4;
  int* mb = meta + (long)b * kMetaStride;
  for (int i = tid; i < m; i += blockDim.x) {
    const double wi = A[pidx(i, i, m)];
    int rk = 0;
    for (int j = 0; j < m; ++j) {
      const double wj = A[pidx(j, j, m)];
      rk += (wj < wi) || (wj == wi && j < i);
    }
    rank[i] = rk;
    mb[1 + i] = rk;
  }
  if (tid == 0) mb[0] = nsw;
  __syncthreads();
  double* W = a.W[b];
  for (int i = tid; i < m; i += blockDim.x) W[rank[i]] = A[pidx(i, i, m)];
}

constexpr int kVecRowsPerWave = 2;
constexpr int kVecWaves = 4;
constexpr int kVecRows = kVecRowsPerWave * kVecWaves;  // rows of V per workgroup
constexpr int kVecPf = 16;                              // rounds of (c, s) loaded ahead

__global__ __launch_bounds__(64 * kVecWaves) void k_syevj_vecs(EigArgs a,
                                                               const double2* __restrict__ rot,
                                                               long rstride,
                                                               const int* __restrict__ meta) {
  __shared__ double Vs[kVecRows][kEigMax];
  const int b = blockIdx.x;
  const int m = a.m[b];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = blockIdx.y * kVecRows + w * kVecRowsPerWave;  // first row of this wavefront
  if (m <= 0 || i0 >= m) return;  // uniform per wavefront; no workgroup barrier follows
  const int M = m + (m & 1), h = M / 2, R = M - 1;
  const int* mb = meta + (long)b * kMetaStride;
  const long total = (long)mb[0] * R;  // rounds to replay
  const bool has1 = i0 + 1 < m;
  double* v0 = Vs[w * kVecRowsPerWave];
  double* v1 = Vs[w * kVecRowsPerWave + 1];
  for (int j = lane; j < m; j += 64) {
    v0[j] = (j == i0) ? 1.0 : 0.0;
    v1[j] = (j == i0 + 1) ? 1.0 : 0.0;
  }
  const bool act = lane < h;
  // players of pair `lane` in round r (the round-robin of k_syevj), advanced by one
  // position per round: 1..R cyclically, player 0 fixed
  int pa = lane, pb = M - 1 - lane;
  const double2* rb = rot + (long)b * rstride + lane;
  double2 cur[kVecPf], nxt[kVecPf];
#pragma unroll
  for (int j = 0; j < kVecPf; ++j)
    cur[j] = (act && j < total) ? rb[(long)j * h] : make_double2(1.0, 0.0);
  for (long g0 = 0; g0 < total; g0 += kVecPf) {
#pragma unroll
    for (int j = 0; j < kVecPf; ++j) {
      const long g = g0 + kVecPf + j;
      nxt[j] = (act && g < total) ? rb[g * h] : make_double2(1.0, 0.0);
    }
#pragma unroll
    for (int j = 0; j < kVecPf; ++j) {
      // guard rather than break: the loop unrolls fully and cur[] stays in registers
      const bool live = g0 + j < total;  // uniform per wavefront
      // the writes of the previous round (other lanes' columns) are read below
      asm volatile("" ::: "memory");
      __builtin_amdgcn_wave_barrier();
      const double c = cur[j].x, s = cur[j].y;
      const int p = min(pa, pb), q = max(pa, pb);
      if (live && act && s != 0.0 && q < m) {
        const double x0 = v0[p], y0 = v0[q];
        v0[p] = c * x0 - s * y0;
        v0[q] = s * x0 + c * y0;
        if (has1) {
          const double x1 = v1[p], y1 = v1[q];
          v1[p] = c * x1 - s * y1;
          v1[q] = s * x1 + c * y1;
        }
      }
      if (lane != 0) pa = (pa == R) ? 1 : pa + 1;
      pb = (pb == R) ? 1 : pb + 1;
    }
#pragma unroll
    for (int j = 0; j < kVecPf; ++j) cur[j] = nxt[j];
  }
  asm volatile("" ::: "memory");
  __builtin_amdgcn_wave_barrier();
  double* Vout = a.V[b];
  const long ldv = a.ldv;
  for (int j = lane; j < m; j += 64) {
    const long col = (long)mb[1 + j] * ldv;
    Vout[i0 + col] = v0[j];
    if (has1) Vout[i0 + 1 + col] = v1[j];
  }
}

size_t eig_lds_bytes(int mmax) {
  const int M = mmax + (mmax & 1);
  const int h = M / 2;
  const size_t npk = (size_t)M * (M + 1);
  return sizeof(double) * (((npk + 1) & ~size_t(1)) + 2 * h) + sizeof(int) * (4 + mmax) + 64;
}

// Rotation records are staged per chunk of the batch so that their workspace
// stays near this size however large the batch is.
constexpr size_t kRotChunkBytes = size_t(256) << 20;

void eig_launch(const EigArgs& a, int batch, int mmax, hipStream_t st) {
  static std::once_flag attr;
  std::call_once(attr, [] {
    SL_HIP(hipFuncSetAttribute((const void*)k_syevj, hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024));
  });
  SL_CHECK_ARG(mmax <= kEigMax, "projected problem too large for the LDS eigensolver");
  SL_CHECK_ARG(a.max_sweeps >= 1, "max_sweeps must be positive");
  if (batch <= 0 || mmax <= 0) return;
  const size_t lds = eig_lds_bytes(mmax);
  sislice_handle* h = current_handle();
  SL_CHECK_ARG(h != nullptr, "no current handle for the eigensolver workspace");
  const int Mx = mmax + (mmax & 1);
  const long rstride = (long)a.max_sweeps * (Mx - 1) * (Mx / 2);  // double2 per matrix
  const size_t rot_bytes = (size_t)rstride * sizeof(double2);
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>(batch, kRotChunkBytes / rot_bytes));
  const size_t meta_off = ((size_t)chunk * rot_bytes + 255) & ~size_t(255);
  char* ws = static_cast<char*>(
      ws_get(h, kBufEigRot, meta_off + (size_t)chunk * kMetaStride * sizeof(int)));
  double2* rot = reinterpret_cast<double2*>(ws);
  int* meta = reinterpret_cast<int*>(ws + meta_off);
  const int tk = prof_begin(h, kProfEig, st);
  for (int c0 = 0; c0 < batch; c0 += chunk) {
    const int nb = std::min(chunk, batch - c0);
    EigArgs c = a;
    c.m = a.m + c0;
    c.A = a.A + c0;
    c.W = a.W + c0;
    c.V = a.V + c0;
    SL_LAUNCH(k_syevj, dim3(nb), dim3(1024), lds, st, c, rot, rstride, meta);
    SL_LAUNCH_CHECK();
    SL_LAUNCH(k_syevj_vecs, dim3(nb, (mmax + kVecRows - 1) / kVecRows), dim3(64 * kVecWaves), 0,
              st, c, rot, rstride, meta);
    SL_LAUNCH_CHECK();
  }
  prof_end(h, tk, st);
}

}  // namespace sislice
