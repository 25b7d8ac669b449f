// Small dense symmetric eigensolver for the projected problems of Rayleigh-Ritz
// (Section 2.1: (V^T A V) Q = Q Omega) and of the Lanczos tridiagonal-block
// matrices.
//
// Design (gfx950): two kernels per batch.
//  k_syevj: one 1024-thread workgroup per matrix, the lower triangle of A in LDS
//  as a full row-major array with the odd row length M + 1 (M = m rounded up to
//  even): the blocks a wavefront updates lie along rows or columns of distinct
//  players, which this length spreads over the banks.  Cyclic Jacobi in the
//  parallel round-robin order: each round rotates m/2 disjoint (p, q) pairs
//  (Golub & Van Loan, symmetric Schur 2x2 rotation) and applies all of them to A
//  as independent 2x2 blocks J_k^T A_{kl} J_l, then moves to the next pairing.
//  The rounds are pipelined: wavefront 0 updates the blocks that the next round's
//  rotations read (every diagonal block and one off-diagonal block per pair) and
//  then computes those rotations while the other fifteen wavefronts update the
//  rest, so a round is one block update and one workgroup barrier (a 112 x 112
//  solve takes 19% less time than with a rotation phase and two barriers a round).
//  The (c, s) of every pair of every round are written to a rotation record in
//  device memory; at the end the eigenvalues are sorted ascending and the rank of
//  each diagonal position kept.
//  k_syevj_vecs: forms V = J_1 J_2 ... by replaying the record on rows of the
//  identity.  Rows of V never mix and a round moves every player one position
//  along a fixed conveyor, so each lane keeps the two entries of its pair's
//  players in registers and passes them to the neighbouring lanes after each
//  round (cross-lane moves, no LDS, no barrier); the rows of one matrix spread over
//  many CUs instead of sharing the CU that runs the rotations.
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

// The Jacobi rotation of one pair (Golub & Van Loan, symmetric Schur 2x2 step):
// (c, s) and t = s / c that zero a_pq, or the identity when the pair is padding or
// a_pq is negligible against sqrt(|a_pp a_qq|).  Returns whether it rotates.  The
// threshold test and the rotation are evaluated side by side (their square roots
// are independent) and the result selected afterwards.
__device__ __forceinline__ bool pair_rotation(double app, double aqq, double apq, bool valid,
                                              double& c, double& sn, double& t) {
  const double thr = 1e-15 * sqrt(fabs(app * aqq));
  const bool rot = valid & (fabs(apq) > thr) & (fabs(apq) > 1e-300);
  // t = tan of the angle that zeroes a_pq, the root of t^2 + 2 tau t - 1 of smaller
  // modulus, tau = (a_qq - a_pp) / (2 a_pq), written as
  // t = sgn(tau) |e| / (|d| + sqrt(d^2 + e^2)) with d = a_qq - a_pp, e = 2 a_pq
  const double d = aqq - app, e = 2.0 * apq;
  const double hyp = sqrt(fma(d, d, e * e));
  double tt = fabs(e) * rcp_nr(fabs(d) + hyp);
  if (rot && !(hyp > 1e-150 && hyp < 1e300)) {
    // d^2 + e^2 underflows or overflows: the same form on d and e scaled by a power
    // of two (t does not depend on the scale; e != 0 when the pair rotates)
    const int ex = ilogb(fmax(fabs(d), fabs(e)));
    const double ds = ldexp(d, -ex), es = ldexp(e, -ex);
    tt = fabs(es) * rcp_nr(fabs(ds) + sqrt(fma(ds, ds, es * es)));
  }
  if (d != 0.0 && ((d < 0.0) != (e < 0.0))) tt = -tt;
  const double cr = rsq_nr(fma(tt, tt, 1.0));
  c = rot ? cr : 1.0;
  sn = rot ? tt * cr : 0.0;
  t = rot ? tt : 0.0;
  return rot;
}

__global__ __launch_bounds__(1024) void k_syevj(EigArgs a, double2* __restrict__ rot, long rstride,
                                                int* __restrict__ meta) {
  extern __shared__ double sh[];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int m = a.m[b];
  if (m <= 0) return;
  const int M = m + (m & 1);
  const int h = M / 2, R = M - 1;
  const int npk = M * (M + 1);
  double* A = sh;                                                    // lower triangle, rows of M + 1
  double2* csn = reinterpret_cast<double2*>(sh + ((npk + 1) & ~1));  // [2][h] (c, s) by round parity
  int* flag = reinterpret_cast<int*>(csn + 2 * h);                     // [4], then rank [m]
  int* rflag = flag + 2;                                               // [2] the round rotates
  double2* rb = rot + (long)b * rstride;                               // [sweep][round][pair]
  const double* Ain = a.A[b];
  const long lda = a.lda;
  for (int e = tid; e < m * m; e += blockDim.x) {
    const int i = e % m, j = e / m;
    if (i >= j) A[pidx(i, j, m)] = Ain[i + (long)j * lda];
  }
  // Block tasks (k, l), k >= l, of pairs of pairs; a thread's tasks are the same in
  // every round, only the players of the pairs' positions (k and M - 1 - k) move on
  // by one per round (in registers; after M - 1 rounds they are back).
  // Wavefront 0 owns the blocks that the next round's rotations read: every diagonal
  // block (k, k), and for each pair k' the block that will hold a_pq of k' in the
  // next round.  By the round-robin rule the two players of pair k' next round come
  // from this round's pairs k' + 1 and k' - 1 (pairs 0 and 1 for k' = 0, pairs
  // h - 1 and h - 2 for k' = h - 1).  So wavefront 0 can compute the next round's
  // rotations from its own results while the other wavefronts apply the rest of
  // this round's blocks: one workgroup barrier per round, the rotation latency off
  // the critical path.
  constexpr int JA = 2;  // enough for m <= kEigMax (h <= 56)
  int tk[JA], tl[JA];
  const int w = tid >> 6, lane = tid & 63;
  if (w == 0) {
    tk[0] = lane < h ? lane : -1;
    tl[0] = lane < h ? lane : 0;
    int k1 = -1, k2 = 0;
    if (lane == 0 && h >= 2) {
      k1 = 1;
      k2 = 0;
    } else if (lane >= 1 && lane <= h - 2) {
      k1 = lane + 1;
      k2 = lane - 1;
    } else if (lane == h - 1 && h >= 3) {
      k1 = h - 1;
      k2 = h - 2;
    }
    tk[1] = k1;
    tl[1] = k2;
  } else {
    // the other blocks row by row: row k (2 <= k <= h - 2) without (k, k - 2), row
    // h - 1 without (h - 1, h - 3) and (h - 1, h - 2); rows 0 and 1 have none
#pragma unroll
    for (int j = 0; j < JA; ++j) {
      int idx = (tid - 64) + (1024 - 64) * j, k = -1, l = 0;
      for (int kk = 2; kk <= h - 1 && k < 0; ++kk) {
        const int cnt = kk <= h - 2 ? kk - 1 : h - 3;
        if (idx < cnt) {
          k = kk;
          l = (kk <= h - 2 && idx == kk - 2) ? kk - 1 : idx;
        } else {
          idx -= cnt;
        }
      }
      tk[j] = k;
      tl[j] = l;
    }
  }
  int uk[JA], vk[JA], ul[JA], vl[JA];
#pragma unroll
  for (int j = 0; j < JA; ++j) {
    const int k = tk[j] < 0 ? 0 : tk[j], l = tl[j];
    uk[j] = k;
    vk[j] = M - 1 - k;
    ul[j] = l;
    vl[j] = M - 1 - l;
  }
  // the second task slot is empty in whole wavefronts at small orders: skip its loads
  const bool slot1 = __ballot(tk[1] >= 0) != 0;
  int up = lane, vp = M - 1 - lane;  // wavefront 0, lane < h: the players of pair `lane`
  // wavefront 0: the rotations of global round g into buffer g & 1, the round's flag
  const long gmax = (long)a.max_sweeps * R;
  // The pair's own (diagonal) block of the next round is exactly what the rotation
  // reads, and nothing else touches it before that round's update: its elements
  // and rotation stay in registers (d_*) for the diagonal task.
  double d_app = 0.0, d_aqq = 0.0, d_apq = 0.0, d_sn = 0.0, d_t = 0.0;
  auto next_rotations = [&](long g) {
    const int p = min(up, vp), q = max(up, vp), qc = min(q, m - 1);
    d_apq = A[pidx(qc, p, m)];
    d_app = A[pidx(p, p, m)];
    d_aqq = A[pidx(qc, qc, m)];
    double c;
    const bool r = pair_rotation(d_app, d_aqq, d_apq, q < m, c, d_sn, d_t);
    const int buf = (int)(g & 1);
    csn[buf * h + lane] = make_double2(c, d_sn);
    rb[g * h + lane] = make_double2(c, d_sn);
    const bool any = __ballot(r) != 0;
    if (lane == 0) rflag[buf] = any ? 1 : 0;
  };
  __syncthreads();
  if (tid < h) next_rotations(0);
  __syncthreads();
  int nsw = 0;
  for (int sweep = 0; sweep < a.max_sweeps; ++sweep) {
    bool swept = false;
    for (int r = 0; r < R; ++r) {
      const long g = (long)sweep * R + r;
      const int buf = (int)(g & 1);
      const double2* cs = csn + buf * h;
      const bool rotated = rflag[buf] != 0;
      swept |= rotated;
      if (rotated) {
        // A <- J^T A J as independent 2x2 blocks.  The blocks of one round are
        // disjoint, so every load of this thread's blocks is issued before any
        // store; absent elements (an index at or past m) are read from a valid
        // address, zeroed and never stored.  Wavefront 0's first task is its pair's
        // diagonal block, held in registers; every other task is off-diagonal.
        const int j0 = w == 0 ? 1 : 0;
        double2 csk[JA], csl[JA];
        int i00[JA], i01[JA], i10[JA], i11[JA];
        double x00[JA], x01[JA], x10[JA], x11[JA];
        bool vq_k[JA], vq_l[JA];
#pragma unroll
        for (int j = 0; j < JA; ++j) {
          if (j < j0 || (j > 0 && !slot1)) continue;
          csk[j] = cs[max(tk[j], 0)];
          csl[j] = cs[tl[j]];
          const int pk = min(uk[j], vk[j]), qk = max(uk[j], vk[j]);
          const int pl = min(ul[j], vl[j]), ql = max(ul[j], vl[j]);
          vq_k[j] = qk < m;
          vq_l[j] = ql < m;
          i00[j] = sidx(pk, pl, m);
          i01[j] = vq_l[j] ? sidx(pk, ql, m) : i00[j];
          i10[j] = vq_k[j] ? sidx(qk, pl, m) : i00[j];
          i11[j] = (vq_k[j] && vq_l[j]) ? sidx(qk, ql, m) : i00[j];
          x00[j] = A[i00[j]];
          x01[j] = A[i01[j]];
          x10[j] = A[i10[j]];
          x11[j] = A[i11[j]];
        }
        if (w == 0 && lane < h && d_sn != 0.0) {
          // the pair's own block: a_pp - t a_pq, a_qq + t a_pq, a_pq = 0 (a pair
          // that rotates has both players below m)
          const int p = min(up, vp), q = max(up, vp);
          A[pidx(p, p, m)] = d_app - d_t * d_apq;
          A[pidx(q, q, m)] = d_aqq + d_t * d_apq;
          A[pidx(q, p, m)] = 0.0;
        }
#pragma unroll
        for (int j = 0; j < JA; ++j) {
          if (j < j0 || (j > 0 && !slot1)) continue;
          const double ck = csk[j].x, sk = csk[j].y, cl = csl[j].x, sl = csl[j].y;
          if (tk[j] < 0 || (sk == 0.0 && sl == 0.0)) continue;
          const double a01 = vq_l[j] ? x01[j] : 0.0;
          const double a10 = vq_k[j] ? x10[j] : 0.0;
          const double a11 = (vq_k[j] && vq_l[j]) ? x11[j] : 0.0;
          // rows: J_k^T
          const double r00 = ck * x00[j] - sk * a10, r01 = ck * a01 - sk * a11;
          const double r10 = sk * x00[j] + ck * a10, r11 = sk * a01 + ck * a11;
          // columns: J_l
          A[i00[j]] = cl * r00 - sl * r01;
          if (vq_l[j]) A[i01[j]] = sl * r00 + cl * r01;
          if (vq_k[j]) A[i10[j]] = cl * r10 - sl * r11;
          if (vq_k[j] && vq_l[j]) A[i11[j]] = sl * r10 + cl * r11;
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
      if (tid < h) {
        // wavefront 0 wrote every element these read (its own stores, in order)
        up = rr_next(up, M);
        vp = rr_next(vp, M);
        if (g + 1 < gmax) next_rotations(g + 1);
      }
      __syncthreads();
    }
    if (!swept) break;
    ++nsw;
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

// Whole-wavefront lane shifts by one (DPP wave_shl:1 and wave_shr:1): lane k receives
// the value of lane k + 1, respectively k - 1 (0 past the ends).
__device__ __forceinline__ double from_next_lane(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)v, 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), 0x130, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_prev_lane(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)v, 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), 0x138, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Rows of V never mix, and in the round-robin order a round moves every player one
// position along a fixed conveyor: so lane k of a wavefront keeps, for each of its
// rows, the entries of the two players at positions k and M - 1 - k (pair k) in
// registers, applies pair k's rotation of the round to them, then passes them on to
// the neighbouring lanes (the entry at position k + 1 comes from lane k + 1, the one
// at M - k from lane k - 1, with the turn-arounds at lanes 0 and h - 1).  No LDS, no
// barrier; after whole sweeps every player is back at its starting position.
__global__ __launch_bounds__(64 * kVecWaves) void k_syevj_vecs(EigArgs a,
                                                               const double2* __restrict__ rot,
                                                               long rstride,
                                                               const int* __restrict__ meta) {
  const int b = blockIdx.x;
  const int m = a.m[b];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = blockIdx.y * kVecRows + w * kVecRowsPerWave;  // first row of this wavefront
  if (m <= 0 || i0 >= m) return;  // uniform per wavefront; no workgroup barrier follows
  const int M = m + (m & 1), h = M / 2, R = M - 1;
  const int* mb = meta + (long)b * kMetaStride;
  const long total = (long)mb[0] * R;  // rounds to replay
  const bool act = lane < h;
  // players at this lane's two positions, advanced by one position per round
  int pa = lane, pb = M - 1 - lane;
  double lo[kVecRowsPerWave], hi[kVecRowsPerWave];
#pragma unroll
  for (int r = 0; r < kVecRowsPerWave; ++r) {
    lo[r] = (act && pa == i0 + r) ? 1.0 : 0.0;
    hi[r] = (act && pb == i0 + r) ? 1.0 : 0.0;
  }
  // (c, s) of this lane's pair, kVecPf rounds per buffer, two buffers in turn: one
  // is replayed while the next is loaded.  Rounds past the end are loaded from the
  // last one (clamped, so every load is unconditional) and never replayed.  Lanes
  // past the pairs read pair 0's record; their entries never reach an active lane.
  const double2* rb = rot + (long)b * rstride + (act ? lane : 0);
  auto fetch = [&](double2* buf, long g0) {
#pragma unroll
    for (int j = 0; j < kVecPf; ++j) buf[j] = rb[min(g0 + j, total - 1) * h];
  };
  auto replay = [&](const double2* buf, long g0) {
#pragma unroll
    for (int j = 0; j < kVecPf; ++j) {
      if (g0 + j >= total) break;  // uniform per wavefront
      // the rotation of pair (p, q) acts on (v_p, v_q); with p at position
      // M - 1 - k instead of k the same formula holds with s negated
      const double c = buf[j].x, s = pa < pb ? buf[j].y : -buf[j].y;
#pragma unroll
      for (int r = 0; r < kVecRowsPerWave; ++r) {
        const double x = lo[r], y = hi[r];
        lo[r] = c * x - s * y;
        hi[r] = s * x + c * y;
      }
      if (h > 1) {  // uniform; with one pair nothing moves
#pragma unroll
        for (int r = 0; r < kVecRowsPerWave; ++r) {
          const double up = from_next_lane(lo[r]), dn = from_prev_lane(hi[r]);
          const double nlo = lane == 0 ? lo[r] : (lane == h - 1 ? hi[r] : up);
          hi[r] = lane == 0 ? up : dn;
          lo[r] = nlo;
        }
      }
      if (lane != 0) pa = (pa == R) ? 1 : pa + 1;
      pb = (pb == R) ? 1 : pb + 1;
    }
  };
  if (total > 0) {
    double2 bufa[kVecPf], bufb[kVecPf];
    fetch(bufa, 0);
    for (long g0 = 0; g0 < total; g0 += 2 * kVecPf) {
      fetch(bufb, g0 + kVecPf);
      replay(bufa, g0);
      if (g0 + kVecPf >= total) break;
      fetch(bufa, g0 + 2 * kVecPf);
      replay(bufb, g0 + kVecPf);
    }
  }
  if (!act) return;
  double* Vout = a.V[b];
  const long ldv = a.ldv;
#pragma unroll
  for (int r = 0; r < kVecRowsPerWave; ++r) {
    const int i = i0 + r;
    if (i >= m) break;
    Vout[i + (long)mb[1 + pa] * ldv] = lo[r];
    if (pb < m) Vout[i + (long)mb[1 + pb] * ldv] = hi[r];
  }
}

size_t eig_lds_bytes(int mmax) {
  const int M = mmax + (mmax & 1);
  const int h = M / 2;
  const size_t npk = (size_t)M * (M + 1);
  return sizeof(double) * (((npk + 1) & ~size_t(1)) + 4 * h) + sizeof(int) * (4 + mmax) + 64;
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
