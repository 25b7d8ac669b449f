// Shift-invert application X = C^{-1} Y = P^T L^{-T} D^{-1} L^{-1} P Y through the
// factors of the Bunch-Kaufman LDL^T (Algorithm 2, third step), for several
// shifts at once.
//
// Design (gfx950): the triangular solves are dependency chains over row blocks
// of 64.  Each solve is one persistent launch per direction: workgroups take
// row blocks in dependency order from a per-shift ticket counter (so a block
// only ever waits for blocks already owned by running workgroups), accumulate
// the off-diagonal contributions of finished blocks as those blocks appear
// (sentinel hand-off below), and finish their block with a precomputed inverse
// of the 64x64 unit-lower diagonal block, so the critical path per block is one
// hand-off plus one 64x64 block product on FP64 MFMA.  L is read once per
// direction.
// The block-diagonal D^{-1} (1x1 and 2x2 pivots) is applied at the start of the
// backward sweep.
#include "common.hpp"
#include "handle.hpp"
#include "solve.hpp"

namespace sislice {

constexpr int SB = kSolveBlock;  // 64 rows per block

// perm p(i) and pivot-block flags (1: 1x1, 2: first row of 2x2, 0: second row)
// from the documented ipiv format.
__global__ __launch_bounds__(256) void k_solve_prep(int n, const int* const* ipivs,
                                                    int* const* perms, int* const* blks) {
  const int s = blockIdx.y;
  const int* ipiv = ipivs[s];
  int* perm = perms[s];
  int* blk = blks[s];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int v = ipiv[i];
    perm[i] = v >= 0 ? v : -v - 1;
    if (v >= 0) {
      blk[i] = 1;
    } else {
      int run = 0;  // consecutive 2x2 rows before i
      for (int q = i - 1; q >= 0 && ipiv[q] < 0; --q) ++run;
      blk[i] = (run & 1) ? 0 : 2;
    }
  }
}

__device__ __forceinline__ double lval(const double* LD, long ldld, const int* blk, int row,
                                       int col) {
  // strictly lower L entry (row > col); inside a 2x2 pivot block the slot holds
  // D's off-diagonal and L's entry is a structural zero
  if (row == col + 1 && blk[col] == 2) return 0.0;
  return LD[row + (long)col * ldld];
}

// Inverse of each 64x64 unit-lower diagonal block of L (rows past n: identity).
// Linv layout per shift: block b at b*SB*SB, column-major 64x64.
__global__ __launch_bounds__(64) void k_diag_inv_blk(int n, const double* const* LDs, long ldld,
                                                     const int* const* blks, double* const* Linvs) {
  __shared__ double sL[SB][SB + 1];
  __shared__ double sX[SB][SB + 1];  // sX[c][i] = X(i, c)
  const int b = blockIdx.x, s = blockIdx.y, t = threadIdx.x;
  const double* LD = LDs[s];
  const int* blk = blks[s];
  const int r0 = b * SB;
  for (int k = 0; k < SB; ++k) {
    const int col = r0 + k, row = r0 + t;
    double v = 0.0;
    if (t > k && row < n) v = lval(LD, ldld, blk, row, col);
    sL[t][k] = v;
  }
  __syncthreads();
  const int c = t;
  for (int i = 0; i < SB; ++i) {
    double acc = (i == c) ? 1.0 : 0.0;
    for (int k = 0; k < i; ++k) acc -= sL[i][k] * sX[c][k];
    sX[c][i] = (i >= c) ? acc : 0.0;
  }
  __syncthreads();
  double* Linv = Linvs[s] + (long)b * SB * SB;
  for (int k = 0; k < SB; ++k) Linv[t + k * SB] = sX[k][t];
}

// Look-ahead blocks of depth d = 1, 2 (per shift, after the nblk diagonal inverses):
//   Mf^d_b = Linv_b L_{b,b-d}           (forward sweep, b >= d)
//   Mb^d_b = Linv_b^T L_{b+d,b}^T       (backward sweep, b + d <= nblk - 1)
// so that a block's result is P_b - sum_d M^d_b x (block b -+ d), with P_b (the
// contributions of blocks further away) formed before the nearest two blocks are
// available.  L's structural zeros inside 2x2 pivots are applied here (lval), so
// the sweeps read these blocks as plain matrices.  Layout: column-major 64x64,
// Mf^d at (2d - 1)*nblk*SB*SB and Mb^d at 2d*nblk*SB*SB of the Linv buffer.
__global__ __launch_bounds__(256) void k_lookahead(int n, const double* const* LDs, long ldld,
                                                   const int* const* blks, double* const* Linvs) {
  __shared__ double sA[SB][SB + 1];  // Linv_b(i, k)
  __shared__ double sB[SB][SB + 1];
  const int b = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int nblk = (n + SB - 1) / SB;
  const double* LD = LDs[s];
  const int* blk = blks[s];
  double* base = Linvs[s];
  const double* Li = base + (long)b * SB * SB;
  const int r0 = b * SB;
  for (int e = tid; e < SB * SB; e += 256) sA[e & 63][e >> 6] = Li[e];
  for (int d = 1; d <= kSolveLook; ++d) {
    // forward: sB[j][k] = L(r0 + j, r0 - d*64 + k)
    if (b >= d) {
      __syncthreads();
      for (int e = tid; e < SB * SB; e += 256) {
        const int j = e & 63, k = e >> 6, row = r0 + j;
        sB[j][k] = (row < n) ? lval(LD, ldld, blk, row, r0 - d * SB + k) : 0.0;
      }
      __syncthreads();
      double* Mf = base + (long)(2 * d - 1) * nblk * SB * SB + (long)b * SB * SB;
      for (int e = tid; e < SB * SB; e += 256) {
        const int i = e & 63, k = e >> 6;
        double v = 0.0;
        for (int j = 0; j <= i; ++j) v += sA[i][j] * sB[j][k];
        Mf[e] = v;
      }
    }
    // backward: G = L_{b+d,b} Linv_b, sB[i][j] = L(r0 + d*64 + i, r0 + j); Mb = G^T
    if (b + d < nblk) {
      __syncthreads();
      for (int e = tid; e < SB * SB; e += 256) {
        const int ii = e & 63, j = e >> 6, row = r0 + d * SB + ii;
        sB[ii][j] = (row < n) ? lval(LD, ldld, blk, row, r0 + j) : 0.0;
      }
      __syncthreads();
      double* Mb = base + (long)(2 * d) * nblk * SB * SB + (long)b * SB * SB;
      for (int e = tid; e < SB * SB; e += 256) {
        const int i = e & 63, k = e >> 6;  // Mb(i, k) = G(k, i) = sum_j L(k, j) Linv(j, i)
        double v = 0.0;
        for (int j = i; j < SB; ++j) v += sB[k][j] * sA[j][i];
        Mb[e] = v;
      }
    }
  }
}

__device__ __forceinline__ unsigned ticket(unsigned* ctr, unsigned nblk) {
  __shared__ unsigned t;
  if (threadIdx.x == 0) {
    t = atomicAdd(ctr, 1u);
    if (t == nblk - 1) atomicExch(ctr, 0u);  // last taker resets for the next launch
  }
  __syncthreads();
  return t;
}

// Hand-off between workgroups without flags.  Before a sweep, its result buffer
// is filled with a signalling-NaN sentinel (no arithmetic result is a signalling
// NaN, and the fill kernel has completed before the sweep starts).  A block is
// published by storing its values as relaxed agent-scope atomics, which go to
// the device coherence point instead of a per-XCD L2 line; a waiter polls the
// block itself with agent-scope loads until no sentinel is left.  One round trip
// per hand-off, no drain on the producer's side.  (Polling a flag with acquire
// loads would invalidate the caches on every poll; with hundreds of waiters that
// serialises the whole chip.)
constexpr unsigned long long kSentinelBits = 0x7FF4000000000001ull;

__device__ __forceinline__ double ld_shared_blk(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_shared_blk(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool is_sentinel(double v) {
  return (unsigned long long)__double_as_longlong(v) == kSentinelBits;
}

// Every wait is bounded: after `limit` unsuccessful polls a waiter stops, raises
// the handle's wait-error word (the host turns it into an error status after the
// call) and goes on with what it read, so the launch always drains.  Correct
// hand-offs finish in microseconds; the default bound is about a second.
struct WaitBound {
  unsigned* err;
  unsigned limit;
};

__device__ __forceinline__ bool wait_expired(const WaitBound& wb, unsigned& polls) {
  if (polls++ < wb.limit) return false;
  __hip_atomic_store(wb.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// sx[c * kLdx + rr] = block rows rr < rows of column c of B (ld ldb), once none is
// the sentinel; rows past `rows` read as zero.  A block that is already complete
// (the common case for a workgroup that started after its predecessors) is read in
// one round trip.  Otherwise one lane waits on a single element first (the last
// one of the block), so the waiting workgroups do not stream the whole block from
// the coherence point on every poll; the block is then loaded and checked in full
// (other lanes' stores may still be on their way).
// LDS column stride of a vector block: odd, so the 16 rows of one column that a
// quarter-wave reads as an MFMA operand fall in 16 different banks
constexpr int kLdx = SB + 1;

__device__ __forceinline__ void poll_block(double* sx, const double* B, long ldb, int nrhs,
                                           int rows, const WaitBound& wb) {
  {
    int ok = 1;
    for (int e = threadIdx.x; e < nrhs * SB; e += 256) {
      const int rr = e & 63, c = e >> 6;
      double v = 0.0;
      if (rr < rows) {
        v = ld_shared_blk(B + rr + (long)c * ldb);
        if (is_sentinel(v)) ok = 0;
      }
      sx[c * kLdx + rr] = v;
    }
    if (__syncthreads_and(ok)) return;
  }
  __shared__ int expired;
  if (threadIdx.x == 0) {
    const double* last = B + (rows - 1) + (long)(nrhs - 1) * ldb;
    unsigned polls = 0;
    int ex = 0;
    while (is_sentinel(ld_shared_blk(last))) {
      if (wait_expired(wb, polls)) {
        ex = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    expired = ex;
  }
  __syncthreads();
  unsigned polls = 0;
  for (;;) {
    int ok = 1;
    for (int e = threadIdx.x; e < nrhs * SB; e += 256) {
      const int rr = e & 63, c = e >> 6;
      double v = 0.0;
      if (rr < rows) {
        v = ld_shared_blk(B + rr + (long)c * ldb);
        if (is_sentinel(v)) ok = 0;
      }
      sx[c * kLdx + rr] = v;
    }
    // a wait that already expired, or one that expires here, goes on with what it read
    // (the decision is uniform: `expired` and the poll count are the same in every lane)
    if (__syncthreads_and(ok) || expired || wait_expired(wb, polls)) return;
    __builtin_amdgcn_s_sleep(2);
  }
}

// The critical hand-off (a block waiting for its immediate predecessor): at most
// one or two workgroups per shift wait here at a time, so every lane spins on its
// own elements and the block is complete one round trip after it lands, instead
// of one round trip for the probe element and another for the block.  A lane
// re-polls all of its still-missing elements together.
template <int NR>
__device__ __forceinline__ void poll_block_spin(double* sx, const double* B, long ldb, int nrhs,
                                                int rows, const WaitBound& wb) {
  constexpr int E = NR * SB / 256;  // elements per lane
  double v[E];
  bool live[E];
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int e = threadIdx.x + 256 * k, rr = e & 63, c = e >> 6;
    live[k] = c < nrhs && rr < rows;
    v[k] = live[k] ? ld_shared_blk(B + rr + (long)c * ldb) : 0.0;
  }
  unsigned polls = 0;
  for (;;) {
    bool missing = false;
#pragma unroll
    for (int k = 0; k < E; ++k) missing |= live[k] && is_sentinel(v[k]);
    if (!missing || wait_expired(wb, polls)) break;
    __builtin_amdgcn_s_sleep(1);
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int e = threadIdx.x + 256 * k, rr = e & 63, c = e >> 6;
      if (live[k] && is_sentinel(v[k])) v[k] = ld_shared_blk(B + rr + (long)c * ldb);
    }
  }
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int e = threadIdx.x + 256 * k, rr = e & 63, c = e >> 6;
    if (c < nrhs) sx[c * kLdx + rr] = v[k];
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_fill_sentinel(int n, int nrhs, int nshift,
                                                       double* const* A, double* const* B, long ld) {
  const int s = blockIdx.y;
  const double sv = __longlong_as_double((long long)kSentinelBits);
  const long tot = (long)n * nrhs;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < tot; e += (long)gridDim.x * 256) {
    const long off = (e % n) + (e / n) * ld;
    if (A) A[s][off] = sv;
    if (B) B[s][off] = sv;
  }
}

// Workgroups are dispatched to the 8 XCDs round-robin by linear id.  Shift s is
// served by the workgroups of XCD s % 8 only, so its dependency chain stays on one
// L2.  On each XCD the shifts are interleaved by rank (local index j = rank * U + u
// serves shift x + 8u, U = ceil(nshift / 8)), so every shift's first workgroups
// are dispatched before any shift's later ones.  Returns -1 for the padding
// workgroups of an unbalanced split.
__device__ __forceinline__ int solve_shift_of(int g, int nshift) {
  const int x = g & 7, j = g >> 3;
  const int U = (nshift + 7) >> 3;
  const int s = x + 8 * (j % U);
  return s < nshift ? s : -1;
}

// The sweeps' 64x64 block products run on FP64 MFMA (v_mfma_f64_16x16x4).  Wavefront
// w owns rows 16w .. 16w+15 of the block; with j = lane % 16 and g = lane / 16, a
// product R = M X (M a 64x64 matrix, X a 64 x nrhs vector block) is accumulated as
// R^T = X^T M^T in 16-column tiles u: step t supplies X(4t + g, 16u + j) as the A
// operand (from LDS) and M(16w + j, 4t + g) as the B operand (from registers), and
// accumulator element r of the lane ends up holding R(16w + j, 16u + g + 4r).  A
// product is subtracted by negating the accumulator around it (y - M x computed as
// -(M x + (-y)), the same rounding), so the matrices are loaded as they are, with
// no arithmetic between a load and its use.  Columns past nrhs are padding: their A
// operands come from zeroed LDS and their results are never stored.
template <int NT>
__device__ __forceinline__ void mfma_block(const double* sx, const double (&mfr)[16], d4 (&acc)[NT]) {
  const int l = threadIdx.x & 63, j = l & 15, g = l >> 4;
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[u] = mfma16x16x4(sx[(16 * u + j) * kLdx + 4 * t + g], mfr[t], acc[u]);
}

// The same product as two independent multiply-add chains (even and odd steps),
// for the products on the critical path.
template <int NT>
__device__ __forceinline__ void mfma_block2(const double* sx, const double (&mfr)[16], d4 (&acc)[NT]) {
  const int l = threadIdx.x & 63, j = l & 15, g = l >> 4;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    d4 h = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 16; t += 2) {
      acc[u] = mfma16x16x4(sx[(16 * u + j) * kLdx + 4 * t + g], mfr[t], acc[u]);
      h = mfma16x16x4(sx[(16 * u + j) * kLdx + 4 * t + 4 + g], mfr[t + 1], h);
    }
    acc[u] += h;
  }
}

// The product with M in LDS instead of registers: M(m, k) at sm[m * kLdx + k].
template <int NT>
__device__ __forceinline__ void mfma_block_lds(const double* sx, const double* sm, d4 (&acc)[NT]) {
  const int tid = threadIdx.x, l = tid & 63, j = l & 15, g = l >> 4, rw = 16 * (tid >> 6) + j;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const double bm = sm[rw * kLdx + 4 * t + g];
#pragma unroll
    for (int u = 0; u < NT; ++u) acc[u] = mfma16x16x4(sx[(16 * u + j) * kLdx + 4 * t + g], bm, acc[u]);
  }
}

// B-operand fragments of a column-major 64x64 matrix M (ld 64): M(16w + j, 4t + g),
// or of its transpose.
template <bool TRANS>
__device__ __forceinline__ void load_frag(const double* M, double (&f)[16]) {
  const int tid = threadIdx.x, l = tid & 63, rw = 16 * (tid >> 6) + (l & 15), g = l >> 4;
#pragma unroll
  for (int t = 0; t < 16; ++t) f[t] = TRANS ? M[(4 * t + g) + 64 * rw] : M[rw + 64 * (4 * t + g)];
}

template <int NT>
__device__ __forceinline__ void negate(d4 (&x)[NT]) {
#pragma unroll
  for (int u = 0; u < NT; ++u) x[u] = -x[u];
}

// Forward sweep: Z = L^{-1} P Y.  The L blocks do not depend on other workgroups,
// so the next one is prefetched into registers while the current result block is
// awaited.  The contributions of blocks 0 .. b-3 are accumulated as they appear,
// P_b = Linv_b acc is formed before block b-2 is available, and after the last
// hand-off only Z_b = P_b - Mf_b Z_{b-1} remains (the look-ahead blocks Mf^1, Mf^2).
template <int NR>
__global__ __launch_bounds__(256) void k_fwd(SolveArgs a) {
  constexpr int NT = (NR + 15) / 16;
  __shared__ double sx[16 * NT * kLdx];
  const int tid = threadIdx.x, l = tid & 63, j = l & 15, g = l >> 4;
  const int n = a.n, nrhs = a.nrhs, nblk = (n + SB - 1) / SB;
  const int s = solve_shift_of(blockIdx.x, a.nshift);
  if (s < 0) return;
  const WaitBound wb{a.wait_err, a.wait_limit};
  const int b = (int)ticket(a.ctr + s, nblk);
  const double* LD = a.LD[s];
  const int* perm = a.perm[s];
  const double* Y = a.Y[s];
  double* Z = a.Z[s];
  const int r0 = b * SB;
  const int row = r0 + 16 * (tid >> 6) + j;
  for (int e = tid; e < 16 * NT * kLdx; e += 256) sx[e] = 0.0;
  // everything that does not depend on other blocks is issued first
  const double* Lbase = a.Linv[s];
  double inv[16];
  load_frag<false>(Lbase + (long)b * SB * SB, inv);
  d4 acc[NT];  // -(P Y - contributions so far)
  {
    // every load from a clamped index, then the selects: one round trip for Y
    const int pr = perm[min(row, n - 1)];
    double y[NT][4];
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) y[u][r] = Y[pr + (long)min(16 * u + g + 4 * r, nrhs - 1) * a.ldy];
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = 16 * u + g + 4 * r;
        acc[u][r] = (c < nrhs && row < n) ? -y[u][r] : 0.0;
      }
  }
  // L(row, c0 + 4t + g) of block cb, the B operand of its contribution.  Rows past n
  // (last block only) read row n - 1: they only reach this block's rows past n,
  // which are cleared before P_b.
  double lcur[16], lnext[16];
  const int rowc = min(row, n - 1);
  auto load_L = [&](int cb) {
    const long c0 = (long)cb * SB;
#pragma unroll
    for (int t = 0; t < 16; ++t) lnext[t] = LD[rowc + (c0 + 4 * t + g) * a.ldld];
  };
  if (b > 2) load_L(0);
  __syncthreads();
  for (int cb = 0; cb + 2 < b; ++cb) {
#pragma unroll
    for (int t = 0; t < 16; ++t) lcur[t] = lnext[t];
    if (cb + 3 < b) load_L(cb + 1);
    poll_block(sx, Z + cb * SB, a.ldz, nrhs, SB, wb);
    mfma_block<NT>(sx, lcur, acc);
    __syncthreads();
  }
  // the look-ahead blocks load while P_b = Linv_b acc is formed
  double mf2[16], mf[16];
  if (b >= 2) load_frag<false>(Lbase + (3L * nblk + b) * SB * SB, mf2);
  if (b >= 1) load_frag<false>(Lbase + (1L * nblk + b) * SB * SB, mf);
  const int rw = 16 * (tid >> 6) + j;
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r) sx[(16 * u + g + 4 * r) * kLdx + rw] = row < n ? -acc[u][r] : 0.0;
  __syncthreads();
  d4 pb[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) pb[u] = d4{0.0, 0.0, 0.0, 0.0};
  mfma_block<NT>(sx, inv, pb);
  negate<NT>(pb);
  if (b >= 2) {  // P_b -= Mf^2_b Z_{b-2}
    __syncthreads();
    poll_block_spin<NR>(sx, Z + (b - 2) * SB, a.ldz, nrhs, SB, wb);
    mfma_block2<NT>(sx, mf2, pb);
  }
  if (b >= 1) {
    __syncthreads();
    poll_block_spin<NR>(sx, Z + (b - 1) * SB, a.ldz, nrhs, SB, wb);
    mfma_block2<NT>(sx, mf, pb);
  }
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = 16 * u + g + 4 * r;
      if (c < nrhs && row < n) st_shared_blk(Z + row + (long)c * a.ldz, -pb[u][r]);
    }
}

// Backward sweep: X = P^T L^{-T} D^{-1} Z, from the last block up, with the same
// look-ahead: V_b = P_b - Mb_b V_{b+1}, P_b = Linv_b^T (D^{-1} Z_b - contributions
// of blocks b+3 ..) - Mb^2_b V_{b+2}.
template <int NR>
__global__ __launch_bounds__(256) void k_bwd(SolveArgs a) {
  constexpr int NT = (NR + 15) / 16;
  __shared__ double sx[16 * NT * kLdx];
  __shared__ double sl[SB * kLdx];  // sl[m * kLdx + k] = L(c0 + k, r0 + m) of the block in use
  const int tid = threadIdx.x, l = tid & 63, j = l & 15, g = l >> 4;
  const int n = a.n, nrhs = a.nrhs, nblk = (n + SB - 1) / SB;
  const int s = solve_shift_of(blockIdx.x, a.nshift);
  if (s < 0) return;
  const WaitBound wb{a.wait_err, a.wait_limit};
  const int tk = (int)ticket(a.ctr + s, nblk);
  const int b = nblk - 1 - tk;
  const double* LD = a.LD[s];
  const int* blk = a.blk[s];
  const int* perm = a.perm[s];
  const double* Z = a.Z[s];
  double* V = a.V[s];
  double* X = a.X[s];
  const int r0 = b * SB;
  const int rw = 16 * (tid >> 6) + j;
  const int row = r0 + rw;
  for (int e = tid; e < 16 * NT * kLdx; e += 256) sx[e] = 0.0;
  const double* Lbase = a.Linv[s];
  double inv[16];  // Linv_b^T
  load_frag<true>(Lbase + (long)b * SB * SB, inv);
  d4 acc[NT];  // -(D^{-1} Z_b - contributions so far)
  // D^{-1} on this block's rows.  The pivot flag, both candidate 2x2 blocks (the row
  // as first or as second row of its pivot) and the rows of Z around this row are
  // loaded at once from clamped indices, and the values are selected afterwards, so
  // the block starts after one round trip instead of a chain of dependent ones.
  {
    const int rc = min(row, n - 1), rup = min(rc + 1, n - 1), rdn = max(rc - 1, 0);
    const int bt_rc = blk[rc];
    const int bt = row < n ? bt_rc : 1;
    const double l_rr = LD[rc + (long)rc * a.ldld], l_ur = LD[rup + (long)rc * a.ldld];
    const double l_uu = LD[rup + (long)rup * a.ldld], l_dd = LD[rdn + (long)rdn * a.ldld];
    const double l_rd = LD[rc + (long)rdn * a.ldld];
    double zs[NT][4], zu[NT][4], zd[NT][4];
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long cc = (long)min(16 * u + g + 4 * r, nrhs - 1) * a.ldz;
        zs[u][r] = Z[rc + cc];
        zu[u][r] = Z[rup + cc];
        zd[u][r] = Z[rdn + cc];
      }
    // 1x1 pivot: d11; first row of a 2x2 pivot (k = row); second row (k = row - 1)
    double d11 = 1.0, d21 = 0.0, d22 = 1.0;
    if (row < n) {
      if (bt == 1) {
        d11 = l_rr;
      } else if (bt == 2) {
        d11 = l_rr;
        d21 = l_ur;
        d22 = l_uu;
      } else {
        d11 = l_dd;
        d21 = l_rd;
        d22 = l_rr;
      }
    }
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = 16 * u + g + 4 * r;
        double v = 0.0;
        if (c < nrhs && row < n) {
          const double z = zs[u][r];
          if (!a.applyD) {
            v = z;
          } else if (bt == 1) {
            v = (d11 != 0.0) ? z / d11 : 0.0;
          } else {
            const double zp = bt == 2 ? zu[u][r] : zd[u][r];
            // [w1 w2] = D^{-1} [z1 z2], scaled by the off-diagonal as in the factorization
            const double z1 = bt == 2 ? z : zp, z2 = bt == 2 ? zp : z;
            const double aa = d11 / d21, gg = d22 / d21;
            const double tt = 1.0 / (d21 * (aa * gg - 1.0));
            v = bt == 2 ? tt * (gg * z1 - z2) : tt * (aa * z2 - z1);
          }
        }
        acc[u][r] = -v;
      }
  }
  // L_{cb,b}^T, the B operand of block cb's contribution, is read along L's columns
  // (element e: row c0 + (e & 63), column r0 + (e >> 6)) and transposed through
  // LDS; the poll's barrier orders those writes before the products.  Rows of L past
  // n (the ragged last block) read row n - 1: they meet the zero rows of that
  // block's V.  A block that accumulates has all its rows below n.
  constexpr int Q = SB * SB / 256;
  double lnext[Q];
  auto load_L = [&](int cb) {
    const int c0 = cb * SB;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = tid + 256 * q;
      lnext[q] = LD[min(c0 + (e & 63), n - 1) + (long)(r0 + (e >> 6)) * a.ldld];
    }
  };
  if (b + 3 < nblk) load_L(nblk - 1);
  __syncthreads();
  for (int cb = nblk - 1; cb > b + 2; --cb) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = tid + 256 * q;
      sl[(e >> 6) * kLdx + (e & 63)] = lnext[q];
    }
    if (cb - 1 > b + 2) load_L(cb - 1);
    poll_block(sx, V + cb * SB, a.ldz, nrhs, min(SB, n - cb * SB), wb);
    mfma_block_lds<NT>(sx, sl, acc);
    __syncthreads();
  }
  // the look-ahead blocks load while P_b = Linv_b^T acc is formed
  double mb2[16], mb[16];
  if (b + 2 < nblk) load_frag<false>(Lbase + (4L * nblk + b) * SB * SB, mb2);
  if (b + 1 < nblk) load_frag<false>(Lbase + (2L * nblk + b) * SB * SB, mb);
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r) sx[(16 * u + g + 4 * r) * kLdx + rw] = -acc[u][r];
  __syncthreads();
  d4 pb[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) pb[u] = d4{0.0, 0.0, 0.0, 0.0};
  mfma_block<NT>(sx, inv, pb);
  negate<NT>(pb);
  if (b + 2 < nblk) {  // P_b -= Mb^2_b V_{b+2}
    __syncthreads();
    poll_block_spin<NR>(sx, V + (b + 2) * SB, a.ldz, nrhs, min(SB, n - (b + 2) * SB), wb);
    mfma_block2<NT>(sx, mb2, pb);
  }
  if (b + 1 < nblk) {
    __syncthreads();
    poll_block_spin<NR>(sx, V + (b + 1) * SB, a.ldz, nrhs, min(SB, n - (b + 1) * SB), wb);
    mfma_block2<NT>(sx, mb, pb);
  }
  const int px = row < n ? perm[row] : 0;
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = 16 * u + g + 4 * r;
      if (c < nrhs && row < n) {
        st_shared_blk(V + row + (long)c * a.ldz, -pb[u][r]);
        X[px + (long)c * a.ldx] = -pb[u][r];
      }
    }
}

// Li (ldli, zero elsewhere) receives the 64x64 inverses of L's diagonal blocks on
// its block diagonal: the starting point of the explicit inverse of L.
__global__ __launch_bounds__(256) void k_diag_inv_scatter(int n, const double* __restrict__ Linv,
                                                          double* __restrict__ Li, long ldli) {
  const int b = blockIdx.x;
  for (int e = threadIdx.x; e < SB * SB; e += 256) {
    const int r = b * SB + (e & 63), c = b * SB + (e >> 6);
    if (r < n && c < n) Li[r + (long)c * ldli] = Linv[(long)b * SB * SB + e];
  }
}

void diag_inv_scatter_launch(int n, const double* Linv, double* Li, long ldli, hipStream_t st) {
  SL_LAUNCH(k_diag_inv_scatter, dim3((unsigned)ceil_div(n, SB)), dim3(256), 0, st, n, Linv, Li,
            ldli);
  SL_LAUNCH_CHECK();
}

void solve_prep_launch(int n, int S, const int* const* d_ipiv, int* const* d_perm,
                       int* const* d_blk, const double* const* d_LD, long ldld,
                       double* const* d_Linv, hipStream_t st) {
  SL_LAUNCH(k_solve_prep, dim3((unsigned)ceil_div(n, 256), S), dim3(256), 0, st, n, d_ipiv,
                     d_perm, d_blk);
  SL_LAUNCH_CHECK();
  SL_LAUNCH(k_diag_inv_blk, dim3((unsigned)ceil_div(n, SB), S), dim3(64), 0, st, n, d_LD,
                     ldld, (const int* const*)d_blk, d_Linv);
  SL_LAUNCH_CHECK();
  SL_LAUNCH(k_lookahead, dim3((unsigned)ceil_div(n, SB), S), dim3(256), 0, st, n, d_LD, ldld,
            (const int* const*)d_blk, d_Linv);
  SL_LAUNCH_CHECK();
}

void solve_launch(SolveArgs a, hipStream_t st, int mode) {
  const int nblk = (int)ceil_div(a.n, SB);
  SL_CHECK_ARG(a.nrhs >= 0 && a.nrhs <= kSolveMaxRhs, "too many right-hand sides for one sweep");
  // 8 XCDs x ceil(nshift / 8) shift slots x nblk blocks (see solve_shift_of)
  const unsigned grid = (unsigned)(8 * ceil_div(a.nshift, 8) * nblk);
  sislice_handle* ph = current_handle();
  a.wait_err = wait_flag(ph);
  a.wait_limit = ph->wait_limit;
  const int tk = prof_begin(ph, kProfSolve);
  // sentinels in the result buffers of the sweeps of this launch
  const long tot = (long)a.n * a.nrhs;
  SL_LAUNCH(k_fill_sentinel, dim3((unsigned)std::min<long>(ceil_div(tot, 256), 1024), a.nshift),
            dim3(256), 0, st, a.n, a.nrhs, a.nshift, (mode == 0 || mode == 1) ? a.Z : nullptr,
            (mode == 0 || mode == 2) ? a.V : nullptr, a.ldz);
  SL_LAUNCH_CHECK();
  const bool small = a.nrhs <= 8;
  if (mode == 0 || mode == 1) {
    if (small)
      SL_LAUNCH(k_fwd<8>, dim3(grid), dim3(256), 0, st, a);
    else
      SL_LAUNCH(k_fwd<kSolveMaxRhs>, dim3(grid), dim3(256), 0, st, a);
    SL_LAUNCH_CHECK();
  }
  if (mode == 0 || mode == 2) {
    if (small)
      SL_LAUNCH(k_bwd<8>, dim3(grid), dim3(256), 0, st, a);
    else
      SL_LAUNCH(k_bwd<kSolveMaxRhs>, dim3(grid), dim3(256), 0, st, a);
    SL_LAUNCH_CHECK();
  }
  prof_end(ph, tk);
}

}  // namespace sislice
