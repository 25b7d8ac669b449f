// Dense FP64 building blocks of the Lanczos / Rayleigh-Ritz / KPM phases:
// batched MFMA GEMM with optional transposes and deterministic split-K,
// symmetrisation of a lower-stored matrix, column dot products / norms, and the
// counter-based Gaussian start blocks.
//
// GEMM design (gfx950): 64x64 output tile per 256-thread workgroup, four
// wavefronts each owning 32x32 as 2x2 v_mfma_f64_16x16x4 blocks; K staged
// through double-buffered LDS in chunks of 16 (sA[k][i], sB[k][j]), the next two
// chunks' loads in flight during the current chunk's MFMAs.  The MFMA A operand carries
// op(B)^T and the B operand op(A)^T so that accumulator register r of lane l
// holds C(i0 + l%16, j0 + l/16 + 4r): sixteen consecutive rows of one column,
// i.e. coalesced column-major stores.  Transposed operands only change the
// global->LDS load pattern (always along the contiguous dimension).
#include "blas.hpp"
#include "common.hpp"
#include "handle.hpp"

namespace sislice {

// p[0] + p[stride] + ... + p[(cnt - 1) stride], added in that order, with eight loads in
// flight (a plain loop issues one load per round trip): the split-K reductions.
__device__ __forceinline__ double ordered_sum(const double* __restrict__ p, long stride, int cnt) {
  double s = 0.0;
  int q = 0;
  for (; q + 8 <= cnt; q += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(long)(q + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; q < cnt; ++q) s += p[(long)q * stride];
  return s;
}

constexpr int GT = 64;   // tile rows/cols
constexpr int GK = 16;   // K chunk

template <bool TA, bool TB>
__global__ __launch_bounds__(256, 4) void k_gemm(GemmArgs g) {
  // row stride GT + 1 (odd): the staging stores along k (16 lanes a quarter-wave) hit
  // 16 different banks
  __shared__ double sA[2][GK][GT + 1];
  __shared__ double sB[2][GK][GT + 1];
  const int zb = blockIdx.z;
  const int b = zb / g.splits, sp = zb % g.splits;
  const int m = g.m ? g.m[b] : g.m0;
  const int n = g.n ? g.n[b] : g.n0;
  const int K = g.k ? g.k[b] : g.k0;
  const int i0 = blockIdx.x * GT, j0 = blockIdx.y * GT;
  if (i0 >= m || j0 >= n) return;
  const double* A = g.A ? g.A[b] : g.A1;
  const double* B = g.B ? g.B[b] : g.B1;
  int kc = (K + g.splits - 1) / g.splits;
  kc = (kc + GK - 1) / GK * GK;
  const int kb = sp * kc, ke = min(K, kb + kc);
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
  const int lr = l & 15, lk = l >> 4;
  d4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
  // Staging: element e = tid + 256 q of a chunk, read along the contiguous
  // dimension of each operand.  Two register sets hold the chunks after the one in
  // LDS: chunk c + 2 is loaded while chunk c feeds the MFMAs and chunk c + 1 is
  // written to the other LDS buffer, one barrier per chunk; two chunks in flight per
  // workgroup are what hides the memory latency at four workgroups per CU.
  // The loads are buffer loads from a descriptor based at the tile's corner of the
  // chunk: a lane's offset is small and fixed, and an element outside the operand
  // gets an offset past the descriptor's range, which the hardware reads as zero.
  constexpr int NQ = GK * GT / 256;
  constexpr unsigned kOut = 0x80000000u;  // past kRange: reads as 0
  constexpr int kRange = 0x7fffffff;
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  double ra[2][NQ], rb[2][NQ];
  // Load q of a thread: A element (row ia0 + q da_i, k ka0 + q da_k) of the chunk,
  // B element (k kb0 + q db_k, column ib0 + q db_j): along the contiguous dimension
  // the 256 threads cover the tile's 64 entries or the chunk's 16 once per q.
  const int ia0 = TA ? tid >> 4 : tid & 63, ka0 = TA ? tid & 15 : tid >> 6;
  constexpr int da_i = TA ? 16 : 0, da_k = TA ? 0 : 4;
  const int ib0 = TB ? tid & 63 : tid >> 4, kb0 = TB ? tid >> 6 : tid & 15;
  constexpr int db_j = TB ? 0 : 16, db_k = TB ? 4 : 0;
  // byte offsets from the chunk's corner and their per-q strides
  const unsigned oa0 = 8u * (unsigned)(TA ? ka0 + ia0 * g.lda : ia0 + ka0 * g.lda);
  const unsigned sa = 8u * (unsigned)(TA ? da_i * g.lda : da_k * g.lda);
  const unsigned ob0 = 8u * (unsigned)(TB ? ib0 + kb0 * g.ldb : kb0 + ib0 * g.ldb);
  const unsigned sbq = 8u * (unsigned)(TB ? db_k * g.ldb : db_j * g.ldb);
  auto fetch = [&](int s, int k0) {
    // corners of the chunk in A (rows i0.., k k0..) and in B (k k0.., columns j0..)
    const double* ca = TA ? A + k0 + (long)i0 * g.lda : A + i0 + (long)k0 * g.lda;
    const double* cb = TB ? B + j0 + (long)k0 * g.ldb : B + k0 + (long)j0 * g.ldb;
    const __amdgpu_buffer_rsrc_t da = __builtin_amdgcn_make_buffer_rsrc((void*)ca, (short)0, kRange, 0x00020000);
    const __amdgpu_buffer_rsrc_t db = __builtin_amdgcn_make_buffer_rsrc((void*)cb, (short)0, kRange, 0x00020000);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const bool va = (i0 + ia0 + q * da_i < m) & (k0 + ka0 + q * da_k < ke);
      const bool vb = (j0 + ib0 + q * db_j < n) & (k0 + kb0 + q * db_k < ke);
      const u2 xa = __builtin_amdgcn_raw_buffer_load_b64(da, (int)(va ? oa0 + q * sa : kOut), 0, 0);
      const u2 xb = __builtin_amdgcn_raw_buffer_load_b64(db, (int)(vb ? ob0 + q * sbq : kOut), 0, 0);
      ra[s][q] = __builtin_bit_cast(double, xa);
      rb[s][q] = __builtin_bit_cast(double, xb);
    }
  };
  auto stage = [&](int buf, int s) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      sA[buf][ka0 + q * da_k][ia0 + q * da_i] = ra[s][q];
      sB[buf][kb0 + q * db_k][ib0 + q * db_j] = rb[s][q];
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const double bA0 = sA[buf][kk + lk][wi + lr], bA1 = sA[buf][kk + lk][wi + 16 + lr];
      const double aB0 = sB[buf][kk + lk][wj + lr], aB1 = sB[buf][kk + lk][wj + 16 + lr];
      acc[0][0] = mfma16x16x4(aB0, bA0, acc[0][0]);
      acc[0][1] = mfma16x16x4(aB1, bA0, acc[0][1]);
      acc[1][0] = mfma16x16x4(aB0, bA1, acc[1][0]);
      acc[1][1] = mfma16x16x4(aB1, bA1, acc[1][1]);
    }
  };
  // Chunk c sits in LDS buffer c & 1 and came through register set c & 1.  The
  // fetches are unconditional (past the end every element reads as zero and is never
  // staged), so the wait before each stage always leaves the newest set in flight.
  const int nch = kb < ke ? (ke - kb + GK - 1) / GK : 0;
  if (nch > 0) {
    fetch(0, kb);
    fetch(1, kb + GK);
    stage(0, 0);
  }
  __syncthreads();
  for (int c = 0; c < nch; c += 2) {
    fetch(0, kb + (c + 2) * GK);
    compute(0);
    if (c + 1 < nch) stage(1, 1);
    __syncthreads();
    if (c + 1 >= nch) break;
    fetch(1, kb + (c + 3) * GK);
    compute(1);
    if (c + 2 < nch) stage(0, 0);
    __syncthreads();
  }
  if (g.splits > 1) {
    double* P = g.partial + ((long)b * g.splits + sp) * g.pstride;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + wi + 16 * x + lr, j = j0 + wj + 16 * y + lk + 4 * r;
          if (i < m && j < n) P[i + (long)j * g.pld] = acc[x][y][r];
        }
    return;
  }
  double* C = g.C ? g.C[b] : g.C1;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wi + 16 * x + lr, j = j0 + wj + 16 * y + lk + 4 * r;
        if (i < m && j < n) {
          double* c = C + i + (long)j * g.ldc;
          const double v = g.alpha * acc[x][y][r];
          *c = (g.beta == 0.0) ? v : v + g.beta * *c;
        }
      }
}

// C = alpha * sum_sp partial[sp] + beta * C, summed in split order (deterministic).
__global__ __launch_bounds__(256) void k_gemm_reduce(GemmArgs g) {
  const int b = blockIdx.y;
  const int m = g.m ? g.m[b] : g.m0;
  const int n = g.n ? g.n[b] : g.n0;
  double* C = g.C ? g.C[b] : g.C1;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < (long)m * n; e += (long)gridDim.x * 256) {
    const int i = (int)(e % m), j = (int)(e / m);
    // summed in split order
    const double s =
        ordered_sum(g.partial + (long)b * g.splits * g.pstride + i + (long)j * g.pld, g.pstride, g.splits);
    double* c = C + i + (long)j * g.ldc;
    const double v = g.alpha * s;
    *c = (g.beta == 0.0) ? v : v + g.beta * *c;
  }
}

void gemm_launch(GemmArgs g, int batch, int mmax, int nmax, bool ta, bool tb, hipStream_t st) {
  if (batch <= 0 || mmax <= 0 || nmax <= 0) return;
  if (g.splits < 1) g.splits = 1;
  if (g.splits > 1) {
    SL_CHECK_ARG(g.partial != nullptr, "split-K GEMM needs a partial buffer");
    g.pld = mmax;
    g.pstride = (long)mmax * nmax;
  }
  dim3 grid((unsigned)ceil_div(mmax, GT), (unsigned)ceil_div(nmax, GT), (unsigned)(batch * g.splits));
  sislice_handle* ph = current_handle();
  const int tk = prof_begin(ph, kProfGemm, st);
  if (!ta && !tb) SL_LAUNCH((k_gemm<false, false>), grid, dim3(256), 0, st, g);
  if (!ta && tb) SL_LAUNCH((k_gemm<false, true>), grid, dim3(256), 0, st, g);
  if (ta && !tb) SL_LAUNCH((k_gemm<true, false>), grid, dim3(256), 0, st, g);
  if (ta && tb) SL_LAUNCH((k_gemm<true, true>), grid, dim3(256), 0, st, g);
  SL_LAUNCH_CHECK();
  if (g.splits > 1) {
    const long tot = (long)mmax * nmax;
    SL_LAUNCH(k_gemm_reduce, dim3((unsigned)std::min<long>(ceil_div(tot, 256), 4096), batch),
                       dim3(256), 0, st, g);
    SL_LAUNCH_CHECK();
  }
  prof_end(ph, tk, st);
}

// ------------------------------------------------------------ skinny products
//
// C = alpha * M X + beta * C with M square n x n (column-major, ldm) and X n x k,
// k <= kSkinnyMaxCol.  The product is bound by reading M once from HBM (8 n^2
// bytes, halved for a triangular M), so it is written for streaming: a
// workgroup owns 64 rows and a K chunk of kSkinnyKc columns of M, each of its
// four wavefronts a quarter of the chunk; lane i of a wavefront holds row i0 + i
// and accumulates NC columns with FMA.  M is read in unconditional 8-deep
// batches of contiguous 512-byte column segments (rows past n are clamped and
// never stored); the X chunk sits in LDS (k-major, so the NC entries a step
// needs are one broadcast read).  The quarters are summed in LDS in order, the
// chunks by k_skinny_reduce in chunk order, so results are deterministic.  A
// triangular M (tri = 1 lower, 2 upper, zeros stored in the other half) skips the
// chunks that do not meet a row tile.

__device__ __forceinline__ bool skinny_chunk_live(int tri, int i0, int kc) {
  if (tri == 1) return kc <= i0 + 63;                    // lower: columns <= row
  if (tri == 2) return kc + kSkinnyKc > i0;               // upper: columns >= row
  return true;
}

template <int NC>
__global__ __launch_bounds__(256) void k_skinny_mm(int n, const double* __restrict__ M, long ldm,
                                                   int tri, const double* __restrict__ X, long ldx,
                                                   double* __restrict__ P, int pcols, int c_off) {
  constexpr int KQ = kSkinnyKc / 4;  // columns of M per wavefront
  constexpr int NCP = NC + (NC & 1);
  __shared__ double sh[(kSkinnyKc * NCP > 3 * NC * 64) ? kSkinnyKc * NCP : 3 * NC * 64];
  const int t = blockIdx.x, q = blockIdx.y;
  const int i0 = t * 64, kc = q * kSkinnyKc;
  if (!skinny_chunk_live(tri, i0, kc)) return;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  // X chunk, k-major: sh[k * NCP + c] = X(kc + k, c)
  for (int e = tid; e < kSkinnyKc * NC; e += 256) {
    const int k = e % kSkinnyKc, c = e / kSkinnyKc;
    sh[k * NCP + c] = (kc + k < n) ? X[kc + k + (long)c * ldx] : 0.0;
  }
  __syncthreads();
  const int row = i0 + l;
  const double* Mr = M + min(row, n - 1);
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0.0;
  const int kb = kc + w * KQ;
  const int ke = min(n, kb + KQ);
  int k = kb;
  for (; k + 8 <= ke; k += 8) {
    double m8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) m8[u] = Mr[(long)(k + u) * ldm];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double* xs = sh + (k - kc + u) * NCP;
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] += m8[u] * xs[c];
    }
  }
  for (; k < ke; ++k) {
    const double mv = Mr[(long)k * ldm];
    const double* xs = sh + (k - kc) * NCP;
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] += mv * xs[c];
  }
  __syncthreads();  // the X chunk is dead: reuse LDS for the quarter sums
  if (w > 0) {
#pragma unroll
    for (int c = 0; c < NC; ++c) sh[((w - 1) * NC + c) * 64 + l] = acc[c];
  }
  __syncthreads();
  if (w == 0 && row < n) {
    double* Pq = P + (long)q * n * pcols + (long)c_off * n;
#pragma unroll
    for (int c = 0; c < NC; ++c)
      Pq[row + (long)c * n] =
          ((acc[c] + sh[(0 * NC + c) * 64 + l]) + sh[(1 * NC + c) * 64 + l]) + sh[(2 * NC + c) * 64 + l];
  }
}

// MFMA form for 8..32 columns.  With the columns broadcast from LDS, the VALU form
// spends ten 16-byte LDS reads per row of M for its 20 FMAs a lane: bound by LDS.  Here
// wavefront w owns rows i0 + 16 w .. + 15 and one or two 16-column blocks of the
// output; per k-step of 4 it streams one entry of M per lane (the MFMA's A operand,
// 16 rows x 4 k) and reads one X entry per lane and block from LDS (the B operand),
// with 16 loads of M in flight.  Columns past NC read a valid column and are zeroed.
// Partial layout and chunk skipping as in k_skinny_mm.
template <int NC>
__global__ __launch_bounds__(256) void k_skinny_mfma(int n, const double* __restrict__ M, long ldm,
                                                     int tri, const double* __restrict__ X,
                                                     long ldx, double* __restrict__ P, int pcols,
                                                     int c_off) {
  constexpr int NB = (NC + 15) / 16;  // 16-column blocks
  constexpr int SP = NC | 1;          // LDS row stride (doubles), odd: conflict-free staging
  constexpr int NS = kSkinnyKc / 4;   // k-steps per chunk
  constexpr int PF = 16;              // loads of M in flight per lane
  __shared__ double sh[kSkinnyKc * SP];
  const int t = blockIdx.x, q = blockIdx.y;
  const int i0 = t * 64, kc = q * kSkinnyKc;
  if (!skinny_chunk_live(tri, i0, kc)) return;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
  // X chunk, k-major: sh[k * SP + c] = X(kc + k, c), zero past n
  for (int e = tid; e < kSkinnyKc * NC; e += 256) {
    const int k = e % kSkinnyKc, c = e / kSkinnyKc;
    sh[k * SP + c] = (kc + k < n) ? X[kc + k + (long)c * ldx] : 0.0;
  }
  __syncthreads();
  const int row = i0 + 16 * w + lr;
  const double* Mr = M + min(row, n - 1);
  // k past n reads a valid entry: its X row is zero
  auto ldm_at = [&](int s) { return Mr[(long)min(kc + 4 * s + lk, n - 1) * ldm]; };
  d4 acc[NB];
#pragma unroll
  for (int bb = 0; bb < NB; ++bb) acc[bb] = d4{0.0, 0.0, 0.0, 0.0};
  double mv[PF];
#pragma unroll
  for (int j = 0; j < PF; ++j) mv[j] = ldm_at(j);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double a = mv[s % PF];
    if (s + PF < NS) mv[s % PF] = ldm_at(s + PF);
    const double* xs = sh + (4 * s + lk) * SP;
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      const int c = 16 * bb + lr;
      const double xv = xs[c < NC ? c : 0];
      acc[bb] = mfma16x16x4(c < NC ? xv : 0.0, a, acc[bb]);
    }
  }
  // acc[bb] register r of lane l: output row i0 + 16 w + lr, column 16 bb + lk + 4 r
  if (row < n) {
    double* Pq = P + (long)q * n * pcols + (long)c_off * n;
#pragma unroll
    for (int bb = 0; bb < NB; ++bb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = 16 * bb + lk + 4 * r;
        if (c < NC) Pq[row + (long)c * n] = acc[bb][r];
      }
  }
}

__global__ __launch_bounds__(256) void k_skinny_reduce(int n, int ncol, int nchunk, int tri,
                                                       const double* __restrict__ P, double alpha,
                                                       double beta, double* __restrict__ C,
                                                       long ldc) {
  const long tot = (long)n * ncol;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < tot; e += (long)gridDim.x * 256) {
    const int i = (int)(e % n), c = (int)(e / n);
    const int i0 = (i / 64) * 64;
    const double* Pe = P + i + (long)c * n;
    // summed in chunk order over the live chunks; eight loads issued at a time (a dead
    // chunk's partial is read but not added)
    double s = 0.0;
    int q = 0;
    for (; q + 8 <= nchunk; q += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = Pe[(long)(q + u) * tot];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (skinny_chunk_live(tri, i0, (q + u) * kSkinnyKc)) s += v[u];
    }
    for (; q < nchunk; ++q)
      if (skinny_chunk_live(tri, i0, q * kSkinnyKc)) s += Pe[(long)q * tot];
    double* cp = C + i + (long)c * ldc;
    const double v = alpha * s;
    *cp = (beta == 0.0) ? v : v + beta * *cp;
  }
}

template <int NC>
static void skinny_part(int n, const double* M, long ldm, int tri, const double* X, long ldx,
                        double* partial, int pcols, int c_off, hipStream_t st) {
  const int nchunk = (int)ceil_div(n, kSkinnyKc);
  if constexpr (NC >= 8)
    SL_LAUNCH((k_skinny_mfma<NC>), dim3((unsigned)ceil_div(n, 64), nchunk), dim3(256), 0, st, n,
              M, ldm, tri, X + (long)c_off * ldx, ldx, partial, pcols, c_off);
  else
    SL_LAUNCH((k_skinny_mm<NC>), dim3((unsigned)ceil_div(n, 64), nchunk), dim3(256), 0, st, n, M,
              ldm, tri, X + (long)c_off * ldx, ldx, partial, pcols, c_off);
  SL_LAUNCH_CHECK();
}

void skinny_launch(int n, int ncol, const double* M, long ldm, int tri, const double* X, long ldx,
                   double alpha, double beta, double* C, long ldc, double* partial,
                   hipStream_t st) {
  if (n <= 0 || ncol <= 0) return;
  SL_CHECK_ARG(ncol <= kSkinnyMaxCol, "skinny product: too many columns");
  sislice_handle* ph = current_handle();
  const int tk = prof_begin(ph, kProfGemm, st);
  // column pieces of instantiated widths (each piece streams M once)
  int c0 = 0;
  while (c0 < ncol) {
    const int r = ncol - c0;
    int wdt;
    if (r >= 32) { skinny_part<32>(n, M, ldm, tri, X, ldx, partial, ncol, c0, st); wdt = 32; }
    else if (r >= 24) { skinny_part<24>(n, M, ldm, tri, X, ldx, partial, ncol, c0, st); wdt = 24; }
    else if (r >= 20) { skinny_part<20>(n, M, ldm, tri, X, ldx, partial, ncol, c0, st); wdt = 20; }
    else if (r >= 16) { skinny_part<16>(n, M, ldm, tri, X, ldx, partial, ncol, c0, st); wdt = 16; }
    else if (r >= 8) { skinny_part<8>(n, M, ldm, tri, X, ldx, partial, ncol, c0, st); wdt = 8; }
    else if (r >= 4) { skinny_part<4>(n, M, ldm, tri, X, ldx, partial, ncol, c0, st); wdt = 4; }
    else if (r >= 2) { skinny_part<2>(n, M, ldm, tri, X, ldx, partial, ncol, c0, st); wdt = 2; }
    else { skinny_part<1>(n, M, ldm, tri, X, ldx, partial, ncol, c0, st); wdt = 1; }
    c0 += wdt;
  }
  const int nchunk = (int)ceil_div(n, kSkinnyKc);
  const long tot = (long)n * ncol;
  SL_LAUNCH(k_skinny_reduce, dim3((unsigned)std::min<long>(ceil_div(tot, 256), 4096)), dim3(256),
            0, st, n, ncol, nchunk, tri, partial, alpha, beta, C, ldc);
  SL_LAUNCH_CHECK();
  prof_end(ph, tk, st);
}

// ------------------------------------------------- tall-skinny products, 8 columns
//
// The Lanczos block is 8 columns wide, so the reorthogonalisation and CholeskyQR
// products are (n x m)^T (n x 8) and (n x m) (m x 8) with n >> m: bound by
// reading the n x m basis once.  The generic 64x64-tile GEMM spends 8x its work on
// padding here; these kernels stream the basis instead.
//
// k_tsmt: C_b = V_b^T X_b (m_b x 8).  A workgroup takes kTsRows rows of one batch
// entry and 64 columns of V, stages 64-row slices of V through LDS (coalesced
// along the rows) and accumulates 8 dot products per column in four row phases;
// per-chunk partials are summed in chunk order by k_tsmt_reduce.
__global__ __launch_bounds__(256) void k_tsmt(TsArgs a) {
  __shared__ double sV[64][65];
  __shared__ double sX[kTsRows][8];
  const int b = blockIdx.z, q = blockIdx.x;
  const int m = a.m[b];
  const int i0 = blockIdx.y * 64;
  if (i0 >= m) return;
  const int n = a.n, r0 = q * kTsRows;
  const double* V = a.V[b];
  const double* X = a.X[b];
  const int tid = threadIdx.x;
  // loads from clamped indices, issued unconditionally through the global address space
  // (flat loads would also wait on the LDS counter), zeroed where they lie outside
  typedef __attribute__((address_space(1))) const double gcd;
  const gcd* Xg = (const gcd*)X;
  const gcd* Vg = (const gcd*)V;
  // the X slice: every load issued before any store (a rolled load / wait / store loop
  // made one memory round trip per element a thread stages)
  constexpr int XE = kTsRows * 8 / 256;
  double xv[XE];
#pragma unroll
  for (int u = 0; u < XE; ++u) {
    const int e = tid + 256 * u, r = e % kTsRows, c = e / kTsRows;
    xv[u] = Xg[min(r0 + r, n - 1) + (long)c * a.ldx];
  }
  const int i = tid & 63, rg = tid >> 6;
  double acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = 0.0;
  // the 64x64 block of the next stage is loaded into registers while the current
  // one is consumed: element e = tid + 256 j -> (row e & 63, column e >> 6)
  double vn[16];
  auto load_v = [&](int st) {
    const int rs = r0 + 64 * st;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int e = tid + 256 * j, r = e & 63, ii = e >> 6;
      vn[j] = Vg[min(rs + r, n - 1) + (long)min(i0 + ii, m - 1) * a.ldv];
    }
  };
  load_v(0);
#pragma unroll
  for (int u = 0; u < XE; ++u) {
    const int e = tid + 256 * u, r = e % kTsRows, c = e / kTsRows;
    sX[r][c] = (r0 + r < n) ? xv[u] : 0.0;
  }
  for (int st = 0; st < kTsRows / 64; ++st) {
    __syncthreads();
    const int rs = r0 + 64 * st;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int e = tid + 256 * j, r = e & 63, ii = e >> 6;
      sV[r][ii] = ((rs + r < n) & (i0 + ii < m)) ? vn[j] : 0.0;
    }
    if (st + 1 < kTsRows / 64) load_v(st + 1);
    __syncthreads();
    for (int rr = rg; rr < 64; rr += 4) {
      const double v = sV[rr][i];
      const double* xr = sX[64 * st + rr];
#pragma unroll
      for (int c = 0; c < 8; ++c) acc[c] += v * xr[c];
    }
  }
  __syncthreads();
  double* red = &sV[0][0];  // [3][64][8]
  if (rg > 0) {
#pragma unroll
    for (int c = 0; c < 8; ++c) red[((rg - 1) * 64 + i) * 8 + c] = acc[c];
  }
  __syncthreads();
  if (rg == 0 && i0 + i < m) {
    double* P = a.partial + (((long)b * a.nchunk + q) * a.mmax + (i0 + i)) * 8;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      P[c] = ((acc[c] + red[(0 * 64 + i) * 8 + c]) + red[(1 * 64 + i) * 8 + c]) + red[(2 * 64 + i) * 8 + c];
  }
}

__global__ __launch_bounds__(256) void k_tsmt_reduce(TsArgs a) {
  const int b = blockIdx.y;
  const int m = a.m[b];
  double* C = a.C[b];
  for (int e = blockIdx.x * 256 + threadIdx.x; e < m * 8; e += gridDim.x * 256) {
    const int i = e >> 3, c = e & 7;
    const double s = ordered_sum(a.partial + ((long)b * a.nchunk * a.mmax + i) * 8 + c, (long)a.mmax * 8, a.nchunk);
    const long ldc = a.ldcb ? a.ldcb[b] : a.ldc;
    C[i + (long)c * ldc] = a.alpha * s;
  }
}

void tsmt_launch(TsArgs a, int batch, int mmax, hipStream_t st) {
  if (batch <= 0 || mmax <= 0) return;
  a.mmax = mmax;
  a.nchunk = (int)ceil_div(a.n, kTsRows);
  sislice_handle* ph = current_handle();
  const int tk = prof_begin(ph, kProfGemm, st);
  SL_LAUNCH(k_tsmt, dim3(a.nchunk, (unsigned)ceil_div(mmax, 64), batch), dim3(256), 0, st, a);
  SL_LAUNCH_CHECK();
  SL_LAUNCH(k_tsmt_reduce, dim3((unsigned)ceil_div(mmax * 8, 256), batch), dim3(256), 0, st, a);
  SL_LAUNCH_CHECK();
  prof_end(ph, tk, st);
}

// k_tsmm: Y_b = beta Y_b + alpha (V_b C_b + V2_b C2_b), n x 8.  The coefficients
// sit in LDS.  Four consecutive lanes share a row and split the columns of V
// (lane g takes k = g mod 4, for all eight outputs), so a wavefront reads 16 rows
// of four different columns per load (four 128-byte segments, none repeated) and
// the four partial sums of a row meet through lane shuffles.
// Coefficient rows sit kTsmmLd = 9 doubles apart: the four rows a quarter-wave reads
// at once (k = g mod 4) then fall in different banks, as do the staging stores.
constexpr int kTsmmLd = 9;
__global__ __launch_bounds__(256) void k_tsmm(TsArgs a) {
  extern __shared__ double sC[];  // [m1 + m2][kTsmmLd]
  const int b = blockIdx.y, tid = threadIdx.x;
  const int m1 = a.m[b], m2 = a.m2 ? a.m2[b] : 0;
  const double* C1 = a.C[b];
  for (int e = tid; e < m1 * 8; e += 256) {
    const int k = e % m1, c = e / m1;
    sC[k * kTsmmLd + c] = C1[k + (long)c * a.ldc];
  }
  if (m2 > 0) {
    const double* C2 = a.C2[b];
    for (int e = tid; e < m2 * 8; e += 256) {
      const int k = e % m2, c = e / m2;
      sC[(m1 + k) * kTsmmLd + c] = C2[k + (long)c * a.ldc2];
    }
  }
  __syncthreads();
  const int n = a.n;
  const int row = blockIdx.x * 64 + (tid >> 2), g = tid & 3;
  const bool rv = row < n;
  const int rc = rv ? row : n - 1;
  double acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = 0.0;
  auto run = [&](const double* Vb, long ldv, const double* sCb, int mb) {
    int k = g;
    for (; k + 12 < mb; k += 16) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = Vb[(long)(k + 4 * u) * ldv];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double* cr = sCb + (k + 4 * u) * kTsmmLd;
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] += v[u] * cr[c];
      }
    }
    for (; k < mb; k += 4) {
      const double v = Vb[(long)k * ldv];
      const double* cr = sCb + k * kTsmmLd;
#pragma unroll
      for (int c = 0; c < 8; ++c) acc[c] += v * cr[c];
    }
  };
  run(a.V[b] + rc, a.ldv, sC, m1);
  if (m2 > 0) run(a.V2[b] + rc, a.ldv2, sC + m1 * kTsmmLd, m2);
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    acc[c] += __shfl_xor(acc[c], 1);
    acc[c] += __shfl_xor(acc[c], 2);
  }
  double acc0 = acc[0], acc1 = acc[1];
#pragma unroll
  for (int q = 1; q < 4; ++q) {
    acc0 = (g == q) ? acc[2 * q] : acc0;
    acc1 = (g == q) ? acc[2 * q + 1] : acc1;
  }
  if (rv) {
    double* Y = a.Y[b] + row;
    double* y0 = Y + (long)(2 * g) * a.ldy;
    double* y1 = Y + (long)(2 * g + 1) * a.ldy;
    *y0 = (a.beta == 0.0) ? a.alpha * acc0 : a.beta * *y0 + a.alpha * acc0;
    *y1 = (a.beta == 0.0) ? a.alpha * acc1 : a.beta * *y1 + a.alpha * acc1;
  }
}

void tsmm_launch(TsArgs a, int batch, int mtot_max, hipStream_t st) {
  if (batch <= 0) return;
  const size_t lds = (size_t)std::max(mtot_max, 1) * kTsmmLd * sizeof(double);
  SL_CHECK_ARG(lds <= kTsmmMaxLds, "tall-skinny product: too many basis columns");
  static std::once_flag attr;
  std::call_once(attr, [] {
    SL_HIP(hipFuncSetAttribute((const void*)k_tsmm, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kTsmmMaxLds));
  });
  sislice_handle* ph = current_handle();
  const int tk = prof_begin(ph, kProfGemm, st);
  SL_LAUNCH(k_tsmm, dim3((unsigned)ceil_div(a.n, 64), batch), dim3(256), lds, st, a);
  SL_LAUNCH_CHECK();
  prof_end(ph, tk, st);
}

// out = f1 * X + f2 * Y + f3 * Z elementwise over n x ncol blocks (ld n); Z may
// be null (f3 ignored).
__global__ __launch_bounds__(256) void k_lincomb3(long tot, double f1, const double* __restrict__ X,
                                                  double f2, const double* __restrict__ Y,
                                                  double f3, const double* __restrict__ Z,
                                                  double* __restrict__ out) {
  for (long e = blockIdx.x * 256L + threadIdx.x; e < tot; e += (long)gridDim.x * 256) {
    double v = f1 * X[e] + f2 * Y[e];
    if (Z) v += f3 * Z[e];
    out[e] = v;
  }
}

void lincomb3_launch(long tot, double f1, const double* X, double f2, const double* Y, double f3,
                     const double* Z, double* out, hipStream_t st) {
  if (tot <= 0) return;
  SL_LAUNCH(k_lincomb3, dim3((unsigned)std::min<long>(ceil_div(tot, 256), 4096)), dim3(256), 0, st,
            tot, f1, X, f2, Y, f3, Z, out);
  SL_LAUNCH_CHECK();
}

// y = x / sqrt(s2[0]) (a zero norm gives y = 0), and rec[0] = sqrt(s2[0]) when rec
// is non-null: normalisation by a norm that stays on the device.
__global__ __launch_bounds__(256) void k_scale_by_norm(int n, const double* __restrict__ s2,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y,
                                                       double* __restrict__ rec) {
  const double nr = sqrt(fmax(s2[0], 0.0));
  const double f = nr > 0.0 ? 1.0 / nr : 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) y[i] = x[i] * f;
  if (rec && blockIdx.x == 0 && threadIdx.x == 0) rec[0] = nr;
}

void scale_by_norm_launch(int n, const double* s2, const double* x, double* y, double* rec,
                          hipStream_t st) {
  SL_LAUNCH(k_scale_by_norm, dim3((unsigned)std::min<long>(ceil_div(n, 256), 1024)), dim3(256), 0,
            st, n, s2, x, y, rec);
  SL_LAUNCH_CHECK();
}

// ------------------------------------------------ single-vector Lanczos step tail
//
// After w = H v_j, one step of the single-vector Lanczos run that bounds the spectrum
// ends with alpha_j = v_j^T w, two classical Gram-Schmidt passes of w against
// V[:, 0..j], beta_j = ||w|| and v_{j+1} = w / beta_j.  V has at most 61 columns and
// stays in L2, so one 1024-thread workgroup does all of it in one launch: eleven short
// launches before, whose gaps cost more than their work.  Every sum is taken in a
// fixed order (a lane's rows in order, the wavefront's butterfly, the sixteen
// wavefronts in order), so the result is deterministic.
__device__ __forceinline__ double lt_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ __launch_bounds__(1024) void k_lanczos_tail(int n, int j, double* __restrict__ V,
                                                       double* __restrict__ wv,
                                                       double* __restrict__ alpha,
                                                       double* __restrict__ s2,
                                                       double* __restrict__ beta) {
  extern __shared__ double sw[];  // w of the pass, n doubles
  __shared__ double coef[kLanczosTailMaxCols];
  __shared__ double red[16];
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
  const int nc = j + 1;
  auto block_sum = [&](double v) -> double {  // every thread gets the sum
    v = lt_wave_sum(v);
    __syncthreads();
    if (l == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += red[q];
    return t;
  };
  {
    const double* vj = V + (long)j * n;
    double s = 0.0;
    for (int r = tid; r < n; r += 1024) s += vj[r] * wv[r];
    const double a = block_sum(s);
    if (tid == 0) alpha[j] = a;
  }
  for (int pass = 0; pass < 2; ++pass) {
    for (int r = tid; r < n; r += 1024) sw[r] = wv[r];
    __syncthreads();
    // coef_i = V[:, i]^T w: wavefront i mod 16 takes column i; eight loads of the
    // column in flight per lane, into eight partial sums added in order
    for (int i = wave; i < nc; i += 16) {
      const double* vi = V + (long)i * n;
      double p8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int r = l;
      for (; r + 7 * 64 < n; r += 8 * 64) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = vi[r + 64 * u];
#pragma unroll
        for (int u = 0; u < 8; ++u) p8[u] += x[u] * sw[r + 64 * u];
      }
      for (int u = 0; r < n; r += 64, ++u) p8[u] += vi[r] * sw[r];
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) s += p8[u];
      s = lt_wave_sum(s);
      if (l == 0) coef[i] = s;
    }
    __syncthreads();
    // w -= V coef (a thread's rows only), eight columns' loads in flight
    for (int r = tid; r < n; r += 1024) {
      double acc = 0.0;
      int i = 0;
      for (; i + 8 <= nc; i += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = V[r + (long)(i + u) * n];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += x[u] * coef[i + u];
      }
      for (; i < nc; ++i) acc += V[r + (long)i * n] * coef[i];
      wv[r] = sw[r] - acc;
    }
    __syncthreads();
  }
  double s = 0.0;
  for (int r = tid; r < n; r += 1024) s += wv[r] * wv[r];
  const double t = block_sum(s);
  const double nr = sqrt(fmax(t, 0.0));
  const double f = nr > 0.0 ? 1.0 / nr : 0.0;
  double* vn = V + (long)(j + 1) * n;
  for (int r = tid; r < n; r += 1024) vn[r] = wv[r] * f;
  if (tid == 0) {
    s2[j] = t;
    beta[j] = nr;
  }
}

void lanczos_tail_launch(int n, int j, double* V, double* w, double* alpha, double* s2,
                         double* beta, hipStream_t st) {
  static std::once_flag attr;
  std::call_once(attr, [] {
    SL_HIP(hipFuncSetAttribute((const void*)k_lanczos_tail,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kLanczosTailMaxN * sizeof(double))));
  });
  SL_CHECK_ARG(n >= 1 && n <= kLanczosTailMaxN, "Lanczos step tail: order out of range");
  SL_CHECK_ARG(j >= 0 && j + 1 <= kLanczosTailMaxCols, "Lanczos step tail: too many columns");
  SL_LAUNCH(k_lanczos_tail, dim3(1), dim3(1024), (size_t)n * sizeof(double), st, n, j, V, w,
            alpha, s2, beta);
  SL_LAUNCH_CHECK();
}

// Y[:, c] = X[:, c] / sqrt(s2[c]) for ncol columns (zero when s2 <= 0), rec[c] = sqrt(s2[c]).
__global__ __launch_bounds__(256) void k_scale_cols(int n, const double* __restrict__ s2,
                                                    const double* __restrict__ X, long ldx,
                                                    double* __restrict__ Y, long ldy,
                                                    double* __restrict__ rec) {
  const int c = blockIdx.y;
  const double nr = sqrt(fmax(s2[c], 0.0));
  const double f = nr > 0.0 ? 1.0 / nr : 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
    Y[i + (long)c * ldy] = X[i + (long)c * ldx] * f;
  if (rec && blockIdx.x == 0 && threadIdx.x == 0) rec[c] = nr;
}

void scale_cols_launch(int n, int ncol, const double* s2, const double* X, long ldx, double* Y,
                       long ldy, double* rec, hipStream_t st) {
  if (n <= 0 || ncol <= 0) return;
  SL_LAUNCH(k_scale_cols, dim3((unsigned)std::min<long>(ceil_div(n, 256), 64), ncol), dim3(256), 0,
            st, n, s2, X, ldx, Y, ldy, rec);
  SL_LAUNCH_CHECK();
}

// Out-of-place transpose T = S^T of an n x n matrix, 32 x 32 tiles through LDS.
__global__ __launch_bounds__(256) void k_transpose(int n, const double* __restrict__ S, long lds,
                                                   double* __restrict__ T, long ldt) {
  __shared__ double t[32][33];
  const int bi = blockIdx.x, bj = blockIdx.y;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < 32; yy += 8) {
    const int i = bi * 32 + tx, j = bj * 32 + yy;
    t[yy][tx] = (i < n && j < n) ? S[i + (long)j * lds] : 0.0;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int i = bj * 32 + tx, j = bi * 32 + yy;
    if (i < n && j < n) T[i + (long)j * ldt] = t[tx][yy];
  }
}

void transpose_launch(int n, const double* S, long lds, double* T, long ldt, hipStream_t st) {
  const unsigned G = (unsigned)ceil_div(n, 32);
  SL_LAUNCH(k_transpose, dim3(G, G), dim3(256), 0, st, n, S, lds, T, ldt);
  SL_LAUNCH_CHECK();
}

// F (n x n, ldf) = symmetric completion of the lower triangle of S (lds), tiled
// through LDS so both the read and the mirrored write are coalesced.
__global__ __launch_bounds__(256) void k_sym_full(int n, const double* __restrict__ S, long lds,
                                                  double* __restrict__ F, long ldf) {
  __shared__ double t[32][33];
  const int bi = blockIdx.x, bj = blockIdx.y;
  if (bi < bj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    const int i = bi * 32 + tx, j = bj * 32 + yy;
    double v = 0.0;
    if (i < n && j < n) {
      v = (i >= j) ? S[i + (long)j * lds] : S[j + (long)i * lds];
      F[i + (long)j * ldf] = v;
    }
    t[yy][tx] = v;
  }
  __syncthreads();
  if (bi == bj) return;
  for (int yy = ty; yy < 32; yy += 8) {
    const int i = bj * 32 + tx, j = bi * 32 + yy;  // mirrored tile
    if (i < n && j < n) F[i + (long)j * ldf] = t[tx][yy];
  }
}

void sym_full_launch(int n, const double* S, long lds, double* F, long ldf, hipStream_t st) {
  const unsigned T = (unsigned)ceil_div(n, 32);
  SL_LAUNCH(k_sym_full, dim3(T, T), dim3(256), 0, st, n, S, lds, F, ldf);
  SL_LAUNCH_CHECK();
}

// Column dots: out[b][c] = sum_i X[i,c] * Y[i,c] (or ||X[:,c] - w_c Y[:,c]||^2 when
// mode == 1), per batch, two-level deterministic reduction.
__global__ __launch_bounds__(256) void k_coldot_partial(ColDotArgs a) {
  const int b = blockIdx.z, c = blockIdx.y, chunk = blockIdx.x;
  const int nc = a.ncol ? a.ncol[b] : a.ncol0;
  if (c >= nc) return;
  const double* X = (a.X ? a.X[b] : a.x1) + (long)c * a.ldx;
  const double* Y = (a.Y ? a.Y[b] : a.y1) + (long)c * a.ldy;
  const double w = (a.mode == 1) ? (a.w ? a.w[b] : a.w1)[c] : 0.0;
  const int r0 = chunk * kDotChunk, r1 = min(a.n, r0 + kDotChunk);
  double s = 0.0;
  for (int i = r0 + threadIdx.x; i < r1; i += 256) {
    if (a.mode == 0) {
      s += X[i] * Y[i];
    } else {
      const double d = X[i] - w * Y[i];
      s += d * d;
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[((long)b * a.maxcol + c) * a.nchunk + chunk] = red[0];
}

__global__ __launch_bounds__(256) void k_coldot_reduce(ColDotArgs a) {
  const int b = blockIdx.x;
  const int nc = a.ncol ? a.ncol[b] : a.ncol0;
  for (int c = threadIdx.x; c < nc; c += 256) {
    const double s = ordered_sum(a.partial + ((long)b * a.maxcol + c) * a.nchunk, 1, a.nchunk);
    (a.out ? a.out[b] : a.out1)[c] = (a.mode == 1) ? sqrt(s) : s;
  }
}

void coldot_launch(ColDotArgs a, int batch, int maxcol, hipStream_t st) {
  a.maxcol = maxcol;
  a.nchunk = (int)ceil_div(a.n, kDotChunk);
  SL_LAUNCH(k_coldot_partial, dim3(a.nchunk, maxcol, batch), dim3(256), 0, st, a);
  SL_LAUNCH_CHECK();
  SL_LAUNCH(k_coldot_reduce, dim3(batch), dim3(256), 0, st, a);
  SL_LAUNCH_CHECK();
}

// Gaussian block from the SplitMix64 stream: entry (i, c) uses stream index
// c * n + i, Box-Muller on outputs 2k and 2k+1 (the library's shared definition).
__device__ __forceinline__ unsigned long long smix(unsigned long long seed, unsigned long long i) {
  unsigned long long z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_gauss_block(int n, int ncol, const unsigned long long* seeds,
                                                     double* const* X, long ldx) {
  const int b = blockIdx.y;
  const unsigned long long sd = seeds[b];
  double* x = X[b];
  for (long e = blockIdx.x * 256L + threadIdx.x; e < (long)n * ncol; e += (long)gridDim.x * 256) {
    const int i = (int)(e % n), c = (int)(e / n);
    const unsigned long long k = (unsigned long long)c * n + i;
    const double u1 = (double)(smix(sd, 2 * k) >> 11) * 0x1.0p-53;
    const double u2 = (double)(smix(sd, 2 * k + 1) >> 11) * 0x1.0p-53;
    x[i + (long)c * ldx] = sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586 * u2);
  }
}

__global__ __launch_bounds__(256) void k_rademacher_block(int n, int ncol, unsigned long long seed,
                                                          double* X, long ldx) {
  for (long e = blockIdx.x * 256L + threadIdx.x; e < (long)n * ncol; e += (long)gridDim.x * 256) {
    const int i = (int)(e % n), c = (int)(e / n);
    const unsigned long long v = smix(seed, (unsigned long long)c * n + i);
    X[i + (long)c * ldx] = (v >> 63) ? -1.0 : 1.0;
  }
}

void gauss_launch(int n, int ncol, int batch, const unsigned long long* d_seeds, double* const* X,
                  long ldx, hipStream_t st) {
  const long tot = (long)n * ncol;
  SL_LAUNCH(k_gauss_block, dim3((unsigned)std::min<long>(ceil_div(tot, 256), 2048), batch),
                     dim3(256), 0, st, n, ncol, d_seeds, X, ldx);
  SL_LAUNCH_CHECK();
}

void rademacher_launch(int n, int ncol, unsigned long long seed, double* X, long ldx,
                       hipStream_t st) {
  const long tot = (long)n * ncol;
  SL_LAUNCH(k_rademacher_block, dim3((unsigned)std::min<long>(ceil_div(tot, 256), 2048)),
                     dim3(256), 0, st, n, ncol, seed, X, ldx);
  SL_LAUNCH_CHECK();
}

}  // namespace sislice
