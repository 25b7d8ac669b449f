// Host-side helpers shared by the drivers: the pinned upload ring for per-launch
// kernel tables and a batched GEMM front end.
#pragma once

#include <chrono>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "blas.hpp"
#include "handle.hpp"
#include "kernels.hpp"

namespace sislice {

using Clock = std::chrono::steady_clock;
inline double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// Pinned host ring + device ring for the small per-launch tables.  put() only
// stages a table in the host ring; the tables staged since the last launch go
// to the device in one copy, issued by the launch macro just before the next
// kernel (stream order then delivers them first).  The host bytes stay untouched
// until the stream has passed that copy: the ring is rewound only after a
// stream synchronisation.
// Rings nest (a driver that calls the planner): both use the handle's one ring
// memory, so a nested ring first uploads the outer one's staged tables, waits
// for the stream and rewinds the outer ring (whose earlier tables have all been
// consumed then); when the nested ring ends it uploads its own, waits again and
// hands the launch hook back to the outer ring.
class Ring {
 public:
  explicit Ring(sislice_handle* h, size_t cap = 16u << 20) : h_(h), cap_(cap) {
    if (h->flush_fn == &Ring::flush_thunk && h->flush_ctx) {
      outer_ = static_cast<Ring*>(h->flush_ctx);
      outer_->flush();
      SL_HIP(hipStreamSynchronize(h->stream));
      outer_->off_ = outer_->pend_ = 0;
      outer_->seen_.clear();
    }
    if (h->ring_cap < cap) {
      if (h->ring_host) {
        SL_HIP(hipStreamSynchronize(h->stream));
        SL_HIP(hipHostFree(h->ring_host));
        h->ring_host = nullptr;
        h->ring_cap = 0;
      }
      SL_HIP(hipHostMalloc(&h->ring_host, cap, hipHostMallocDefault));
      h->ring_cap = cap;
    }
    host_ = static_cast<char*>(h->ring_host);
    dev_ = static_cast<char*>(ws_get(h, kBufRing, cap));
    h->flush_fn = &Ring::flush_thunk;
    h->flush_ctx = this;
  }
  ~Ring() {
    if (h_->flush_ctx == this) {
      try {
        flush();
        if (outer_) (void)hipStreamSynchronize(h_->stream);
      } catch (...) {
      }
      h_->flush_fn = outer_ ? &Ring::flush_thunk : nullptr;
      h_->flush_ctx = outer_;
    }
  }
  Ring(const Ring&) = delete;
  Ring& operator=(const Ring&) = delete;
  // A table identical to one staged since the last rewind is not staged again: the
  // device copy at that offset is not overwritten before the next rewind, so the
  // launch reads it from there, and a launch whose tables all repeat needs no upload.
  void* put(const void* src, size_t bytes) {
    if (bytes == 0) bytes = 8;
    const size_t b = (bytes + 255) & ~size_t(255);
    SL_CHECK_ARG(b <= cap_, "table too large for the upload ring");
    uint64_t key = 0;
    if (src) {
      key = 1469598103934665603ull ^ bytes;  // FNV-1a over the bytes
      const unsigned char* c = static_cast<const unsigned char*>(src);
      for (size_t i = 0; i < bytes; ++i) key = (key ^ c[i]) * 1099511628211ull;
      auto it = seen_.find(key);
      if (it != seen_.end() && it->second.second == bytes &&
          std::memcmp(host_ + it->second.first, src, bytes) == 0)
        return dev_ + it->second.first;
    }
    if (off_ + b > cap_) {
      flush();
      SL_HIP(hipStreamSynchronize(h_->stream));
      off_ = pend_ = 0;
      seen_.clear();
    }
    if (src)
      std::memcpy(host_ + off_, src, bytes);
    else
      std::memset(host_ + off_, 0, bytes);
    if (src) seen_[key] = {off_, bytes};
    void* r = dev_ + off_;
    off_ += b;
    return r;
  }
  void flush() {
    if (off_ > pend_) {
      SL_HIP(hipMemcpyAsync(dev_ + pend_, host_ + pend_, off_ - pend_, hipMemcpyHostToDevice,
                            h_->stream));
      pend_ = off_;
    }
  }
  template <class T>
  T* vec(const std::vector<T>& v) {
    return static_cast<T*>(put(v.empty() ? nullptr : v.data(), v.size() * sizeof(T)));
  }
  template <class T>
  T* const* ptrs(const std::vector<T*>& v) {
    return reinterpret_cast<T* const*>(put(v.empty() ? nullptr : v.data(), v.size() * sizeof(T*)));
  }
  template <class T>
  const T* const* cptrs(const std::vector<T*>& v) {
    return reinterpret_cast<const T* const*>(
        put(v.empty() ? nullptr : v.data(), v.size() * sizeof(T*)));
  }
  // caller has synchronised the stream: every uploaded table has been consumed;
  // tables still staged are uploaded (and waited for) before the ring rewinds
  void synced() {
    if (off_ > pend_) {
      flush();
      SL_HIP(hipStreamSynchronize(h_->stream));
    }
    off_ = pend_ = 0;
    seen_.clear();
  }

 private:
  static void flush_thunk(void* self) { static_cast<Ring*>(self)->flush(); }
  sislice_handle* h_;
  Ring* outer_ = nullptr;
  size_t cap_;
  char* host_;
  char* dev_;
  size_t off_ = 0;
  size_t pend_ = 0;
  std::unordered_map<uint64_t, std::pair<size_t, size_t>> seen_;  // key -> (offset, bytes)
};

struct Ctx {
  sislice_handle* h;
  hipStream_t st;
  Ring* ring;
};

// A device allocation owned by one call, for rare paths that need memory beyond
// the handle's workspaces (hipFree waits for the device before releasing it).
struct DevBuf {
  void* p = nullptr;
  void alloc(size_t bytes) {
    release();
    if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
      p = nullptr;
      throw Error(SISLICE_ERR_ALLOC, "device allocation failed");
    }
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
  }
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
};

// Batched GEMM helper: per-batch sizes, pointer tables through the ring (a batch of
// one passes its sizes and operands in the arguments instead), split-K (ordered
// partials) when the reduction is long and the output small.
inline void gemm(Ctx& c, bool ta, bool tb, const std::vector<int>& m, const std::vector<int>& nn,
          const std::vector<int>& k, const std::vector<const double*>& A, long lda,
          const std::vector<const double*>& B, long ldb, const std::vector<double*>& C, long ldc,
          double alpha, double beta) {
  const int batch = (int)m.size();
  if (batch == 0) return;
  int mmax = 0, nmax = 0, kmax = 0;
  for (int b = 0; b < batch; ++b) {
    mmax = std::max(mmax, m[b]);
    nmax = std::max(nmax, nn[b]);
    kmax = std::max(kmax, k[b]);
  }
  if (mmax == 0 || nmax == 0) return;
  GemmArgs g;
  if (batch == 1) {
    g.m0 = m[0];
    g.n0 = nn[0];
    g.k0 = k[0];
    g.A1 = A[0];
    g.B1 = B[0];
    g.C1 = C[0];
  } else {
    g.m = c.ring->vec(m);
    g.n = c.ring->vec(nn);
    g.k = c.ring->vec(k);
    g.A = c.ring->cptrs(A);
    g.B = c.ring->cptrs(B);
    g.C = c.ring->ptrs(C);
  }
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.alpha = alpha;
  g.beta = beta;
  int splits = 1;
  const long tiles = ceil_div(mmax, 64) * ceil_div(nmax, 64) * (long)batch;
  if (kmax >= 1024 && tiles < 512) {
    // splits at least 256 deep; 64 deep (four K chunks) for outputs of a few tiles,
    // the Gram-type products V^T w of the reorthogonalisations
    splits = (int)std::min<long>(std::max<long>(1, 1024 / tiles), kmax / (tiles < 16 ? 64 : 256));
    splits = std::max(1, std::min(splits, 64));
  }
  g.splits = splits;
  if (splits > 1)
    g.partial = static_cast<double*>(
        ws_get(c.h, kBufMisc, sizeof(double) * (size_t)batch * splits * mmax * nmax));
  gemm_launch(g, batch, mmax, nmax, ta, tb, c.st);
}

// Driver workspace of one pencil: full copies of A and B (adjacent: [A B] is an
// n x 2n matrix with leading dimension n), the factorizations of
// A - pts[s] B (LD, ipiv) with room for their solve preparation (perm, blk,
// Linv), and small scratch.  driver_factor carves it, factors every point in
// lock step, reads the inertias (synchronising) and, when no pivot is an exact
// zero, records the factorizations in the handle's cache (h->fc.id != 0).
struct DriverWs {
  double* Af = nullptr;
  double* Bf = nullptr;
  std::vector<double*> LD;
  std::vector<int32_t*> ipv;
  std::vector<int*> perm, blk;
  std::vector<double*> Linv;
  double* nsmall = nullptr;
  double* nX = nullptr;
  int* nflag = nullptr;
  FactorPlan fp;
  std::vector<int64_t> inert;
};
DriverWs driver_factor(sislice_handle* h, Ring& ring, int n, const double* A, long lda,
                       const double* B, long ldb, const std::vector<double>& pts, int nb);

// The shift planners and the plain per-pencil path (argument checks done by the
// entry points).  plan_impl runs the KPM planner, or with dos_mode 0 / 1 the
// paper's Lanczos DOS planner (dos_nv runs of dos_k steps; equal-count roots or
// DOSCluster).  solve_impl's optional `start` (device n x 8 n_s, ld n) gives
// each probe's Lanczos start block (warm start) instead of a Gaussian one (with
// the subspace-iteration driver, opts.driver == 1: n x start_cols per probe, the
// leading columns of its start basis), and `probe_of` (host int32[n_e]) receives
// the probe that validated each returned eigenpair.
sislice_status plan_impl(sislice_handle* h, int64_t n64, const double* A, int64_t lda,
                         const double* B, int64_t ldb, int64_t n_e, int64_t n_s,
                         const sislice_opts& o, double* sig, double* top, double* mom_out,
                         double* bounds_out, int dos_mode = -1, int dos_k = 0, int dos_nv = 0);
sislice_status solve_impl(sislice_handle* h, int64_t n64, const double* A, int64_t lda,
                          const double* B, int64_t ldb, int64_t n_e, int64_t n_s,
                          const double* sigmas_in, double* omega_top_io, const sislice_opts& o,
                          double* evals, double* evecs, int64_t ldx, double* resid_out,
                          sislice_report* rep, const double* start = nullptr,
                          int32_t* probe_of = nullptr, int start_cols = 8);
void check_opts(const sislice_opts& o);

}  // namespace sislice
