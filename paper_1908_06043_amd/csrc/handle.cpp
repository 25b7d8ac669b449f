// Handle lifecycle, workspaces, status strings and the factorization entry points.
#include "handle.hpp"

#include <algorithm>
#include <cstring>
#include <string>

#include "factor_api.hpp"
#include "kernels.hpp"

namespace sislice {

static thread_local sislice_handle* g_current = nullptr;
sislice_handle* current_handle() { return g_current; }
void set_current_handle(sislice_handle* h) { g_current = h; }

void check_handle(sislice_handle* h) {
  SL_CHECK_ARG(h != nullptr, "null handle");
  SL_HIP(hipSetDevice(h->device));
  set_current_handle(h);
}

void* ws_get(sislice_handle* h, int id, size_t bytes) {
  auto& b = h->bufs[id];
  if (bytes == 0) bytes = 256;
  if (b.cap < bytes) {
    if (id == kBufDriver) h->fc.id = 0;  // the cached factorizations move
    if (b.ptr) {
      SL_HIP(hipStreamSynchronize(h->stream));
      SL_HIP(hipFree(b.ptr));
      b.ptr = nullptr;
      b.cap = 0;
    }
    size_t cap = bytes + bytes / 8;
    if (hipMalloc(&b.ptr, cap) != hipSuccess) {
      b.ptr = nullptr;
      throw Error(SISLICE_ERR_ALLOC, "device workspace allocation failed");
    }
    b.cap = cap;
  }
  return b.ptr;
}

void* host_stage(sislice_handle* h, size_t bytes) {
  if (h->host_cap < bytes) {
    if (h->host_stage) {
      SL_HIP(hipStreamSynchronize(h->stream));
      SL_HIP(hipHostFree(h->host_stage));
      h->host_stage = nullptr;
      h->host_cap = 0;
    }
    size_t cap = bytes + bytes / 4 + 4096;
    if (hipHostMalloc(&h->host_stage, cap, hipHostMallocDefault) != hipSuccess) {
      h->host_stage = nullptr;
      throw Error(SISLICE_ERR_ALLOC, "pinned host allocation failed");
    }
    h->host_cap = cap;
  }
  return h->host_stage;
}

unsigned* sync_words(sislice_handle* h, size_t words) {
  if (h->sync_cap < words) {
    if (h->sync) {
      SL_HIP(hipStreamSynchronize(h->stream));
      SL_HIP(hipFree(h->sync));
      h->sync = nullptr;
      h->sync_cap = 0;
    }
    const size_t cap = words + 4096;
    if (hipMalloc(&h->sync, cap * sizeof(unsigned)) != hipSuccess) {
      h->sync = nullptr;
      throw Error(SISLICE_ERR_ALLOC, "sync area allocation failed");
    }
    SL_HIP(hipMemsetAsync(h->sync, 0, cap * sizeof(unsigned), h->stream));
    h->sync_cap = cap;
  }
  return h->sync;
}

unsigned* wait_flag(sislice_handle* h) {
  if (!h->wait_word) {
    if (hipMalloc(&h->wait_word, 256) != hipSuccess) {
      h->wait_word = nullptr;
      throw Error(SISLICE_ERR_ALLOC, "wait-flag allocation failed");
    }
    SL_HIP(hipMemsetAsync(h->wait_word, 0, 256, h->stream));
  }
  return h->wait_word;
}

void check_waits(sislice_handle* h) {
  if (!h || !h->wait_word) return;
  // a local word, not the pinned staging area: callers may still hold results there
  unsigned hv = 0;
  SL_HIP(hipMemcpyAsync(&hv, h->wait_word, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
  SL_HIP(hipStreamSynchronize(h->stream));
  if (hv == 0) return;
  SL_HIP(hipMemsetAsync(h->wait_word, 0, sizeof(unsigned), h->stream));
  SL_HIP(hipStreamSynchronize(h->stream));
  throw Error(SISLICE_ERR_HIP, "a triangular-solve hand-off wait exceeded its bound of " +
                                   std::to_string(h->wait_limit) + " polls");
}

hipStream_t group_stream(sislice_handle* h, int g) {
  while ((int)h->group_streams.size() <= g) {
    hipStream_t s = nullptr;
    SL_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    h->group_streams.push_back(s);
  }
  return h->group_streams[g];
}

hipEvent_t group_event(sislice_handle* h, int g) {
  while ((int)h->group_events.size() <= g) {
    hipEvent_t e = nullptr;
    SL_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->group_events.push_back(e);
  }
  return h->group_events[g];
}

int prof_begin(sislice_handle* h, int cat, hipStream_t on) {
  if (!h || !h->prof || !((h->prof_mask >> cat) & 1u)) return -1;
  if (h->evnext + 2 > h->evpool.size()) {
    const size_t grow = std::max<size_t>(256, h->evpool.size());
    for (size_t q = 0; q < grow; ++q) {
      hipEvent_t e;
      SL_HIP(hipEventCreate(&e));
      h->evpool.push_back(e);
    }
  }
  hipEvent_t a = h->evpool[h->evnext++];
  hipEvent_t b = h->evpool[h->evnext++];
  SL_HIP(hipEventRecord(a, on ? on : h->stream));
  h->recs.push_back({cat, a, b});
  return (int)h->recs.size() - 1;
}

void prof_end(sislice_handle* h, int ticket, hipStream_t on) {
  if (!h || ticket < 0) return;
  SL_HIP(hipEventRecord(h->recs[ticket].b, on ? on : h->stream));
}

void prof_collect(sislice_handle* h, double* ms, int64_t* count) {
  for (const auto& r : h->recs) {
    float t = 0.f;
    SL_HIP(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.cat] += t;
    count[r.cat] += 1;
  }
}

void prof_reset(sislice_handle* h) {
  h->recs.clear();
  h->evnext = 0;
}

int default_nb(int n) { return n >= 2048 ? 64 : 32; }

FactorPlan build_factor(sislice_handle* h, int bufid, int n, const double* A, long lda,
                        const double* B, long ldb, int S, const double* sigmas_host,
                        double* const* LD_host, long ldld, int32_t* const* ipiv_host, int nb,
                        bool pivot) {
  const FactorPlan defaults;
  const int nbpiv = h->cur_nbpiv > 0 ? h->cur_nbpiv : defaults.nbpiv;
  const int npmax = factor_npanel_max(n, nb, nbpiv, defaults.fast != 0);
  const long ldw = n;
  Sizer z;
  z.take<double>(S);                          // sigmas
  z.take<double>((size_t)S * ldw * (nb + 2));  // W
  for (int q = 0; q < 4; ++q) z.take<int>((size_t)S * n);
  z.take<int>((size_t)S * npmax);
  z.take<int>((size_t)S * npmax * n);
  z.take<FactorState>(S);
  z.take<int64_t>(3 * (size_t)S);
  z.take<void*>(10 * (size_t)S);
  z.take<double>((size_t)S * (3 * nb + nb * nb));   // aux
  Carver c(ws_get(h, bufid, z.off));
  FactorPlan fp;
  fp.n = n;
  fp.nshift = S;
  fp.nb = nb;
  fp.pivot = pivot;
  fp.A = A;
  fp.B = B;
  fp.lda = lda;
  fp.ldb = ldb;
  fp.ldld = ldld;
  fp.ldw = ldw;
  double* d_sig = c.take<double>(S);
  double* W = c.take<double>((size_t)S * ldw * (nb + 2));
  int* perm = c.take<int>((size_t)S * n);
  int* sw = c.take<int>((size_t)S * n);
  int* blk = c.take<int>((size_t)S * n);
  int* cp = c.take<int>((size_t)S * n);
  int* ps = c.take<int>((size_t)S * npmax);
  int* snap = c.take<int>((size_t)S * npmax * n);
  fp.d_state = c.take<FactorState>(S);
  fp.d_inertia = c.take<int64_t>(3 * (size_t)S);
  void** tab = c.take<void*>(10 * (size_t)S);
  double* aux = c.take<double>((size_t)S * (3 * nb + nb * nb));
  // host staging: sigmas then the pointer tables
  size_t hbytes = sizeof(double) * S + sizeof(void*) * 10 * S;
  char* hs = static_cast<char*>(host_stage(h, hbytes));
  std::memcpy(hs, sigmas_host, sizeof(double) * S);
  void** ht = reinterpret_cast<void**>(hs + sizeof(double) * S);
  for (int s = 0; s < S; ++s) {
    ht[0 * S + s] = LD_host[s];
    ht[1 * S + s] = W + (size_t)s * ldw * (nb + 2);
    ht[2 * S + s] = perm + (size_t)s * n;
    ht[3 * S + s] = sw + (size_t)s * n;
    ht[4 * S + s] = blk + (size_t)s * n;
    ht[5 * S + s] = cp + (size_t)s * n;
    ht[6 * S + s] = ps + (size_t)s * npmax;
    ht[7 * S + s] = snap + (size_t)s * npmax * n;
    ht[8 * S + s] = ipiv_host[s];
    ht[9 * S + s] = aux + (size_t)s * (3 * nb + nb * nb);
  }
  SL_HIP(hipMemcpyAsync(d_sig, hs, sizeof(double) * S, hipMemcpyHostToDevice, h->stream));
  SL_HIP(hipMemcpyAsync(tab, ht, sizeof(void*) * 10 * S, hipMemcpyHostToDevice, h->stream));
  fp.d_sigmas = d_sig;
  fp.d_LD = reinterpret_cast<double* const*>(tab + 0 * S);
  fp.d_W = reinterpret_cast<double* const*>(tab + 1 * S);
  fp.d_perm = reinterpret_cast<int* const*>(tab + 2 * S);
  fp.d_sw = reinterpret_cast<int* const*>(tab + 3 * S);
  fp.d_blk = reinterpret_cast<int* const*>(tab + 4 * S);
  fp.d_colpanel = reinterpret_cast<int* const*>(tab + 5 * S);
  fp.d_pstart = reinterpret_cast<int* const*>(tab + 6 * S);
  fp.pstart_base = ps;
  fp.npmax = npmax;
  fp.d_snap = reinterpret_cast<int* const*>(tab + 7 * S);
  fp.d_ipiv = reinterpret_cast<int* const*>(tab + 8 * S);
  fp.d_aux = reinterpret_cast<double* const*>(tab + 9 * S);
  fp.nbpiv = nbpiv;
  fp.cus = h->cus;
  // two shift groups on two streams overlap one group's panels with the other's
  // updates where the updates are long (measured at n = 12288, 49 shifts: 1080
  // against 1122 ms; at n = 4096 the lock-step form is faster)
  fp.groups = (n >= 8192 && S >= 8) ? 2 : 1;
  if (h->cur_wide_min > 0) fp.wide_min = h->cur_wide_min;
  return fp;
}

void factor_run(sislice_handle* h, const FactorPlan& fp, hipStream_t st) {
  // (the null stream cannot be captured)
  if (!h->use_graphs || h->stream == nullptr || !fp.pivot || fp.n <= 0 || fp.nshift <= 0) {
    factor_launch(fp, st);
    return;
  }
  factor_shift_form_launch(fp, st);
  sislice_handle::FactorGraph* g = nullptr;
  for (auto& q : h->fgraphs)
    if (q.n == fp.n && q.S == fp.nshift && q.nb == fp.nb && q.nbpiv == fp.nbpiv &&
        q.wide_min == fp.wide_min && q.ldld == fp.ldld && q.state == fp.d_state)
      g = &q;
  if (!g) {
    factor_prepare();
    flush_uploads();  // nothing staged may become a node of the graph
    auto fn = h->flush_fn;
    const bool prof = h->prof;
    h->flush_fn = nullptr;
    h->prof = false;
    sislice_handle::FactorGraph ng;
    ng.n = fp.n;
    ng.S = fp.nshift;
    ng.nb = fp.nb;
    ng.nbpiv = fp.nbpiv;
    ng.wide_min = fp.wide_min;
    ng.ldld = fp.ldld;
    ng.state = fp.d_state;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      try {
        factor_steps_launch(fp, st, false);
      } catch (...) {
        hipGraph_t dead = nullptr;
        (void)hipStreamEndCapture(st, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        h->flush_fn = fn;
        h->prof = prof;
        throw;
      }
      e = hipStreamEndCapture(st, &ng.graph);
    }
    h->flush_fn = fn;
    h->prof = prof;
    SL_HIP(e);
    SL_HIP(hipGraphInstantiate(&ng.exec, ng.graph, nullptr, nullptr, 0));
    // a graph of the same shape over a workspace that has moved is stale
    for (auto it = h->fgraphs.begin(); it != h->fgraphs.end();) {
      if (it->n == ng.n && it->S == ng.S && it->nb == ng.nb && it->nbpiv == ng.nbpiv &&
          it->wide_min == ng.wide_min) {
        (void)hipGraphExecDestroy(it->exec);
        (void)hipGraphDestroy(it->graph);
        it = h->fgraphs.erase(it);
      } else {
        ++it;
      }
    }
    h->fgraphs.push_back(ng);
    g = &h->fgraphs.back();
    ++h->graphs_built;
  }
  SL_HIP(hipGraphLaunch(g->exec, st));
  ++h->graph_replays;
}

}  // namespace sislice

using namespace sislice;

#define SL_API_BEGIN try {
#define SL_API_END                                          \
  }                                                         \
  catch (const sislice::Error& e) {                         \
    std::fprintf(stderr, "sislice: %s\n", e.what());        \
    return e.status;                                        \
  }                                                         \
  catch (const std::exception& e) {                         \
    std::fprintf(stderr, "sislice: %s\n", e.what());        \
    return SISLICE_ERR_HIP;                                 \
  }

extern "C" {

void sislice_default_opts(sislice_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->block = 8;
  o->max_basis = 112;
  o->max_cycles = 40;
  o->kpm_moments = 64;
  o->kpm_vectors = 20;
  o->bounds_steps = 30;
  o->nb = 0;
  o->tol = 1e-10;
  o->top_margin = 2.0;
  o->seed = 0;
  o->profile = 0;
  o->driver = 0;
  o->subspace_iters = 4;
  o->max_recovery = 2;
  o->graphs = 1;
}

const char* sislice_status_string(sislice_status s) {
  switch (s) {
    case SISLICE_OK: return "ok";
    case SISLICE_ERR_ARG: return "invalid argument";
    case SISLICE_ERR_HIP: return "HIP runtime error";
    case SISLICE_ERR_ALLOC: return "allocation failed";
    case SISLICE_ERR_NO_DEVICE: return "no gfx950 device";
    case SISLICE_SINGULAR_SHIFT: return "a shift is an eigenvalue (exact zero pivot)";
    case SISLICE_NOT_CONVERGED: return "residual tolerance not reached";
    case SISLICE_MISSING_EIGS: return "eigenvalues missing from a slice or below the top boundary";
  }
  return "unknown status";
}

sislice_status sislice_create(sislice_handle** out, int device, void* stream) {
  SL_API_BEGIN
  SL_CHECK_ARG(out != nullptr, "null output pointer");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return SISLICE_ERR_NO_DEVICE;
  hipDeviceProp_t prop;
  SL_HIP(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SISLICE_ERR_NO_DEVICE;
  SL_HIP(hipSetDevice(device));
  auto* h = new sislice_handle();
  h->device = device;
  h->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  h->stream = static_cast<hipStream_t>(stream);
  try {
    for (auto& e : h->ev) SL_HIP(hipEventCreate(&e));
    // set-up of the allocation-free entry point: the wait word exists from the
    // start and the scratch array's address on this device is known
    wait_flag(h);
    h->scratch = noalloc_scratch_setup(device);
    SL_HIP(hipStreamSynchronize(h->stream));
  } catch (...) {
    sislice_destroy(h);
    throw;
  }
  *out = h;
  return SISLICE_OK;
  SL_API_END
}

sislice_status sislice_destroy(sislice_handle* h) {
  if (!h) return SISLICE_OK;
  for (auto* w : h->workers) sislice_destroy(w);
  for (auto s : h->worker_streams) {
    hipStreamSynchronize(s);
    hipStreamDestroy(s);
  }
  for (auto s : h->group_streams) {
    hipStreamSynchronize(s);
    hipStreamDestroy(s);
  }
  for (auto e : h->group_events) hipEventDestroy(e);
  hipSetDevice(h->device);
  hipStreamSynchronize(h->stream);
  for (auto& b : h->bufs)
    if (b.ptr) hipFree(b.ptr);
  if (h->host_stage) hipHostFree(h->host_stage);
  if (h->sync) hipFree(h->sync);
  if (h->wait_word) hipFree(h->wait_word);
  if (h->ring_host) hipHostFree(h->ring_host);
  for (auto& g : h->fgraphs) {
    hipGraphExecDestroy(g.exec);
    hipGraphDestroy(g.graph);
  }
  for (auto e : h->evpool) hipEventDestroy(e);
  for (auto& e : h->ev)
    if (e) hipEventDestroy(e);
  delete h;
  return SISLICE_OK;
}

sislice_status sislice_set_stream(sislice_handle* h, void* stream) {
  SL_API_BEGIN
  check_handle(h);
  h->stream = static_cast<hipStream_t>(stream);
  return SISLICE_OK;
  SL_API_END
}

sislice_status sislice_set_wait_limit(sislice_handle* h, int64_t polls) {
  SL_API_BEGIN
  check_handle(h);
  SL_CHECK_ARG(polls >= 0 && polls <= 0xFFFFFFFFll, "wait limit out of range");
  h->wait_limit = (unsigned)polls;
  for (auto* w : h->workers) w->wait_limit = (unsigned)polls;
  return SISLICE_OK;
  SL_API_END
}

sislice_status sislice_ldlt_factor_multi(sislice_handle* h, int64_t n, const double* A, int64_t lda,
                                         const double* B, int64_t ldb, int64_t n_shifts,
                                         const double* sigmas, double* const* LD, int64_t ldld,
                                         int32_t* const* ipiv, int64_t* inertia) {
  SL_API_BEGIN
  check_handle(h);
  SL_CHECK_ARG(n >= 0 && n <= (int64_t)1 << 20, "n out of range");
  SL_CHECK_ARG(n_shifts >= 1 && n_shifts <= 4096, "n_shifts out of range");
  SL_CHECK_ARG(inertia && sigmas && LD && ipiv, "null pointer argument");
  if (n == 0) {
    for (int64_t s = 0; s < 3 * n_shifts; ++s) inertia[s] = 0;
    return SISLICE_OK;
  }
  SL_CHECK_ARG(A && B && lda >= n && ldb >= n && ldld >= n, "bad matrix argument");
  for (int64_t s = 0; s < n_shifts; ++s) SL_CHECK_ARG(LD[s] && ipiv[s], "null LD/ipiv pointer");
  SL_CHECK_ARG(n <= 20000, "n too large for the factorization kernels (LDS-resident column)");
  const int nb = default_nb((int)n);
  FactorPlan fp = build_factor(h, kBufFactor, (int)n, A, lda, B, ldb, (int)n_shifts, sigmas, LD,
                               ldld, ipiv, nb, true);
  factor_launch(fp, h->stream);
  auto* hi = static_cast<int64_t*>(host_stage(h, sizeof(int64_t) * 3 * n_shifts));
  SL_HIP(hipMemcpyAsync(hi, fp.d_inertia, sizeof(int64_t) * 3 * n_shifts, hipMemcpyDeviceToHost,
                        h->stream));
  SL_HIP(hipStreamSynchronize(h->stream));
  bool singular = false;
  for (int64_t s = 0; s < 3 * n_shifts; ++s) inertia[s] = hi[s];
  check_waits(h);
  for (int64_t s = 0; s < n_shifts; ++s) singular |= inertia[3 * s + 1] > 0;
  return singular ? SISLICE_SINGULAR_SHIFT : SISLICE_OK;
  SL_API_END
}

sislice_status sislice_ldlt_factor(sislice_handle* h, int64_t n, const double* A, int64_t lda,
                                   const double* B, int64_t ldb, double sigma, double* LD,
                                   int64_t ldld, int32_t* ipiv, int64_t inertia[3]) {
  double* lds[1] = {LD};
  int32_t* ips[1] = {ipiv};
  return sislice_ldlt_factor_multi(h, n, A, lda, B, ldb, 1, &sigma, lds, ldld, ips, inertia);
}

}  // extern "C"
