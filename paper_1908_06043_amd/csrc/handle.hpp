// Library handle: device, stream and growable device workspaces.
#pragma once

#include <map>
#include <vector>

#include "common.hpp"

struct sislice_handle {
  int device = 0;
  int cus = 256;  // compute units of the device
  hipStream_t stream = nullptr;
  hipEvent_t ev[8] = {};
  struct Buf {
    void* ptr = nullptr;
    size_t cap = 0;
  };
  Buf bufs[10];
  void* host_stage = nullptr;  // pinned staging for small host<->device records
  size_t host_cap = 0;
  unsigned* sync = nullptr;  // epoch flags and ticket counters of the persistent solves
  size_t sync_cap = 0;       // in unsigned words
  unsigned epoch = 0;
  // bounded device waits: polls before a waiter gives up, and the device word it
  // raises then (allocated on first use, zero while no wait has expired)
  unsigned wait_limit = 1u << 21;
  unsigned* wait_word = nullptr;
  // device address of the allocation-free solve's scratch array on this device
  void* scratch = nullptr;
  void* ring_host = nullptr;  // pinned ring for per-step pointer tables
  size_t ring_cap = 0;
  // staged-but-not-uploaded tables: flushed (one copy) before the next launch
  void (*flush_fn)(void*) = nullptr;
  void* flush_ctx = nullptr;
  // kernel-class timing with HIP events (enabled per call)
  bool prof = false;
  unsigned prof_mask = 0x3F;  // bit c: kernel class c is timed
  std::vector<hipEvent_t> evpool;
  size_t evnext = 0;
  struct ProfRec {
    int cat;
    hipEvent_t a, b;
  };
  std::vector<ProfRec> recs;
  // Factorizations of the last sislice_solve (its shifts, then the top boundary),
  // which stay in the driver workspace for sislice_adjoint.  id 0: none valid.
  struct FactorCache {
    uint64_t id = 0;
    int n = 0;
    const double* A = nullptr;
    const double* B = nullptr;
    long lda = 0, ldb = 0;
    double* Af = nullptr;  // full A, followed by full B (an n x 2n matrix)
    std::vector<double> pts;
    std::vector<double*> LD;
    std::vector<int32_t*> ipv;
    std::vector<int*> perm, blk;
    std::vector<double*> Linv;
    std::vector<int64_t> inertia;  // 3 per point
    std::vector<char> prepped;     // solve preparation done for the point
  } fc;
  uint64_t fc_counter = 0;
  // Batched solves: worker handles (each with its own stream and workspaces)
  // and the factorization parameters chosen by the autotuner per order n.
  std::vector<sislice_handle*> workers;
  std::vector<hipStream_t> worker_streams;  // created by the library, owned
  // Extra streams of a factorization run in shift groups (created by the
  // library, owned) and the events that fork them from and join them to the
  // handle's stream.
  std::vector<hipStream_t> group_streams;
  std::vector<hipEvent_t> group_events;
  struct FactorTune {
    int nb = 0, nbpiv = 0, wide_min = 0;
  };
  std::map<int, FactorTune> tuned;
  // panel parameters for the next factorizations (0: the library defaults)
  int cur_nbpiv = 0, cur_wide_min = 0;
  // Captured factorization sequences (panel/update steps, interchanges, inertia)
  // replayed with hipGraphLaunch when graphs are on: one per (order, shift
  // count, panel parameters) and factorization workspace.
  struct FactorGraph {
    int n = 0, S = 0, nb = 0, nbpiv = 0, wide_min = 0;
    long ldld = 0;
    const void* state = nullptr;  // the workspace the graph's kernels address
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<FactorGraph> fgraphs;
  bool use_graphs = false;
  int64_t graph_replays = 0;
  int64_t graphs_built = 0;
};

namespace sislice {

enum BufId {
  kBufFactor = 0,
  kBufSolve = 1,
  kBufDriver = 2,
  kBufKpm = 3,
  kBufEig = 4,
  kBufMisc = 5,
  kBufLanczos = 6,
  kBufRing = 7,
  kBufAdjoint = 8,
  kBufEigRot = 9
};

// Returns a device buffer of at least `bytes`, reallocating (contents lost) if needed.
void* ws_get(sislice_handle* h, int id, size_t bytes);
void* host_stage(sislice_handle* h, size_t bytes);

// Bump allocator over one workspace block.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* p) : base(static_cast<char*>(p)) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* r = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return r;
  }
  static size_t round(size_t b) { return (b + 255) & ~size_t(255); }
};

// Counting pass with the same layout rules as Carver.
struct Sizer {
  size_t off = 0;
  template <class T>
  void take(size_t count) {
    off = (off + 255) & ~size_t(255);
    off += count * sizeof(T);
  }
};

void check_handle(sislice_handle* h);

// Zero-initialised flag/counter words for persistent launches; grows (and
// re-zeroes) on demand.  Returns the base pointer.
unsigned* sync_words(sislice_handle* h, size_t words);
// The wait-error word of the handle's bounded device waits (allocated and zeroed
// on first use).
unsigned* wait_flag(sislice_handle* h);
// Device address of the allocation-free solve's scratch array on `device`
// (looked up once per device; the device becomes current).
void* noalloc_scratch_setup(int device);
// After a stream synchronisation: throws SISLICE_ERR_HIP (and clears the word)
// when a device wait of an earlier launch expired.
void check_waits(sislice_handle* h);
inline unsigned next_epoch(sislice_handle* h) { return ++h->epoch; }

// Kernel-class timing: prof_begin records an event before a launch on the
// handle's stream and returns a ticket; prof_end records the closing event.
// prof_collect (after a stream synchronisation) sums durations per class.
enum ProfCat { kProfPanel = 0, kProfUpdate = 1, kProfSolve = 2, kProfGemm = 3, kProfEig = 4, kProfOther = 5 };
// With a stream argument the events go on that stream (work launched on a
// stream other than the handle's).
int prof_begin(sislice_handle* h, int cat, hipStream_t on = nullptr);
void prof_end(sislice_handle* h, int ticket, hipStream_t on = nullptr);
// The handle's g-th group stream (non-blocking, default priority; created on
// first use) and its g-th fork/join event.
hipStream_t group_stream(sislice_handle* h, int g);
hipEvent_t group_event(sislice_handle* h, int g);
void prof_collect(sislice_handle* h, double* ms, int64_t* count);
void prof_reset(sislice_handle* h);

// The handle whose stream receives the current launches (set by entry points).
sislice_handle* current_handle();
void set_current_handle(sislice_handle* h);

// Uploads the kernel-argument tables staged since the last launch (one
// host-to-device copy on the handle's stream); called before every launch.
inline void flush_uploads() {
  sislice_handle* h = current_handle();
  if (h && h->flush_fn) h->flush_fn(h->flush_ctx);
}

}  // namespace sislice

// Every kernel launch of the library goes through this macro.
#define SL_LAUNCH(...)             \
  do {                             \
    ::sislice::flush_uploads();    \
    hipLaunchKernelGGL(__VA_ARGS__); \
  } while (0)

namespace sislice {

}  // namespace sislice
