// sislice_ldlt_solve_noalloc: the shift-invert solve of sislice_ldlt_solve for
// callers that cannot allocate (code under graph capture, tight serving loops).
//
// It runs the same kernels as sislice_ldlt_solve (the preparation of the
// diagonal-block inverses and look-ahead blocks, then the forward and backward
// sweeps), but every buffer beyond the caller's factors and right-hand sides
// lives in one file-scope device array of fixed size.  Nothing is allocated:
// no workspace growth, no pinned staging, no pointer tables uploaded from the
// host (a one-thread kernel writes them into the array), no synchronisation.
//
// Each GPU holds its own copy of the array; its address on a device is taken
// once, when the first handle on that device is created, and used from then
// on.  The array keeps the contents of the last call; the ticket counter that
// must start at zero is cleared by that same kernel at the start of each call.
// Calls that overlap on one GPU (two streams, two handles) share the array and
// race.
#include <mutex>
#include <vector>

#include "handle.hpp"
#include "solve.hpp"

// Largest order the array is sized for (right-hand sides up to 64, in chunks of
// 32): about 12.6 MB at n = 4096.
constexpr int64_t kNoallocMaxN = 4096;
constexpr size_t kScratchBytes = 13u << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace sislice {

namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;  // per device: device address of `scratch`

struct Layout {
  size_t perm, blk, linv, z, v, tab, ctr, total;
};

// byte offset of the next 256-aligned region of `bytes`
size_t place(size_t& off, size_t bytes) {
  off = (off + 255) & ~size_t(255);
  const size_t o = off;
  off += bytes;
  return o;
}

Layout layout(int64_t n) {
  Layout L;
  size_t off = 0;
  L.perm = place(off, sizeof(int) * (size_t)n);
  L.blk = place(off, sizeof(int) * (size_t)n);
  L.linv = place(off, sizeof(double) * solve_linv_size(n));
  L.z = place(off, sizeof(double) * (size_t)n * kSolveMaxRhs);
  L.v = place(off, sizeof(double) * (size_t)n * kSolveMaxRhs);
  L.tab = place(off, sizeof(void*) * 16);
  L.ctr = place(off, sizeof(unsigned) * 64);
  L.total = off;
  return L;
}

// Pointer tables of the single-shift launches (LD, ipiv, perm, blk, Linv, Z, V,
// then one X slot per right-hand-side chunk) and the cleared ticket counter.
__global__ void k_noalloc_tables(void** tab, const double* LD, const int32_t* ipiv, int* perm,
                                 int* blk, double* Linv, double* Z, double* V, double* X0,
                                 double* X1, unsigned* ctr) {
  if (threadIdx.x != 0) return;
  tab[0] = const_cast<double*>(LD);
  tab[1] = const_cast<int32_t*>(ipiv);
  tab[2] = perm;
  tab[3] = blk;
  tab[4] = Linv;
  tab[5] = Z;
  tab[6] = V;
  tab[8] = X0;
  tab[9] = X1;
  ctr[0] = 0u;
}

}  // namespace

void* noalloc_scratch_setup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_addr.size() <= device) g_scratch_addr.resize(device + 1, nullptr);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    SL_HIP(hipSetDevice(device));
    SL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    SL_CHECK_ARG(p != nullptr, "no device address for the solve scratch array");
    g_scratch_addr[device] = p;
  }
  return g_scratch_addr[device];
}

}  // namespace sislice

using namespace sislice;

extern "C" sislice_status sislice_ldlt_solve_noalloc(sislice_handle* h, int64_t n, const double* LD,
                                                     int64_t ldld, const int32_t* ipiv,
                                                     int64_t nrhs, double* X, int64_t ldx) {
  try {
    check_handle(h);
    SL_CHECK_ARG(n >= 0 && n <= kNoallocMaxN,
                 "n exceeds the allocation-free solve's scratch array (n <= 4096)");
    SL_CHECK_ARG(nrhs >= 0 && nrhs <= 64, "nrhs must be in [0, 64]");
    if (n == 0 || nrhs == 0) return SISLICE_OK;
    SL_CHECK_ARG(LD && ipiv && X && ldld >= n && ldx >= n, "bad argument");
    SL_CHECK_ARG(h->scratch != nullptr && h->wait_word != nullptr,
                 "handle has no scratch array or wait word");
    const Layout L = layout(n);
    SL_CHECK_ARG(L.total <= kScratchBytes, "scratch layout exceeds the array");
    char* base = static_cast<char*>(h->scratch);
    void** tab = reinterpret_cast<void**>(base + L.tab);
    unsigned* ctr = reinterpret_cast<unsigned*>(base + L.ctr);
    struct NoProf {  // no timing events here: creating them may allocate
      sislice_handle* h;
      bool was;
      ~NoProf() { h->prof = was; }
    } np{h, h->prof};
    h->prof = false;
    hipLaunchKernelGGL(k_noalloc_tables, dim3(1), dim3(64), 0, h->stream, tab, LD, ipiv,
                       reinterpret_cast<int*>(base + L.perm), reinterpret_cast<int*>(base + L.blk),
                       reinterpret_cast<double*>(base + L.linv), reinterpret_cast<double*>(base + L.z),
                       reinterpret_cast<double*>(base + L.v), X,
                       X + (nrhs > kSolveMaxRhs ? kSolveMaxRhs * ldx : 0), ctr);
    SL_LAUNCH_CHECK();
    solve_prep_launch((int)n, 1, reinterpret_cast<const int* const*>(tab + 1),
                      reinterpret_cast<int* const*>(tab + 2), reinterpret_cast<int* const*>(tab + 3),
                      reinterpret_cast<const double* const*>(tab + 0), ldld,
                      reinterpret_cast<double* const*>(tab + 4), h->stream);
    for (int64_t c0 = 0; c0 < nrhs; c0 += kSolveMaxRhs) {
      double** dx = reinterpret_cast<double**>(tab + 8 + c0 / kSolveMaxRhs);
      SolveArgs a;
      a.n = (int)n;
      a.nshift = 1;
      a.nrhs = (int)std::min<int64_t>(kSolveMaxRhs, nrhs - c0);
      a.LD = reinterpret_cast<const double* const*>(tab + 0);
      a.ldld = ldld;
      a.perm = reinterpret_cast<const int* const*>(tab + 2);
      a.blk = reinterpret_cast<const int* const*>(tab + 3);
      a.Linv = reinterpret_cast<const double* const*>(tab + 4);
      a.Y = dx;
      a.ldy = ldx;
      a.X = dx;
      a.ldx = ldx;
      a.Z = reinterpret_cast<double* const*>(tab + 5);
      a.V = reinterpret_cast<double* const*>(tab + 6);
      a.ldz = n;
      a.ctr = ctr;
      solve_launch(a, h->stream);
    }
    return SISLICE_OK;
  } catch (const Error& e) {
    std::fprintf(stderr, "sislice: %s\n", e.what());
    return e.status;
  }
}
