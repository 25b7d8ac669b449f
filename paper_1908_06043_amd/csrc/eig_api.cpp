// sislice_sym_eig: batched small symmetric eigensolver entry point.
#include "eig.hpp"
#include "handle.hpp"

using namespace sislice;

extern "C" sislice_status sislice_sym_eig(sislice_handle* h, int32_t m, int32_t batch,
                                          const double* A, int64_t lda, double* W, double* V) {
  try {
    check_handle(h);
    SL_CHECK_ARG(m >= 0 && m <= kEigMax, "order must be in [0, 112]");
    SL_CHECK_ARG(batch >= 0 && batch <= 65535, "batch out of range");
    if (m == 0 || batch == 0) return SISLICE_OK;
    SL_CHECK_ARG(A && W && V && lda >= m, "bad argument");
    Sizer z;
    z.take<int>(batch);
    z.take<void*>(3 * (size_t)batch);
    Carver c(ws_get(h, kBufEig, z.off));
    int* dm = c.take<int>(batch);
    void** tab = c.take<void*>(3 * (size_t)batch);
    const size_t hb = sizeof(int) * batch + 256 + sizeof(void*) * 3 * batch;
    char* hs = static_cast<char*>(host_stage(h, hb));
    int* hm = reinterpret_cast<int*>(hs);
    void** ht = reinterpret_cast<void**>(hs + ((sizeof(int) * batch + 255) & ~size_t(255)));
    for (int b = 0; b < batch; ++b) {
      hm[b] = m;
      ht[b] = const_cast<double*>(A + (size_t)b * lda * m);
      ht[batch + b] = W + (size_t)b * m;
      ht[2 * batch + b] = V + (size_t)b * m * m;
    }
    SL_HIP(hipMemcpyAsync(dm, hm, sizeof(int) * batch, hipMemcpyHostToDevice, h->stream));
    SL_HIP(hipMemcpyAsync(tab, ht, sizeof(void*) * 3 * batch, hipMemcpyHostToDevice, h->stream));
    EigArgs a;
    a.m = dm;
    a.A = reinterpret_cast<const double* const*>(tab);
    a.lda = lda;
    a.W = reinterpret_cast<double* const*>(tab + batch);
    a.V = reinterpret_cast<double* const*>(tab + 2 * batch);
    a.ldv = m;
    eig_launch(a, batch, m, h->stream);
    SL_HIP(hipStreamSynchronize(h->stream));  // the host staging is reused by the next call
    return SISLICE_OK;
  } catch (const Error& e) {
    std::fprintf(stderr, "sislice: %s\n", e.what());
    return e.status;
  }
}

extern "C" sislice_status sislice_sym_eig_var(sislice_handle* h, int32_t batch, const int32_t* m,
                                              int32_t mmax, const double* A, int64_t lda, double* W,
                                              double* V) {
  try {
    check_handle(h);
    SL_CHECK_ARG(mmax >= 0 && mmax <= kEigMax, "largest order must be in [0, 112]");
    SL_CHECK_ARG(batch >= 0 && batch <= 65535, "batch out of range");
    if (mmax == 0 || batch == 0) return SISLICE_OK;
    SL_CHECK_ARG(m && A && W && V && lda >= mmax, "bad argument");
    for (int b = 0; b < batch; ++b) SL_CHECK_ARG(m[b] >= 0 && m[b] <= mmax, "order out of range");
    Sizer z;
    z.take<int>(batch);
    z.take<void*>(3 * (size_t)batch);
    Carver c(ws_get(h, kBufEig, z.off));
    int* dm = c.take<int>(batch);
    void** tab = c.take<void*>(3 * (size_t)batch);
    const size_t hb = sizeof(int) * batch + 256 + sizeof(void*) * 3 * batch;
    char* hs = static_cast<char*>(host_stage(h, hb));
    int* hm = reinterpret_cast<int*>(hs);
    void** ht = reinterpret_cast<void**>(hs + ((sizeof(int) * batch + 255) & ~size_t(255)));
    for (int b = 0; b < batch; ++b) {
      hm[b] = m[b];
      ht[b] = const_cast<double*>(A + (size_t)b * lda * mmax);
      ht[batch + b] = W + (size_t)b * mmax;
      ht[2 * batch + b] = V + (size_t)b * mmax * mmax;
    }
    SL_HIP(hipMemcpyAsync(dm, hm, sizeof(int) * batch, hipMemcpyHostToDevice, h->stream));
    SL_HIP(hipMemcpyAsync(tab, ht, sizeof(void*) * 3 * batch, hipMemcpyHostToDevice, h->stream));
    EigArgs a;
    a.m = dm;
    a.A = reinterpret_cast<const double* const*>(tab);
    a.lda = lda;
    a.W = reinterpret_cast<double* const*>(tab + batch);
    a.V = reinterpret_cast<double* const*>(tab + 2 * batch);
    a.ldv = mmax;
    eig_launch(a, batch, mmax, h->stream);
    SL_HIP(hipStreamSynchronize(h->stream));  // the host staging is reused by the next call
    return SISLICE_OK;
  } catch (const Error& e) {
    std::fprintf(stderr, "sislice: %s\n", e.what());
    return e.status;
  }
}
