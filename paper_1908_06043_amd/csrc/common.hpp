// Shared definitions of the gfx950 spectrum-slicing library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>
#include <stdexcept>
#include <string>

#include "sislice.h"

namespace sislice {

// Errors inside the library are C++ exceptions carrying a status; every C entry
// point catches them and returns the status.
struct Error : std::runtime_error {
  sislice_status status;
  Error(sislice_status s, const std::string& what) : std::runtime_error(what), status(s) {}
};

#define SL_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::sislice::Error(SISLICE_ERR_HIP, std::string(#call) + ": " +                 \
                                                  hipGetErrorString(e_));                 \
  } while (0)

#define SL_CHECK_ARG(cond, msg)                                                           \
  do {                                                                                    \
    if (!(cond)) throw ::sislice::Error(SISLICE_ERR_ARG, msg);                            \
  } while (0)

#define SL_LAUNCH_CHECK() SL_HIP(hipGetLastError())

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4_f64 on gfx950, one wavefront: D(16x16) += A(16x4) * B(4x16).
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator element r
// of lane l is D[l / 16 + 4 r][l % 16] (rows interleaved by 4; measured on the
// device with random operands).
__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Bunch-Kaufman pivot threshold alpha = (1 + sqrt(17)) / 8 (Bunch & Kaufman 1977).
constexpr double kBkAlpha = 0.6403882032022076;

// Per-shift factorization state kept in device memory, so that a fixed sequence
// of launches can advance panels whose width depends on the pivots chosen.
struct FactorState {
  int32_t k0;        // first column of the panel factored last
  int32_t kb;        // columns factored by that panel
  int32_t done;      // 1 once every column is factored
  int32_t npanel;    // panels factored so far
  int64_t neg, zero, pos;  // inertia of D accumulated over the pivots
  int32_t jstart;    // columns of the current panel accepted by the pivot-free path
  int32_t pad;
};

// Largest panel width the factorization kernels are built for.
constexpr int kMaxNb = 64;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace sislice
