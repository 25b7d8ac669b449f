// Factorization workspace builder shared by the entry points and the driver.
#pragma once

#include "handle.hpp"
#include "kernels.hpp"

namespace sislice {

int default_nb(int n);

// Carves the per-shift factorization workspace from workspace `bufid`, uploads
// the shift values and pointer tables (host arrays of device pointers) and
// returns the launch plan.
FactorPlan build_factor(sislice_handle* h, int bufid, int n, const double* A, long lda,
                        const double* B, long ldb, int S, const double* sigmas_host,
                        double* const* LD_host, long ldld, int32_t* const* ipiv_host, int nb,
                        bool pivot);

// Runs the factorization of a plan: directly (factor_launch), or, with the
// handle's graphs on and a pivoting plan, the shift-form followed by the replay
// of the captured step sequence for the plan's shape and workspace (captured on
// first use).
void factor_run(sislice_handle* h, const FactorPlan& fp, hipStream_t st);

}  // namespace sislice
