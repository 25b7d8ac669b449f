// Host-side planning helpers (validation, KPM CDOS, k-means, SplitMix64).
#pragma once

#include <cstdint>
#include <vector>

#include "sislice.h"

namespace sislice {

// Sub-stream tags of the SplitMix64 draws (seed of a stream = output 0 of seed ^ tag).
constexpr uint64_t kTagKpm = 0x4B504Dull;        // Rademacher probe vectors
constexpr uint64_t kTagBounds = 0x424E44ull;     // spectral-bounds Lanczos start
constexpr uint64_t kTagLanczos = 0x4C4E43ull;    // probe start blocks (^ shift index << 32)
constexpr uint64_t kTagKmeansPP = 0x4B4D50ull;   // k-means++ seeding
constexpr uint64_t kTagDos = 0x444F53ull;        // start vectors of the Lanczos DOS runs

uint64_t splitmix64(uint64_t seed, uint64_t i);
double rng_uniform(uint64_t seed, uint64_t i);
uint64_t rng_derive(uint64_t seed, uint64_t tag);

void jackson(int M, double* g);
double kpm_cdos(const double* mu, const double* g, int M, double a, double b, int64_t n,
                double omega);
void kpm_place(const double* mu, int M, double a, double b, int64_t n, int64_t n_e, int64_t n_s,
               double top_margin, double* sigmas, double* omega_top);
void kmeanspp(const double* x, int64_t n, int k, uint64_t seed, double* out);
void lloyd(const double* x, int64_t n, int k, double* c, int32_t* lab, int max_iter);
// Probe migration between SCF steps (Section 3.2): k-means of the validated values
// seeded with the previous shifts (or k-means++), clusters mapped to the probe of
// maximal overlap, merged, unmapped probes deleted and the largest probe split by
// 2-means until n_s probes exist again.  Shifts ascending; value_probe[i] = new
// probe seeded by value i; origin[r] = previous probe continued (-1: inserted).
struct ScfMigration {
  std::vector<double> shifts;
  std::vector<int> origin;
  std::vector<int> value_probe;
  int merged = 0, deleted = 0, inserted = 0;
};
ScfMigration scf_migrate(const double* x, const int32_t* probe_of, int64_t n, const double* prev,
                         int n_s, bool use_kmeanspp, uint64_t seed);

// The paper's Lanczos DOS estimate (Section 3.1, eq. dos / cdos) from n_v runs of
// k-step Lanczos (Ritz values theta and squared first components zeta2, run r at
// offset r * k), with widths nu = d / 3 (d = the larger neighbour gap, floored at
// 1e-3 (b - a) / k), and the two planners: equal-count roots (mode 0) and
// DOSCluster with refinement, safeguards and DOS-expectation shifts (mode 1).
struct LanczosDos {
  int64_t n = 0;
  int k = 0, nv = 0;
  double a = 0, b = 0;
  std::vector<double> th, z2, nu;  // nv * k each
  LanczosDos(const double* theta, const double* zeta2, int k, int nv, int64_t n);
  double phi(double w) const;
  double cdos(double w) const;
  double expectation(double l, double u) const;
  double root(double target, double lo, double hi) const;
};
void dos_plan(const LanczosDos& d, int64_t n_e, int64_t n_s, int mode, double top_margin,
              double* sigmas, double* omega_top);

int64_t validate(int64_t ns, const double* sig, const int64_t* nu, double omega_top, int64_t nu_top,
                 const int64_t* off, const int64_t* cnt, const double* th, const double* rs,
                 int32_t* scase, int32_t* sexact, int32_t* scand, int32_t* chosen);

}  // namespace sislice
