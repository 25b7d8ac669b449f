// Host-side planning: slice validation (Section 2.2), the KPM cumulative DOS and
// equal-count shift placement (Section 3.1), k-means shift migration (Section
// 3.2) and the SplitMix64 counter generator used for every random draw.
#include "planner.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

namespace sislice {

// SplitMix64 (Steele, Lea & Flood 2014), counter form: output i of seed s is the
// finaliser applied to s + (i + 1) * golden-ratio increment.
uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double rng_uniform(uint64_t seed, uint64_t i) { return (double)(splitmix64(seed, i) >> 11) * 0x1.0p-53; }

uint64_t rng_derive(uint64_t seed, uint64_t tag) { return splitmix64(seed ^ tag, 0); }

// ------------------------------------------------------------------ KPM

void jackson(int M, double* g) {
  const double q = M_PI / (M + 1);
  const double cotq = std::cos(q) / std::sin(q);
  for (int k = 0; k < M; ++k)
    g[k] = ((M - k + 1) * std::cos(q * k) + std::sin(q * k) * cotq) / (M + 1);
}

// Phi(omega) = N [g0 mu0 (1 - th/pi) - (2/pi) sum_{k>=1} g_k mu_k sin(k th)/k],
// th = arccos((omega - c)/d): the integral of the Jackson-damped Chebyshev
// density from the bottom of [a, b] up to omega.  With the coefficients
// e_0 = g0 mu0 and e_k = (2/pi) g_k mu_k / k (k >= 1) formed once,
// Phi = N [e_0 (1 - th/pi) - sum_k e_k sin(k th)].
static void cdos_coefs(const double* mu, const double* g, int M, double* e) {
  e[0] = g[0] * mu[0];
  for (int k = 1; k < M; ++k) e[k] = (2.0 / M_PI) * g[k] * mu[k] / k;
}

static double cdos_eval(const double* e, int M, double a, double b, int64_t n, double omega) {
  const double c = 0.5 * (a + b), d = 0.5 * (b - a);
  double t = (omega - c) / d;
  t = std::min(1.0, std::max(-1.0, t));
  const double th = std::acos(t);
  double acc = e[0] * (1.0 - th / M_PI);
  // sin(k th) from the rotation (cos kth, sin kth) <- (cos th, sin th) (cos (k-1)th, sin (k-1)th):
  // one sine and one cosine per evaluation instead of one sine per term (the bisections of
  // the placement evaluate this a few hundred times); the rotation's error grows linearly in k
  const double c1 = std::cos(th), s1 = std::sin(th);
  double ck = c1, sk = s1;
  for (int k = 1; k < M; ++k) {
    acc -= e[k] * sk;
    const double cn = ck * c1 - sk * s1;
    sk = sk * c1 + ck * s1;
    ck = cn;
  }
  return (double)n * acc;
}

double kpm_cdos(const double* mu, const double* g, int M, double a, double b, int64_t n,
                double omega) {
  std::vector<double> e(M);
  cdos_coefs(mu, g, M, e.data());
  return cdos_eval(e.data(), M, a, b, n, omega);
}

// bisection to 1e-12 (b - a) on the coefficients of cdos_coefs
static double kpm_root(double target, const double* e, int M, double a, double b, int64_t n) {
  double lo = a, hi = b;
  const double tol = 1e-12 * (b - a);
  while (hi - lo > tol) {
    const double mid = 0.5 * (lo + hi);
    if (cdos_eval(e, M, a, b, n, mid) < target)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

void kpm_place(const double* mu, int M, double a, double b, int64_t n, int64_t n_e, int64_t n_s,
               double top_margin, double* sigmas, double* omega_top) {
  std::vector<double> g(M), e(M);
  jackson(M, g.data());
  cdos_coefs(mu, g.data(), M, e.data());
  const double K = (double)n_e / (double)n_s;
  const double top_count = (double)n_e + top_margin * K;
  *omega_top = kpm_root(top_count, e.data(), M, a, b, n);
  const double Kp = top_count / (double)n_s;
  double prev = a;
  for (int64_t j = 1; j <= n_s; ++j) {
    const double w = kpm_root(j * Kp, e.data(), M, a, b, n);
    sigmas[j - 1] = 0.5 * (prev + w);
    prev = w;
  }
}

// ------------------------------------------------------------------ k-means

static int nearest(const double* c, int k, double x) {
  int best = 0;
  double bd = std::fabs(x - c[0]);
  for (int j = 1; j < k; ++j) {
    const double d = std::fabs(x - c[j]);
    if (d < bd) {  // strict: ties stay with the lower centroid
      bd = d;
      best = j;
    }
  }
  return best;
}

void kmeanspp(const double* x, int64_t n, int k, uint64_t seed, double* out) {
  const uint64_t s = rng_derive(seed, kTagKmeansPP);
  uint64_t draw = 0;
  double u = rng_uniform(s, draw++);
  int64_t first = std::min<int64_t>((int64_t)(u * (double)n), n - 1);
  out[0] = x[first];
  std::vector<double> d2(n);
  for (int64_t i = 0; i < n; ++i) d2[i] = (x[i] - out[0]) * (x[i] - out[0]);
  for (int c = 1; c < k; ++c) {
    double total = 0.0;
    for (int64_t i = 0; i < n; ++i) total += d2[i];
    u = rng_uniform(s, draw++);
    if (total == 0.0) {
      out[c] = out[c - 1];
      continue;
    }
    const double target = u * total;
    double cum = 0.0;
    int64_t pick = n - 1;
    for (int64_t i = 0; i < n; ++i) {
      cum += d2[i];
      if (cum > target) {
        pick = i;
        break;
      }
    }
    out[c] = x[pick];
    for (int64_t i = 0; i < n; ++i) {
      const double e = (x[i] - x[pick]) * (x[i] - x[pick]);
      if (e < d2[i]) d2[i] = e;
    }
  }
}

void lloyd(const double* x, int64_t n, int k, double* c, int32_t* lab_out, int max_iter) {
  std::vector<int32_t> lab(n, -1), nl(n);
  for (int it = 0; it < max_iter; ++it) {
    for (int64_t i = 0; i < n; ++i) nl[i] = nearest(c, k, x[i]);
    if (it > 0 && nl == lab) break;
    lab = nl;
    for (int j = 0; j < k; ++j) {
      double sum = 0.0;
      int64_t cnt = 0;
      for (int64_t i = 0; i < n; ++i)
        if (lab[i] == j) {
          sum += x[i];
          ++cnt;
        }
      if (cnt > 0) c[j] = sum / (double)cnt;
    }
  }
  if (lab_out)
    for (int64_t i = 0; i < n; ++i) lab_out[i] = lab[i];
}

// ------------------------------------------------------------------ SCF probe migration

static double mean_of(const double* x, const std::vector<int>& idx) {
  double t = 0.0;
  for (int i : idx) t += x[i];  // left to right, ascending index
  return t / (double)idx.size();
}

ScfMigration scf_migrate(const double* x, const int32_t* probe_of, int64_t n,
                         const double* prev, int n_s, bool use_kmeanspp, uint64_t seed) {
  std::vector<double> c(n_s);
  if (use_kmeanspp)
    kmeanspp(x, n, n_s, seed, c.data());
  else
    for (int j = 0; j < n_s; ++j) c[j] = prev[j];
  std::sort(c.begin(), c.end());
  std::vector<int32_t> lab(n);
  lloyd(x, n, n_s, c.data(), lab.data(), 300);
  // cluster -> probe of maximal overlap (ties: previous shift nearest the centroid,
  // then the lower probe); empty clusters map nowhere
  std::vector<int> cmap(n_s, -1);
  for (int k = 0; k < n_s; ++k) {
    std::vector<int64_t> cnt(n_s, 0);
    int64_t members = 0;
    for (int64_t i = 0; i < n; ++i)
      if (lab[i] == k) {
        ++cnt[probe_of[i]];
        ++members;
      }
    if (members == 0) continue;
    int best = -1;
    for (int p = 0; p < n_s; ++p)
      if (best < 0 || cnt[p] > cnt[best] ||
          (cnt[p] == cnt[best] && std::fabs(prev[p] - c[k]) < std::fabs(prev[best] - c[k])))
        best = p;
    cmap[k] = best;
  }
  struct Pr {
    int origin;
    double ref;
    std::vector<int> m;
  };
  std::vector<Pr> pr;
  ScfMigration out;
  for (int p = 0; p < n_s; ++p) {
    int nk = 0;
    for (int k = 0; k < n_s; ++k) nk += cmap[k] == p;
    if (nk == 0) continue;
    out.merged += nk - 1;
    Pr q{p, prev[p], {}};
    for (int64_t i = 0; i < n; ++i)
      if (lab[i] >= 0 && cmap[lab[i]] == p) q.m.push_back((int)i);
    pr.push_back(std::move(q));
  }
  out.deleted = n_s - (int)pr.size();
  while ((int)pr.size() < n_s) {
    int big = 0;
    for (int q = 1; q < (int)pr.size(); ++q)
      if (pr[q].m.size() > pr[big].m.size()) big = q;
    if (pr[big].m.size() < 2) break;
    // 2-means of the probe's values from their smallest and largest
    std::vector<double> v;
    for (int i : pr[big].m) v.push_back(x[i]);
    double c2[2] = {*std::min_element(v.begin(), v.end()), *std::max_element(v.begin(), v.end())};
    std::vector<int32_t> l2(v.size());
    lloyd(v.data(), (int64_t)v.size(), 2, c2, l2.data(), 300);
    std::vector<int> lo, hi;
    for (size_t t = 0; t < v.size(); ++t) (l2[t] == 0 ? lo : hi).push_back(pr[big].m[t]);
    if (lo.empty() || hi.empty()) break;
    const double ref = pr[big].ref;
    const bool keep_lo = std::fabs(mean_of(x, lo) - ref) <= std::fabs(mean_of(x, hi) - ref);
    std::vector<int> go = keep_lo ? hi : lo;
    pr[big].m = keep_lo ? lo : hi;
    Pr nw{-1, mean_of(x, go), go};
    pr.push_back(std::move(nw));
    ++out.inserted;
  }
  std::vector<double> sh(pr.size());
  for (size_t q = 0; q < pr.size(); ++q) sh[q] = mean_of(x, pr[q].m);
  std::vector<int> order(pr.size());
  for (size_t q = 0; q < pr.size(); ++q) order[q] = (int)q;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sh[a] < sh[b]; });
  out.value_probe.assign(n, -1);
  for (size_t r = 0; r < order.size(); ++r) {
    const Pr& q = pr[order[r]];
    out.shifts.push_back(sh[order[r]]);
    out.origin.push_back(q.origin);
    for (int i : q.m) out.value_probe[i] = (int)r;
  }
  return out;
}

// ------------------------------------------------------------------ Lanczos DOS

LanczosDos::LanczosDos(const double* theta, const double* zeta2, int k_, int nv_, int64_t n_)
    : n(n_), k(k_), nv(nv_) {
  th.assign(theta, theta + (size_t)k * nv);
  z2.assign(zeta2, zeta2 + (size_t)k * nv);
  a = *std::min_element(th.begin(), th.end());
  b = *std::max_element(th.begin(), th.end());
  const double floor = 1e-3 * (b - a) / k;
  nu.resize(th.size());
  for (int r = 0; r < nv; ++r)
    for (int j = 0; j < k; ++j) {
      const double* t = th.data() + (size_t)r * k;
      const double left = j > 0 ? t[j] - t[j - 1] : -1e300;
      const double right = j + 1 < k ? t[j + 1] - t[j] : -1e300;
      nu[(size_t)r * k + j] = std::max(std::max(left, right), floor) / 3.0;
    }
}

double LanczosDos::phi(double w) const {
  double tot = 0.0;
  for (int r = 0; r < nv; ++r) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) {
      const size_t q = (size_t)r * k + j;
      const double kap = (w - th[q]) / (nu[q] * std::sqrt(2.0));
      s += z2[q] / nu[q] * std::exp(-kap * kap);
    }
    tot += s;
  }
  return (double)n / std::sqrt(2.0 * M_PI) * tot / nv;
}

double LanczosDos::cdos(double w) const {
  double tot = 0.0;
  for (int r = 0; r < nv; ++r) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) {
      const size_t q = (size_t)r * k + j;
      const double kap = (w - th[q]) / (nu[q] * std::sqrt(2.0));
      s += z2[q] * (std::erf(kap) + 1.0);
    }
    tot += s;
  }
  return (double)n / 2.0 * tot / nv;
}

double LanczosDos::expectation(double l, double u) const {
  double tot = 0.0;
  for (int r = 0; r < nv; ++r) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) {
      const size_t q = (size_t)r * k + j;
      auto psi = [&](double w) {
        const double kap = (w - th[q]) / (nu[q] * std::sqrt(2.0));
        return th[q] / 2.0 * std::erf(kap) - nu[q] / std::sqrt(2.0 * M_PI) * std::exp(-kap * kap);
      };
      s += z2[q] * (psi(u) - psi(l));
    }
    tot += s;
  }
  return (double)n * tot / nv / (cdos(u) - cdos(l));
}

double LanczosDos::root(double target, double lo, double hi) const {
  if (cdos(lo) - target >= 0) return lo;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (cdos(mid) - target < 0)
      lo = mid;
    else
      hi = mid;
    if (hi - lo <= 1e-12 * (b - a)) break;
  }
  return 0.5 * (lo + hi);
}

namespace {

using Iv = std::pair<double, double>;

double gamma_of(const LanczosDos& d, const Iv& iv) { return d.cdos(iv.second) - d.cdos(iv.first); }

std::vector<Iv> dos_cluster(const LanczosDos& d, double lo, double hi, int nw) {
  std::vector<double> w(nw), f(nw);
  for (int i = 0; i < nw; ++i) {
    w[i] = lo + (hi - lo) / (nw - 1) * i;
    f[i] = d.phi(w[i]);
  }
  std::vector<int> mx;
  for (int i = 0; i < nw; ++i)
    if ((i == 0 || f[i] > f[i - 1]) && (i == nw - 1 || f[i] >= f[i + 1])) mx.push_back(i);
  if (mx.size() <= 1) return {Iv(lo, hi)};
  std::vector<double> mu{lo};
  for (size_t j = 0; j + 1 < mx.size(); ++j) {
    int best = mx[j];
    if (mx[j + 1] - mx[j] > 1) {
      best = mx[j] + 1;
      for (int t = mx[j] + 1; t < mx[j + 1]; ++t)
        if (f[t] < f[best]) best = t;
    }
    mu.push_back(w[best]);
  }
  mu.push_back(hi);
  std::vector<Iv> out;
  for (size_t j = 0; j + 1 < mu.size(); ++j) {
    if (!(mu[j + 1] > mu[j])) continue;
    bool has = false;
    for (double t : d.th) has |= t > mu[j] && t <= mu[j + 1];
    if (has) out.emplace_back(mu[j], mu[j + 1]);
  }
  return out;
}

std::vector<Iv> merge_small(const LanczosDos& d, std::vector<Iv> I, double tol = 2.0) {
  bool changed = true;
  while (changed) {
    changed = false;
    for (size_t j = 0; j < I.size(); ++j) {
      if (I.size() == 1 || gamma_of(d, I[j]) >= tol) continue;
      std::vector<size_t> cands;
      if (j > 0 && I[j - 1].second == I[j].first) cands.push_back(j - 1);
      if (j + 1 < I.size() && I[j + 1].first == I[j].second) cands.push_back(j + 1);
      if (cands.empty()) continue;
      size_t t = cands[0];
      for (size_t q : cands)
        if (gamma_of(d, I[q]) < gamma_of(d, I[t])) t = q;
      const Iv m(std::min(I[t].first, I[j].first), std::max(I[t].second, I[j].second));
      std::vector<Iv> keep;
      for (size_t q = 0; q < I.size(); ++q)
        if (q != j && q != t) keep.push_back(I[q]);
      keep.push_back(m);
      std::sort(keep.begin(), keep.end());
      I = keep;
      changed = true;
      break;
    }
  }
  return I;
}

}  // namespace

void dos_plan(const LanczosDos& d, int64_t n_e, int64_t n_s, int mode, double top_margin,
              double* sigmas, double* omega_top) {
  const double span = d.b - d.a;
  const double a = d.a - 0.01 * span;
  const double top = d.root((double)n_e + top_margin * (double)n_e / (double)n_s, a, d.b + 0.01 * span);
  *omega_top = top;
  if (mode == 0) {
    const double pa = d.cdos(a);
    const double K = (d.cdos(top) - pa) / (double)n_s;
    std::vector<double> pts{a};
    for (int64_t j = 1; j < n_s; ++j) pts.push_back(d.root(pa + (double)j * K, a, top));
    pts.push_back(top);
    for (int64_t j = 0; j < n_s; ++j) sigmas[j] = 0.5 * (pts[j] + pts[j + 1]);
    return;
  }
  const int nw = 10 * d.k;
  // C(l, u) = ceil(gamma(l, u)) is the paper's approximate count (Sec. 3.1); the
  // refined grid has 2 C(l, u) / C(a, top) nw points, rounded half up, at least 10
  const double c_all = std::ceil(gamma_of(d, Iv(a, top)));
  std::vector<Iv> I = dos_cluster(d, a, top, nw);
  for (int round = 0; round < 20; ++round) {
    I = merge_small(d, I);
    std::vector<Iv> nwI;
    bool grew = false;
    for (const Iv& iv : I) {
      const double g = gamma_of(d, iv);
      if (g > 50.0) {
        const int nw2 = std::max(10, (int)std::floor(2.0 * std::ceil(g) / c_all * nw + 0.5));
        std::vector<Iv> sub = dos_cluster(d, iv.first, iv.second, nw2);
        if (sub.size() >= 2) {
          nwI.insert(nwI.end(), sub.begin(), sub.end());
          grew = true;
          continue;
        }
      }
      nwI.push_back(iv);
    }
    std::sort(nwI.begin(), nwI.end());
    I = nwI;
    if (!grew) break;
  }
  while ((int64_t)I.size() < n_s) {
    size_t j = 0;
    for (size_t q = 1; q < I.size(); ++q)
      if (gamma_of(d, I[q]) > gamma_of(d, I[j])) j = q;
    const double l = I[j].first, u = I[j].second;
    const double mid = d.root(0.5 * (d.cdos(l) + d.cdos(u)), l, u);
    std::vector<Iv> nwI(I.begin(), I.begin() + j);
    nwI.emplace_back(l, mid);
    nwI.emplace_back(mid, u);
    nwI.insert(nwI.end(), I.begin() + j + 1, I.end());
    std::sort(nwI.begin(), nwI.end());
    I = nwI;
  }
  while ((int64_t)I.size() > n_s) {
    size_t j = 0;
    for (size_t q = 1; q < I.size(); ++q)
      if (gamma_of(d, I[q]) < gamma_of(d, I[j])) j = q;
    std::vector<size_t> cands, adj;
    if (j > 0) cands.push_back(j - 1);
    if (j + 1 < I.size()) cands.push_back(j + 1);
    for (size_t q : cands)
      if (I[q].second == I[j].first || I[q].first == I[j].second) adj.push_back(q);
    const std::vector<size_t>& pool = adj.empty() ? cands : adj;
    size_t t = pool[0];
    for (size_t q : pool)
      if (gamma_of(d, I[q]) < gamma_of(d, I[t])) t = q;
    const Iv m(std::min(I[t].first, I[j].first), std::max(I[t].second, I[j].second));
    std::vector<Iv> keep;
    for (size_t q = 0; q < I.size(); ++q)
      if (q != j && q != t) keep.push_back(I[q]);
    keep.push_back(m);
    std::sort(keep.begin(), keep.end());
    I = keep;
  }
  std::vector<double> sh;
  for (const Iv& iv : I) sh.push_back(d.expectation(iv.first, iv.second));
  std::sort(sh.begin(), sh.end());
  for (int64_t j = 0; j < n_s; ++j) sigmas[j] = sh[j];
}

// ------------------------------------------------------------------ validation

int64_t validate(int64_t ns, const double* sig, const int64_t* nu, double omega_top, int64_t nu_top,
                 const int64_t* off, const int64_t* cnt, const double* th, const double* rs,
                 int32_t* scase, int32_t* sexact, int32_t* scand, int32_t* chosen) {
  int64_t total = 0;
  for (int64_t j = 0; j < ns; ++j) total = std::max(total, off[j] + cnt[j]);
  for (int64_t t = 0; t < total; ++t) chosen[t] = 0;
  int64_t nval = 0;
  struct Cand {
    double v, r, dist;
    int64_t idx;
  };
  std::vector<Cand> cs;
  for (int64_t s = 0; s <= ns; ++s) {
    const double lo = (s == 0) ? -std::numeric_limits<double>::infinity() : sig[s - 1];
    const double hi = (s == ns) ? omega_top : sig[s];
    const int64_t nlo = (s == 0) ? 0 : nu[s - 1];
    const int64_t nhi = (s == ns) ? nu_top : nu[s];
    const int64_t n_exact = nhi - nlo;
    cs.clear();
    auto add = [&](int64_t p, double a, double b, bool lo_closed, bool hi_closed) {
      for (int64_t q = 0; q < cnt[p]; ++q) {
        const int64_t t = off[p] + q;
        const double v = th[t];
        const bool in_lo = lo_closed ? (v >= a) : (v > a);
        const bool in_hi = hi_closed ? (v <= b) : (v < b);
        if (in_lo && in_hi) cs.push_back({v, rs[t], std::fabs(v - sig[p]), t});
      }
    };
    if (s == 0) {
      add(0, lo, hi, false, false);
    } else if (s == ns) {
      add(ns - 1, lo, hi, true, false);
    } else {
      const double tau = 0.5 * (lo + hi);
      add(s - 1, lo, tau, true, true);  // a value at tau belongs to the lower probe
      add(s, tau, hi, false, false);
    }
    const int64_t n_cand = (int64_t)cs.size();
    int32_t cse = 0;
    if (n_exact > n_cand) cse = 1;
    if (n_exact < n_cand) {
      cse = 2;
      std::sort(cs.begin(), cs.end(), [](const Cand& a, const Cand& b) {
        if (a.r != b.r) return a.r < b.r;
        if (a.dist != b.dist) return a.dist < b.dist;
        return a.v < b.v;
      });
      cs.resize(std::max<int64_t>(n_exact, 0));
    }
    for (const auto& c : cs) {
      chosen[c.idx] = 1;
      ++nval;
    }
    if (scase) scase[s] = cse;
    if (sexact) sexact[s] = (int32_t)n_exact;
    if (scand) scand[s] = (int32_t)n_cand;
  }
  return nval;
}

}  // namespace sislice

using namespace sislice;

extern "C" {

uint64_t sislice_splitmix64(uint64_t seed, uint64_t i) { return splitmix64(seed, i); }

double sislice_kpm_cdos(const double* mu, int32_t M, double a, double b, int64_t n, double omega) {
  if (!mu || M <= 0 || !(b > a)) return std::numeric_limits<double>::quiet_NaN();
  std::vector<double> g(M);
  jackson(M, g.data());
  return kpm_cdos(mu, g.data(), M, a, b, n, omega);
}

sislice_status sislice_kpm_place(const double* mu, int32_t M, double a, double b, int64_t n,
                                 int64_t n_e, int64_t n_s, double top_margin, double* sigmas,
                                 double* omega_top) {
  if (!mu || !sigmas || !omega_top || M <= 0 || !(b > a) || n_s <= 0 || n_e <= 0 || n_e > n)
    return SISLICE_ERR_ARG;
  kpm_place(mu, M, a, b, n, n_e, n_s, top_margin, sigmas, omega_top);
  return SISLICE_OK;
}

sislice_status sislice_kmeans_shifts(const double* ritz, int64_t n, const double* prev_shifts,
                                     int64_t n_s, int32_t use_kmeanspp, uint64_t seed,
                                     double* new_shifts, int32_t* labels) {
  if (!ritz || !new_shifts || n <= 0 || n_s <= 0 || n_s > n) return SISLICE_ERR_ARG;
  if (!use_kmeanspp && !prev_shifts) return SISLICE_ERR_ARG;
  std::vector<double> c(n_s);
  if (use_kmeanspp)
    kmeanspp(ritz, n, (int)n_s, seed, c.data());
  else
    for (int64_t j = 0; j < n_s; ++j) c[j] = prev_shifts[j];
  std::sort(c.begin(), c.end());
  lloyd(ritz, n, (int)n_s, c.data(), labels, 300);
  // labels refer to the sorted initial order; the final centroids keep that order
  // unless two crossed, so report them sorted together with relabelled members
  std::vector<int> order(n_s);
  for (int64_t j = 0; j < n_s; ++j) order[j] = (int)j;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return c[a] < c[b]; });
  std::vector<int> rank(n_s);
  for (int64_t j = 0; j < n_s; ++j) {
    new_shifts[j] = c[order[j]];
    rank[order[j]] = (int)j;
  }
  if (labels)
    for (int64_t i = 0; i < n; ++i) labels[i] = rank[labels[i]];
  return SISLICE_OK;
}

sislice_status sislice_dos_plan(const double* theta, const double* zeta2, int32_t k, int32_t nv,
                                int64_t n, int64_t n_e, int64_t n_s, int32_t mode,
                                double top_margin, double* sigmas, double* omega_top) {
  if (!theta || !zeta2 || !sigmas || !omega_top || k < 2 || nv < 1 || n < 1 || n_e < 1 ||
      n_s < 1 || (mode != 0 && mode != 1))
    return SISLICE_ERR_ARG;
  const LanczosDos d(theta, zeta2, k, nv, n);
  dos_plan(d, n_e, n_s, mode, top_margin, sigmas, omega_top);
  return SISLICE_OK;
}

sislice_status sislice_scf_migrate(const double* ritz, const int32_t* probe_of, int64_t n,
                                   const double* prev_shifts, int64_t n_s, int32_t use_kmeanspp,
                                   uint64_t seed, double* new_shifts, int32_t* value_probe,
                                   int32_t* origin, int32_t* n_new, int32_t* stats) {
  if (!ritz || !probe_of || !prev_shifts || !new_shifts || !n_new || n <= 0 || n_s <= 0 ||
      n_s > n)
    return SISLICE_ERR_ARG;
  for (int64_t i = 0; i < n; ++i)
    if (probe_of[i] < 0 || probe_of[i] >= n_s) return SISLICE_ERR_ARG;
  const ScfMigration m = scf_migrate(ritz, probe_of, n, prev_shifts, (int)n_s, use_kmeanspp != 0, seed);
  *n_new = (int32_t)m.shifts.size();
  for (size_t r = 0; r < m.shifts.size(); ++r) {
    new_shifts[r] = m.shifts[r];
    if (origin) origin[r] = m.origin[r];
  }
  if (value_probe)
    for (int64_t i = 0; i < n; ++i) value_probe[i] = m.value_probe[i];
  if (stats) {
    stats[0] = m.merged;
    stats[1] = m.deleted;
    stats[2] = m.inserted;
  }
  return SISLICE_OK;
}

int64_t sislice_validate(int64_t n_s, const double* sigmas, const int64_t* nu, double omega_top,
                         int64_t nu_top, const int64_t* offsets, const int64_t* counts,
                         const double* thetas, const double* resids, int32_t* slice_case,
                         int32_t* slice_exact, int32_t* slice_cand, int32_t* chosen) {
  if (n_s <= 0 || !sigmas || !nu || !offsets || !counts || !chosen) return SISLICE_ERR_ARG;
  for (int64_t j = 0; j < n_s; ++j)
    if (counts[j] > 0 && (!thetas || !resids)) return SISLICE_ERR_ARG;
  return validate(n_s, sigmas, nu, omega_top, nu_top, offsets, counts, thetas, resids, slice_case,
                  slice_exact, slice_cand, chosen);
}

}  // extern "C"
