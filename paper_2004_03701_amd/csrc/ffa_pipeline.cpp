// Multi-DM pipeline pieces around the search (Sec. 5.7): the DM trials to
// search, clusters of peaks in frequency, harmonic flags. Host code: these
// work on lists of a few thousand entries.
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "../../include/ffa.h"

namespace {

constexpr double kDispersion = 4.148808e3;  // s MHz^2 pc^-1 cm^3

bool finite_all(const double* v, int32_t n) {
  for (int32_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// "a is brighter than b": higher S/N, or equal S/N and a lower index.
inline bool brighter(const float* snr, int32_t a, int32_t b) {
  return snr[a] > snr[b] || (snr[a] == snr[b] && a < b);
}

}  // namespace

extern "C" {

ffa_status ffa_select_dm_trials(const double* dm, int32_t n, double f_lo_mhz, double f_hi_mhz,
                                double max_smear_s, int32_t* keep, int32_t* nkeep) {
  if (!dm || !keep || !nkeep || n < 0) return FFA_ERR_INVALID_ARG;
  if (!(f_lo_mhz > 0.0) || !(f_hi_mhz > f_lo_mhz) || !(max_smear_s > 0.0) ||
      !std::isfinite(f_hi_mhz) || !std::isfinite(max_smear_s))
    return FFA_ERR_INVALID_ARG;
  if (!finite_all(dm, n)) return FFA_ERR_INVALID_ARG;
  for (int32_t i = 1; i < n; ++i)
    if (dm[i] < dm[i - 1]) return FFA_ERR_INVALID_ARG;
  // the DM error whose smearing across the band is max_smear_s, doubled
  const double step =
      2.0 * max_smear_s / (kDispersion * (std::pow(f_lo_mhz, -2.0) - std::pow(f_hi_mhz, -2.0)));
  const double half = 0.5 * step;
  int32_t count = 0;
  const double* end = dm + n;
  int32_t i = 0;
  while (i < n) {
    // the highest trial within half a step above the first uncovered one ...
    int32_t j = i;
    while (j + 1 < n && dm[j + 1] - dm[i] <= half) ++j;
    keep[count++] = j;
    // ... covers every trial up to half a step above itself
    const double* next = std::upper_bound(dm + j, end, dm[j],
                                          [half](double base, double v) { return v - base > half; });
    i = (int32_t)(next - dm);
  }
  *nkeep = count;
  return FFA_OK;
}

ffa_status ffa_cluster_frequencies(const double* freq, const float* snr, int32_t n, double tol_hz,
                                   int32_t* cluster_of, int32_t* brightest, int32_t* members,
                                   int32_t* nclusters) {
  if (!freq || !snr || !cluster_of || !brightest || !members || !nclusters || n < 0)
    return FFA_ERR_INVALID_ARG;
  if (!(tol_hz >= 0.0) || !std::isfinite(tol_hz) || !finite_all(freq, n)) return FFA_ERR_INVALID_ARG;
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [freq](int32_t a, int32_t b) {
    return freq[a] < freq[b] || (freq[a] == freq[b] && a < b);
  });
  int32_t c = -1;
  for (int32_t q = 0; q < n; ++q) {
    const int32_t a = order[q];
    if (q == 0 || freq[a] - freq[order[q - 1]] > tol_hz) {  // a gap: a new cluster
      ++c;
      brightest[c] = a;
      members[c] = 0;
    }
    cluster_of[a] = c;
    ++members[c];
    if (brighter(snr, a, brightest[c])) brightest[c] = a;
  }
  *nclusters = c + 1;
  return FFA_OK;
}

ffa_status ffa_flag_harmonics(const double* freq, const float* snr, int32_t n, double tol_hz,
                              int32_t max_order, int32_t* parent, int32_t* harm_num,
                              int32_t* harm_den) {
  if (!freq || !snr || !parent || !harm_num || !harm_den || n < 0) return FFA_ERR_INVALID_ARG;
  if (!(tol_hz >= 0.0) || !std::isfinite(tol_hz) || max_order < 1 || max_order > 64)
    return FFA_ERR_INVALID_ARG;
  for (int32_t i = 0; i < n; ++i)
    if (!(freq[i] > 0.0) || !std::isfinite(freq[i])) return FFA_ERR_INVALID_ARG;
  // the ratios, in the order of preference
  struct Ratio {
    int32_t num, den;
    double r;
  };
  std::vector<Ratio> ratios;
  for (int32_t a = 1; a <= max_order; ++a)
    for (int32_t b = 1; b <= max_order; ++b)
      if ((a != 1 || b != 1) && std::gcd(a, b) == 1) ratios.push_back({a, b, (double)a / (double)b});
  std::sort(ratios.begin(), ratios.end(), [](const Ratio& x, const Ratio& y) {
    return x.num + x.den < y.num + y.den || (x.num + x.den == y.num + y.den && x.num < y.num);
  });
  // entries by frequency, so that the entries near (n / m) f_i are found by
  // binary search
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [freq](int32_t a, int32_t b) { return freq[a] < freq[b]; });
  std::vector<double> sorted(n);
  for (int32_t q = 0; q < n; ++q) sorted[q] = freq[order[q]];
  std::vector<int32_t> best_rank(n, INT32_MAX);  // rank of the chosen ratio for the parent
  for (int32_t j = 0; j < n; ++j) {
    parent[j] = -1;
    harm_num[j] = 0;
    harm_den[j] = 0;
  }
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t rk = 0; rk < (int32_t)ratios.size(); ++rk) {
      const Ratio& ra = ratios[rk];
      const double centre = ra.r * freq[i];
      const double half = tol_hz * (1.0 + ra.r);
      // a slightly wider window than the test below, which decides exactly
      const double slack = 1e-12 * (fabs(centre) + half);
      auto lo = std::lower_bound(sorted.begin(), sorted.end(), centre - half - slack);
      for (auto it = lo; it != sorted.end() && *it <= centre + half + slack; ++it) {
        const int32_t j = order[it - sorted.begin()];
        if (j == i || !brighter(snr, i, j)) continue;
        if (!(fabs(freq[j] - ra.r * freq[i]) <= half)) continue;
        const int32_t p = parent[j];
        // the brightest parent; for one parent, its first ratio
        if (p < 0 || brighter(snr, i, p) || (p == i && rk < best_rank[j])) {
          parent[j] = i;
          harm_num[j] = ra.num;
          harm_den[j] = ra.den;
          best_rank[j] = rk;
        }
      }
    }
  }
  return FFA_OK;
}

}  // extern "C"
