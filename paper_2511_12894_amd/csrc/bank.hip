// Organisation of a template bank into sets of one reference and its dependent
// templates (sec. III.A, template bank construction), host code:
//   1. order the bank by chirp mass and split it in halves, recursively, until
//      in every subset the longest and shortest durations differ by at most
//      max_spread;
//   2. split every subset with more than max_size templates in halves along
//      its symmetric-mass-ratio order, recursively, until none is larger;
//   3. in every set take as reference the template whose summed absolute
//      duration difference to the others is smallest (a median duration).
// Durations are tau(f_low) = t_c - t(f_low) of the TaylorF2 phase (sec. II.C).
#include <algorithm>
#include <cmath>
#include <vector>

#include "rf_internal.h"

namespace rf {
namespace {

struct Item {
  int64_t idx;
  double mc, eta, tau;
};

// halves [lo, mid), [mid, hi) with mid = lo + (hi - lo) / 2 until pred(range) holds
template <typename Pred>
void bisect(int64_t lo, int64_t hi, const Pred& ok, std::vector<std::pair<int64_t, int64_t>>& out) {
  if (hi - lo <= 1 || ok(lo, hi)) {
    out.emplace_back(lo, hi);
    return;
  }
  const int64_t mid = lo + (hi - lo) / 2;
  bisect(lo, mid, ok, out);
  bisect(mid, hi, ok, out);
}

}  // namespace
}  // namespace rf

using namespace rf;

extern "C" {

rf_status rf_template_durations(const rf_tmpl* t, int64_t n, double f_low, double* tau) {
  return guarded(nullptr, [&] {
    RF_CHECK(t && tau && n >= 0, "rf_template_durations: bad arguments");
    RF_CHECK(std::isfinite(f_low) && f_low > 0, "rf_template_durations: f_low must be positive");
    for (int64_t i = 0; i < n; ++i) {
      RF_CHECK(std::isfinite(t[i].m1) && std::isfinite(t[i].m2) && t[i].m1 > 0 && t[i].m2 > 0,
               "rf_template_durations: template masses must be positive");
      tau[i] = -tf2_t(tf2_coef(t[i]), f_low);
    }
  });
}

rf_status rf_bank_organise(const rf_tmpl* t, const double* tau, int64_t n, double max_spread, int32_t max_size,
                           int32_t* group, int64_t* reference, int32_t* ngroups) {
  return guarded(nullptr, [&] {
    RF_CHECK(t && tau && group && reference && ngroups && n >= 1, "rf_bank_organise: bad arguments");
    RF_CHECK(std::isfinite(max_spread) && max_spread >= 0, "rf_bank_organise: bad duration spread");
    RF_CHECK(max_size >= 1, "rf_bank_organise: max_size must be >= 1");
    std::vector<Item> v(n);
    for (int64_t i = 0; i < n; ++i) {
      const double m1 = t[i].m1, m2 = t[i].m2;
      RF_CHECK(std::isfinite(m1) && std::isfinite(m2) && m1 > 0 && m2 > 0 && std::isfinite(tau[i]),
               "rf_bank_organise: bad template");
      const double m = m1 + m2, eta = m1 * m2 / (m * m);
      v[i] = Item{i, m * std::pow(eta, 0.6), eta, tau[i]};
    }
    // 1. chirp-mass order (ties by index), bisection on the duration spread
    std::stable_sort(v.begin(), v.end(), [](const Item& a, const Item& b) { return a.mc < b.mc; });
    auto spread_ok = [&](int64_t lo, int64_t hi) {
      double a = v[lo].tau, b = v[lo].tau;
      for (int64_t i = lo + 1; i < hi; ++i) {
        a = std::min(a, v[i].tau);
        b = std::max(b, v[i].tau);
      }
      return b - a <= max_spread;
    };
    std::vector<std::pair<int64_t, int64_t>> sets;
    bisect(0, n, spread_ok, sets);
    // 2. symmetric-mass-ratio order inside each set (ties by chirp-mass order), bisection on the size
    std::vector<std::pair<int64_t, int64_t>> groups;
    for (const auto& s : sets) {
      std::stable_sort(v.begin() + s.first, v.begin() + s.second,
                       [](const Item& a, const Item& b) { return a.eta < b.eta; });
      bisect(s.first, s.second, [&](int64_t lo, int64_t hi) { return hi - lo <= max_size; }, groups);
    }
    RF_CHECK(groups.size() <= size_t(INT32_MAX), "rf_bank_organise: too many groups");
    // 3. reference: the summed absolute duration difference is smallest at the
    //    median durations (for an even count, anywhere between the two middle
    //    ones); take the lower median value, first in the set's order
    std::vector<double> d;
    for (size_t g = 0; g < groups.size(); ++g) {
      const int64_t lo = groups[g].first, hi = groups[g].second;
      d.resize(size_t(hi - lo));
      for (int64_t i = lo; i < hi; ++i) d[size_t(i - lo)] = v[i].tau;
      const size_t h = (d.size() - 1) / 2;
      std::nth_element(d.begin(), d.begin() + h, d.end());
      const double med = d[h];
      int64_t r = lo;
      while (v[r].tau != med) ++r;
      reference[g] = v[r].idx;
      for (int64_t i = lo; i < hi; ++i) group[v[i].idx] = int32_t(g);
    }
    *ngroups = int32_t(groups.size());
  });
}

}  // extern "C"
