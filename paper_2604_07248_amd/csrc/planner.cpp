// Screen placement along a path (Sec. 2.4, Eq. 7; App. C Eq. S18-S21):
// host arithmetic behind turpy_place_screens.  The steps and their order are
// documented with the declaration in include/turpy.h.
#include <algorithm>
#include <cmath>
#include <vector>

#include "report.hpp"
#include "turpy.h"

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxIntervals = 65536;
constexpr int kPanels = 64;  // Gauss-Legendre panels per interval (plus table nodes)

// 8-point Gauss-Legendre rule on [-1, 1] (Abramowitz & Stegun, Table 25.4).
constexpr double kGlX[4] = {0.1834346424956498049, 0.5255324099163289858, 0.7966664774136267396,
                            0.9602898564975362317};
constexpr double kGlW[4] = {0.3626837833783619830, 0.3137066458778872873, 0.2223810344533744706,
                            0.1012285362903762592};

struct Profile {
  int kind = 0;
  double cn2 = 0, A = 0, V = 0;
  const double* z = nullptr;
  const double* v = nullptr;
  int64_t count = 0;

  double at(double h) const {
    switch (kind) {
      case TURPY_CN2_UNIFORM:
        return cn2;
      case TURPY_CN2_HUFNAGEL_VALLEY: {
        const double s = 1e-5 * h;
        const double s2 = s * s, s4 = s2 * s2, s8 = s4 * s4;
        return 0.00594 * (V / 27.0) * (V / 27.0) * s8 * s2 * std::exp(-h / 1000.0) +
               2.7e-16 * std::exp(-h / 1500.0) + A * std::exp(-h / 100.0);
      }
      default: {
        if (h <= z[0]) return v[0];
        if (h >= z[count - 1]) return v[count - 1];
        const int64_t i = std::upper_bound(z, z + count, h) - z;  // z[i-1] <= h < z[i]
        const double t = (h - z[i - 1]) / (z[i] - z[i - 1]);
        return v[i - 1] + t * (v[i] - v[i - 1]);
      }
    }
  }

  // Panel edges over [a, b]: kPanels equal panels plus the table's nodes inside.
  std::vector<double> edges(double a, double b) const {
    std::vector<double> e;
    e.reserve(kPanels + 2);
    for (int i = 0; i <= kPanels; ++i) e.push_back(a + (b - a) * i / kPanels);
    if (kind == TURPY_CN2_TABLE) {
      for (int64_t i = 0; i < count; ++i)
        if (z[i] > a && z[i] < b) e.push_back(z[i]);
      std::sort(e.begin(), e.end());
      e.erase(std::unique(e.begin(), e.end()), e.end());
      e.back() = b;
    }
    return e;
  }
};

template <class F>
double gauss8(F&& f, double lo, double hi) {
  const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
  double s = 0;
  for (int i = 0; i < 4; ++i) s += kGlW[i] * (f(c - h * kGlX[i]) + f(c + h * kGlX[i]));
  return s * h;
}

// Integral of Cn2 over [a, b].
double integral(const Profile& p, double a, double b) {
  const std::vector<double> e = p.edges(a, b);
  double s = 0;
  for (size_t i = 0; i + 1 < e.size(); ++i) s += gauss8([&](double h) { return p.at(h); }, e[i], e[i + 1]);
  return s;
}

// Integral of Cn2(z) (1 - (z - a)/D)^(5/3) over [a, b], D = b - a.  On the
// panel that ends at b the weight is not smooth; there z = b - w u^3 turns the
// integrand into Cn2(b - w u^3) 3 w^(8/3) u^7 / D^(5/3), which is.
double weighted(const Profile& p, double a, double b) {
  const double d = b - a;
  const std::vector<double> e = p.edges(a, b);
  double s = 0;
  for (size_t i = 0; i + 2 < e.size(); ++i)
    s += gauss8([&](double h) { return p.at(h) * std::pow((b - h) / d, 5.0 / 3.0); }, e[i], e[i + 1]);
  const double w = b - e[e.size() - 2];
  s += gauss8([&](double u) { return p.at(b - w * u * u * u) * u * u * u * u * u * u * u; }, 0.0, 1.0) * 3.0 *
       std::pow(w, 8.0 / 3.0) / std::pow(d, 5.0 / 3.0);
  return s;
}

// Eq. S19 over [a, b].
double rytov(const Profile& p, double a, double b, double k) {
  return 3.27 * std::pow(k, 7.0 / 6.0) * std::pow(b - a, 5.0 / 6.0) * weighted(p, a, b);
}

// Halve intervals of `bounds` while `over(lo, hi)` holds; false when the
// interval count would exceed kMaxIntervals.
template <class Over>
bool split(std::vector<double>& bounds, Over&& over) {
  std::vector<double> out{bounds.front()};
  for (size_t i = 1; i < bounds.size(); ++i) {
    std::vector<std::pair<double, double>> stack{{out.back(), bounds[i]}};
    while (!stack.empty()) {
      const auto [lo, hi] = stack.back();
      stack.pop_back();
      if (over(lo, hi)) {
        const double mid = 0.5 * (lo + hi);
        stack.push_back({mid, hi});
        stack.push_back({lo, mid});
      } else {
        out.push_back(hi);
        if (static_cast<int>(out.size()) > kMaxIntervals + 1) return false;
      }
    }
  }
  bounds.swap(out);
  return true;
}

turpy_status check_profile(const turpy_cn2_profile* prof, Profile* p) {
  if (!prof) return turpy::report(TURPY_E_INVALID, "place_screens: NULL profile");
  p->kind = prof->kind;
  switch (prof->kind) {
    case TURPY_CN2_UNIFORM:
      if (!(prof->cn2 >= 0) || !std::isfinite(prof->cn2))
        return turpy::report(TURPY_E_INVALID, "place_screens: uniform Cn2 must be finite and >= 0");
      p->cn2 = prof->cn2;
      return TURPY_OK;
    case TURPY_CN2_HUFNAGEL_VALLEY:
      if (!(prof->A >= 0) || !(prof->V >= 0) || !std::isfinite(prof->A) || !std::isfinite(prof->V))
        return turpy::report(TURPY_E_INVALID, "place_screens: Hufnagel-Valley A and V must be finite and >= 0");
      p->A = prof->A;
      p->V = prof->V;
      return TURPY_OK;
    case TURPY_CN2_TABLE:
      if (!prof->z || !prof->values || prof->count < 1)
        return turpy::report(TURPY_E_INVALID, "place_screens: table needs z, values and count >= 1");
      for (int64_t i = 0; i < prof->count; ++i) {
        if (!(prof->values[i] >= 0) || !std::isfinite(prof->values[i]) || !std::isfinite(prof->z[i]))
          return turpy::report(TURPY_E_INVALID, "place_screens: table entry %lld is not finite / >= 0",
                               static_cast<long long>(i));
        if (i > 0 && !(prof->z[i] > prof->z[i - 1]))
          return turpy::report(TURPY_E_INVALID, "place_screens: table z must increase strictly");
      }
      p->z = prof->z;
      p->v = prof->values;
      p->count = prof->count;
      return TURPY_OK;
    default:
      return turpy::report(TURPY_E_INVALID, "place_screens: unknown profile kind %d", prof->kind);
  }
}

}  // namespace

extern "C" turpy_status turpy_place_screens(const turpy_cn2_profile* profile, double length, double wavelength,
                                            double n0, int32_t n, double dx, double rytov_limit, int32_t initial,
                                            int32_t max_screens, int32_t* num_screens, double* dz, double* cn2dz,
                                            double* rytov_out) {
  Profile p;
  if (turpy_status s = check_profile(profile, &p)) return s;
  if (!(length > 0) || !(wavelength > 0) || !(n0 > 0) || !(dx > 0) || n < 2 || !(rytov_limit > 0) ||
      initial < 1 || initial > kMaxIntervals || !std::isfinite(length) || !std::isfinite(rytov_limit))
    return turpy::report(TURPY_E_INVALID, "place_screens: length, wavelength, n0, dx, rytov_limit must be > 0, "
                                          "n >= 2 and 1 <= initial <= %d", kMaxIntervals);
  if (!num_screens || !dz || !cn2dz || max_screens < 0)
    return turpy::report(TURPY_E_INVALID, "place_screens: NULL output or negative capacity");
  const double k = 2.0 * kPi * n0 / wavelength;
  const double k0 = 2.0 * kPi / wavelength, kap = 2.0 * kPi / dx;
  const double arg = n0 * n0 * k0 * k0 - kap * kap;
  if (!(arg > 0)) return turpy::report(TURPY_E_INVALID, "place_screens: dx <= wavelength / n0, Eq. 7 has no step");
  const double dz_max = 0.5 * n * dx * std::sqrt(arg) / kap;

  std::vector<double> b(static_cast<size_t>(initial) + 1);
  for (int i = 0; i <= initial; ++i) b[i] = length * i / initial;
  b.back() = length;
  auto over = [&](double lo, double hi) { return rytov(p, lo, hi, k) > rytov_limit; };
  const char* too_many = "place_screens: more than %d intervals needed";
  // (2) halve intervals above the limit
  if (!split(b, over)) return turpy::report(TURPY_E_INVALID, too_many, kMaxIntervals);
  // (3) merge neighbours left to right while the merged interval stays within the limit
  std::vector<double> m{b[0], b[1]};
  for (size_t i = 2; i < b.size(); ++i) {
    if (rytov(p, m[m.size() - 2], b[i], k) <= rytov_limit)
      m.back() = b[i];
    else
      m.push_back(b[i]);
  }
  b.swap(m);
  // (4) equal shares of the cumulative strength, interpolated linearly, then (2) again
  const size_t M = b.size() - 1;
  if (M > 1) {
    std::vector<double> cum(M + 1, 0.0);
    for (size_t i = 0; i < M; ++i) cum[i + 1] = cum[i] + rytov(p, b[i], b[i + 1], k);
    std::vector<double> nb{0.0};
    size_t seg = 0;
    for (size_t j = 1; j < M; ++j) {
      const double target = cum[M] * static_cast<double>(j) / static_cast<double>(M);
      while (seg + 1 < M && cum[seg + 1] < target) ++seg;
      const double span = cum[seg + 1] - cum[seg];
      const double t = span > 0 ? (target - cum[seg]) / span : 0.0;
      nb.push_back(b[seg] + t * (b[seg + 1] - b[seg]));
    }
    nb.push_back(length);
    b.swap(nb);
    if (!split(b, over)) return turpy::report(TURPY_E_INVALID, too_many, kMaxIntervals);
  }
  // (5) Eq. 7
  if (!split(b, [&](double lo, double hi) { return hi - lo > dz_max; }))
    return turpy::report(TURPY_E_INVALID, too_many, kMaxIntervals);

  const int32_t count = static_cast<int32_t>(b.size() - 1);
  *num_screens = count;
  if (count > max_screens)
    return turpy::report(TURPY_E_CAPACITY, "place_screens: %d screens, capacity %d", count, max_screens);
  for (int32_t i = 0; i < count; ++i) {
    const double w = b[i + 1] - b[i];
    dz[i] = 0.5 * w + (i > 0 ? 0.5 * (b[i] - b[i - 1]) : 0.0);
    cn2dz[i] = integral(p, b[i], b[i + 1]);
    if (rytov_out) rytov_out[i] = rytov(p, b[i], b[i + 1], k);
  }
  dz[count] = 0.5 * (b[count] - b[count - 1]);
  return TURPY_OK;
}
