// Test driver for the host-only part of the library (descriptor validation,
// screen placement), built with the host compiler's address and
// undefined-behaviour sanitizers by tests/test_host_asan.py.  Reads one case
// per line from stdin and prints one result line per case:
//   V flags n M dx wavelength n0 l0 L0 sh tf conv R alpha nodz nocn2 dz[0..M] cn2dz[0..M-1]
//     -> V status message
//   P kind cn2 A V count length wavelength n0 n dx rytov_limit initial max_screens z[count] values[count]
//     -> P status M dz[0..M] cn2dz[0..M-1] rytov[0..M-1]   (M and arrays only when status is 0)
#include <cstdio>
#include <cstdlib>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "report.hpp"
#include "turpy.h"

namespace {

double num(std::istringstream& in) {
  std::string s;
  in >> s;
  return std::strtod(s.c_str(), nullptr);  // accepts nan and inf
}

void validate(std::istringstream& in) {
  turpy_path p{};
  const uint32_t flags = static_cast<uint32_t>(num(in));
  p.n = static_cast<int32_t>(num(in));
  p.num_screens = static_cast<int32_t>(num(in));
  p.dx = num(in);
  p.wavelength = num(in);
  p.n0 = num(in);
  p.l0 = num(in);
  p.L0 = num(in);
  p.sh_levels = static_cast<int32_t>(num(in));
  p.tf_kind = static_cast<int32_t>(num(in));
  p.inner_scale_conv = static_cast<int32_t>(num(in));
  p.realizations = static_cast<int64_t>(num(in));
  p.psd_alpha = num(in);
  const bool no_dz = num(in) != 0, no_cn2 = num(in) != 0;
  const int m = p.num_screens > 0 && p.num_screens <= (1 << 20) ? p.num_screens : 0;
  // exactly the entries the descriptor promises, so that a read past them is caught
  std::vector<double> dz, cn2;
  for (int i = 0; i <= m; ++i) dz.push_back(num(in));
  for (int i = 0; i < m; ++i) cn2.push_back(num(in));
  p.dz = no_dz ? nullptr : dz.data();
  p.cn2dz = no_cn2 || m == 0 ? nullptr : cn2.data();
  const turpy_status st = turpy::validate_path(&p, flags);
  std::printf("V %d %s\n", static_cast<int>(st), st ? turpy_last_error() : "");
}

void place(std::istringstream& in) {
  turpy_cn2_profile prof{};
  prof.kind = static_cast<int32_t>(num(in));
  prof.cn2 = num(in);
  prof.A = num(in);
  prof.V = num(in);
  prof.count = static_cast<int64_t>(num(in));
  const double length = num(in), wavelength = num(in), n0 = num(in);
  const int32_t n = static_cast<int32_t>(num(in));
  const double dx = num(in), limit = num(in);
  const int32_t initial = static_cast<int32_t>(num(in)), cap = static_cast<int32_t>(num(in));
  std::vector<double> z, v;
  for (int64_t i = 0; i < prof.count; ++i) z.push_back(num(in));
  for (int64_t i = 0; i < prof.count; ++i) v.push_back(num(in));
  prof.z = z.empty() ? nullptr : z.data();
  prof.values = v.empty() ? nullptr : v.data();
  std::vector<double> dz(cap + 1), cn2(cap), ry(cap);
  int32_t m = -1;
  const turpy_status st = turpy_place_screens(&prof, length, wavelength, n0, n, dx, limit, initial, cap, &m,
                                              dz.data(), cn2.data(), ry.data());
  std::printf("P %d", static_cast<int>(st));
  if (st == TURPY_OK) {
    std::printf(" %d", m);
    for (int i = 0; i <= m; ++i) std::printf(" %.17g", dz[i]);
    for (int i = 0; i < m; ++i) std::printf(" %.17g", cn2[i]);
    for (int i = 0; i < m; ++i) std::printf(" %.17g", ry[i]);
  }
  std::printf("\n");
}

}  // namespace

int main() {
  std::string line;
  while (std::getline(std::cin, line)) {
    std::istringstream in(line);
    std::string kind;
    in >> kind;
    if (kind == "V") validate(in);
    else if (kind == "P") place(in);
    else if (!kind.empty()) return 2;
  }
  return 0;
}
