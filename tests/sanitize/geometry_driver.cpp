// Host-only driver for the library's geometry tables, built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitize_host.py.
// Builds the tables for many shapes, orders and coordinate parameters and
// checks basic invariants; any out-of-bounds access or undefined behaviour
// aborts the run.
#include <cmath>
#include <cstdio>
#include <string>

#include "../../paper_2501_14030_amd/csrc/hr_internal.h"

namespace hr {
void set_error(const std::string&) {}
}

int main() {
  int checked = 0;
  const int shapes[][3] = {{5, 5, 2}, {8, 4, 2}, {32, 16, 4}, {37, 19, 6}, {64, 64, 8}, {128, 64, 8}};
  const int orders[] = {2, 4, 6, 8, 10};
  for (int coords = 0; coords < 2; ++coords)
    for (const auto& sh : shapes)
      for (int order : orders) {
        const int NG = order / 2;
        if (sh[0] < NG || sh[1] < NG) continue;
        hr::Dims d{};
        d.N0 = sh[0];
        d.N1 = sh[1];
        d.N2 = sh[2];
        d.NG = NG;
        d.P0 = sh[0] + NG;
        d.nint = sh[0] * sh[1] * sh[2];
        d.nout = NG * sh[1] * sh[2];
        d.sph = coords;
        hr_grid_params p{1.0e6, 0.07, 1.5, 100.0, 0.5};
        hr::HostTables t;
        std::string err;
        if (!hr::build_tables((hr_coords)coords, d, p, t, err)) {
          std::printf("build_tables failed: %s\n", err.c_str());
          return 1;
        }
        if (!(t.ds_g > 0)) return 2;
        for (double c : t.crat)
          if (!(c >= 1.0 - 1e-12)) return 3;  // every interior cell is at least ds_g
        for (double r : t.orinv)
          if (!(r > 0) || !std::isfinite(r)) return 4;
        ++checked;
      }
  std::printf("geometry tables checked: %d\n", checked);
  return 0;
}
