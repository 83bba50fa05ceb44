#include <algorithm>
// Host-only driver for the library's geometry tables and the resident
// kernel's patch partition, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitize_host.py. Builds the tables
// for many shapes, orders and coordinate parameters and checks basic
// invariants; checks the partition against the rim cells the resident kernel
// enumerates (walked here independently, in the kernel's order); any
// out-of-bounds access or undefined behaviour aborts the run.
#include <cmath>
#include <cstdio>
#include <set>
#include <string>
#include <vector>

#include "../../paper_2501_14030_amd/csrc/hr_internal.h"

namespace hr {
void set_error(const std::string&) {}
}

// Owner patch of every rim cell of patch b (8 columns x ry rows), as the
// kernel walks them: per plane, NG x ry cells on each x0 side (low, high),
// then NG x 8 cells on each x1 side (low, high).
static std::set<int> rim_owners(const hr::Dims& d, int ry, int nbx, int b) {
  const int RB = hr::kResPatch, NG = d.NG;
  const int x0b = (b % nbx) * RB, x1b = (b / nbx) * ry;
  const int nrx = 2 * NG * ry;
  std::set<int> out;
  for (int w = 0; w < nrx + 2 * NG * RB; ++w) {
    int l0, l1;
    if (w < nrx) {
      const int side = w / (NG * ry), w2 = w % (NG * ry);
      l0 = (side == 0 ? 0 : NG + RB) + w2 % NG;
      l1 = NG + w2 / NG;
    } else {
      const int side = (w - nrx) / (NG * RB), w2 = (w - nrx) % (NG * RB);
      l0 = NG + w2 % RB;
      l1 = (side == 0 ? 0 : NG + ry) + w2 / RB;
    }
    int s0 = x0b + l0 - NG, s1 = x1b + l1 - NG;
    if (s0 < 0) {
      s0 = -1 - s0;
      if (d.sph) s1 = d.N1 - 1 - s1;
    } else if (s1 < 0) {
      s1 = -1 - s1;
    } else if (s1 >= d.N1) {
      s1 = 2 * d.N1 - 1 - s1;
    }
    if (s0 < 0 || s0 >= d.P0 || s1 < 0 || s1 >= d.N1) return {-1};
    const int bx = s0 >= d.N0 ? nbx - 1 : s0 / RB;
    out.insert(bx + nbx * (s1 / ry));
  }
  out.erase(b);
  return out;
}

static int check_plans() {
  int checked = 0;
  const int shapes[][3] = {{8, 8, 2}, {16, 8, 2}, {64, 32, 8}, {64, 64, 8}, {128, 128, 16},
                           {24, 40, 14}, {256, 256, 8}};
  for (int ry : {8, 4})
  for (int sph = 0; sph < 2; ++sph)
    for (const auto& sh : shapes)
      for (int NG : {4, 5}) {
        hr::Dims d{};
        d.N0 = sh[0]; d.N1 = sh[1]; d.N2 = sh[2]; d.NG = NG; d.P0 = sh[0] + NG; d.sph = sph;
        d.R1 = sh[1];
        std::vector<int> w;
        int nbx = 0, nby = 0;
        if (ry == 4 && (d.N0 / 8) * (d.N1 / 4) > hr::kResMaxBlocks) continue;
        if (!hr::resident_plan(d, ry, w, nbx, nby)) return 10;
        if (nbx != d.N0 / 8 || nby != d.N1 / ry) return 11;
        const int W = hr::kResMaxWait + 1;
        for (int b = 0; b < nbx * nby; ++b) {
          const int n = w[(size_t)b * W];
          std::set<int> part(w.begin() + (size_t)b * W + 1, w.begin() + (size_t)b * W + 1 + n);
          if ((int)part.size() != n || part.count(b)) return 12;
          for (int o : rim_owners(d, ry, nbx, b))
            if (o < 0 || !part.count(o)) return 13;       // a rim owner is a partner
          for (int o : part) {                            // the relation is symmetric
            const int m = w[(size_t)o * W];
            bool back = false;
            for (int k = 1; k <= m; ++k) back = back || w[(size_t)o * W + k] == b;
            if (!back) return 14;
          }
        }
        ++checked;
      }
  // shapes the partition refuses
  const int bad[][4] = {{37, 19, 6, 5}, {32, 16, 18, 4}, {12, 8, 4, 4}, {16, 16, 4, 9}};
  for (const auto& sh : bad) {
    hr::Dims d{};
    d.N0 = sh[0]; d.N1 = sh[1]; d.N2 = sh[2]; d.NG = sh[3]; d.P0 = sh[0] + sh[3];
    d.R1 = sh[1];
    std::vector<int> w;
    int nbx = 1, nby = 1;
    if (hr::resident_plan(d, 8, w, nbx, nby) || nbx || nby) return 15;
  }
  {
    // 8 x 4 patches on N1 = 12 (not a multiple of 8); no other patch rows
    hr::Dims d{};
    d.N0 = 16; d.N1 = 12; d.N2 = 4; d.NG = 4; d.P0 = 20; d.R1 = 12;
    std::vector<int> w;
    int nbx = 0, nby = 0;
    if (!hr::resident_plan(d, 4, w, nbx, nby) || nbx != 2 || nby != 3) return 16;
    if (hr::resident_plan(d, 8, w, nbx, nby) || hr::resident_plan(d, 2, w, nbx, nby)) return 17;
  }
  std::printf("resident partitions checked: %d\n", checked);
  return 0;
}

int main() {
  if (int rc = check_plans()) {
    std::printf("partition check failed: %d\n", rc);
    return rc;
  }
  int checked = 0;
  const int shapes[][3] = {{5, 5, 2}, {8, 4, 2}, {32, 16, 4}, {37, 19, 6}, {64, 64, 8}, {128, 64, 8}};
  const int orders[] = {2, 4, 6, 8, 10};
  for (int coords = 0; coords < 5; ++coords)
    for (const auto& sh : shapes)
      for (int order : orders) {
        const int NG = order / 2;
        if (sh[0] < NG || sh[1] < NG) continue;
        const bool cart = coords == 4;
        if (cart && (sh[2] < NG || sh[2] < 2)) continue;
        hr::Dims d{};
        d.N0 = sh[0];
        d.N1 = sh[1];
        d.N2 = sh[2];
        d.NG = NG;
        d.P0 = sh[0] + NG + (cart ? NG : 0);
        d.nint = sh[0] * sh[1] * sh[2];
        d.nout = NG * sh[1] * sh[2];
        d.sph = coords == 1 || coords == 2 ? 1 : 0;
        // SinhCylindrical: outer rows on both z faces; Cartesian: outer
        // layers beyond all six faces
        d.zo = coords == 3 || cart ? NG : 0;
        d.R1 = sh[1] + 2 * d.zo;
        d.cart = cart ? 1 : 0;
        hr_grid_params p{1.0e6, 0.07, 1.5, 100.0, 0.5};
        hr::HostTables t;
        std::string err;
        if (!hr::build_tables((hr_coords)coords, d, p, t, err)) {
          std::printf("build_tables failed: %s\n", err.c_str());
          return 1;
        }
        if (cart) {
          // constant Laplacian factors, uniform cells, and one coordinate per
          // stored column, row and plane, increasing along each axis
          if ((int)t.cx.size() != d.P0 + d.R1 + hr::planes_of(d)) return 20;
          for (double c : t.crat)
            if (c != 1.0) return 21;
          const int n[3] = {d.N0, d.N1, d.N2};
          int off = 0;
          for (int a = 0; a < 3; ++a) {
            for (int j = 1; j < n[a] + 2 * NG; ++j)
              if (!(t.cx[off + j] > t.cx[off + j - 1])) return 22;
            off += n[a] + 2 * NG;
          }
          // stored indices of the padded box stay below its size
          const long last = hr::sidx(d, d.N0 + NG - 1, d.N1 + NG - 1, d.N2 + NG - 1);
          if (last != (long)d.P0 * d.R1 * hr::planes_of(d) - 1 || hr::sidx(d, -NG, -NG, -NG) != 0)
            return 23;
          ++checked;
          continue;
        }
        if (!(t.ds_g > 0)) return 2;
        for (double c : t.crat)
          if (!(c >= 1.0 - 1e-12)) return 3;  // every interior cell is at least ds_g
        for (double r : t.orinv)
          if (!(r > 0) || !std::isfinite(r)) return 4;
        for (double r : t.zrinv)
          if (!(r > 0) || !std::isfinite(r)) return 5;
        for (double q : t.zq)
          if (q == 0.0 || !std::isfinite(q)) return 6;
        // z-face points: up to four steps toward the interior stay on stored
        // points (rows in [-zo, N1 + zo), columns in [0, P0))
        for (int zr = 0; zr < 2 * d.zo; ++zr)
          for (int i0 = 0; i0 < d.P0; ++i0) {
            const int k = i0 + d.P0 * zr;
            const int i1 = zr < d.zo ? zr - d.zo : d.N1 + (zr - d.zo);
            const int st = (int)t.zstep[k];
            if (st != d.P0 && st != -d.P0 && st != -1) return 7;
            for (int q = 1; q <= 4 && q <= std::min(d.N0, d.N1); ++q) {
              const int j0 = st == -1 ? i0 - q : i0;
              const int j1 = st == -1 ? i1 : i1 + (st > 0 ? q : -q);
              if (j0 < 0 || j0 >= d.P0 || j1 < -d.zo || j1 >= d.N1 + d.zo) return 8;
            }
          }
        ++checked;
      }
  std::printf("geometry tables checked: %d\n", checked);
  return 0;
}
