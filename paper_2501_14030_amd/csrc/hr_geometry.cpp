// Host-side geometry of the relaxation grids: coordinate maps, scale
// factors, flat-space Laplacian coefficients, the variable wave speed and the
// outer-boundary factors. Runs once per grid; the results are uploaded as
// small 1D/2D tables (every factor depends on xx0 and xx1 only).
//
// Coordinates (companion-paper families named in the paper's "Basic
// equations" section and conclusions; the exact maps are readings):
//   SinhSymTP  prolate spheroidal with a sinh-stretched radial coordinate,
//              rho = A(xx0) sin xx1, z = sqrt(A^2 + b^2) cos xx1,
//              A(xx0) = amax sinh(xx0/w) / sinh(1/w), xx0 in [0,1];
//   Spherical  rho = r sin xx1, z = r cos xx1, r = xx0 in [0, rmax];
//   SinhSpherical  the same with r = A(xx0), xx0 in [0,1] (one of the further
//              coordinate families the paper's conclusions name);
// with xx1 in [0,pi] and xx2 = phi in [-pi,pi], cell-centred;
//   SinhCylindrical  (the cylindrical-like family of the conclusions)
//              rho = A(xx0), z = A(xx1) with xx1 in [-1,1], phi = xx2; both z
//              faces are outer boundaries with NG stored rows each.
//
// Both metrics are diagonal, so with scale factors h_i and J = h0 h1 h2
//   lap f = sum_i  f,ii / h_i^2 + (1/J) d_i (J / h_i^2) f,i .
// The wave speed is c(x) = kappa ds_min(x)/ds_g with ds_min(x) the smallest
// proper cell width h_i dxx_i at x and ds_g its interior minimum, so that
// the local Courant number is the same everywhere (end of the "Basic
// equations" section: wave speed proportional to the local grid spacing).

#include <algorithm>
#include <cmath>
#include <set>

#include "hr_internal.h"

namespace hr {
namespace {

constexpr double kPi = 3.14159265358979323846;

struct Local {
  double h0, h1, h2;   // scale factors
  double a0, a1, a2;   // 1 / h_i^2
  double b0, b1;       // (1/J) d_i (J / h_i^2), i = 0, 1 (the phi term vanishes)
  double rho, z;       // cylindrical position at phi = 0
  double drdx0;        // d r_cartesian / d xx0 along the coordinate line
  double drdx1;        // d r_cartesian / d xx1 (SinhCylindrical's z faces)
};

Local local_sinhsymtp(const hr_grid_params& p, double x0, double x1) {
  const double w = p.sinhwaa, b = p.bscale;
  const double norm = std::sinh(1.0 / w);
  const double A = p.amax * std::sinh(x0 / w) / norm;
  const double dA = p.amax * std::cosh(x0 / w) / (w * norm);
  const double d2A = A / (w * w);
  const double sn = std::sin(x1), cs = std::cos(x1);
  const double R2 = A * A + b * b;
  const double S = A * A + b * b * sn * sn;
  Local L;
  L.h0 = dA * std::sqrt(S) / std::sqrt(R2);
  L.h1 = std::sqrt(S);
  L.h2 = A * sn;
  L.a0 = R2 / (dA * dA * S);
  L.a1 = 1.0 / S;
  L.a2 = 1.0 / (A * A * sn * sn);
  // J/h0^2 = A sqrt(R2) sin(x1) / A'  ->  derivative along xx0 over J
  L.b0 = (2.0 * A * A + b * b - A * R2 * d2A / (dA * dA)) / (A * dA * S);
  // J/h1^2 = A A' sin(x1) / sqrt(R2) ->  derivative along xx1 over J
  L.b1 = cs / (sn * S);
  L.rho = A * sn;
  L.z = std::sqrt(R2) * cs;
  const double r = std::sqrt(L.rho * L.rho + L.z * L.z);
  L.drdx0 = A * dA / r;  // r^2 = A^2 + b^2 cos^2 xx1
  L.drdx1 = 0.0;
  return L;
}

// SinhSpherical: r = A(xx0) with SinhSymTP's sinh stretching, spherical angles.
// Scale factors (A', A, A sin xx1); with J = A' A^2 sin xx1,
//   (1/J) d_0 (J / A'^2) = (1/J) d_0 (A^2 sin xx1 / A') = 2/(A A') - A''/A'^3.
Local local_sinhspherical(const hr_grid_params& p, double x0, double x1) {
  const double w = p.sinhwaa;
  const double norm = std::sinh(1.0 / w);
  const double A = p.amax * std::sinh(x0 / w) / norm;
  const double dA = p.amax * std::cosh(x0 / w) / (w * norm);
  const double d2A = A / (w * w);
  const double sn = std::sin(x1), cs = std::cos(x1);
  Local L;
  L.h0 = dA;
  L.h1 = A;
  L.h2 = A * sn;
  L.a0 = 1.0 / (dA * dA);
  L.a1 = 1.0 / (A * A);
  L.a2 = 1.0 / (A * A * sn * sn);
  L.b0 = 2.0 / (A * dA) - d2A / (dA * dA * dA);
  L.b1 = cs / (sn * A * A);
  L.rho = A * sn;
  L.z = A * cs;
  L.drdx0 = dA;
  L.drdx1 = 0.0;
  return L;
}

// SinhCylindrical: rho = A(xx0), z = A(xx1), both with SinhSymTP's sinh
// stretching; scale factors (A'(xx0), A'(xx1), rho), J = A'(xx0) A'(xx1) rho:
//   (1/J) d_0 (J / h0^2) = (A'^2 - A A'') / (A'^3 A)  at xx0,
//   (1/J) d_1 (J / h1^2) = -Z'' / Z'^3                at xx1 (Z = A(xx1)),
// where A'^2 - A A'' = (amax / (w sinh(1/w)))^2 exactly (the difference of
// the two terms would lose most digits where xx0 >> w).
Local local_sinhcylindrical(const hr_grid_params& p, double x0, double x1) {
  const double w = p.sinhwaa;
  const double norm = std::sinh(1.0 / w);
  const double A = p.amax * std::sinh(x0 / w) / norm;
  const double dA = p.amax * std::cosh(x0 / w) / (w * norm);
  const double d2A = A / (w * w);
  const double Z = p.amax * std::sinh(x1 / w) / norm;
  const double dZ = p.amax * std::cosh(x1 / w) / (w * norm);
  const double d2Z = Z / (w * w);
  Local L;
  L.h0 = dA;
  L.h1 = dZ;
  L.h2 = A;
  L.a0 = 1.0 / (dA * dA);
  L.a1 = 1.0 / (dZ * dZ);
  L.a2 = 1.0 / (A * A);
  const double kk = p.amax / (w * norm);
  L.b0 = kk * kk / (dA * dA * dA * A);
  L.b1 = -d2Z / (dZ * dZ * dZ);
  L.rho = A;
  L.z = Z;
  const double r = std::sqrt(A * A + Z * Z);
  L.drdx0 = A * dA / r;
  L.drdx1 = Z * dZ / r;
  return L;
}

Local local_spherical(double x0, double x1) {
  const double r = x0, sn = std::sin(x1), cs = std::cos(x1);
  Local L;
  L.h0 = 1.0;
  L.h1 = r;
  L.h2 = r * sn;
  L.a0 = 1.0;
  L.a1 = 1.0 / (r * r);
  L.a2 = 1.0 / (r * r * sn * sn);
  L.b0 = 2.0 / r;
  L.b1 = cs / (sn * r * r);
  L.rho = r * sn;
  L.z = r * cs;
  L.drdx0 = 1.0;
  L.drdx1 = 0.0;
  return L;
}

}  // namespace

// Cartesian grids: the cube [-rmax, rmax]^3 with unit scale factors. The
// Laplacian factors are the constants 1/dx_d^2 (no first-derivative terms),
// every cell has the same width (c = kappa everywhere) and volume; the face
// points' radiation condition takes r and d r / d x_d from the stored
// coordinates (cx) in the kernel.
static bool build_tables_cartesian(const Dims& d, const hr_grid_params& p, HostTables& t,
                                   std::string& err) {
  const double L = p.rmax;
  const int n[3] = {d.N0, d.N1, d.N2};
  double dx[3];
  for (int a = 0; a < 3; ++a) dx[a] = 2.0 * L / n[a];
  const int n2d = d.N0 * d.N1, o2d = d.NG * d.N1, e2d = d.P0 * d.R1, z2d = d.P0 * 2 * d.zo;
  t.alpha.assign(5 * (size_t)n2d, 0.0);
  for (int k = 0; k < n2d; ++k) {
    t.alpha[0 * (size_t)n2d + k] = 1.0 / (dx[0] * dx[0]);
    t.alpha[1 * (size_t)n2d + k] = 1.0 / (dx[1] * dx[1]);
    t.alpha[2 * (size_t)n2d + k] = 1.0 / (dx[2] * dx[2]);
  }
  t.crat.assign(n2d, 1.0);
  t.ocrat.assign(o2d, 0.0);
  t.orinv.assign(o2d, 0.0);
  t.oq.assign(o2d, 0.0);
  t.zcrat.assign(z2d, 0.0);
  t.zrinv.assign(z2d, 0.0);
  t.zq.assign(z2d, 0.0);
  t.zstep.assign(z2d, 0.0);
  t.rho.assign(e2d, 0.0);
  t.zc.assign(e2d, 0.0);
  t.rcart.assign(e2d, 0.0);
  t.cphi.assign(d.N2, 0.0);
  t.sphi.assign(d.N2, 0.0);
  t.vol.assign(n2d, dx[0] * dx[1] * dx[2]);
  t.vol_total = dx[0] * dx[1] * dx[2] * (double)d.nint;
  t.volw = t.vol;
  t.volw_total = t.vol_total;
  t.ds_g = std::fmin(dx[0], std::fmin(dx[1], dx[2]));
  // cell centres of the stored columns, rows and planes (NG beyond each face)
  t.cx.clear();
  for (int a = 0; a < 3; ++a)
    for (int j = -d.NG; j < n[a] + d.NG; ++j) t.cx.push_back(-L + (j + 0.5) * dx[a]);
  if (!(t.ds_g > 0.0) || !std::isfinite(t.ds_g)) {
    err = "grid has a non-positive or non-finite cell width";
    return false;
  }
  return true;
}

bool build_tables(hr_coords coords, const Dims& d, const hr_grid_params& p,
                  HostTables& t, std::string& err) {
  if (coords == HR_CARTESIAN) return build_tables_cartesian(d, p, t, err);
  const bool cyl = coords == HR_SINHCYLINDRICAL;
  const double x0max = (coords == HR_SPHERICAL) ? p.rmax : 1.0;
  const double dx[3] = {x0max / d.N0, (cyl ? 2.0 : kPi) / d.N1, 2.0 * kPi / d.N2};
  auto coord = [&](int dir, int j) {  // j = stored index (0 = first interior)
    const double lo = (dir == 2) ? -kPi : (dir == 1 && cyl) ? -1.0 : 0.0;
    return lo + (j + 0.5) * dx[dir];
  };
  auto local = [&](int i0, int i1) {
    if (coords == HR_SINHSYMTP) return local_sinhsymtp(p, coord(0, i0), coord(1, i1));
    if (coords == HR_SINHSPHERICAL) return local_sinhspherical(p, coord(0, i0), coord(1, i1));
    if (cyl) return local_sinhcylindrical(p, coord(0, i0), coord(1, i1));
    return local_spherical(coord(0, i0), coord(1, i1));
  };
  auto dsmin = [&](const Local& L) {
    double s = std::fabs(L.h0) * dx[0];
    s = std::fmin(s, std::fabs(L.h1) * dx[1]);
    s = std::fmin(s, std::fabs(L.h2) * dx[2]);
    return s;
  };
  const int n2d = d.N0 * d.N1, o2d = d.NG * d.N1, e2d = d.P0 * d.R1, z2d = d.P0 * 2 * d.zo;
  t.alpha.assign(5 * (size_t)n2d, 0.0);
  t.crat.assign(n2d, 0.0);
  t.ocrat.assign(o2d, 0.0);
  t.orinv.assign(o2d, 0.0);
  t.oq.assign(o2d, 0.0);
  t.zcrat.assign(z2d, 0.0);
  t.zrinv.assign(z2d, 0.0);
  t.zq.assign(z2d, 0.0);
  t.zstep.assign(z2d, 0.0);
  t.rho.assign(e2d, 0.0);
  t.zc.assign(e2d, 0.0);
  t.rcart.assign(e2d, 0.0);
  t.cphi.assign(d.N2, 0.0);
  t.sphi.assign(d.N2, 0.0);
  t.vol.assign(n2d, 0.0);
  t.vol_total = 0.0;

  std::vector<double> ds(e2d);
  double dsg = INFINITY;
  for (int i1 = -d.zo; i1 < d.N1 + d.zo; ++i1)
    for (int i0 = 0; i0 < d.P0; ++i0) {
      const Local L = local(i0, i1);
      const int e = i0 + d.P0 * (i1 + d.zo);
      ds[e] = dsmin(L);
      t.rho[e] = L.rho;
      t.zc[e] = L.z;
      t.rcart[e] = std::sqrt(L.rho * L.rho + L.z * L.z);
      if (i1 < 0 || i1 >= d.N1) {
        // an outer row of a z face: lower rows first, then upper ones. The
        // radiation condition's one-sided difference runs along xx1 where
        // |z| >= rho, else along xx0 (only corner points beyond the rho face
        // qualify), so the direction is within 45 degrees of the radial one
        const int zr = i1 < 0 ? i1 + d.zo : d.zo + (i1 - d.N1);
        const int k = i0 + d.P0 * zr;
        t.zrinv[k] = 1.0 / t.rcart[e];
        if (std::fabs(L.z) >= L.rho) {
          t.zq[k] = (i1 < 0 ? -1.0 : 1.0) / (2.0 * dx[1] * L.drdx1);
          t.zstep[k] = i1 < 0 ? d.P0 : -d.P0;
        } else {
          t.zq[k] = 1.0 / (2.0 * dx[0] * L.drdx0);
          t.zstep[k] = -1.0;
        }
      } else if (i0 < d.N0) {
        const int k = i0 + d.N0 * i1;
        t.alpha[0 * (size_t)n2d + k] = L.a0 / (dx[0] * dx[0]);
        t.alpha[1 * (size_t)n2d + k] = L.a1 / (dx[1] * dx[1]);
        t.alpha[2 * (size_t)n2d + k] = L.a2 / (dx[2] * dx[2]);
        t.alpha[3 * (size_t)n2d + k] = L.b0 / dx[0];
        t.alpha[4 * (size_t)n2d + k] = L.b1 / dx[1];
        t.vol[k] = std::fabs(L.h0 * L.h1 * L.h2) * dx[0] * dx[1] * dx[2];
        t.vol_total += t.vol[k] * d.N2;
        dsg = std::fmin(dsg, ds[e]);
      } else {
        const int k = (i0 - d.N0) + d.NG * i1;
        t.orinv[k] = 1.0 / t.rcart[e];
        t.oq[k] = 1.0 / (2.0 * dx[0] * L.drdx0);
      }
    }
  if (!(dsg > 0.0) || !std::isfinite(dsg)) {
    err = "grid has a non-positive or non-finite cell width";
    return false;
  }
  t.ds_g = dsg;
  t.volw = t.vol;
  t.volw_total = t.vol_total;
  for (int i1 = -d.zo; i1 < d.N1 + d.zo; ++i1)
    for (int i0 = 0; i0 < d.P0; ++i0) {
      const int e = i0 + d.P0 * (i1 + d.zo);
      if (i1 < 0 || i1 >= d.N1)
        t.zcrat[i0 + d.P0 * (i1 < 0 ? i1 + d.zo : d.zo + (i1 - d.N1))] = ds[e] / dsg;
      else if (i0 < d.N0)
        t.crat[i0 + d.N0 * i1] = ds[e] / dsg;
      else
        t.ocrat[(i0 - d.N0) + d.NG * i1] = ds[e] / dsg;
    }
  for (int i2 = 0; i2 < d.N2; ++i2) {
    const double ph = coord(2, i2);
    t.cphi[i2] = std::cos(ph);
    t.sphi[i2] = std::sin(ph);
  }
  for (double a : t.alpha)
    if (!std::isfinite(a)) {
      err = "non-finite Laplacian coefficient (check coordinate parameters)";
      return false;
    }
  return true;
}

// Partition of a grid into the resident kernel's 8 x ry (x0, x1) patches and
// the exchange partners of each patch: the owners of the stored points its
// rim taps read (inner-boundary images resolved as in the stage kernels), and
// the patches whose rims read it, so that every reader of a patch's exchange
// slot is one of its partners (the double-buffered exchange relies on it).
bool resident_plan(const Dims& d, int ry, std::vector<int>& waits, int& nbx, int& nby) {
  constexpr int RB = kResPatch;
  nbx = nby = 0;
  if (ry != 8 && ry != 4) return false;
  // stored outer rows on the x1 faces (SinhCylindrical) are not handled by the
  // resident kernel: such grids run on the stage kernels
  if (d.zo) return false;
  if (d.N0 % RB || d.N1 % ry || d.NG > RB || d.N2 > 16 || d.N2 < 2) return false;
  const int bx_n = d.N0 / RB, by_n = d.N1 / ry, nb = bx_n * by_n;
  if (nb > kResMaxBlocks) return false;
  const int NG = d.NG;
  // owner patch of a stored (s0, s1); outer points belong to the last x0 patch
  auto owner = [&](int s0, int s1) { return std::min(s0 / RB, bx_n - 1) + bx_n * (s1 / ry); };
  std::vector<std::set<int>> rel(nb);
  for (int b = 0; b < nb; ++b) {
    const int x0b = (b % bx_n) * RB, x1b = (b / bx_n) * ry;
    auto tap = [&](int j0, int j1) {
      int s0 = j0, s1 = j1;
      if (j0 < 0) {
        s0 = -1 - j0;
        s1 = d.sph ? d.N1 - 1 - j1 : j1;
      } else if (j1 < 0) {
        s1 = -1 - j1;
      } else if (j1 >= d.N1) {
        s1 = 2 * d.N1 - 1 - j1;
      }
      const int o = owner(s0, s1);
      if (o != b) {
        rel[b].insert(o);
        rel[o].insert(b);
      }
    };
    for (int k = 1; k <= NG; ++k) {
      for (int r = 0; r < ry; ++r) {
        tap(x0b - k, x1b + r);
        tap(x0b + RB - 1 + k, x1b + r);
      }
      for (int c = 0; c < RB; ++c) {
        tap(x0b + c, x1b - k);
        tap(x0b + c, x1b + ry - 1 + k);
      }
    }
  }
  waits.assign((size_t)nb * (kResMaxWait + 1), 0);
  for (int b = 0; b < nb; ++b) {
    if ((int)rel[b].size() > kResMaxWait) return false;
    waits[(size_t)b * (kResMaxWait + 1)] = (int)rel[b].size();
    int k = 1;
    for (int o : rel[b]) waits[(size_t)b * (kResMaxWait + 1) + k++] = o;
  }
  nbx = bx_n;
  nby = by_n;
  return true;
}

}  // namespace hr
