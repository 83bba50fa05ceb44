// Plain FP64 reference implementation ("oracle") of hyperbolic relaxation for
// conformally flat binary-black-hole puncture initial data.
//
// TEST INFRASTRUCTURE ONLY. This file is compiled into oracle/libhr_oracle.so
// and is loaded by the tests, by the smoke check and by the CPU-baseline leg of
// the benchmark. The product library never links, includes or calls it, and it
// shares no code, headers or tables with the HIP path.
//
// What it computes (paper: "Basic equations" section):
//   * Eq. (4): the Hamiltonian constraint for the regular part u of the
//     conformal factor, psi = psi_singular + u,
//         lap(u) + (1/8) A_ij A^ij (psi_singular + u)^-7 = 0,
//     with lap the Laplacian of the flat conformal metric in curvilinear
//     coordinates and A_ij the Bowen-York (Brandt-Bruegmann puncture)
//     trace-free extrinsic curvature, which solves the momentum constraint
//     analytically.
//   * Eq. (5): the damped wave system whose steady state solves Eq. (4),
//         d_t u = v - eta u,   d_t v = c^2 [ lap(u) + (1/8) A A (psi_s+u)^-7 ],
//     integrated by the method of lines with classic RK4 (the driver
//     algorithm of the "Adapting NRPy for CUDA" section: RHS, then boundary
//     conditions, then the Runge-Kutta substep, with the residual H and its
//     grid L2 norm computed once per outer iteration).
//   * A wave speed proportional to the local grid spacing so that the CFL
//     condition holds everywhere (end of the "Basic equations" section).
//
// The paper delegates the coordinate definitions, boundary conditions and
// norm to earlier work; the readings used here are (each also listed in the
// design notes):
//   * cell-centred grids; NG = fd_order/2 ghost zones on every face;
//   * SinhSymTP: prolate-spheroidal coordinates with a sinh-stretched radial
//     coordinate, x = A sin(xx1) cos(xx2), y = A sin(xx1) sin(xx2),
//     z = sqrt(A^2+b^2) cos(xx1), A = AMAX sinh(xx0/w)/sinh(1/w), xx0 in [0,1];
//     the two foci (0,0,+-b) carry the punctures;
//   * Spherical: uniform r in [0,RMAX], theta in [0,pi], phi in [-pi,pi];
//   * SinhSpherical (one of the further coordinate families the paper's
//     conclusions list): r = A(xx0) with the same sinh stretching, xx0 in
//     [0,1], theta, phi as for Spherical;
//   * SinhCylindrical (the cylindrical-like family of the conclusions):
//     rho = A(xx0), z = A(xx1) with the same sinh stretching, xx0 in [0,1],
//     xx1 in [-1,1], phi = xx2 in [-pi,pi]; x = rho cos(phi), y = rho sin(phi).
//     Both z faces are outer boundaries (stored outer points, radiation
//     condition), the xx0 = 0 face reflects through the axis with phi + pi,
//     phi is periodic. An outer point beyond a z face takes its one-sided
//     difference along xx1 where |z| >= rho and along xx0 elsewhere (the
//     corners toward the rho face), so that the chosen direction is within
//     45 degrees of the radial one and d r / d xx_i never becomes small;
//   * Cartesian (the Cartesian-like family of the conclusions): the cube
//     [-RMAX, RMAX]^3 with xx0, xx1, xx2 = x, y, z. All six faces are outer
//     boundaries with NG stored layers; a layer point takes its one-sided
//     difference along its face normal x_d, with d r / d x_d = x_d / r. The
//     edge and corner points (beyond two or three faces) are read neither by
//     the star stencil nor by a face point's difference and are not evolved;
//     there are no parity images;
//   * psi_singular = 1 + sum_n m_n / (2 r_n);
//   * A^ij = sum_n 3/(2 r^2) [P^i n^j + P^j n^i - (delta^ij - n^i n^j) P.n]
//              + 3/r^3 [(S x n)^i n^j + (S x n)^j n^i];
//   * centred finite differences of order fd_order (Fornberg weights),
//     no dissipation;
//   * c(x) = kappa * ds_min(x) / ds_g, dt = CFL * ds_g, where ds_min(x) is the
//     smallest proper cell width at x and ds_g its minimum over the interior;
//   * boundary conditions act on each stage right-hand side k: at outer points
//     (xx0 beyond its maximum) k_f = -c (f/r + d_r f) for f in {u, v}
//     (radiation condition, f -> 0 as 1/r), d_r f from a second-order one-sided
//     xx0 difference; every other ghost copies k from the interior or outer
//     point at the same Cartesian position (parity +1, u is a scalar);
//   * residual_l2 = sqrt( sum_interior H^2 / N_interior ).
//
// Everything is plain loops in double precision. Build flags: -O2 -fopenmp
// -ffp-contract=off, no fast-math.

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace {

const double kPi = 3.14159265358979323846;

enum { OR_SINHSYMTP = 0, OR_SPHERICAL = 1, OR_SINHSPHERICAL = 2, OR_SINHCYLINDRICAL = 3,
       OR_CARTESIAN = 4 };

// Fornberg's algorithm (B. Fornberg, "Generation of finite difference formulas
// on arbitrarily spaced grids", Math. Comp. 51 (1988) 699): weights c[j][k] of
// the k-th derivative at z from samples at x[0..n-1], k = 0..m. Written from
// the recurrences of that paper.
void fornberg_weights(double z, const std::vector<double>& x, int m,
                      std::vector<std::vector<double>>& c) {
  const int n = (int)x.size();
  c.assign(n, std::vector<double>(m + 1, 0.0));
  double c1 = 1.0;
  double c4 = x[0] - z;
  c[0][0] = 1.0;
  for (int i = 1; i < n; ++i) {
    const int mn = std::min(i, m);
    double c2 = 1.0;
    const double c5 = c4;
    c4 = x[i] - z;
    for (int j = 0; j < i; ++j) {
      const double c3 = x[i] - x[j];
      c2 = c2 * c3;
      if (j == i - 1) {
        for (int k = mn; k >= 1; --k)
          c[i][k] = c1 * (k * c[i - 1][k - 1] - c5 * c[i - 1][k]) / c2;
        c[i][0] = -c1 * c5 * c[i - 1][0] / c2;
      }
      for (int k = mn; k >= 1; --k)
        c[j][k] = (c4 * c[j][k] - k * c[j][k - 1]) / c3;
      c[j][0] = c4 * c[j][0] / c3;
    }
    c1 = c2;
  }
}

struct Grid {
  int coords;
  int N[3];
  int NG;
  int Nx[3];
  int fd_order;
  double amax, w, b, rmax;
  double xxmin[3], xxmax[3], dxx[3];
  std::vector<double> xx[3];
  // centred-difference weights for offsets -NG..NG (index k+NG)
  std::vector<double> w1, w2;
  // Laplacian factors on the padded (i0,i1) plane: lap = a0 f,00 + a1 f,11
  // + a2 f,22 + b0 f,0 + b1 f,1
  std::vector<double> a0, a1, a2, b0, b1;
  // local smallest cell width on the padded (i0,i1) plane, and its interior
  // minimum
  std::vector<double> dsmin;
  double ds_g;
  // outer-boundary geometry on the padded (i0,i1) plane (d r / d xx1: the
  // z faces of SinhCylindrical)
  std::vector<double> rcart, drdxx0, drdxx1;
  // SinhCylindrical outer points beyond a z face: 1 where the radiation
  // condition's difference runs along xx1 (|z| >= rho), 0 along xx0
  std::vector<char> along1;
  // radiation condition: order of the one-sided xx0 difference (2 or 4) and
  // its weights for the offsets 0, -1, ..., -order (Fornberg, spacing 1)
  int bc_order = 2;
  std::vector<double> wbc;
  // Cartesian coordinates of every padded point
  std::vector<double> X, Y, Z;
  // constant sources on every padded point
  std::vector<double> psi, ssrc;
  // inner-ghost images: -1 interior, -2 outer, else flat index of image
  std::vector<long> img;
  // state
  std::vector<double> u, v;
  // RK4 work arrays (stage slopes and stage input)
  std::vector<double> k1u, k1v, k2u, k2v, k3u, k3v, k4u, k4v, yu, yv;

  long npad() const { return (long)Nx[0] * Nx[1] * Nx[2]; }
  long idx(int i0, int i1, int i2) const {
    return i0 + (long)Nx[0] * (i1 + (long)Nx[1] * i2);
  }
  long idx2(int i0, int i1) const { return i0 + (long)Nx[0] * i1; }
  bool interior(int i0, int i1, int i2) const {
    return i0 >= NG && i0 < NG + N[0] && i1 >= NG && i1 < NG + N[1] &&
           i2 >= NG && i2 < NG + N[2];
  }
  // stored outer points: beyond xx0's maximum (interior xx1), and for
  // SinhCylindrical also every point beyond either z face with xx0 >= 0; for
  // Cartesian every point beyond exactly one of the six faces (the edge and
  // corner points beyond two or three faces are never read by the star
  // stencil or by a face point's normal difference, and are not evolved)
  bool outer(int i0, int i1, int i2) const {
    if (coords == 4) {
      const int i[3] = {i0, i1, i2};
      int out = 0;
      for (int d = 0; d < 3; ++d) out += (i[d] < NG || i[d] >= NG + N[d]) ? 1 : 0;
      return out == 1;
    }
    if (i2 < NG || i2 >= NG + N[2]) return false;
    const bool in1 = i1 >= NG && i1 < NG + N[1];
    if (coords == 3 && !in1) return i0 >= NG;
    return i0 >= NG + N[0] && in1;
  }
  // outer point on a z face (SinhCylindrical), corners included
  bool zface(int i0, int i1, int i2) const {
    return coords == 3 && outer(i0, i1, i2) && (i1 < NG || i1 >= NG + N[1]);
  }
};

// Sinh-stretched radial map A(xx0) (SinhSymTP's A, SinhSpherical's r) and its
// first two derivatives.
void sinh_radial(const Grid& g, double x0, double& A, double& Ap, double& App) {
  const double s1 = std::sinh(1.0 / g.w);
  A = g.amax * std::sinh(x0 / g.w) / s1;
  Ap = g.amax * std::cosh(x0 / g.w) / (g.w * s1);
  App = A / (g.w * g.w);
}

// Cartesian position of the point with coordinates (x0, x1, x2).
void to_cart(const Grid& g, double x0, double x1, double x2, double& x,
             double& y, double& z) {
  if (g.coords == OR_CARTESIAN) {
    x = x0;
    y = x1;
    z = x2;
  } else if (g.coords == OR_SINHSYMTP) {
    double A, Ap, App;
    sinh_radial(g, x0, A, Ap, App);
    const double R = std::sqrt(A * A + g.b * g.b);
    x = A * std::sin(x1) * std::cos(x2);
    y = A * std::sin(x1) * std::sin(x2);
    z = R * std::cos(x1);
  } else if (g.coords == OR_SINHCYLINDRICAL) {
    double rho, Zc, d1, d2;
    sinh_radial(g, x0, rho, d1, d2);
    sinh_radial(g, x1, Zc, d1, d2);
    x = rho * std::cos(x2);
    y = rho * std::sin(x2);
    z = Zc;
  } else {
    // spherical: r = xx0 (Spherical) or the sinh-stretched A(xx0) (SinhSpherical)
    double r = x0;
    if (g.coords == OR_SINHSPHERICAL) {
      double Ap, App;
      sinh_radial(g, x0, r, Ap, App);
    }
    x = r * std::sin(x1) * std::cos(x2);
    y = r * std::sin(x1) * std::sin(x2);
    z = r * std::cos(x1);
  }
}

// Scale factors h_i (proper length per unit coordinate) and Laplacian factors
// at (x0, x1). The flat metric is diagonal in all three coordinate systems, so
// lap f = sum_i [ f,ii / h_i^2 + (1/J) d_i(J/h_i^2) f,i ],  J = h0 h1 h2.
void metric_at(const Grid& g, double x0, double x1, double h[3], double* a,
               double* bb) {
  const double s = std::sin(x1), c = std::cos(x1);
  if (g.coords == OR_CARTESIAN) {
    // the identity map: unit scale factors, no first-derivative terms
    h[0] = h[1] = h[2] = 1.0;
    if (a) {
      a[0] = a[1] = a[2] = 1.0;
      bb[0] = bb[1] = 0.0;
    }
  } else if (g.coords == OR_SINHSYMTP) {
    double A, Ap, App;
    sinh_radial(g, x0, A, Ap, App);
    const double R2 = A * A + g.b * g.b;
    const double S = A * A + g.b * g.b * s * s;
    h[0] = Ap * std::sqrt(S) / std::sqrt(R2);
    h[1] = std::sqrt(S);
    h[2] = A * s;
    if (a) {
      a[0] = R2 / (Ap * Ap * S);
      a[1] = 1.0 / S;
      a[2] = 1.0 / (A * A * s * s);
      // (1/J) d_0 (J/h0^2) with J/h0^2 = A R sin(x1)/A'
      bb[0] = (2.0 * A * A + g.b * g.b - A * R2 * App / (Ap * Ap)) / (A * Ap * S);
      // (1/J) d_1 (J/h1^2) with J/h1^2 = A A' sin(x1)/R
      bb[1] = c / (s * S);
    }
  } else if (g.coords == OR_SINHCYLINDRICAL) {
    // rho = A(xx0), z = Z(xx1): h = (A', Z', A), J = A' Z' A
    double A, Ap, App, Z, Zp, Zpp;
    sinh_radial(g, x0, A, Ap, App);
    sinh_radial(g, x1, Z, Zp, Zpp);
    h[0] = Ap;
    h[1] = Zp;
    h[2] = A;
    if (a) {
      a[0] = 1.0 / (Ap * Ap);
      a[1] = 1.0 / (Zp * Zp);
      a[2] = 1.0 / (A * A);
      // (1/J) d_0 (J/h0^2), J/h0^2 = Z' A / A': Z' (A'^2 - A A'')/A'^2 / (A' Z' A),
      // with A'^2 - A A'' = (amax / (w sinh(1/w)))^2 exactly (cosh^2 - sinh^2 = 1;
      // the difference itself cancels to a few digits where xx0 >> w)
      const double k = g.amax / (g.w * std::sinh(1.0 / g.w));
      bb[0] = k * k / (Ap * Ap * Ap * A);
      // (1/J) d_1 (J/h1^2), J/h1^2 = A' A / Z': -A' A Z''/Z'^2 / (A' Z' A)
      bb[1] = -Zpp / (Zp * Zp * Zp);
    }
  } else if (g.coords == OR_SINHSPHERICAL) {
    // r = A(xx0): h = (A', A, A sin x1), J = A' A^2 sin x1
    double A, Ap, App;
    sinh_radial(g, x0, A, Ap, App);
    h[0] = Ap;
    h[1] = A;
    h[2] = A * s;
    if (a) {
      a[0] = 1.0 / (Ap * Ap);
      a[1] = 1.0 / (A * A);
      a[2] = 1.0 / (A * A * s * s);
      // (1/J) d_0 (J/h0^2) with J/h0^2 = A^2 sin(x1)/A':
      //   d_0 (A^2/A') = (2 A A'^2 - A^2 A'')/A'^2, divided by A' A^2
      bb[0] = (2.0 * A * Ap * Ap - A * A * App) / (Ap * Ap * Ap * A * A);
      // (1/J) d_1 (J/h1^2), J/h1^2 = A' sin(x1)
      bb[1] = c / (s * A * A);
    }
  } else {
    const double r = x0;
    h[0] = 1.0;
    h[1] = r;
    h[2] = r * s;
    if (a) {
      a[0] = 1.0;
      a[1] = 1.0 / (r * r);
      a[2] = 1.0 / (r * r * s * s);
      bb[0] = 2.0 / r;
      bb[1] = c / (s * r * r);
    }
  }
}

// Image of a padded ghost index: reflections through xx0 = 0, theta = 0 and
// theta = pi (each adds pi to phi), and phi periodicity, applied in that order
// until the index is interior or outer.
long image_of(const Grid& g, int i0, int i1, int i2) {
  const int NG = g.NG, N1 = g.N[1], N2 = g.N[2];
  for (int guard = 0; guard < 8; ++guard) {
    if (i0 < NG) {
      // spherical: theta mirrors; SinhSymTP and SinhCylindrical keep xx1
      if (g.coords == OR_SPHERICAL || g.coords == OR_SINHSPHERICAL)
        i1 = N1 + 2 * NG - 1 - i1;
      i0 = 2 * NG - 1 - i0;
      i2 += N2 / 2;
    } else if (g.coords != OR_SINHCYLINDRICAL && i1 < NG) {
      i1 = 2 * NG - 1 - i1;
      i2 += N2 / 2;
    } else if (g.coords != OR_SINHCYLINDRICAL && i1 >= NG + N1) {
      i1 = 2 * N1 + 2 * NG - 1 - i1;
      i2 += N2 / 2;
    } else if (i2 < NG || i2 >= NG + N2) {
      i2 = NG + (((i2 - NG) % N2) + N2) % N2;
    } else {
      return g.idx(i0, i1, i2);
    }
  }
  return -3;  // unreachable for valid grids
}

void build_grid(Grid& g) {
  g.NG = g.fd_order / 2;
  for (int d = 0; d < 3; ++d) g.Nx[d] = g.N[d] + 2 * g.NG;
  g.xxmin[0] = 0.0;
  g.xxmax[0] = (g.coords == OR_SPHERICAL) ? g.rmax : 1.0;
  g.xxmin[1] = (g.coords == OR_SINHCYLINDRICAL) ? -1.0 : 0.0;
  g.xxmax[1] = (g.coords == OR_SINHCYLINDRICAL) ? 1.0 : kPi;
  g.xxmin[2] = -kPi;
  g.xxmax[2] = kPi;
  if (g.coords == OR_CARTESIAN)   // the cube [-rmax, rmax]^3
    for (int d = 0; d < 3; ++d) {
      g.xxmin[d] = -g.rmax;
      g.xxmax[d] = g.rmax;
    }
  for (int d = 0; d < 3; ++d) {
    g.dxx[d] = (g.xxmax[d] - g.xxmin[d]) / g.N[d];
    g.xx[d].resize(g.Nx[d]);
    for (int j = 0; j < g.Nx[d]; ++j)
      g.xx[d][j] = g.xxmin[d] + (j - g.NG + 0.5) * g.dxx[d];
  }
  // finite-difference weights on offsets -NG..NG
  std::vector<double> off(2 * g.NG + 1);
  for (int k = -g.NG; k <= g.NG; ++k) off[k + g.NG] = (double)k;
  std::vector<std::vector<double>> c;
  fornberg_weights(0.0, off, 2, c);
  g.w1.resize(2 * g.NG + 1);
  g.w2.resize(2 * g.NG + 1);
  for (int j = 0; j < 2 * g.NG + 1; ++j) {
    g.w1[j] = c[j][1];
    g.w2[j] = c[j][2];
  }
  // 2D factors over the padded (i0, i1) plane
  const long n2d = (long)g.Nx[0] * g.Nx[1];
  g.a0.assign(n2d, 0);
  g.a1.assign(n2d, 0);
  g.a2.assign(n2d, 0);
  g.b0.assign(n2d, 0);
  g.b1.assign(n2d, 0);
  g.dsmin.assign(n2d, 0);
  g.rcart.assign(n2d, 0);
  g.drdxx0.assign(n2d, 0);
  g.drdxx1.assign(n2d, 0);
  g.along1.assign(n2d, 0);
  g.ds_g = 1e300;
  for (int i1 = 0; i1 < g.Nx[1]; ++i1)
    for (int i0 = 0; i0 < g.Nx[0]; ++i0) {
      const long k = g.idx2(i0, i1);
      double h[3], a[3], bb[2];
      metric_at(g, g.xx[0][i0], g.xx[1][i1], h, a, bb);
      g.a0[k] = a[0];
      g.a1[k] = a[1];
      g.a2[k] = a[2];
      g.b0[k] = bb[0];
      g.b1[k] = bb[1];
      double ds = std::fabs(h[0]) * g.dxx[0];
      ds = std::min(ds, std::fabs(h[1]) * g.dxx[1]);
      ds = std::min(ds, std::fabs(h[2]) * g.dxx[2]);
      g.dsmin[k] = ds;
      const bool int01 = i0 >= g.NG && i0 < g.NG + g.N[0] && i1 >= g.NG &&
                         i1 < g.NG + g.N[1];
      if (int01) g.ds_g = std::min(g.ds_g, ds);
      // Cartesian radius and d r / d xx0 (independent of phi)
      double x, y, z;
      to_cart(g, g.xx[0][i0], g.xx[1][i1], 0.0, x, y, z);
      const double r = std::sqrt(x * x + y * y + z * z);
      g.rcart[k] = r;
      if (g.coords == OR_SINHSYMTP) {
        double A, Ap, App;
        sinh_radial(g, g.xx[0][i0], A, Ap, App);
        g.drdxx0[k] = A * Ap / r;
      } else if (g.coords == OR_SINHCYLINDRICAL) {
        // r^2 = rho^2 + z^2: dr/dxx0 = rho rho'/r, dr/dxx1 = z z'/r
        double A, Ap, App, Z, Zp, Zpp;
        sinh_radial(g, g.xx[0][i0], A, Ap, App);
        sinh_radial(g, g.xx[1][i1], Z, Zp, Zpp);
        g.drdxx0[k] = Ap * A / r;
        g.drdxx1[k] = Z * Zp / r;
        g.along1[k] = std::fabs(Z) >= A ? 1 : 0;
      } else if (g.coords == OR_SINHSPHERICAL) {
        double A, Ap, App;
        sinh_radial(g, g.xx[0][i0], A, Ap, App);
        g.drdxx0[k] = Ap;
      } else {
        g.drdxx0[k] = 1.0;
      }
    }
  // Cartesian coordinates and ghost images of every padded point
  const long np = g.npad();
  g.X.resize(np);
  g.Y.resize(np);
  g.Z.resize(np);
  g.img.resize(np);
  for (int i2 = 0; i2 < g.Nx[2]; ++i2)
    for (int i1 = 0; i1 < g.Nx[1]; ++i1)
      for (int i0 = 0; i0 < g.Nx[0]; ++i0) {
        const long id = g.idx(i0, i1, i2);
        to_cart(g, g.xx[0][i0], g.xx[1][i1], g.xx[2][i2], g.X[id], g.Y[id],
                g.Z[id]);
        if (g.interior(i0, i1, i2))
          g.img[id] = -1;
        else if (g.outer(i0, i1, i2))
          g.img[id] = -2;
        else if (g.coords == OR_CARTESIAN)
          g.img[id] = -4;   // edge or corner point: never read, not evolved
        else
          g.img[id] = image_of(g, i0, i1, i2);
      }
  g.psi.assign(np, 1.0);
  g.ssrc.assign(np, 0.0);
  g.u.assign(np, 0.0);
  g.v.assign(np, 0.0);
}

// Bowen-York conformal extrinsic curvature A^ij (row-major 3x3) at (x,y,z).
void bowen_york(int n, const double* m, const double* xp, const double* P,
                const double* S, double x, double y, double z, double Aij[9]) {
  (void)m;
  for (int k = 0; k < 9; ++k) Aij[k] = 0.0;
  for (int p = 0; p < n; ++p) {
    const double dx[3] = {x - xp[3 * p], y - xp[3 * p + 1], z - xp[3 * p + 2]};
    const double r = std::sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
    const double nv[3] = {dx[0] / r, dx[1] / r, dx[2] / r};
    const double* Pp = P + 3 * p;
    const double* Sp = S + 3 * p;
    const double Pn = Pp[0] * nv[0] + Pp[1] * nv[1] + Pp[2] * nv[2];
    const double sxn[3] = {Sp[1] * nv[2] - Sp[2] * nv[1],
                           Sp[2] * nv[0] - Sp[0] * nv[2],
                           Sp[0] * nv[1] - Sp[1] * nv[0]};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double delta = (i == j) ? 1.0 : 0.0;
        const double lin = 3.0 / (2.0 * r * r) *
                           (Pp[i] * nv[j] + Pp[j] * nv[i] -
                            (delta - nv[i] * nv[j]) * Pn);
        const double spin = 3.0 / (r * r * r) *
                            (sxn[i] * nv[j] + sxn[j] * nv[i]);
        Aij[3 * i + j] += lin + spin;
      }
  }
}

// Centred first and second derivatives along direction d at padded point
// (i0,i1,i2), in coordinate units.
inline void derivs(const Grid& g, const double* f, int i0, int i1, int i2,
                   int d, double& d1, double& d2) {
  const int NG = g.NG;
  double s1 = 0.0, s2 = 0.0;
  for (int k = -NG; k <= NG; ++k) {
    const int j0 = i0 + (d == 0 ? k : 0);
    const int j1 = i1 + (d == 1 ? k : 0);
    const int j2 = i2 + (d == 2 ? k : 0);
    const double fv = f[g.idx(j0, j1, j2)];
    s1 += g.w1[k + NG] * fv;
    s2 += g.w2[k + NG] * fv;
  }
  d1 = s1 / g.dxx[d];
  d2 = s2 / (g.dxx[d] * g.dxx[d]);
}

inline double laplacian_at(const Grid& g, const double* f, int i0, int i1,
                           int i2) {
  double d1[3], d2[3];
  for (int d = 0; d < 3; ++d) derivs(g, f, i0, i1, i2, d, d1[d], d2[d]);
  const long k = g.idx2(i0, i1);
  return g.a0[k] * d2[0] + g.a1[k] * d2[1] + g.a2[k] * d2[2] +
         g.b0[k] * d1[0] + g.b1[k] * d1[1];
}

// The nonlinear source (1/8) A_ij A^ij (psi_s + u)^-7.
inline double source_at(const Grid& g, long id, double uval) {
  return g.ssrc[id] * std::pow(g.psi[id] + uval, -7.0);
}

// Eq. (5) right-hand side plus boundary conditions, on every padded point.
void rhs(const Grid& g, double eta, double kappa, const double* u,
         const double* v, double* ku, double* kv) {
  const int NG = g.NG;
#pragma omp parallel for collapse(2) schedule(static)
  for (int i2 = NG; i2 < NG + g.N[2]; ++i2)
    for (int i1 = NG; i1 < NG + g.N[1]; ++i1)
      for (int i0 = NG; i0 < NG + g.N[0]; ++i0) {
        const long id = g.idx(i0, i1, i2);
        const long k2 = g.idx2(i0, i1);
        const double c = kappa * g.dsmin[k2] / g.ds_g;
        const double lap = laplacian_at(g, u, i0, i1, i2);
        ku[id] = v[id] - eta * u[id];
        kv[id] = c * c * (lap + source_at(g, id, u[id]));
      }
  // outer points beyond xx0's maximum: radiation condition (Cartesian grids
  // take all six faces below)
  if (g.coords != OR_CARTESIAN)
#pragma omp parallel for collapse(2) schedule(static)
  for (int i2 = NG; i2 < NG + g.N[2]; ++i2)
    for (int i1 = NG; i1 < NG + g.N[1]; ++i1)
      for (int i0 = NG + g.N[0]; i0 < g.Nx[0]; ++i0) {
        const long id = g.idx(i0, i1, i2);
        const long k2 = g.idx2(i0, i1);
        const double c = kappa * g.dsmin[k2] / g.ds_g;
        const double r = g.rcart[k2];
        const double drdx = g.drdxx0[k2];
        double dudx, dvdx;
        if (g.bc_order == 2) {
          const long im1 = g.idx(i0 - 1, i1, i2), im2 = g.idx(i0 - 2, i1, i2);
          dudx = (3.0 * u[id] - 4.0 * u[im1] + u[im2]) / (2.0 * g.dxx[0]);
          dvdx = (3.0 * v[id] - 4.0 * v[im1] + v[im2]) / (2.0 * g.dxx[0]);
        } else {
          dudx = 0.0;
          dvdx = 0.0;
          for (int k = 0; k <= g.bc_order; ++k) {
            const long ik = g.idx(i0 - k, i1, i2);
            dudx += g.wbc[k] * u[ik];
            dvdx += g.wbc[k] * v[ik];
          }
          dudx /= g.dxx[0];
          dvdx /= g.dxx[0];
        }
        ku[id] = -c * (u[id] / r + dudx / drdx);
        kv[id] = -c * (v[id] / r + dvdx / drdx);
      }
  // outer points of the z faces (SinhCylindrical, corners included): the same
  // condition, with the radial derivative from a one-sided difference taken
  // toward the interior along xx1 where |z| >= rho,
  // d_r f = (d f / d xx1) / (d r / d xx1), and along xx0 elsewhere
  if (g.coords == OR_SINHCYLINDRICAL) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int i2 = NG; i2 < NG + g.N[2]; ++i2)
      for (int i1 = 0; i1 < g.Nx[1]; ++i1) {
        if (i1 >= NG && i1 < NG + g.N[1]) continue;
        for (int i0 = NG; i0 < g.Nx[0]; ++i0) {
          const long id = g.idx(i0, i1, i2);
          const long k2 = g.idx2(i0, i1);
          const double c = kappa * g.dsmin[k2] / g.ds_g;
          const double r = g.rcart[k2];
          const bool a1 = g.along1[k2] != 0;
          // outward direction and the index step toward the interior
          const int dir = a1 ? (i1 < NG ? -1 : 1) : 1;
          auto at = [&](int q) {
            return a1 ? g.idx(i0, i1 - q * dir, i2) : g.idx(i0 - q, i1, i2);
          };
          const double h = a1 ? g.dxx[1] : g.dxx[0];
          double dudx = 0.0, dvdx = 0.0;
          if (g.bc_order == 2) {
            dudx = dir * (3.0 * u[id] - 4.0 * u[at(1)] + u[at(2)]) / (2.0 * h);
            dvdx = dir * (3.0 * v[id] - 4.0 * v[at(1)] + v[at(2)]) / (2.0 * h);
          } else {
            for (int q = 0; q <= g.bc_order; ++q) {
              dudx += g.wbc[q] * u[at(q)];
              dvdx += g.wbc[q] * v[at(q)];
            }
            dudx *= dir / h;
            dvdx *= dir / h;
          }
          const double drdx = a1 ? g.drdxx1[k2] : g.drdxx0[k2];
          ku[id] = -c * (u[id] / r + dudx / drdx);
          kv[id] = -c * (v[id] / r + dvdx / drdx);
        }
      }
  }
  // Cartesian face points: the same condition with the radial derivative
  // from a one-sided difference along the face normal d toward the interior,
  // d_r f = (d f / d x_d) / (d r / d x_d), d r / d x_d = x_d / r
  if (g.coords == OR_CARTESIAN) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int i2 = 0; i2 < g.Nx[2]; ++i2)
      for (int i1 = 0; i1 < g.Nx[1]; ++i1)
        for (int i0 = 0; i0 < g.Nx[0]; ++i0) {
          if (!g.outer(i0, i1, i2)) continue;
          const int ii[3] = {i0, i1, i2};
          int d = 0;
          while (ii[d] >= NG && ii[d] < NG + g.N[d]) ++d;
          const int dir = ii[d] < NG ? -1 : 1;   // outward along x_d
          auto at = [&](int q) {
            int j[3] = {i0, i1, i2};
            j[d] -= q * dir;
            return g.idx(j[0], j[1], j[2]);
          };
          const long id = g.idx(i0, i1, i2);
          const double c = kappa * g.dsmin[g.idx2(i0, i1)] / g.ds_g;
          const double x = g.X[id], y = g.Y[id], z = g.Z[id];
          const double r = std::sqrt(x * x + y * y + z * z);
          const double xd = d == 0 ? x : (d == 1 ? y : z);
          const double h = g.dxx[d];
          double dudx = 0.0, dvdx = 0.0;
          if (g.bc_order == 2) {
            dudx = dir * (3.0 * u[id] - 4.0 * u[at(1)] + u[at(2)]) / (2.0 * h);
            dvdx = dir * (3.0 * v[id] - 4.0 * v[at(1)] + v[at(2)]) / (2.0 * h);
          } else {
            for (int q = 0; q <= g.bc_order; ++q) {
              dudx += g.wbc[q] * u[at(q)];
              dvdx += g.wbc[q] * v[at(q)];
            }
            dudx *= dir / h;
            dvdx *= dir / h;
          }
          const double drdx = xd / r;
          ku[id] = -c * (u[id] / r + dudx / drdx);
          kv[id] = -c * (v[id] / r + dvdx / drdx);
        }
  }
  // inner ghosts: copy from images (parity +1)
  const long np = g.npad();
#pragma omp parallel for schedule(static)
  for (long id = 0; id < np; ++id) {
    const long im = g.img[id];
    if (im >= 0) {
      ku[id] = ku[im];
      kv[id] = kv[im];
    }
  }
}

void rk4_step(Grid& g, double eta, double kappa, double dt) {
  const long np = g.npad();
  if ((long)g.yu.size() != np) {
    for (auto* a : {&g.k1u, &g.k1v, &g.k2u, &g.k2v, &g.k3u, &g.k3v, &g.k4u,
                    &g.k4v, &g.yu, &g.yv})
      a->assign(np, 0.0);
  }
  double* u = g.u.data();
  double* v = g.v.data();
  double *k1u = g.k1u.data(), *k1v = g.k1v.data(), *k2u = g.k2u.data(),
         *k2v = g.k2v.data(), *k3u = g.k3u.data(), *k3v = g.k3v.data(),
         *k4u = g.k4u.data(), *k4v = g.k4v.data(), *yu = g.yu.data(),
         *yv = g.yv.data();
  rhs(g, eta, kappa, u, v, k1u, k1v);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < np; ++i) {
    yu[i] = u[i] + 0.5 * dt * k1u[i];
    yv[i] = v[i] + 0.5 * dt * k1v[i];
  }
  rhs(g, eta, kappa, yu, yv, k2u, k2v);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < np; ++i) {
    yu[i] = u[i] + 0.5 * dt * k2u[i];
    yv[i] = v[i] + 0.5 * dt * k2v[i];
  }
  rhs(g, eta, kappa, yu, yv, k3u, k3v);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < np; ++i) {
    yu[i] = u[i] + dt * k3u[i];
    yv[i] = v[i] + dt * k3v[i];
  }
  rhs(g, eta, kappa, yu, yv, k4u, k4v);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < np; ++i) {
    u[i] = u[i] + dt / 6.0 * (k1u[i] + 2.0 * k2u[i] + 2.0 * k3u[i] + k4u[i]);
    v[i] = v[i] + dt / 6.0 * (k1v[i] + 2.0 * k2v[i] + 2.0 * k3v[i] + k4v[i]);
  }
}

// One-sided first-derivative weights of the radiation condition: the
// derivative at offset 0 of the polynomial through the offsets 0, -1, ...,
// -order (unit spacing), order 2 or 4. Order 2 is evaluated in the rhs as
// (3 f0 - 4 f1 + f2) / 2 directly.
bool set_bc_order(Grid& g, int order) {
  if (order != 2 && order != 4) return false;
  if (g.N[0] < order) return false;  // the difference stays on interior points
  if (g.coords == OR_SINHCYLINDRICAL && g.N[1] < order) return false;  // z faces too
  if (g.coords == OR_CARTESIAN && (g.N[1] < order || g.N[2] < order)) return false;
  std::vector<double> off(order + 1);
  for (int k = 0; k <= order; ++k) off[k] = -k;
  std::vector<std::vector<double>> c;
  fornberg_weights(0.0, off, 1, c);
  g.wbc.assign(order + 1, 0.0);
  for (int k = 0; k <= order; ++k) g.wbc[k] = c[k][1];
  g.bc_order = order;
  return true;
}

// Volume-weighted mean of f over the interior cells: sum f J dV / sum J dV
// with J = |h0 h1 h2| at the cell centre and dV = dxx0 dxx1 dxx2 (the
// midpoint rule for the integral of f over the domain, divided by its volume).
// radius > 0 keeps only the cells whose centre lies at a Cartesian distance
// below radius (an integration sphere). With vol_out, also returns the total
// volume sum J dV of the cells taken.
double volume_mean(const Grid& g, const double* f, double radius, double* vol_out) {
  const int NG = g.NG;
  double num = 0.0, den = 0.0;
  const double dV = g.dxx[0] * g.dxx[1] * g.dxx[2];
  for (int i2 = NG; i2 < NG + g.N[2]; ++i2)
    for (int i1 = NG; i1 < NG + g.N[1]; ++i1)
      for (int i0 = NG; i0 < NG + g.N[0]; ++i0) {
        if (radius > 0.0) {
          double x, y, z;
          to_cart(g, g.xx[0][i0], g.xx[1][i1], g.xx[2][i2], x, y, z);
          if (!(std::sqrt(x * x + y * y + z * z) < radius)) continue;
        }
        double h[3];
        metric_at(g, g.xx[0][i0], g.xx[1][i1], h, nullptr, nullptr);
        const double w = std::fabs(h[0] * h[1] * h[2]) * dV;
        num += f[g.idx(i0, i1, i2)] * w;
        den += w;
      }
  if (vol_out) *vol_out = den;
  return num / den;
}

// Hamiltonian-constraint residual H (left-hand side of Eq. 4) on interior
// points, and its grid L2 norm. Partial sums per (i1,i2) row are added in a
// fixed order so the result does not depend on the thread count.
double residual(const Grid& g, const double* u, double* Hout) {
  const int NG = g.NG;
  const int n1 = g.N[1], n2 = g.N[2];
  std::vector<double> rows((size_t)n1 * n2, 0.0);
#pragma omp parallel for collapse(2) schedule(static)
  for (int i2 = NG; i2 < NG + n2; ++i2)
    for (int i1 = NG; i1 < NG + n1; ++i1) {
      double s = 0.0;
      for (int i0 = NG; i0 < NG + g.N[0]; ++i0) {
        const long id = g.idx(i0, i1, i2);
        const double H = laplacian_at(g, u, i0, i1, i2) + source_at(g, id, u[id]);
        if (Hout) Hout[id] = H;
        s += H * H;
      }
      rows[(size_t)(i1 - NG) + (size_t)n1 * (i2 - NG)] = s;
    }
  double tot = 0.0;
  for (double s : rows) tot += s;
  const double nint = (double)g.N[0] * g.N[1] * g.N[2];
  return std::sqrt(tot / nint);
}

}  // namespace

extern "C" {

// Returns NULL on invalid arguments.
void* or_create(int coords, int N0, int N1, int N2, int fd_order, double amax,
                double sinhwaa, double bscale, double rmax) {
  if (coords != OR_SINHSYMTP && coords != OR_SPHERICAL && coords != OR_SINHSPHERICAL &&
      coords != OR_SINHCYLINDRICAL && coords != OR_CARTESIAN)
    return nullptr;
  if (fd_order < 2 || fd_order % 2 || fd_order > 12) return nullptr;
  const int NG = fd_order / 2;
  if (coords == OR_CARTESIAN) {
    // no phi: any N2; every axis carries a face's normal difference
    if (N0 < std::max(NG, 2) || N1 < std::max(NG, 2) || N2 < std::max(NG, 2)) return nullptr;
  } else if (N0 < NG || N1 < NG || N2 < 2 || N2 % 2) {
    return nullptr;
  }
  Grid* g = new Grid();
  g->coords = coords;
  g->N[0] = N0;
  g->N[1] = N1;
  g->N[2] = N2;
  g->fd_order = fd_order;
  g->amax = amax;
  g->w = sinhwaa;
  g->b = bscale;
  g->rmax = rmax;
  build_grid(*g);
  set_bc_order(*g, 2);
  return g;
}

void or_destroy(void* h) { delete (Grid*)h; }

// dims: NG, Nx0, Nx1, Nx2
void or_dims(void* h, int* out) {
  Grid* g = (Grid*)h;
  out[0] = g->NG;
  out[1] = g->Nx[0];
  out[2] = g->Nx[1];
  out[3] = g->Nx[2];
}

void or_xx(void* h, int d, double* out) {
  Grid* g = (Grid*)h;
  std::memcpy(out, g->xx[d].data(), sizeof(double) * g->Nx[d]);
}

void or_dxx(void* h, double* out) {
  Grid* g = (Grid*)h;
  for (int d = 0; d < 3; ++d) out[d] = g->dxx[d];
}

// Cartesian coordinates of all padded points (each npad long).
void or_cart(void* h, double* X, double* Y, double* Z) {
  Grid* g = (Grid*)h;
  const long np = g->npad();
  std::memcpy(X, g->X.data(), sizeof(double) * np);
  std::memcpy(Y, g->Y.data(), sizeof(double) * np);
  std::memcpy(Z, g->Z.data(), sizeof(double) * np);
}

// Laplacian factors a0,a1,a2,b0,b1 and dsmin, each over the padded (i0,i1)
// plane (Nx0*Nx1, i0 fastest), packed one after another into out[6*n2d].
void or_metric(void* h, double* out) {
  Grid* g = (Grid*)h;
  const long n = (long)g->Nx[0] * g->Nx[1];
  const std::vector<double>* arr[6] = {&g->a0, &g->a1, &g->a2,
                                       &g->b0, &g->b1, &g->dsmin};
  for (int a = 0; a < 6; ++a)
    std::memcpy(out + a * n, arr[a]->data(), sizeof(double) * n);
}

// Scale factors h0,h1,h2 at arbitrary coordinates (for tests).
void or_scale_factors(void* h, double x0, double x1, double* hout) {
  metric_at(*(Grid*)h, x0, x1, hout, nullptr, nullptr);
}

void or_to_cart(void* h, double x0, double x1, double x2, double* out) {
  to_cart(*(Grid*)h, x0, x1, x2, out[0], out[1], out[2]);
}

double or_ds_g(void* h) { return ((Grid*)h)->ds_g; }

double or_suggest_dt(void* h, double cfl) { return cfl * ((Grid*)h)->ds_g; }

// Centred finite-difference weights for offsets -NG..NG (2*NG+1 values each).
int or_fd_weights(int fd_order, double* w1, double* w2) {
  if (fd_order < 2 || fd_order % 2 || fd_order > 12) return -1;
  const int NG = fd_order / 2;
  std::vector<double> off(2 * NG + 1);
  for (int k = -NG; k <= NG; ++k) off[k + NG] = (double)k;
  std::vector<std::vector<double>> c;
  fornberg_weights(0.0, off, 2, c);
  for (int j = 0; j < 2 * NG + 1; ++j) {
    w1[j] = c[j][1];
    w2[j] = c[j][2];
  }
  return 0;
}

// Generic Fornberg weights (for tests): z, x[n], derivative order m;
// out[(m+1)*n], derivative-major.
void or_fornberg(double z, const double* x, int n, int m, double* out) {
  std::vector<double> xs(x, x + n);
  std::vector<std::vector<double>> c;
  fornberg_weights(z, xs, m, c);
  for (int k = 0; k <= m; ++k)
    for (int j = 0; j < n; ++j) out[k * n + j] = c[j][k];
}

// Bowen-York A^ij at npts points (pts: 3*npts), out: 9*npts.
void or_bowen_york(int n, const double* m, const double* xp, const double* P,
                   const double* S, const double* pts, long npts, double* out) {
  for (long i = 0; i < npts; ++i)
    bowen_york(n, m, xp, P, S, pts[3 * i], pts[3 * i + 1], pts[3 * i + 2],
               out + 9 * i);
}

// Sources on every padded point; resets u = v = 0.
int or_set_punctures(void* h, int n, const double* m, const double* xp,
                     const double* P, const double* S) {
  Grid* g = (Grid*)h;
  const long np = g->npad();
#pragma omp parallel for schedule(static)
  for (long id = 0; id < np; ++id) {
    double psi = 1.0;
    for (int p = 0; p < n; ++p) {
      const double dx = g->X[id] - xp[3 * p], dy = g->Y[id] - xp[3 * p + 1],
                   dz = g->Z[id] - xp[3 * p + 2];
      const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
      psi += m[p] / (2.0 * r);
    }
    double A[9];
    bowen_york(n, m, xp, P, S, g->X[id], g->Y[id], g->Z[id], A);
    double aa = 0.0;
    for (int k = 0; k < 9; ++k) aa += A[k] * A[k];
    g->psi[id] = psi;
    g->ssrc[id] = aa / 8.0;
  }
  std::fill(g->u.begin(), g->u.end(), 0.0);
  std::fill(g->v.begin(), g->v.end(), 0.0);
  return 0;
}

void or_get_sources(void* h, double* psi, double* ssrc) {
  Grid* g = (Grid*)h;
  const long np = g->npad();
  std::memcpy(psi, g->psi.data(), sizeof(double) * np);
  std::memcpy(ssrc, g->ssrc.data(), sizeof(double) * np);
}

void or_bc_images(void* h, long* out) {
  Grid* g = (Grid*)h;
  std::memcpy(out, g->img.data(), sizeof(long) * g->npad());
}

void or_set_state(void* h, const double* u, const double* v) {
  Grid* g = (Grid*)h;
  const long np = g->npad();
  std::memcpy(g->u.data(), u, sizeof(double) * np);
  std::memcpy(g->v.data(), v, sizeof(double) * np);
}

void or_get_state(void* h, double* u, double* v) {
  Grid* g = (Grid*)h;
  const long np = g->npad();
  std::memcpy(u, g->u.data(), sizeof(double) * np);
  std::memcpy(v, g->v.data(), sizeof(double) * np);
}

// Copy every inner ghost from its image (warm starts and tests).
void or_fill_ghosts(void* h, double* f) {
  Grid* g = (Grid*)h;
  const long np = g->npad();
  for (long id = 0; id < np; ++id)
    if (g->img[id] >= 0) f[id] = f[g->img[id]];
}

// Laplacian of a padded grid function on the interior (other points: 0).
void or_laplacian(void* h, const double* f, double* out) {
  Grid* g = (Grid*)h;
  const int NG = g->NG;
  std::fill(out, out + g->npad(), 0.0);
#pragma omp parallel for collapse(2) schedule(static)
  for (int i2 = NG; i2 < NG + g->N[2]; ++i2)
    for (int i1 = NG; i1 < NG + g->N[1]; ++i1)
      for (int i0 = NG; i0 < NG + g->N[0]; ++i0)
        out[g->idx(i0, i1, i2)] = laplacian_at(*g, f, i0, i1, i2);
}

void or_rhs(void* h, double eta, double kappa, const double* u,
            const double* v, double* ku, double* kv) {
  Grid* g = (Grid*)h;
  std::fill(ku, ku + g->npad(), 0.0);
  std::fill(kv, kv + g->npad(), 0.0);
  rhs(*g, eta, kappa, u, v, ku, kv);
}

// Residual of the current state (Hout may be NULL).
double or_residual(void* h, double* Hout) {
  Grid* g = (Grid*)h;
  if (Hout) std::fill(Hout, Hout + g->npad(), 0.0);
  return residual(*g, g->u.data(), Hout);
}

// sum f J dV / sum J dV over the interior cells within radius (all if
// radius <= 0; f padded); *vol = sum J dV.
double or_volume_mean(void* h, const double* f, double radius, double* vol) {
  return volume_mean(*static_cast<Grid*>(h), f, radius, vol);
}

// Volume-weighted residual norm sqrt(sum H^2 J dV / sum J dV) of the state,
// over the cells within radius (all if radius <= 0).
double or_residual_volume(void* h, double radius) {
  Grid& g = *static_cast<Grid*>(h);
  std::vector<double> H(g.npad(), 0.0);
  residual(g, g.u.data(), H.data());
  for (double& x : H) x = x * x;
  return std::sqrt(volume_mean(g, H.data(), radius, nullptr));
}

double or_residual_of(void* h, const double* u, double* Hout) {
  Grid* g = (Grid*)h;
  if (Hout) std::fill(Hout, Hout + g->npad(), 0.0);
  return residual(*g, u, Hout);
}

void or_rk4_steps(void* h, double eta, double kappa, double dt, long nsteps) {
  Grid* g = (Grid*)h;
  for (long s = 0; s < nsteps; ++s) rk4_step(*g, eta, kappa, dt);
}

// Relaxation loop: RK4 steps; after every check_every steps the residual is
// recorded into hist (if not NULL, capacity hist_cap) and the loop stops when
// it is not finite (return 2) or, for tol > 0, when it falls below tol
// (return 0). With tol > 0 and the cap reached, returns 1; with tol <= 0,
// returns 0 after n_steps. steps_taken and n_hist report progress.
int or_relax(void* h, double eta, double kappa, double dt, long n_steps,
             double tol, long check_every, double* hist, long hist_cap,
             long* steps_taken, long* n_hist) {
  Grid* g = (Grid*)h;
  long nh = 0;
  long s = 0;
  int status = (tol > 0) ? 1 : 0;
  while (s < n_steps) {
    rk4_step(*g, eta, kappa, dt);
    ++s;
    if (check_every > 0 && s % check_every == 0) {
      const double res = residual(*g, g->u.data(), nullptr);
      if (hist && nh < hist_cap) hist[nh] = res;
      ++nh;
      if (!std::isfinite(res)) {
        status = 2;
        break;
      }
      if (tol > 0 && res < tol) {
        status = 0;
        break;
      }
    }
  }
  if (steps_taken) *steps_taken = s;
  if (n_hist) *n_hist = nh;
  return status;
}

// Order (2 or 4) of the one-sided xx0 difference in the radiation
// condition; returns 0, or -1 for another order.
int or_set_bc_order(void* h, int order) {
  return set_bc_order(*static_cast<Grid*>(h), order) ? 0 : -1;
}

int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

}  // extern "C"
