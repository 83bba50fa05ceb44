// Internal declarations of the hyperbolic-relaxation library: the grid
// handle, the device workspace layout and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/hrelax.h"

namespace hr {

constexpr int kBlock = 256;        // threads per block for every grid kernel
constexpr int kMaxPunctures = 4;

// Puncture parameters, passed by value to the source kernel.
struct Punctures {
  int n;
  double m[kMaxPunctures];
  double x[kMaxPunctures][3];
  double P[kMaxPunctures][3];
  double S[kMaxPunctures][3];
};

// One precision's set of grid functions and coefficient tables.
template <typename T>
struct Fields {
  T* un;    // state y_n: u
  T* vn;    //            v
  T* ua;    // stage input/output ping-pong buffer A
  T* va;
  T* ub;    // stage input/output ping-pong buffer B
  T* vb;
  T* au;    // RK4 accumulator
  T* av;
  T* psi;   // psi_singular
  T* ssrc;  // (1/8) A_ij A^ij
  T* fac;   // 6 planes of N0*N1: alpha0, alpha1, alpha2, beta0, beta1, c^2
  T* ofac;  // 3 planes of NG*N1: c, 1/r, 1/(2 dxx0 dr/dxx0)
};

// Geometry of one grid, shared by every kernel launch on it.
struct Dims {
  int N0, N1, N2;  // interior points
  int NG;          // ghost depth = fd_order / 2
  int P0;          // row length of the extended layout, N0 + NG
  int nint;        // N0*N1*N2
  int nout;        // NG*N1*N2
  int sph;         // 1 for Spherical (x0 reflection also flips theta)
};

// Stage kernel arguments (RK4 stage s of 4, classic Butcher tableau).
template <typename T>
struct StageArgs {
  Dims d;
  const T* uin;   // stage input Y_s
  const T* vin;
  const T* un;    // y_n (stages 2, 3)
  const T* vn;
  T* au;          // accumulator
  T* av;
  T* uout;        // Y_{s+1} (stages 1-3) or y_{n+1} (stage 4)
  T* vout;
  const T* psi;
  const T* ssrc;
  const T* fac;
  const T* ofac;
  T eta;
  T cy;           // Y_{s+1} = y_n + cy * k   (cy = dt/2, dt/2, dt)
  T ca;           // acc weight (dt/6, dt/3, dt/3, dt/6)
  int streaming;  // 1: non-temporal access to fields touched once per stage
  int variant;    // 1: plane tiles, 2: phi-marching columns
  int chunk;      // phi planes per block (variant 2)
};

struct ResidualArgs {
  Dims d;
  const void* u;        // state u (double or float)
  const double* psi;
  const double* ssrc;
  const double* fac;    // FP64 table (alpha/beta planes used)
  double* partial;      // one per block
};

// Launchers (hr_kernels.hip). All return the hipError_t of the launch.
// Stage launches; with non-null t0/t1 the dispatch records those events
// around the kernel itself (used for timing).
hipError_t launch_stage(int order, int stage, const StageArgs<double>& a,
                        hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_stage(int order, int stage, const StageArgs<float>& a,
                        hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
// Number of partial sums (blocks) the residual kernel writes for these dims.
int residual_blocks(const Dims& d);
hipError_t launch_residual(int order, bool fp32_state, const ResidualArgs& a,
                           hipStream_t s);
hipError_t launch_finalize(const double* partial, int nparts, int nint,
                           double* out, hipStream_t s);
hipError_t launch_sources(const Dims& d, const double* rho, const double* zc,
                          const double* cphi, const double* sphi,
                          const Punctures& p, double* psi64, double* ssrc64,
                          float* psi32, float* ssrc32, hipStream_t s);
hipError_t launch_to_fp32(const double* src, float* dst, int n, hipStream_t s);
hipError_t launch_to_fp64(const float* src, double* dst, int n, hipStream_t s);
hipError_t launch_fill(double* dst, double value, int n, hipStream_t s);
hipError_t launch_fill(float* dst, float value, int n, hipStream_t s);

// Host geometry (hr_geometry.cpp).
struct HostTables {
  double ds_g;                 // smallest proper cell width over the interior
  std::vector<double> alpha;   // 5 planes of N0*N1: a_i/dxx_i^2 (3), b_i/dxx_i (2)
  std::vector<double> crat;    // N0*N1: ds_min/ds_g at interior (i0,i1)
  std::vector<double> ocrat;   // NG*N1: ds_min/ds_g at outer (i0,i1)
  std::vector<double> orinv;   // NG*N1: 1/r
  std::vector<double> oq;      // NG*N1: 1/(2 dxx0 dr/dxx0)
  std::vector<double> rho;     // P0*N1: cylindrical radius at phi = 0
  std::vector<double> zc;      // P0*N1: z
  std::vector<double> rcart;   // P0*N1: Cartesian radius
  std::vector<double> cphi;    // N2
  std::vector<double> sphi;    // N2
};

bool build_tables(hr_coords coords, const Dims& d, const hr_grid_params& p,
                  HostTables& t, std::string& err);

void set_error(const std::string& msg);

}  // namespace hr

struct hr_grid {
  hr_coords coords;
  int fd_order;
  hr_grid_params prm;
  hr::Dims d;
  hr::HostTables tab;
  size_t G;             // elements reserved per grid function (aligned)
  int nblk_res;         // residual partial-sum blocks

  // device binding
  bool bound = false;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  hr::Fields<double> f64{};
  hr::Fields<float> f32{};
  double* rho = nullptr;   // device copies of the coordinate tables
  double* zc = nullptr;
  double* cphi = nullptr;
  double* sphi = nullptr;
  double* partial = nullptr;
  double* result = nullptr;
  double* host_res = nullptr;   // pinned readback slot
  bool have_sources = false;
  double kappa_loaded = -1.0;   // wave-speed scale currently in fac/ofac

  int variant = 0;              // kernel variant: 0 auto, 1 plane tiles, 2 phi columns
  int streaming = -1;           // non-temporal field access: -1 auto (by size), 0, 1
  int chunk = 0;                // phi planes per block of the column variant (0 auto)

  // FP32 -> FP64 switch rule
  double sw_residual = 1e-6;
  int sw_stall = 2;
  long sw_max_steps = 0;
};
