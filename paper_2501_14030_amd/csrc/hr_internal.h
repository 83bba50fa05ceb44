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
  T* zfac;  // SinhCylindrical z faces, 4 planes of P0*2NG (lower rows, then
            // upper): c, 1/r, q = +-1/(2 dxx dr/dxx) of the point's difference
            // direction (sign: outward), and the index step to the next point
            // toward the interior (+-P0 along xx1, -1 along xx0)
  // split-state single-precision form (FP32 set only): slopes of the FP64 base
  // state, base p = psi_s + u_base and S_src p^-7
  T* khu;
  T* khv;
  T* pb;
  T* sp7;
  // bfloat16 copy of the six factor planes (FP32 set only), read by the
  // single-precision stages when 16-bit factor storage is selected
  unsigned short* facb;
};

// Geometry of one grid, shared by every kernel launch on it.
struct Dims {
  int N0, N1, N2;  // interior points
  int NG;          // ghost depth = fd_order / 2
  int P0;          // row length of the extended layout, N0 + NG
  int nint;        // N0*N1*N2
  int nout;        // NG*N1*N2
  int sph;         // 1 for Spherical (x0 reflection also flips theta)
  int zo;          // stored outer rows on each x1 face: NG for SinhCylindrical
                   // (its z faces are outer boundaries) and Cartesian, else 0
  int R1;          // stored rows per plane, N1 + 2 zo
  int cart;        // 1 for Cartesian: NG stored outer layers beyond all six
                   // faces (P0 = N0 + 2 NG, planes N2 + 2 NG), no images
};

// Stored planes of a grid: N2, plus the two outer slabs of a Cartesian grid.
__host__ __device__ __forceinline__ int planes_of(const Dims& d) {
  return d.N2 + (d.cart ? 2 * d.NG : 0);
}

// Flat index of the stored point (i0, i1, i2): i0 in [0, P0) (Cartesian:
// [-NG, N0 + NG)), i1 in [-zo, N1 + zo), i2 in [0, N2) (Cartesian:
// [-NG, N2 + NG)).
__host__ __device__ __forceinline__ unsigned sidx(const Dims& d, int i0, int i1, int i2) {
  const int o = d.cart ? d.NG : 0;
  return (unsigned)(i0 + o) +
         (unsigned)d.P0 * ((unsigned)(i1 + d.zo) + (unsigned)d.R1 * (unsigned)(i2 + o));
}

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
  // split-state form: the state is an increment e on an FP64 base y_b and the
  // slope is k(y_b) + L e + S_src [(p_b + e_u)^-7 - p_b^-7]; psi/ssrc then hold
  // p_b and S_src p_b^-7
  int corr;
  const T* khu;
  const T* khv;
  int bc4;        // fourth-order one-sided difference in the radiation condition
  const unsigned short* facb;  // bfloat16 factor planes (replace fac when set)
  const T* zfac;  // z-face planes (SinhCylindrical, d.zo > 0)
};

// Base-state slopes for the split-state form (FP64 in, FP32 out).
struct BaseArgs {
  Dims d;
  const double* u;
  const double* v;
  const double* psi;
  const double* ssrc;
  const double* fac;
  const double* ofac;
  double eta;
  float* khu;
  float* khv;
  float* pb;
  float* sp7;
  float* eu;   // increment state, zeroed
  float* ev;
  int bc4;     // fourth-order one-sided difference in the radiation condition
  const double* zfac;  // z-face planes (SinhCylindrical)
};

struct ResidualArgs {
  Dims d;
  const void* u;        // state u (double or float)
  const double* psi;
  const double* ssrc;
  const double* fac;    // FP64 table (alpha/beta planes used)
  const double* wt;     // N0*N1 cell volumes (volume-weighted norm) or null
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
// out[0] = sqrt(sum(partial) / divisor), out[1] = sum(partial).
hipError_t launch_finalize(const double* partial, int nparts, double divisor,
                           double* out, hipStream_t s);
hipError_t launch_sources(const Dims& d, const double* rho, const double* zc,
                          const double* cphi, const double* sphi,
                          const Punctures& p, double* psi64, double* ssrc64,
                          float* psi32, float* ssrc32, hipStream_t s);
// Sources at every stored point of a Cartesian grid; cx holds the stored
// columns' x, rows' y and planes' z (the grid's coordinate table).
hipError_t launch_cart_sources(const Dims& d, const double* cx, const Punctures& p,
                               double* psi64, double* ssrc64, float* psi32, float* ssrc32,
                               hipStream_t s);
hipError_t launch_to_fp32(const double* src, float* dst, int n, hipStream_t s);
hipError_t launch_to_fp64(const float* src, double* dst, int n, hipStream_t s);
struct RebaseArgs {
  double* ub;
  double* vb;
  const float* eu;
  const float* ev;
  int n;
};

hipError_t launch_base(int order, const BaseArgs& a, hipStream_t s);

// Batched launchers: persistent grids walking device work lists whose lengths
// are read from device memory (*nitems). Stage items are (grid, x0 tile,
// x1 tile, phi chunk); residual and base items (grid, x0 tile, x1 tile,
// plane); rebase items (grid, element block). descs of the stage launcher
// are StageArgs<float> (split form) or StageArgs<double>, four per grid.
// zfaces: some grid of the batch stores outer rows on its x1 faces
// (SinhCylindrical); the kernels then run the instances that handle them.
hipError_t launch_batch_stage(int order, int stage, bool fp32_split, bool zfaces,
                              const void* descs, const int4* items, const int* nitems,
                              int nblocks_persistent, hipStream_t s);
hipError_t launch_batch_residual(int order, bool zfaces, const ResidualArgs* descs,
                                 const int4* items, const int* nitems, double* partial,
                                 int nblocks_persistent, hipStream_t s);
hipError_t launch_batch_finalize(const int4* ranges, const double* partial, double* out,
                                 int ngrids, hipStream_t s);
hipError_t launch_batch_base(int order, bool zfaces, const BaseArgs* descs, const int4* items,
                             const int* nitems, int nblocks_persistent, hipStream_t s);
hipError_t launch_batch_rebase(const RebaseArgs* descs, const int2* items, const int* nitems,
                               int nblocks_persistent, hipStream_t s);
// y_b += e over n stored elements (FP64 += FP32), both fields.
hipError_t launch_rebase(double* ub, double* vb, const float* eu, const float* ev, int n,
                         hipStream_t s);
hipError_t launch_fill(double* dst, double value, int n, hipStream_t s);
// dst = a * src over n values.
hipError_t launch_scale(double* dst, const double* src, double a, int n, hipStream_t s);
hipError_t launch_fill(float* dst, float value, int n, hipStream_t s);

// Resident RK4 kernel (hr_resident.hip): one launch runs nsteps
// whole RK4 steps of a small grid with the state held on chip. Every block owns
// an 8 x 8 patch of (x0, x1) columns over all phi planes (the last x0 patch also
// the outer points), keeps y_n, the stage input and the accumulator of its
// points in registers, and exchanges the stage input u with the blocks whose
// points its stencils reach through a double-buffered global array, ordered by
// per-block stage counters.
constexpr int kResPatch = 8;          // patch width along x0 and x1
// Stage-kernel tile: one wavefront along x0 times kTileY rows along x1.
constexpr int kTileX = 64;
constexpr int kTileY = 8;
constexpr int kResMaxWait = 16;       // blocks one block exchanges with, at most
constexpr int kResFlagStride = 32;    // one 128-byte line per block counter
constexpr int kResMaxBlocks = 1024;

// T = double: the FP64 state. T = float: the split-state form's FP32
// increment e on the FP64 base (psi/ssrc then hold p_b and S_src p_b^-7, and
// khu/khv the base slopes k(y_b); the slope is k(y_b) + L e + source
// difference, as in the stage kernels).
template <typename T>
struct ResidentArgsT {
  Dims d;
  T* u;                 // state (extended layout), read at start, written at the end
  T* v;
  const T* psi;
  const T* ssrc;
  const T* khu;         // split form only
  const T* khv;
  const T* fac;         // 6 planes of N0*N1
  const T* ofac;        // 3 planes of NG*N1
  T* x0;                // exchange buffers (extended layout), by stage parity
  T* x1;
  unsigned* flags;      // per-block stage counters, zero at launch
  const int* waits;     // per block: count, then up to kResMaxWait block ids
  unsigned* err;        // bit 0: a wait timed out
  T eta;
  T cy[4];              // Y_{s+1} = y_n + cy[s] k (stage 4: y_{n+1} = acc + ca[3] k)
  T ca[4];              // accumulator weights
  int nbx, nby;         // patches along x0 and x1
  int ry;               // patch rows along x1 (8 or 4; 8 columns along x0)
  int nsteps;
  unsigned spin_limit;  // polls of one counter before a wait gives up
  int bc4;              // fourth-order one-sided difference in the radiation condition
  const unsigned short* facb;  // bfloat16 factor planes (replace fac when set)
  int block0;           // first block of this grid in a multi-grid launch (else 0)
};
using ResidentArgs = ResidentArgsT<double>;

// Exchange partners of every patch (count, then ids; kResMaxWait + 1 ints per
// block) for dims d: the owners of every stencil tap outside the patch,
// including inner-boundary images, and every patch whose taps reach this one.
// Patches are 8 columns (x0) by ry = 8 or 4 rows (x1). False if the grid is
// not made of whole patches or has too many blocks.
bool resident_plan(const Dims& d, int ry, std::vector<int>& waits, int& nbx, int& nby);
// Dynamic LDS bytes of the resident kernel for these dims, element size and
// patch rows (at least enough to keep one block per compute unit).
size_t resident_lds_bytes(const Dims& d, size_t elem, int ry);
// Largest number of co-resident blocks of the resident kernel (FP64 form, or
// the split form with split = true) on the current device for these dims and
// patch rows (0 if the order or N2 is not supported).
int resident_capacity(int order, const Dims& d, bool split, int ry);
// Resets the counters and launches the resident kernel (one block per
// compute unit, all resident at once); events (optional) bracket the kernel.
hipError_t launch_resident(int order, const ResidentArgsT<double>& a, hipStream_t s,
                           hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_resident(int order, const ResidentArgsT<float>& a, hipStream_t s,
                           hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
// Several grids in one resident launch: host_tab[i] is a host copy of
// dev_tab[i] (which must be in device memory, in stream order, before the
// launch) and describes grid i, whose blocks start at host_tab[i].block0, the
// sum of the earlier grids' patches. All grids take the same kernel instance
// (order, patch rows and plane group: resident_kernel_key); each keeps its own
// counters (zeroed here), partners and exchange buffers.
hipError_t launch_resident_multi(int order, const ResidentArgsT<double>* dev_tab,
                                 const ResidentArgsT<double>* host_tab, int n, hipStream_t s);
hipError_t launch_resident_multi(int order, const ResidentArgsT<float>* dev_tab,
                                 const ResidentArgsT<float>* host_tab, int n, hipStream_t s);
// Identifies the kernel instance of a grid with N2 planes (null: none); grids
// with equal keys can share a launch.
const void* resident_kernel_key(int order, int N2, bool split, int ry);
// Co-resident blocks of a multi-grid launch of that instance with lds bytes of
// LDS per block (the largest of its grids').
int resident_multi_capacity(int order, int N2, bool split, int ry, size_t lds);

// Host geometry (hr_geometry.cpp).
struct HostTables {
  double ds_g;                 // smallest proper cell width over the interior
  std::vector<double> alpha;   // 5 planes of N0*N1: a_i/dxx_i^2 (3), b_i/dxx_i (2)
  std::vector<double> crat;    // N0*N1: ds_min/ds_g at interior (i0,i1)
  std::vector<double> ocrat;   // NG*N1: ds_min/ds_g at outer (i0,i1)
  std::vector<double> orinv;   // NG*N1: 1/r
  std::vector<double> oq;      // NG*N1: 1/(2 dxx0 dr/dxx0)
  std::vector<double> zcrat;   // P0*2NG (SinhCylindrical z faces): ds_min/ds_g
  std::vector<double> zrinv;   // P0*2NG: 1/r
  std::vector<double> zq;      // P0*2NG: +-1/(2 dxx dr/dxx), outward sign
  std::vector<double> zstep;   // P0*2NG: index step toward the interior: +-P0
                               // (along xx1, where |z| >= rho), -1 (along xx0)
  std::vector<double> rho;     // P0*R1: cylindrical radius at phi = 0
  std::vector<double> zc;      // P0*R1: z
  std::vector<double> rcart;   // P0*R1: Cartesian radius
  std::vector<double> cphi;    // N2
  std::vector<double> sphi;    // N2
  std::vector<double> vol;     // N0*N1: cell volume |h0 h1 h2| dxx0 dxx1 dxx2 (any plane)
  double vol_total = 0.0;      // sum of the cell volumes over the interior
  std::vector<double> volw;    // N0*N1: weights of the volume norm (vol, zero for cells
                               // whose centre lies beyond the integration radius)
  double volw_total = 0.0;     // sum of the weights over the interior
  std::vector<double> cx;      // Cartesian: x of the P0 stored columns, y of the R1
                               // stored rows, z of the N2 + 2 NG stored planes
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
  double* vol = nullptr;        // device copy of the cell volumes (N0*N1)
  double* partial = nullptr;
  double* result = nullptr;
  double* host_res = nullptr;   // pinned readback slot
  bool have_sources = false;
  hr::Punctures pz{};           // punctures of the last hr_set_punctures
  double kappa_loaded = -1.0;   // wave-speed scale currently in fac/ofac

  int norm = 0;                 // residual norm: 0 over points, 1 volume-weighted
  double norm_radius = 0.0;     // integration radius of the volume norm (<= 0: whole grid)
  int bc_order = 2;             // one-sided difference order of the radiation condition
  int factors16 = 0;            // single-precision stages read bfloat16 factor planes
  int variant = 0;              // kernel variant: 0 auto, 1 plane tiles, 2 phi columns,
                                // 3 resident (FP64 steps in one launch, state on chip)
  // resident-kernel partitions, [0]: 8 x 8 patches, [1]: 8 x 4 patches
  struct ResPlan {
    int ry = 8;
    int nbx = 0, nby = 0;       // patches (0: grid not eligible)
    int cap = 0, cap32 = 0;     // co-resident blocks the device allows (FP64, split FP32)
    std::vector<int> plan;      // exchange partners (host copy, uploaded at bind)
    int* waits = nullptr;       // device copy
    int blocks() const { return nbx * nby; }
  } res[2];
  unsigned res_wait_limit = 1u << 19;  // polls of one partner counter before giving up
  bool res_off = false;         // resident launches off for the rest of this hr_relax call
                                // (a resident launch's exchange wait timed out)
  long res_fallbacks = 0;       // intervals rerun on the stage kernels in this call
  unsigned* res_flags = nullptr;  // stage counters, sized for the larger partition
  unsigned* res_err = nullptr;
  int streaming = -1;           // non-temporal field access: -1 auto (by size), 0, 1
  int chunk = 0;                // phi planes per block of the column variant (0 auto)
  int graph = -1;               // graph capture of check intervals: -1 auto (on), 0, 1
  hipGraphExec_t gexec = nullptr;  // captured check interval and its key
  int g_kind = -1, g_K = 0, g_variant = 0, g_chunk = 0, g_streaming = 0, g_norm = 0, g_bc = 2,
      g_f16 = 0;
  double g_eta = 0, g_dt = 0, g_kappa = 0, g_norm_radius = 0;

  // FP32 -> FP64 switch rule (sw_residual 0: ten times the tolerance)
  double sw_residual = 0.0;
  int sw_stall = 8;
  long sw_max_steps = 0;

  // Durations of the resident launches that hr_relax issues
  // (hr_set_launch_timing): one event pair per launch, recorded inside the
  // dispatch, read after the interval's synchronisation.
  int time_launches = 0;
  std::vector<hipEvent_t> tev;  // event pairs (2 per launch), created on demand, reused
  int tev_used = 0;             // pairs recorded and not yet read
  long tev_stages[8] = {};      // RK stages run by each recorded launch
  double t_us = 0.0;            // summed launch durations
  long t_launches = 0;
  long t_stages = 0;
};

namespace hr {

// Kernel variant and phi chunk of a grid (explicit configuration, else by size;
// the automatic chunk also by precision: fp64 for the FP64 stage kernels).
// Variant 3 (resident) applies to FP64 steps only; stage launches of the
// single-precision forms use plane tiles in its place.
void resolve_variant(const hr_grid* g, int& variant, int& chunk, bool fp64 = true);
// The grid can run the resident kernel on its device.
bool resident_ok(const hr_grid* g);

// Uploads the wave-speed planes (c, c^2) for scale kappa if not loaded (synchronous).
hr_status load_kappa(hr_grid* g, double kappa);

// Resident-kernel arguments of grid g with patch partition p: the FP64 state,
// or the split form's FP32 increment on its FP64 base (hr_abi.hip).
ResidentArgsT<double> resident_args_part(hr_grid* g, const hr_grid::ResPlan* p, double eta,
                                         double dt, int nsteps);
ResidentArgsT<float> resident_args_split_part(hr_grid* g, const hr_grid::ResPlan* p, float eta,
                                              float dt, int nsteps);
// Partition with which grid g runs resident in a batch (null: stage kernels).
const hr_grid::ResPlan* batch_resident_part(const hr_grid* g, bool split);

// Stage-s arguments of grid g in precision T; corr selects the split-state form.
template <typename T>
StageArgs<T> stage_args(const hr_grid* g, const Fields<T>& F, int stage, T eta, T dt,
                        bool corr = false) {
  StageArgs<T> a{};
  a.d = g->d;
  a.psi = corr ? F.pb : F.psi;
  a.ssrc = corr ? F.sp7 : F.ssrc;
  a.corr = corr ? 1 : 0;
  a.khu = F.khu;
  a.khv = F.khv;
  a.fac = F.fac;
  a.ofac = F.ofac;
  a.zfac = F.zfac;
  a.eta = eta;
  a.bc4 = g->bc_order == 4 ? 1 : 0;
  a.facb = g->factors16 ? F.facb : nullptr;
  // non-temporal access measured no faster at any size: off unless asked for
  a.streaming = g->streaming > 0 ? 1 : 0;
  resolve_variant(g, a.variant, a.chunk, sizeof(T) == 8);
  if (a.variant == 3) a.variant = 1;
  a.un = F.un;
  a.vn = F.vn;
  a.au = F.au;
  a.av = F.av;
  switch (stage) {
    case 1:  // Y1 = y_n -> A
      a.uin = F.un; a.vin = F.vn; a.uout = F.ua; a.vout = F.va;
      a.cy = dt / (T)2; a.ca = dt / (T)6;
      break;
    case 2:  // A -> B
      a.uin = F.ua; a.vin = F.va; a.uout = F.ub; a.vout = F.vb;
      a.cy = dt / (T)2; a.ca = dt / (T)3;
      break;
    case 3:  // B -> A
      a.uin = F.ub; a.vin = F.vb; a.uout = F.ua; a.vout = F.va;
      a.cy = dt; a.ca = dt / (T)3;
      break;
    default:  // A, acc -> y_{n+1}
      a.uin = F.ua; a.vin = F.va; a.uout = F.un; a.vout = F.vn;
      a.cy = dt; a.ca = dt / (T)6;
      break;
  }
  return a;
}

}  // namespace hr
