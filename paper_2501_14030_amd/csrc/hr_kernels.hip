// HIP kernels (gfx950) of the hyperbolic-relaxation hot path.
//
// One fused kernel per RK4 stage does, for every stored point, the paper's
// RHS, BC and RK steps (Algorithm 1, inner loop):
//   interior points  k_u = v - eta u,
//                    k_v = c^2 [ lap(u) + S_src (psi_s + u)^-7 ]   (Eq. 5)
//   outer points     k_f = -c (f/r + d_r f), f in {u, v}  (radiation condition)
//   then the classic RK4 stage combine into the next stage input and the
//   accumulator.
// Inner ghost zones are never stored: a stencil tap that falls outside the
// stored range reads the interior point at the same Cartesian position
// (reflection through xx0 = 0, theta = 0 or theta = pi, each with phi + pi,
// and phi periodicity). Since a ghost's RHS is a copy of its image's and both
// start equal, this gives the same values as filling ghost zones.
//
// Layout: every grid function is "extended": (N0+NG) x N1 x N2, x0 fastest,
// the last NG points of each x0 row being the outer boundary points. Laplacian
// coefficients live in 2D (x0, x1) tables, since they do not depend on phi.
//
// The residual H (left-hand side of Eq. 4) is always evaluated in double
// precision; each block reduces its H^2 with wavefront shuffles and writes one
// partial, and a single block adds the partials in a fixed order.

#include <hip/hip_ext.h>

#include <type_traits>

#include "hr_internal.h"
#include "hr_stencil.h"

namespace hr {
namespace {

// ---------------------------------------------------------------------------
// Block tiling. A block owns a TX x TY patch of one (x0, x1) plane of the
// interior. The patch plus an NG-deep rim is staged in LDS once, with rim
// taps outside the stored range replaced by their images: reflection through
// xx0 = 0 (the same plane for SinhSymTP rows, theta mirrored for Spherical,
// phi + pi), through theta = 0 or pi (phi + pi). The x0 and x1 stencil taps
// then read LDS; the x2 taps (periodic in phi) read global memory directly,
// where neighbouring planes' blocks make them cache hits.
constexpr int TX = kTileX;  // threads along x0 (one wavefront)
constexpr int TY = kTileY;  // threads along x1
constexpr int kTileThreads = TX * TY;

template <int NG>
struct TileShape {
  static constexpr int W = TX + 2 * NG;
  static constexpr int H = TY + 2 * NG;
};

// Stored-row geometry seen by a kernel instance: instances built with
// ZF = false serve grids without stored outer rows on the x1 faces (zo = 0,
// R1 = N1 as compile-time facts, so those kernels are unchanged by them); ZF =
// true instances serve SinhCylindrical grids.
template <bool ZF>
__device__ __forceinline__ int zo_of(const Dims& d) { return ZF ? d.zo : 0; }
template <bool ZF>
__device__ __forceinline__ int rows_of(const Dims& d) { return ZF ? d.R1 : d.N1; }
template <bool ZF>
__device__ __forceinline__ unsigned sidx_t(const Dims& d, int i0, int i1, int i2) {
  return (unsigned)i0 +
         (unsigned)d.P0 * ((unsigned)(i1 + zo_of<ZF>(d)) + (unsigned)rows_of<ZF>(d) * (unsigned)i2);
}

// Loads and stores of fields that are touched once per point and stage. With
// NT (large grids) they bypass cache retention so that L2 keeps the u planes
// the stencil re-reads; small grids keep everything cached between launches.
template <bool NT, typename T>
__device__ __forceinline__ T ld(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// XCD-aware tile order for the phi-column kernel. The hardware hands block b of
// a launch to XCD b mod 8, and each XCD has its own L2. Block b is given tile
// number (b mod 8) * (T / 8) + b / 8 (T tiles, remainder spread over the first
// XCDs), so that every XCD works through a contiguous run of tiles, x0
// fastest: the rim rows a tile shares with its x0 and x1 neighbours were most
// likely just loaded into the same L2 (512x512x64 FP64: 414 -> 353 us per
// stage).
constexpr int kXcds = 8;

struct TileId {
  int x, y, z;
};

__device__ __forceinline__ TileId xcd_tile_of(unsigned b, unsigned gx, unsigned gy, unsigned gz) {
  const unsigned n = gx * gy * gz;
  const unsigned per = n / kXcds, rem = n % kXcds;
  const unsigned x = b % kXcds, k = b / kXcds;
  const unsigned t = x * per + (x < rem ? x : rem) + k;
  TileId id;
  id.x = (int)(t % gx);
  id.y = (int)((t / gx) % gy);
  id.z = (int)(t / (gx * gy));
  return id;
}

__device__ __forceinline__ TileId xcd_tile() {
  return xcd_tile_of(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), gridDim.x,
                     gridDim.y, gridDim.z);
}

// Stage the rim-extended patch of plane i2 of field U into tile (type C).
template <int NG, typename C, typename S, bool ZF = false>
__device__ __forceinline__ void load_tile(C* __restrict__ tile, const S* __restrict__ U,
                                          const Dims& d, int x0b, int x1b, int i2) {
  constexpr int W = TileShape<NG>::W, H = TileShape<NG>::H;
  const int tid = threadIdx.x + TX * threadIdx.y;
  const unsigned plane = (unsigned)d.P0 * (unsigned)rows_of<ZF>(d);
  const unsigned b0 = plane * (unsigned)i2;
  const unsigned bh = plane * (unsigned)half_turn(i2, d.N2);
  for (int e = tid; e < W * H; e += kTileThreads) {
    const int l1 = e / W;
    const int l0 = e - l1 * W;
    const int j0 = x0b + l0 - NG;
    const int j1 = x1b + l1 - NG;
    C val = (C)0;
    // stored rows: the interior ones and, with zo_of<ZF>(d), the z faces' outer rows
    if (j1 >= -zo_of<ZF>(d) && j1 < d.N1 + zo_of<ZF>(d)) {
      if (j0 >= 0) {
        if (j0 < d.P0) val = (C)U[b0 + (unsigned)j0 + (unsigned)d.P0 * (unsigned)(j1 + zo_of<ZF>(d))];
      } else {  // reflection through xx0 = 0
        const int r1 = d.sph ? d.N1 - 1 - j1 : j1;
        val = (C)U[bh + (unsigned)(-1 - j0) + (unsigned)d.P0 * (unsigned)(r1 + zo_of<ZF>(d))];
      }
    } else if (j0 >= 0 && j0 < d.P0 && j1 >= -NG && j1 < d.N1 + NG) {
      // reflection through theta = 0 or theta = pi (no stored outer rows here)
      const int r1 = j1 < 0 ? -1 - j1 : 2 * d.N1 - 1 - j1;
      val = (C)U[bh + (unsigned)j0 + (unsigned)d.P0 * (unsigned)r1];
    }
    tile[e] = val;
  }
}

// Un-normalised centred sums along the three directions, compute type C.
template <typename C>
struct Sums {
  C d0, d1, dd0, dd1, dd2, uc;
};

// The 2*NG phi-direction taps of point (i0, i1, i2) (periodic in phi), read
// from global memory; issued before the tile barrier so that they are in
// flight together with every other load of the point.
template <int NG, typename C, typename S>
struct PhiTaps {
  C p[NG], m[NG];
  template <bool ZF = false>
  __device__ __forceinline__ void load(const S* __restrict__ U, const Dims& d, int i0, int i1,
                                       int i2) {
    const unsigned col = (unsigned)i0 + (unsigned)d.P0 * (unsigned)(i1 + zo_of<ZF>(d));
    const unsigned plane = (unsigned)d.P0 * (unsigned)rows_of<ZF>(d);
    // planes i2 + k and i2 - k (mod N2), stepped one at a time
    int jp = i2, jm = i2;
#pragma unroll
    for (int k = 1; k <= NG; ++k) {
      jp = (jp + 1 == d.N2) ? 0 : jp + 1;
      jm = (jm == 0) ? d.N2 - 1 : jm - 1;
      p[k - 1] = (C)U[col + plane * (unsigned)jp];
      m[k - 1] = (C)U[col + plane * (unsigned)jm];
    }
  }
};

template <int NG, typename C, typename S>
__device__ __forceinline__ Sums<C> stencil(const C* __restrict__ tile,
                                           const PhiTaps<NG, C, S>& ph) {
  constexpr Weights<NG> Wt{};
  constexpr int W = TileShape<NG>::W;
  const C* r = tile + (threadIdx.y + NG) * W + (threadIdx.x + NG);
  Sums<C> s;
  const C uc = r[0];
  C d0 = 0, d1 = 0, e0 = 0, e1 = 0, e2 = 0;
#pragma unroll
  for (int k = 1; k <= NG; ++k) {
    const C p0 = r[k], m0 = r[-k];
    const C p1 = r[k * W], m1 = r[-k * W];
    d0 += (C)Wt.d1[k] * (p0 - m0);
    d1 += (C)Wt.d1[k] * (p1 - m1);
    e0 += (C)Wt.d2[k] * (p0 + m0);
    e1 += (C)Wt.d2[k] * (p1 + m1);
    e2 += (C)Wt.d2[k] * (ph.p[k - 1] + ph.m[k - 1]);
  }
  const C w0 = (C)Wt.d2[0];
  s.uc = uc;
  s.d0 = d0;
  s.d1 = d1;
  s.dd0 = e0 + w0 * uc;
  s.dd1 = e1 + w0 * uc;
  s.dd2 = e2 + w0 * uc;
  return s;
}

// (psi + u)^-7 times the source, in the compute type.
template <typename C>
__device__ __forceinline__ C source(C ssrc, C psi, C u) {
  const C p = psi + u;
  const C p2 = p * p;
  const C p4 = p2 * p2;
  return ssrc / (p4 * p2 * p);
}

// Per-point operands of the stage combine, loaded ahead of the tile barrier.
template <int STAGE, bool NT, typename T>
struct CombineIn {
  T un, vn, au, av;
  __device__ __forceinline__ void load(const StageArgs<T>& a, unsigned idx) {
    if constexpr (STAGE == 2 || STAGE == 3) {
      un = ld<NT>(a.un + idx);
      vn = ld<NT>(a.vn + idx);
    }
    if constexpr (STAGE != 1) {
      au = ld<NT>(a.au + idx);
      av = ld<NT>(a.av + idx);
    }
  }
};


// RK4 stage combine for one point, given the stage slopes. The next stage
// input (uout) is re-read with stencils, so it is always a cached store.
template <int STAGE, bool NT, typename T>
__device__ __forceinline__ void combine(const StageArgs<T>& a, unsigned idx,
                                        const CombineIn<STAGE, NT, T>& c, T uin, T vin, T ku,
                                        T kv) {
  if constexpr (STAGE == 1) {
    a.uout[idx] = uin + a.cy * ku;
    st<NT>(a.vout + idx, vin + a.cy * kv);
    st<NT>(a.au + idx, uin + a.ca * ku);
    st<NT>(a.av + idx, vin + a.ca * kv);
  } else if constexpr (STAGE == 4) {
    a.uout[idx] = c.au + a.ca * ku;
    st<NT>(a.vout + idx, c.av + a.ca * kv);
  } else {
    a.uout[idx] = c.un + a.cy * ku;
    st<NT>(a.vout + idx, c.vn + a.cy * kv);
    st<NT>(a.au + idx, c.au + a.ca * ku);
    st<NT>(a.av + idx, c.av + a.ca * kv);
  }
}

// Stage update at an outer point of a z face (SinhCylindrical: stored rows
// i1 in [-zo, 0) and [N1, N1 + zo), any stored i0): the radiation condition
// k_f = -c (f/r + d_r f) with d_r f a one-sided difference toward the
// interior divided by d r / d xx of its direction (along xx1 where
// |z| >= rho, else along xx0; the table holds the index step and q with the
// outward sign folded in), then the stage combine. Reads only the stage
// input.
template <int STAGE, bool NT, bool CORR, typename T>
__device__ __forceinline__ void zface_point(const StageArgs<T>& a, int i0, int i1, int i2) {
  const Dims& d = a.d;
  const int zr = i1 < 0 ? i1 + d.zo : d.zo + (i1 - d.N1);
  const unsigned z2d = (unsigned)d.P0 * 2u * (unsigned)d.zo;
  const unsigned kz = (unsigned)i0 + (unsigned)d.P0 * (unsigned)zr;
  const T c = a.zfac[kz], rinv = a.zfac[z2d + kz], qd = a.zfac[2 * z2d + kz];
  const int in = (int)a.zfac[3 * z2d + kz];   // one point toward the interior
  const unsigned o = sidx(d, i0, i1, i2);
  const T* U = a.uin + o;
  const T* V = a.vin + o;
  const bool bc4 = a.bc4 != 0;
  const T u0 = U[0], u1 = U[in], u2 = U[2 * in];
  const T v0 = V[0], v1 = V[in], v2 = V[2 * in];
  const T u3 = bc4 ? U[3 * in] : (T)0, u4 = bc4 ? U[4 * in] : (T)0;
  const T v3 = bc4 ? V[3 * in] : (T)0, v4 = bc4 ? V[4 * in] : (T)0;
  CombineIn<STAGE, NT, T> co;
  co.load(a, o);
  T kuo = -c * (u0 * rinv + outer_diff(u0, u1, u2, u3, u4, qd, bc4));
  T kvo = -c * (v0 * rinv + outer_diff(v0, v1, v2, v3, v4, qd, bc4));
  if constexpr (CORR) {
    kuo = a.khu[o] + kuo;
    kvo = a.khv[o] + kvo;
  }
  combine<STAGE, NT, T>(a, o, co, u0, v0, kuo, kvo);
}

// The z-face outer points of a block's x0 range in plane i2: the first x1
// tile takes the lower rows, the last one the upper rows, one row per thread
// row ty < zo; threads among the last NG interior columns also take the outer
// column i0 + NG (the corners).
template <int STAGE, bool NT, bool CORR, typename T>
__device__ __forceinline__ void zface_rows(const StageArgs<T>& a, int x0b, int by, int i2) {
  const Dims& d = a.d;
  if (!d.zo || (int)threadIdx.y >= d.zo) return;
  const int nby = (d.N1 + TY - 1) / TY;
  const int i0 = x0b + (int)threadIdx.x;
  if (i0 >= d.N0) return;
  for (int side = 0; side < 2; ++side) {
    if (side == 0 ? by != 0 : by != nby - 1) continue;
    const int i1 = side == 0 ? (int)threadIdx.y - d.zo : d.N1 + (int)threadIdx.y;
    zface_point<STAGE, NT, CORR, T>(a, i0, i1, i2);
    if (i0 >= d.N0 - d.NG) zface_point<STAGE, NT, CORR, T>(a, i0 + d.NG, i1, i2);
  }
}

// One RK4 stage: RHS + boundary conditions + stage combine. Grid:
// (ceil(N0/TX), ceil(N1/TY), N2). Each interior point is one thread; the
// threads with i0 in [N0-NG, N0) also update the outer point i0 + NG of their
// row. Every global load of the interior point is issued before the tile
// barrier so that the point waits for one memory round trip.
template <typename T, int NG, int STAGE, bool NT, bool CORR, bool ZF>
__global__ void __launch_bounds__(kTileThreads) k_stage(StageArgs<T> a) {
  constexpr int W = TileShape<NG>::W, H = TileShape<NG>::H;
  __shared__ T tile[W * H];
  const Dims& d = a.d;
  // hardware block order: the blocks of one (x0, x1) tile at every plane share
  // an XCD (gridDim.x * gridDim.y is a multiple of 8 for the shapes where this
  // matters), so the phi taps of neighbouring planes hit the same L2
  const int x0b = blockIdx.x * TX, x1b = blockIdx.y * TY, i2 = blockIdx.z;
  const int i0 = x0b + threadIdx.x, i1 = x1b + threadIdx.y;
  const bool active = i0 < d.N0 && i1 < d.N1;
  const unsigned n2d = (unsigned)d.N0 * (unsigned)d.N1;
  const unsigned k2 = (unsigned)i0 + (unsigned)d.N0 * (unsigned)i1;
  const unsigned row = sidx_t<ZF>(d, 0, i1, i2);
  const unsigned idx = row + (unsigned)i0;
  PhiTaps<NG, T, T> ph;
  CombineIn<STAGE, NT, T> cin;
  T v = 0, psi = 0, ssrc = 0, f[6], khu = 0, khv = 0;
  if (active) {
    ph.template load<ZF>(a.uin, d, i0, i1, i2);
    v = ld<NT>(a.vin + idx);
    psi = ld<NT>(a.psi + idx);
    ssrc = ld<NT>(a.ssrc + idx);
    if constexpr (CORR) {
      khu = a.khu[idx];
      khv = a.khv[idx];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) f[q] = load_factor(a.fac, a.facb, q * n2d + k2);
    cin.load(a, idx);
  }
  load_tile<NG, T, T, ZF>(tile, a.uin, d, x0b, x1b, i2);
  __syncthreads();
  if constexpr (ZF) zface_rows<STAGE, NT, CORR, T>(a, x0b, (int)blockIdx.y, i2);
  if (!active) return;
  const Sums<T> s = stencil<NG, T, T>(tile, ph);
  const T lap = f[0] * s.dd0 + f[1] * s.dd1 + f[2] * s.dd2 + f[3] * s.d0 + f[4] * s.d1;
  const T u = s.uc;
  T ku, kv;
  if constexpr (CORR) {
    ku = khu + (v - a.eta * u);
    kv = khv + f[5] * (lap + source_delta(ssrc, psi, u));
  } else {
    ku = v - a.eta * u;
    kv = f[5] * (lap + source<T>(ssrc, psi, u));
  }
  combine<STAGE, NT, T>(a, idx, cin, u, v, ku, kv);
  if (i0 >= d.N0 - NG) {
    // outer point: radiation condition with a one-sided xx0 derivative
    const int q = i0 + NG - d.N0;
    const unsigned o = row + (unsigned)(i0 + NG);
    const unsigned ko = (unsigned)q + (unsigned)NG * (unsigned)i1;
    const unsigned o2d = (unsigned)NG * (unsigned)d.N1;
    const T c = a.ofac[ko], rinv = a.ofac[o2d + ko], qd = a.ofac[2 * o2d + ko];
    const T u0 = a.uin[o], u1 = a.uin[o - 1], u2 = a.uin[o - 2];
    const T v0 = a.vin[o], v1 = a.vin[o - 1], v2 = a.vin[o - 2];
    const bool bc4 = a.bc4 != 0;
    const T u3 = bc4 ? a.uin[o - 3] : (T)0, u4 = bc4 ? a.uin[o - 4] : (T)0;
    const T v3 = bc4 ? a.vin[o - 3] : (T)0, v4 = bc4 ? a.vin[o - 4] : (T)0;
    CombineIn<STAGE, NT, T> co;
    co.load(a, o);
    T kuo = -c * (u0 * rinv + outer_diff(u0, u1, u2, u3, u4, qd, bc4));
    T kvo = -c * (v0 * rinv + outer_diff(v0, v1, v2, v3, v4, qd, bc4));
    if constexpr (CORR) {
      kuo = a.khu[o] + kuo;
      kvo = a.khv[o] + kvo;
    }
    combine<STAGE, NT, T>(a, o, co, u0, v0, kuo, kvo);
  }
}

// ---------------------------------------------------------------------------
// Phi-marching variant of the stage kernel. A block owns a TX x TY patch of
// (x0, x1) columns and walks `chunk` consecutive phi planes. The 2*NG+1 phi
// taps of each column sit in a register queue (each u value is loaded once per
// column instead of once per tap), the rim-extended x0-x1 tile is double
// buffered in LDS, and the next plane's tile, queue value and per-point
// operands are prefetched while the current plane is computed. The 2D
// Laplacian coefficients are loaded once per column.

// The rim-extended tile of one plane, split into a global-to-register fetch and
// a register-to-LDS store so the fetch can run one plane ahead.
template <int NG, typename T>
struct TileRegs {
  static constexpr int W = TileShape<NG>::W, H = TileShape<NG>::H;
  static constexpr int NE = (W * H + kTileThreads - 1) / kTileThreads;
  T v[NE];
  template <bool ZF = false>
  __device__ __forceinline__ void fetch(const T* __restrict__ U, const Dims& d, int x0b, int x1b,
                                        int i2) {
    const int tid = threadIdx.x + TX * threadIdx.y;
    const unsigned plane = (unsigned)d.P0 * (unsigned)rows_of<ZF>(d);
    const unsigned b0 = plane * (unsigned)i2;
    const unsigned bh = plane * (unsigned)half_turn(i2, d.N2);
#pragma unroll
    for (int r = 0; r < NE; ++r) {
      const int e = tid + r * kTileThreads;
      const int l1 = e / W;
      const int l0 = e - l1 * W;
      const int j0 = x0b + l0 - NG;
      const int j1 = x1b + l1 - NG;
      T val = (T)0;
      if (e < W * H) {
        if (j1 >= -zo_of<ZF>(d) && j1 < d.N1 + zo_of<ZF>(d)) {   // stored rows (z-face rows too)
          if (j0 >= 0) {
            if (j0 < d.P0)
              val = U[b0 + (unsigned)j0 + (unsigned)d.P0 * (unsigned)(j1 + zo_of<ZF>(d))];
          } else {
            const int r1 = d.sph ? d.N1 - 1 - j1 : j1;
            val = U[bh + (unsigned)(-1 - j0) + (unsigned)d.P0 * (unsigned)(r1 + zo_of<ZF>(d))];
          }
        } else if (j0 >= 0 && j0 < d.P0 && j1 >= -NG && j1 < d.N1 + NG) {
          const int r1 = j1 < 0 ? -1 - j1 : 2 * d.N1 - 1 - j1;
          val = U[bh + (unsigned)j0 + (unsigned)d.P0 * (unsigned)r1];
        }
      }
      v[r] = val;
    }
  }
  __device__ __forceinline__ void store(T* __restrict__ tile) const {
    const int tid = threadIdx.x + TX * threadIdx.y;
#pragma unroll
    for (int r = 0; r < NE; ++r) {
      const int e = tid + r * kTileThreads;
      if (e < W * H) tile[e] = v[r];
    }
  }
};

// Operands of one interior point that are read once per stage.
template <int STAGE, bool CORR, typename T>
struct PointIn {
  T v, psi, ssrc, un, vn, au, av, khu, khv;
  __device__ __forceinline__ void load(const StageArgs<T>& a, unsigned idx) {
    v = a.vin[idx];
    psi = a.psi[idx];
    ssrc = a.ssrc[idx];
    if constexpr (CORR) {
      khu = a.khu[idx];
      khv = a.khv[idx];
    }
    if constexpr (STAGE == 2 || STAGE == 3) {
      un = a.un[idx];
      vn = a.vn[idx];
    }
    if constexpr (STAGE != 1) {
      au = a.au[idx];
      av = a.av[idx];
    }
  }
};

template <int STAGE, bool CORR, typename T>
__device__ __forceinline__ void combine_pt(const StageArgs<T>& a, unsigned idx,
                                           const PointIn<STAGE, CORR, T>& c, T uin, T ku, T kv) {
  if constexpr (STAGE == 1) {
    a.uout[idx] = uin + a.cy * ku;
    a.vout[idx] = c.v + a.cy * kv;
    a.au[idx] = uin + a.ca * ku;
    a.av[idx] = c.v + a.ca * kv;
  } else if constexpr (STAGE == 4) {
    a.uout[idx] = c.au + a.ca * ku;
    a.vout[idx] = c.av + a.ca * kv;
  } else {
    a.uout[idx] = c.un + a.cy * ku;
    a.vout[idx] = c.vn + a.cy * kv;
    a.au[idx] = c.au + a.ca * ku;
    a.av[idx] = c.av + a.ca * kv;
  }
}

template <int NG>
__device__ __forceinline__ int step_up(int j, int N) { return j + 1 == N ? 0 : j + 1; }

// Stage update at outer point t = q + NG (i1 + N1 i2) of the xx0 face (stored
// i0 = N0 + q): the radiation condition with its one-sided xx0 difference,
// then the stage combine; reads only the stage input. The phi-column kernels
// run these as work of their own after the column tiles: inside a tile's
// plane loop, the few lanes holding them stalled every plane of the last x0
// tiles on a memory round trip (256x256x32 FP64: 46 -> 35 us per stage
// without them).
template <typename T, int NG, int STAGE, bool CORR, bool ZF>
__device__ __forceinline__ void outer_point_stage(const StageArgs<T>& a, int t) {
  const Dims& d = a.d;
  const int qo = t % NG, r = t / NG;
  const int i1 = r % d.N1, i2 = r / d.N1;
  const unsigned o = sidx_t<ZF>(d, d.N0 + qo, i1, i2);
  const unsigned ko = (unsigned)qo + (unsigned)NG * (unsigned)i1;
  const unsigned o2d = (unsigned)NG * (unsigned)d.N1;
  const T c = a.ofac[ko], rinv = a.ofac[o2d + ko], qd = a.ofac[2 * o2d + ko];
  const T u0 = a.uin[o], u1 = a.uin[o - 1], u2 = a.uin[o - 2];
  const T v0 = a.vin[o], v1 = a.vin[o - 1], v2 = a.vin[o - 2];
  const bool bc4 = a.bc4 != 0;
  const T u3 = bc4 ? a.uin[o - 3] : (T)0, u4 = bc4 ? a.uin[o - 4] : (T)0;
  const T v3 = bc4 ? a.vin[o - 3] : (T)0, v4 = bc4 ? a.vin[o - 4] : (T)0;
  CombineIn<STAGE, false, T> co;
  co.load(a, o);
  T kuo = -c * (u0 * rinv + outer_diff(u0, u1, u2, u3, u4, qd, bc4));
  T kvo = -c * (v0 * rinv + outer_diff(v0, v1, v2, v3, v4, qd, bc4));
  if constexpr (CORR) {
    kuo = a.khu[o] + kuo;
    kvo = a.khv[o] + kvo;
  }
  combine<STAGE, false, T>(a, o, co, u0, v0, kuo, kvo);
}

// The boundary work a phi-column launch runs in blocks of its own: the NG N1 N2
// outer points of the xx0 face, then (grids with stored z-face rows) the
// 2 zo P0 N2 points of those rows. Work item t of it:
template <typename T, int NG, int STAGE, bool CORR, bool ZF>
__device__ __forceinline__ void outer_work(const StageArgs<T>& a, int t) {
  const Dims& d = a.d;
  const int nx = NG * d.N1 * d.N2;
  if (t < nx) {
    outer_point_stage<T, NG, STAGE, CORR, ZF>(a, t);
  } else if constexpr (ZF) {
    t -= nx;
    if (t >= 2 * d.zo * d.P0 * d.N2) return;
    const int i0 = t % d.P0, r = t / d.P0;
    const int row = r % (2 * d.zo), i2 = r / (2 * d.zo);
    zface_point<STAGE, false, CORR, T>(a, i0, row < d.zo ? row - d.zo : d.N1 + row - d.zo, i2);
  }
}

// Blocks of kTileThreads threads (or batch work items) that cover a grid's
// boundary work (outer_work).
__host__ __device__ __forceinline__ int outer_blocks(const Dims& d) {
  return (d.NG * d.N1 * d.N2 + 2 * d.zo * d.P0 * d.N2 + kTileThreads - 1) / kTileThreads;
}

// Rows of the phi-column kernel's LDS factor table: the FP64 instances keep a
// column's six Laplacian factors in LDS, each thread reading only its own (in
// registers they push stages 2 and 3 into spills: 428 -> 411 us per stage at
// 512x512x64); the FP32 instances do not spill and keep them in registers.
template <typename T>
constexpr int kFacRows = sizeof(T) == 8 ? 6 : 1;

template <typename T, int NG, int STAGE, bool CORR, bool ZF>
__device__ __forceinline__ void stage_col_body(const StageArgs<T>& a, int bx, int by, int bz,
                                               int chunk,
                                               T (&tile)[2][TileShape<NG>::W * TileShape<NG>::H],
                                               T (&fl)[kFacRows<T>][kTileThreads]) {
  constexpr int W = TileShape<NG>::W;
  constexpr Weights<NG> Wt{};
  const Dims& d = a.d;
  const int x0b = bx * TX, x1b = by * TY;
  const int z0 = bz * chunk;
  const int z1 = min(z0 + chunk, d.N2);
  const int i0 = x0b + threadIdx.x, i1 = x1b + threadIdx.y;
  const bool active = i0 < d.N0 && i1 < d.N1;
  const unsigned plane = (unsigned)d.P0 * (unsigned)rows_of<ZF>(d);
  const unsigned col = (unsigned)i0 + (unsigned)d.P0 * (unsigned)(i1 + zo_of<ZF>(d));
  const unsigned n2d = (unsigned)d.N0 * (unsigned)d.N1;
  const unsigned k2 = (unsigned)i0 + (unsigned)d.N0 * (unsigned)i1;

  // phi register queue q[j] = u(z - NG + j), j = 0..2NG, for z = z0
  T q[2 * NG + 1];
  int jq = z0;  // (z0 - NG) mod N2, stepping down one plane at a time
#pragma unroll
  for (int k = 0; k < NG; ++k) jq = (jq == 0) ? d.N2 - 1 : jq - 1;
  // the column's six Laplacian factors: in LDS (FP64) or registers (FP32)
  const int ft = threadIdx.x + TX * threadIdx.y;
  T f[6];
  auto fac = [&](int r) -> T {
    if constexpr (kFacRows<T> == 6) return fl[r][ft];
    else return f[r];
  };
  PointIn<STAGE, CORR, T> cur;
  if (active) {
#pragma unroll
    for (int j = 0; j <= 2 * NG; ++j) {
      q[j] = a.uin[col + plane * (unsigned)jq];
      jq = step_up<NG>(jq, d.N2);
    }
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      if constexpr (kFacRows<T> == 6) fl[r][ft] = load_factor(a.fac, a.facb, r * n2d + k2);
      else f[r] = load_factor(a.fac, a.facb, r * n2d + k2);
    }
    cur.load(a, col + plane * (unsigned)z0);
  }
  // jq now holds (z0 + NG + 1) mod N2: the plane the queue needs next
  {
    TileRegs<NG, T> t0;
    t0.template fetch<ZF>(a.uin, d, x0b, x1b, z0);
    t0.store(tile[0]);
  }
  __syncthreads();
  for (int z = z0; z < z1; ++z) {
    const int buf = (z - z0) & 1;
    const bool more = z + 1 < z1;
    // prefetch plane z + 1
    TileRegs<NG, T> tn;
    PointIn<STAGE, CORR, T> nxt;
    T qn = (T)0;
    if (more) {
      tn.template fetch<ZF>(a.uin, d, x0b, x1b, z + 1);
      if (active) {
        qn = a.uin[col + plane * (unsigned)jq];
        nxt.load(a, col + plane * (unsigned)(z + 1));
      }
    }
    if (active) {
      const T* r = tile[buf] + (threadIdx.y + NG) * W + (threadIdx.x + NG);
      const T uc = r[0];
      T d0 = 0, d1 = 0, e0 = 0, e1 = 0, e2 = 0;
#pragma unroll
      for (int k = 1; k <= NG; ++k) {
        const T p0 = r[k], m0 = r[-k];
        const T p1 = r[k * W], m1 = r[-k * W];
        d0 += (T)Wt.d1[k] * (p0 - m0);
        d1 += (T)Wt.d1[k] * (p1 - m1);
        e0 += (T)Wt.d2[k] * (p0 + m0);
        e1 += (T)Wt.d2[k] * (p1 + m1);
        e2 += (T)Wt.d2[k] * (q[NG + k] + q[NG - k]);
      }
      const T w0 = (T)Wt.d2[0];
      const T lap = fac(0) * (e0 + w0 * uc) + fac(1) * (e1 + w0 * uc) +
                    fac(2) * (e2 + w0 * uc) + fac(3) * d0 + fac(4) * d1;
      T ku, kv;
      if constexpr (CORR) {
        ku = cur.khu + (cur.v - a.eta * uc);
        kv = cur.khv + fac(5) * (lap + source_delta(cur.ssrc, cur.psi, uc));
      } else {
        ku = cur.v - a.eta * uc;
        kv = fac(5) * (lap + source<T>(cur.ssrc, cur.psi, uc));
      }
      const unsigned idx = col + plane * (unsigned)z;
      combine_pt<STAGE, CORR, T>(a, idx, cur, uc, ku, kv);
    }
    if (more) {
      tn.store(tile[buf ^ 1]);
#pragma unroll
      for (int j = 0; j < 2 * NG; ++j) q[j] = q[j + 1];
      q[2 * NG] = qn;
      cur = nxt;
      jq = step_up<NG>(jq, d.N2);
    }
    __syncthreads();
  }
}

// One dimension of blocks: the column tiles (XCD-aware order), then the
// outer-point blocks.
template <typename T, int NG, int STAGE, bool CORR, bool ZF>
__global__ void __launch_bounds__(kTileThreads, 4) k_stage_col(StageArgs<T> a, int chunk) {
  __shared__ T tile[2][TileShape<NG>::W * TileShape<NG>::H];
  __shared__ T fl[kFacRows<T>][kTileThreads];
  const Dims& d = a.d;
  const unsigned gx = (d.N0 + TX - 1) / TX, gy = (d.N1 + TY - 1) / TY;
  const unsigned gz = (d.N2 + chunk - 1) / chunk;
  const unsigned ncol = gx * gy * gz;
  if (blockIdx.x < ncol) {
    const TileId tid = xcd_tile_of(blockIdx.x, gx, gy, gz);
    stage_col_body<T, NG, STAGE, CORR, ZF>(a, tid.x, tid.y, tid.z, chunk, tile, fl);
  } else {
    outer_work<T, NG, STAGE, CORR, ZF>(
        a, (int)(blockIdx.x - ncol) * kTileThreads + threadIdx.x + TX * threadIdx.y);
  }
}

// ---------------------------------------------------------------------------
// Batched kernels: many grids (same order) relaxed by one launch per RK stage.
// A persistent grid of blocks walks a device work list; each item is
// (grid, x0 tile, x1 tile, phi chunk or plane), or in a stage list (grid, -1,
// k, 0): outer-point block k of the grid. Per-grid stage arguments live
// in device memory (four entries per grid, one per stage). The list lengths
// are read from device memory, so a captured launch sequence stays valid when
// converged grids are dropped from the lists.
template <typename T, int NG, int STAGE, bool CORR, bool ZF>
__device__ __forceinline__ void batch_stage_item(const StageArgs<T>* __restrict__ descs,
                                                 const int4 w,
                                                 T (&tile)[2][TileShape<NG>::W * TileShape<NG>::H],
                                                 T (&fl)[kFacRows<T>][kTileThreads]) {
  const StageArgs<T>& a = descs[4 * w.x + (STAGE - 1)];
  if (w.y >= 0) {
    stage_col_body<T, NG, STAGE, CORR, ZF>(a, w.y, w.z, w.w, a.chunk, tile, fl);
  } else {
    outer_work<T, NG, STAGE, CORR, ZF>(a, w.z * kTileThreads + threadIdx.x + TX * threadIdx.y);
  }
}

template <typename T, int NG, int STAGE, bool CORR, bool ZF>
__global__ void __launch_bounds__(kTileThreads, 4)
    k_batch_stage(const StageArgs<T>* __restrict__ descs, const int4* __restrict__ items,
                  const int* __restrict__ nitems) {
  __shared__ T tile[2][TileShape<NG>::W * TileShape<NG>::H];
  __shared__ T fl[kFacRows<T>][kTileThreads];
  const int n = *nitems;
  const int G = gridDim.x;
  if (G % kXcds == 0) {
    // XCD-aware walk: the blocks on XCD x (b mod 8 == x) share the contiguous
    // run x of the list (items are grid-major, x0 tile fastest), so tiles and
    // their neighbours meet in one L2
    const int x = blockIdx.x % kXcds, k = blockIdx.x / kXcds, gk = G / kXcds;
    const int per = n / kXcds, rem = n % kXcds;
    const int lo = x * per + (x < rem ? x : rem), hi = lo + per + (x < rem ? 1 : 0);
    for (int it = lo + k; it < hi; it += gk) batch_stage_item<T, NG, STAGE, CORR, ZF>(descs, items[it], tile, fl);
  } else {
    for (int it = blockIdx.x; it < n; it += G) batch_stage_item<T, NG, STAGE, CORR, ZF>(descs, items[it], tile, fl);
  }
}


// Slopes k(y_b) of the FP64 base state for the split-state single-precision
// form, stored in FP32 with p_b = psi_s + u_b and S_src p_b^-7; the FP32
// increment state is reset to zero. Same tiling as the plane stage kernel.
// Base slopes at an outer point of a z face (SinhCylindrical; see
// zface_point), with the other base quantities as at the xx0 face's points.
__device__ __forceinline__ void base_zface_point(const BaseArgs& a, int i0, int i1, int i2) {
  const Dims& d = a.d;
  const int zr = i1 < 0 ? i1 + d.zo : d.zo + (i1 - d.N1);
  const unsigned z2d = (unsigned)d.P0 * 2u * (unsigned)d.zo;
  const unsigned kz = (unsigned)i0 + (unsigned)d.P0 * (unsigned)zr;
  const double c = a.zfac[kz], rinv = a.zfac[z2d + kz], qd = a.zfac[2 * z2d + kz];
  const int in = (int)a.zfac[3 * z2d + kz];   // one point toward the interior
  const unsigned o = sidx(d, i0, i1, i2);
  const double* U = a.u + o;
  const double* V = a.v + o;
  const bool bc4 = a.bc4 != 0;
  const double u0 = U[0], u1 = U[in], u2 = U[2 * in];
  const double v0 = V[0], v1 = V[in], v2 = V[2 * in];
  const double u3 = bc4 ? U[3 * in] : 0.0, u4 = bc4 ? U[4 * in] : 0.0;
  const double v3 = bc4 ? V[3 * in] : 0.0, v4 = bc4 ? V[4 * in] : 0.0;
  a.khu[o] = (float)(-c * (u0 * rinv + outer_diff(u0, u1, u2, u3, u4, qd, bc4)));
  a.khv[o] = (float)(-c * (v0 * rinv + outer_diff(v0, v1, v2, v3, v4, qd, bc4)));
  a.pb[o] = (float)(a.psi[o] + u0);
  a.sp7[o] = 0.0f;
  a.eu[o] = 0.0f;
  a.ev[o] = 0.0f;
}

template <int NG, bool ZF>
__device__ __forceinline__ void base_body(const BaseArgs& a, int bx, int by, int i2,
                                          double* __restrict__ tile) {
  const Dims& d = a.d;
  const int x0b = bx * TX, x1b = by * TY;
  const int i0 = x0b + threadIdx.x, i1 = x1b + threadIdx.y;
  const bool active = i0 < d.N0 && i1 < d.N1;
  const unsigned n2d = (unsigned)d.N0 * (unsigned)d.N1;
  const unsigned k2 = (unsigned)i0 + (unsigned)d.N0 * (unsigned)i1;
  const unsigned row = sidx_t<ZF>(d, 0, i1, i2);
  const unsigned idx = row + (unsigned)i0;
  PhiTaps<NG, double, double> ph;
  double v = 0, psi = 0, ssrc = 0, f[6];
  if (active) {
    ph.template load<ZF>(a.u, d, i0, i1, i2);
    v = a.v[idx];
    psi = a.psi[idx];
    ssrc = a.ssrc[idx];
#pragma unroll
    for (int q = 0; q < 6; ++q) f[q] = a.fac[q * n2d + k2];
  }
  load_tile<NG, double, double, ZF>(tile, a.u, d, x0b, x1b, i2);
  __syncthreads();
  if (ZF && (int)threadIdx.y < d.zo && i0 < d.N0) {
    // z-face outer points: lower rows from the first x1 tile, upper rows from
    // the last (corners by the last NG interior columns)
    const int nby = (d.N1 + TY - 1) / TY;
    for (int side = 0; side < 2; ++side) {
      if (side == 0 ? by != 0 : by != nby - 1) continue;
      const int z1 = side == 0 ? (int)threadIdx.y - d.zo : d.N1 + (int)threadIdx.y;
      base_zface_point(a, i0, z1, i2);
      if (i0 >= d.N0 - NG) base_zface_point(a, i0 + NG, z1, i2);
    }
  }
  if (!active) return;
  const Sums<double> s = stencil<NG, double, double>(tile, ph);
  const double lap = f[0] * s.dd0 + f[1] * s.dd1 + f[2] * s.dd2 + f[3] * s.d0 + f[4] * s.d1;
  const double u = s.uc;
  const double p = psi + u;
  const double p2 = p * p, p4 = p2 * p2, p7 = p4 * p2 * p;
  a.khu[idx] = (float)(v - a.eta * u);
  a.khv[idx] = (float)(f[5] * (lap + ssrc / p7));
  a.pb[idx] = (float)p;
  a.sp7[idx] = (float)(ssrc / p7);
  a.eu[idx] = 0.0f;
  a.ev[idx] = 0.0f;
  if (i0 >= d.N0 - NG) {
    const int q = i0 + NG - d.N0;
    const unsigned o = row + (unsigned)(i0 + NG);
    const unsigned ko = (unsigned)q + (unsigned)NG * (unsigned)i1;
    const unsigned o2d = (unsigned)NG * (unsigned)d.N1;
    const double c = a.ofac[ko], rinv = a.ofac[o2d + ko], qd = a.ofac[2 * o2d + ko];
    const double u0 = a.u[o], u1 = a.u[o - 1], u2 = a.u[o - 2];
    const double v0 = a.v[o], v1 = a.v[o - 1], v2 = a.v[o - 2];
    const bool bc4 = a.bc4 != 0;
    const double u3 = bc4 ? a.u[o - 3] : 0.0, u4 = bc4 ? a.u[o - 4] : 0.0;
    const double v3 = bc4 ? a.v[o - 3] : 0.0, v4 = bc4 ? a.v[o - 4] : 0.0;
    a.khu[o] = (float)(-c * (u0 * rinv + outer_diff(u0, u1, u2, u3, u4, qd, bc4)));
    a.khv[o] = (float)(-c * (v0 * rinv + outer_diff(v0, v1, v2, v3, v4, qd, bc4)));
    a.pb[o] = (float)(a.psi[o] + u0);
    a.sp7[o] = 0.0f;
    a.eu[o] = 0.0f;
    a.ev[o] = 0.0f;
  }
}

template <int NG, bool ZF>
__global__ void __launch_bounds__(kTileThreads) k_base(BaseArgs a) {
  __shared__ double tile[TileShape<NG>::W * TileShape<NG>::H];
  base_body<NG, ZF>(a, blockIdx.x, blockIdx.y, blockIdx.z, tile);
}

__global__ void __launch_bounds__(kBlock) k_rebase(double* __restrict__ ub,
                                                   double* __restrict__ vb,
                                                   const float* __restrict__ eu,
                                                   const float* __restrict__ ev, int n) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t < n) {
    ub[t] = ub[t] + (double)eu[t];
    vb[t] = vb[t] + (double)ev[t];
  }
}

// Sum over a 64-wide wavefront, then over the block's wavefronts in a fixed
// order. Returns the block total in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double x) {
  __shared__ double wsum[NT / 64];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  const int t = threadIdx.x + blockDim.x * threadIdx.y;
  const int lane = t & 63, wid = t >> 6;
  if (lane == 0) wsum[wid] = x;
  __syncthreads();
  double tot = 0.0;
  if (t == 0)
    for (int w = 0; w < NT / 64; ++w) tot += wsum[w];
  return tot;
}

// Residual H (left-hand side of Eq. 4) in FP64 from a state of storage type S;
// returns the block's sum of H^2 (valid in thread 0), same tiling as the plane
// stage kernel.
template <typename S, int NG, bool ZF>
__device__ __forceinline__ double residual_body(const ResidualArgs& a, int bx, int by, int i2,
                                               double* __restrict__ tile) {
  const Dims& d = a.d;
  const int x0b = bx * TX, x1b = by * TY;
  const S* U = static_cast<const S*>(a.u);
  const int i0 = x0b + threadIdx.x, i1 = x1b + threadIdx.y;
  const bool active = i0 < d.N0 && i1 < d.N1;
  const unsigned n2d = (unsigned)d.N0 * (unsigned)d.N1;
  const unsigned k2 = (unsigned)i0 + (unsigned)d.N0 * (unsigned)i1;
  const unsigned idx = sidx_t<ZF>(d, i0, i1, i2);
  PhiTaps<NG, double, S> ph;
  double psi = 0, ssrc = 0, f[5];
  if (active) {
    ph.template load<ZF>(U, d, i0, i1, i2);
    psi = a.psi[idx];
    ssrc = a.ssrc[idx];
#pragma unroll
    for (int q = 0; q < 5; ++q) f[q] = a.fac[q * n2d + k2];
  }
  load_tile<NG, double, S, ZF>(tile, U, d, x0b, x1b, i2);
  __syncthreads();
  double h2 = 0.0;
  if (active) {
    const Sums<double> s = stencil<NG, double, S>(tile, ph);
    const double lap = f[0] * s.dd0 + f[1] * s.dd1 + f[2] * s.dd2 + f[3] * s.d0 + f[4] * s.d1;
    const double Hv = lap + source<double>(ssrc, psi, s.uc);
    h2 = Hv * Hv;
    if (a.wt) h2 *= a.wt[k2];  // volume-weighted norm: H^2 times the cell volume
  }
  return block_sum<kTileThreads>(h2);
}

template <typename S, int NG, bool ZF>
__global__ void __launch_bounds__(kTileThreads) k_residual(ResidualArgs a) {
  __shared__ double tile[TileShape<NG>::W * TileShape<NG>::H];
  const double tot = residual_body<S, NG, ZF>(a, blockIdx.x, blockIdx.y, blockIdx.z, tile);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    a.partial[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = tot;
}

// Batched residual: items (grid, x0 tile, x1 tile, plane); the block sum of
// item `it` goes to partial[it]. FP64 states only.
template <int NG, bool ZF>
__global__ void __launch_bounds__(kTileThreads)
    k_batch_residual(const ResidualArgs* __restrict__ descs, const int4* __restrict__ items,
                     const int* __restrict__ nitems, double* __restrict__ partial) {
  __shared__ double tile[TileShape<NG>::W * TileShape<NG>::H];
  const int n = *nitems;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int4 w = items[it];
    const ResidualArgs a = descs[w.x];
    const double tot = residual_body<double, NG, ZF>(a, w.y, w.z, w.w, tile);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[it] = tot;
  }
}

// Per-grid L2 norms from the batched partials: block g adds partial[start_g ..
// start_g + count_g) in a fixed order; ranges[g] = (start, count, N_interior).
__global__ void __launch_bounds__(kBlock)
    k_batch_finalize(const int4* __restrict__ ranges, const double* __restrict__ partial,
                     double* __restrict__ out) {
  const int4 r = ranges[blockIdx.x];
  double s = 0.0;
  for (int j = threadIdx.x; j < r.y; j += kBlock) s += partial[r.x + j];
  const double tot = block_sum<kBlock>(s);
  if (threadIdx.x == 0) out[blockIdx.x] = r.y > 0 ? sqrt(tot / (double)r.z) : 0.0;
}

// Batched base slopes of the split-state form.
template <int NG, bool ZF>
__global__ void __launch_bounds__(kTileThreads)
    k_batch_base(const BaseArgs* __restrict__ descs, const int4* __restrict__ items,
                 const int* __restrict__ nitems) {
  __shared__ double tile[TileShape<NG>::W * TileShape<NG>::H];
  const int n = *nitems;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int4 w = items[it];
    const BaseArgs a = descs[w.x];
    base_body<NG, ZF>(a, w.y, w.z, w.w, tile);
    __syncthreads();
  }
}

// Batched rebase y_b += e: items (grid, element block of 256).
__global__ void __launch_bounds__(kBlock)
    k_batch_rebase(const RebaseArgs* __restrict__ descs, const int2* __restrict__ items,
                   const int* __restrict__ nitems) {
  const int n = *nitems;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 w = items[it];
    const RebaseArgs a = descs[w.x];
    const int t = w.y * kBlock + threadIdx.x;
    if (t < a.n) {
      a.ub[t] = a.ub[t] + (double)a.eu[t];
      a.vb[t] = a.vb[t] + (double)a.ev[t];
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_finalize(const double* __restrict__ partial,
                                                     int nparts, double divisor,
                                                     double* __restrict__ out) {
  double s = 0.0;
  for (int j = threadIdx.x; j < nparts; j += kBlock) s += partial[j];
  const double tot = block_sum<kBlock>(s);
  if (threadIdx.x == 0) {
    out[0] = sqrt(tot / divisor);
    out[1] = tot;
  }
}

// psi_singular and (1/8) A_ij A^ij at every stored point (interior and outer).
// psi_s = 1 + sum m/(2 r) and the source factor (1/8) A_ij A^ij of the
// Bowen-York extrinsic curvature at the Cartesian position X.
__device__ __forceinline__ void bowen_york_point(const Punctures& pz, const double X[3],
                                                 double& psi_out, double& src_out) {
  double psi = 1.0;
  double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int p = 0; p < pz.n; ++p) {
    double n[3];
    double r2 = 0.0;
    for (int i = 0; i < 3; ++i) {
      n[i] = X[i] - pz.x[p][i];
      r2 += n[i] * n[i];
    }
    const double r = sqrt(r2);
    for (int i = 0; i < 3; ++i) n[i] = n[i] / r;
    psi += pz.m[p] / (2.0 * r);
    const double* P = pz.P[p];
    const double* S = pz.S[p];
    const double pn = P[0] * n[0] + P[1] * n[1] + P[2] * n[2];
    const double sn[3] = {S[1] * n[2] - S[2] * n[1], S[2] * n[0] - S[0] * n[2],
                          S[0] * n[1] - S[1] * n[0]};
    const double cl = 3.0 / (2.0 * r * r);
    const double cs = 3.0 / (r * r * r);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double proj = (i == j ? 1.0 : 0.0) - n[i] * n[j];
        A[i][j] += cl * (P[i] * n[j] + P[j] * n[i] - proj * pn) +
                   cs * (sn[i] * n[j] + sn[j] * n[i]);
      }
  }
  double aa = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) aa += A[i][j] * A[i][j];
  psi_out = psi;
  src_out = aa / 8.0;
}

__global__ void __launch_bounds__(kBlock) k_sources(Dims d, const double* __restrict__ rho,
                                                    const double* __restrict__ zc,
                                                    const double* __restrict__ cphi,
                                                    const double* __restrict__ sphi,
                                                    Punctures pz, double* __restrict__ psi64,
                                                    double* __restrict__ ssrc64,
                                                    float* __restrict__ psi32,
                                                    float* __restrict__ ssrc32) {
  const int next = d.P0 * d.R1 * d.N2;
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= next) return;
  const int e = t % (d.P0 * d.R1);   // (i0, stored row) of the 2D tables
  const int i2 = t / (d.P0 * d.R1);
  const double X[3] = {rho[e] * cphi[i2], rho[e] * sphi[i2], zc[e]};
  double psi, src;
  bowen_york_point(pz, X, psi, src);
  psi64[t] = psi;
  ssrc64[t] = src;
  psi32[t] = (float)psi;
  ssrc32[t] = (float)src;
}

// ---------------------------------------------------------------------------
// Cartesian grids (the cube [-rmax, rmax]^3, x, y, z along x0, x1, x2). Every
// stored point beyond one face is an outer point; there are no images, so a
// plane tile's rim and the z taps read the stored outer layers directly. The
// Laplacian factors (1/dx_d^2, no first-derivative terms) and c^2 come from
// the same 2D tables as on the curvilinear grids; the face points take r and
// d r / d x_d from the stored coordinates cx (a.zfac): the P0 column
// x's, the R1 row y's, the planes' z's, then kappa and dx_0, dx_1, dx_2.

// Index of coordinate axis `ax` in cx.
__device__ __forceinline__ int cart_off(const Dims& d, int ax) {
  return ax == 0 ? 0 : ax == 1 ? d.P0 : d.P0 + d.R1;
}

// Interior points: one thread each on the plane-tile grid. CORR: the split-state
// form's single-precision increment (slopes as in the curvilinear kernels).
template <typename T, int NG, int STAGE, bool CORR>
__global__ void __launch_bounds__(kTileThreads) k_cart_stage(StageArgs<T> a) {
  constexpr int W = TileShape<NG>::W, H = TileShape<NG>::H;
  constexpr Weights<NG> Wt{};
  __shared__ T tile[W * H];
  const Dims& d = a.d;
  const int x0b = blockIdx.x * TX, x1b = blockIdx.y * TY, i2 = blockIdx.z;
  const int i0 = x0b + threadIdx.x, i1 = x1b + threadIdx.y;
  const bool active = i0 < d.N0 && i1 < d.N1;
  const unsigned plane = (unsigned)d.P0 * (unsigned)d.R1;
  const unsigned idx = sidx(d, active ? i0 : 0, active ? i1 : 0, i2);
  const unsigned n2d = (unsigned)d.N0 * (unsigned)d.N1;
  const unsigned k2 = active ? (unsigned)i0 + (unsigned)d.N0 * (unsigned)i1 : 0u;
  // z taps and point operands, issued before the tile barrier
  T zp[NG], zm[NG], v = 0, psi = 0, ssrc = 0, f[6], hu = 0, hv = 0;
  CombineIn<STAGE, false, T> co;
  if (active) {
#pragma unroll
    for (int k = 1; k <= NG; ++k) {
      zp[k - 1] = a.uin[idx + (unsigned)k * plane];
      zm[k - 1] = a.uin[idx - (unsigned)k * plane];
    }
    v = a.vin[idx];
    psi = a.psi[idx];
    ssrc = a.ssrc[idx];
    if constexpr (CORR) {
      hu = a.khu[idx];
      hv = a.khv[idx];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) f[q] = load_factor(a.fac, a.facb, q * n2d + k2);
    co.load(a, idx);
  }
  const int tid = threadIdx.x + TX * threadIdx.y;
  for (int e = tid; e < W * H; e += kTileThreads) {
    const int l1 = e / W;
    const int l0 = e - l1 * W;
    const int j0 = x0b + l0 - NG, j1 = x1b + l1 - NG;   // both >= -NG
    tile[e] = (j0 < d.N0 + NG && j1 < d.N1 + NG) ? a.uin[sidx(d, j0, j1, i2)] : (T)0;
  }
  __syncthreads();
  if (!active) return;
  const T* r = tile + (threadIdx.y + NG) * W + (threadIdx.x + NG);
  const T uc = r[0];
  T d0 = 0, d1 = 0, e0 = 0, e1 = 0, e2 = 0;
#pragma unroll
  for (int k = 1; k <= NG; ++k) {
    const T p0 = r[k], m0 = r[-k];
    const T p1 = r[k * W], m1 = r[-k * W];
    d0 += (T)Wt.d1[k] * (p0 - m0);
    d1 += (T)Wt.d1[k] * (p1 - m1);
    e0 += (T)Wt.d2[k] * (p0 + m0);
    e1 += (T)Wt.d2[k] * (p1 + m1);
    e2 += (T)Wt.d2[k] * (zp[k - 1] + zm[k - 1]);
  }
  const T w0 = (T)Wt.d2[0];
  const T lap = f[0] * (e0 + w0 * uc) + f[1] * (e1 + w0 * uc) + f[2] * (e2 + w0 * uc) +
                f[3] * d0 + f[4] * d1;
  T ku, kv;
  if constexpr (CORR) {
    ku = hu + (v - a.eta * uc);
    kv = hv + f[5] * (lap + source_delta(ssrc, psi, uc));
  } else {
    ku = v - a.eta * uc;
    kv = f[5] * (lap + source<T>(ssrc, psi, uc));
  }
  combine<STAGE, false, T>(a, idx, co, uc, v, ku, kv);
}

// Number of outer points on the two faces normal to axis ax.
__device__ __forceinline__ int cart_face_points(const Dims& d, int ax) {
  const int n1 = ax == 0 ? d.N1 : d.N0, n2 = ax == 2 ? d.N1 : d.N2;
  return 2 * d.NG * n1 * n2;
}

// Face point number t (all faces, x faces first): its stored index, the
// index step toward the interior, the wave speed, r and q = 1 / (2 dx dr/dn).
// False past the last face point.
template <typename T>
struct FacePoint {
  unsigned o;
  int in;
  T kappa, rr, qd;
};

template <typename T, int NG>
__device__ __forceinline__ bool cart_face_point(const Dims& d, const T* __restrict__ cx, int t,
                                                FacePoint<T>& fp) {
  int ax = 0;
  while (ax < 3 && t >= cart_face_points(d, ax)) t -= cart_face_points(d, ax++);
  if (ax == 3) return false;
  const int nf = ax == 0 ? d.N1 : d.N0, ns = ax == 2 ? d.N1 : d.N2;
  int fast, slow, out, side;
  if (ax == 0) {
    // x faces: t = layer + NG (y + N1 (z + N2 side)); a row's NG layer points
    // on one side are contiguous in memory, so the layer runs fastest
    const int layer = t % NG;
    t /= NG;
    fast = t % nf;
    t /= nf;
    slow = t % ns;
    side = t / ns;
    out = side ? d.N0 + layer : layer - NG;
  } else {
    // y and z faces: t = x + N0 (slow + n_slow (layer + NG side))
    fast = t % nf;
    t /= nf;
    slow = t % ns;
    t /= ns;
    const int layer = t % NG;
    side = t / NG;
    const int n_ax = ax == 1 ? d.N1 : d.N2;
    out = side ? n_ax + layer : -1 - layer;
  }
  int i0, i1, i2;
  if (ax == 0) { i0 = out; i1 = fast; i2 = slow; }
  else if (ax == 1) { i0 = fast; i1 = out; i2 = slow; }
  else { i0 = fast; i1 = slow; i2 = out; }
  const int q2 = planes_of(d);
  fp.kappa = cx[d.P0 + d.R1 + q2];
  const T dxa = cx[d.P0 + d.R1 + q2 + 1 + ax];
  const T x = cx[i0 + d.NG], y = cx[d.P0 + i1 + d.NG], z = cx[d.P0 + d.R1 + i2 + d.NG];
  fp.rr = sqrt(x * x + y * y + z * z);
  const T xa = ax == 0 ? x : ax == 1 ? y : z;
  fp.qd = fp.rr / ((T)2 * dxa * fabs(xa));   // 1 / (2 dx d r / d n)
  const int stride = ax == 0 ? 1 : ax == 1 ? d.P0 : d.P0 * d.R1;
  fp.in = side ? -stride : stride;            // one point toward the interior
  fp.o = sidx(d, i0, i1, i2);
  return true;
}

// The radiation condition's slope -kappa (f/r + d_r f) at a face point, f read
// at the point and its inward neighbours.
template <typename T>
__device__ __forceinline__ T cart_face_slope(const T* __restrict__ F, const FacePoint<T>& fp,
                                             bool bc4) {
  const T f0 = F[fp.o], f1 = F[fp.o + fp.in], f2 = F[fp.o + 2 * fp.in];
  const T f3 = bc4 ? F[fp.o + 3 * fp.in] : (T)0, f4 = bc4 ? F[fp.o + 4 * fp.in] : (T)0;
  return -fp.kappa * (f0 / fp.rr + outer_diff(f0, f1, f2, f3, f4, fp.qd, bc4));
}

// Stage update at face point t (none past the last): the radiation condition,
// then the stage combine; CORR adds the base slopes (the condition is linear).
template <typename T, int NG, int STAGE, bool CORR>
__device__ __forceinline__ void cart_face_stage(const StageArgs<T>& a, int t) {
  FacePoint<T> fp;
  if (!cart_face_point<T, NG>(a.d, a.zfac, t, fp)) return;
  const bool bc4 = a.bc4 != 0;
  CombineIn<STAGE, false, T> co;
  co.load(a, fp.o);
  T kuo = cart_face_slope(a.uin, fp, bc4);
  T kvo = cart_face_slope(a.vin, fp, bc4);
  if constexpr (CORR) {
    kuo = a.khu[fp.o] + kuo;
    kvo = a.khv[fp.o] + kvo;
  }
  combine<STAGE, false, T>(a, fp.o, co, a.uin[fp.o], a.vin[fp.o], kuo, kvo);
}

// Interior points in columns: a block walks `chunk` z planes of one (x0, x1)
// tile, as the curvilinear column kernel does along phi, without images: the
// padded box stores the tile's rim and the NG planes beyond each z face, so the
// z taps are a register queue filled by one load per plane, and the
// rim-extended tile of the next plane is fetched into registers while the
// current one is computed from LDS. The arithmetic is that of k_cart_stage.
template <typename T, int NG, int STAGE, bool CORR>
__global__ void __launch_bounds__(kTileThreads, 4) k_cart_col(StageArgs<T> a, int chunk) {
  constexpr int W = TileShape<NG>::W, H = TileShape<NG>::H;
  constexpr int NE = (W * H + kTileThreads - 1) / kTileThreads;
  constexpr Weights<NG> Wt{};
  __shared__ T tile[2][W * H];
  __shared__ T fl[kFacRows<T>][kTileThreads];
  const Dims& d = a.d;
  const int ft = threadIdx.x + TX * threadIdx.y;
  // one dimension of blocks: the column tiles (XCD-aware order), then the
  // face points, kTileThreads per block
  const unsigned gx = (d.N0 + TX - 1) / TX, gy = (d.N1 + TY - 1) / TY;
  const unsigned gz = (d.N2 + chunk - 1) / chunk;
  if (blockIdx.x >= gx * gy * gz) {
    cart_face_stage<T, NG, STAGE, CORR>(a, (int)(blockIdx.x - gx * gy * gz) * kTileThreads + ft);
    return;
  }
  const TileId id = xcd_tile_of(blockIdx.x, gx, gy, gz);
  const int x0b = id.x * TX, x1b = id.y * TY;
  const int z0 = id.z * chunk, z1 = min(z0 + chunk, d.N2);
  const int i0 = x0b + threadIdx.x, i1 = x1b + threadIdx.y;
  const bool active = i0 < d.N0 && i1 < d.N1;
  const unsigned plane = (unsigned)d.P0 * (unsigned)d.R1;
  // stored plane p = z + NG of the padded box starts at p * plane
  const unsigned col = sidx(d, active ? i0 : 0, active ? i1 : 0, -NG);
  const unsigned n2d = (unsigned)d.N0 * (unsigned)d.N1;
  const unsigned k2 = active ? (unsigned)i0 + (unsigned)d.N0 * (unsigned)i1 : 0u;
  // this thread's tile elements: offset within a stored plane, or none (the
  // cells past the far rim; the tile's corners are loaded but never read)
  unsigned toff[NE];
  bool tin[NE];
#pragma unroll
  for (int r = 0; r < NE; ++r) {
    const int e = ft + r * kTileThreads;
    const int l1 = e / W;
    const int l0 = e - l1 * W;
    const int j0 = x0b + l0 - NG, j1 = x1b + l1 - NG;   // both >= -NG
    tin[r] = e < W * H && j0 < d.N0 + NG && j1 < d.N1 + NG;
    toff[r] = tin[r] ? sidx(d, j0, j1, -NG) : 0u;
  }
  auto fetch = [&](T (&v)[NE], int z) {
    const unsigned pb = plane * (unsigned)(z + NG);
#pragma unroll
    for (int r = 0; r < NE; ++r) v[r] = tin[r] ? a.uin[toff[r] + pb] : (T)0;
  };
  auto store = [&](const T (&v)[NE], T* t) {
#pragma unroll
    for (int r = 0; r < NE; ++r) {
      const int e = ft + r * kTileThreads;
      if (e < W * H) t[e] = v[r];
    }
  };
  // z queue q[j] = u(z - NG + j), j = 0..2NG, for z = z0 (stored planes z0 ... z0 + 2NG)
  T q[2 * NG + 1];
  T f[6];
  auto fac = [&](int r) -> T {
    if constexpr (kFacRows<T> == 6) return fl[r][ft];
    else return f[r];
  };
  PointIn<STAGE, CORR, T> cur;
  if (active) {
#pragma unroll
    for (int j = 0; j <= 2 * NG; ++j) q[j] = a.uin[col + plane * (unsigned)(z0 + j)];
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      if constexpr (kFacRows<T> == 6) fl[r][ft] = load_factor(a.fac, a.facb, r * n2d + k2);
      else f[r] = load_factor(a.fac, a.facb, r * n2d + k2);
    }
    cur.load(a, col + plane * (unsigned)(z0 + NG));
  }
  {
    T t0[NE];
    fetch(t0, z0);
    store(t0, tile[0]);
  }
  __syncthreads();
  for (int z = z0; z < z1; ++z) {
    const int buf = (z - z0) & 1;
    const bool more = z + 1 < z1;
    // prefetch plane z + 1 (its queue entry is u(z + 1 + NG), stored plane z + 1 + 2NG)
    T tn[NE];
    PointIn<STAGE, CORR, T> nxt;
    T qn = (T)0;
    if (more) {
      fetch(tn, z + 1);
      if (active) {
        qn = a.uin[col + plane * (unsigned)(z + 1 + 2 * NG)];
        nxt.load(a, col + plane * (unsigned)(z + 1 + NG));
      }
    }
    if (active) {
      const T* r = tile[buf] + (threadIdx.y + NG) * W + (threadIdx.x + NG);
      const T uc = r[0];
      T d0 = 0, d1 = 0, e0 = 0, e1 = 0, e2 = 0;
#pragma unroll
      for (int k = 1; k <= NG; ++k) {
        const T p0 = r[k], m0 = r[-k];
        const T p1 = r[k * W], m1 = r[-k * W];
        d0 += (T)Wt.d1[k] * (p0 - m0);
        d1 += (T)Wt.d1[k] * (p1 - m1);
        e0 += (T)Wt.d2[k] * (p0 + m0);
        e1 += (T)Wt.d2[k] * (p1 + m1);
        e2 += (T)Wt.d2[k] * (q[NG + k] + q[NG - k]);
      }
      const T w0 = (T)Wt.d2[0];
      const T lap = fac(0) * (e0 + w0 * uc) + fac(1) * (e1 + w0 * uc) +
                    fac(2) * (e2 + w0 * uc) + fac(3) * d0 + fac(4) * d1;
      T ku, kv;
      if constexpr (CORR) {
        ku = cur.khu + (cur.v - a.eta * uc);
        kv = cur.khv + fac(5) * (lap + source_delta(cur.ssrc, cur.psi, uc));
      } else {
        ku = cur.v - a.eta * uc;
        kv = fac(5) * (lap + source<T>(cur.ssrc, cur.psi, uc));
      }
      combine_pt<STAGE, CORR, T>(a, col + plane * (unsigned)(z + NG), cur, uc, ku, kv);
    }
    if (more) {
      store(tn, tile[buf ^ 1]);
#pragma unroll
      for (int j = 0; j < 2 * NG; ++j) q[j] = q[j + 1];
      q[2 * NG] = qn;
      cur = nxt;
    }
    __syncthreads();
  }
}

// Face points, one thread each: the radiation condition k_f = -c (f/r + d_r
// f) with d_r f = (d f / d n) / (d r / d n) along the outward normal n = +-x_d
// (d r / d n = |x_d| / r), the one-sided difference toward the interior, then
// the stage combine. Threads run along x0: on the y and z faces over a row,
// on the x faces over a row end's NG layer points.
template <typename T, int NG, int STAGE, bool CORR>
__global__ void __launch_bounds__(kBlock) k_cart_faces(StageArgs<T> a) {
  cart_face_stage<T, NG, STAGE, CORR>(a, blockIdx.x * kBlock + threadIdx.x);
}

// The split-state form's base evaluation on a Cartesian grid (FP64 state u, v):
// interior points on plane tiles, the slopes k(y_b) of Eq. 5, p_b = psi_s + u
// and S_src p_b^-7 in single precision, the increment zeroed.
template <int NG>
__global__ void __launch_bounds__(kTileThreads) k_cart_base(BaseArgs a) {
  constexpr int W = TileShape<NG>::W, H = TileShape<NG>::H;
  constexpr Weights<NG> Wt{};
  __shared__ double tile[W * H];
  const Dims& d = a.d;
  const int x0b = blockIdx.x * TX, x1b = blockIdx.y * TY, i2 = blockIdx.z;
  const int i0 = x0b + threadIdx.x, i1 = x1b + threadIdx.y;
  const bool active = i0 < d.N0 && i1 < d.N1;
  const unsigned plane = (unsigned)d.P0 * (unsigned)d.R1;
  const unsigned idx = sidx(d, active ? i0 : 0, active ? i1 : 0, i2);
  const unsigned n2d = (unsigned)d.N0 * (unsigned)d.N1;
  const unsigned k2 = active ? (unsigned)i0 + (unsigned)d.N0 * (unsigned)i1 : 0u;
  double zp[NG], zm[NG], v = 0, psi = 0, ssrc = 0, f[6];
  if (active) {
#pragma unroll
    for (int k = 1; k <= NG; ++k) {
      zp[k - 1] = a.u[idx + (unsigned)k * plane];
      zm[k - 1] = a.u[idx - (unsigned)k * plane];
    }
    v = a.v[idx];
    psi = a.psi[idx];
    ssrc = a.ssrc[idx];
#pragma unroll
    for (int q = 0; q < 6; ++q) f[q] = a.fac[q * n2d + k2];
  }
  const int tid = threadIdx.x + TX * threadIdx.y;
  for (int e = tid; e < W * H; e += kTileThreads) {
    const int l1 = e / W;
    const int l0 = e - l1 * W;
    const int j0 = x0b + l0 - NG, j1 = x1b + l1 - NG;   // both >= -NG
    tile[e] = (j0 < d.N0 + NG && j1 < d.N1 + NG) ? a.u[sidx(d, j0, j1, i2)] : 0.0;
  }
  __syncthreads();
  if (!active) return;
  const double* r = tile + (threadIdx.y + NG) * W + (threadIdx.x + NG);
  const double uc = r[0];
  double d0 = 0, d1 = 0, e0 = 0, e1 = 0, e2 = 0;
#pragma unroll
  for (int k = 1; k <= NG; ++k) {
    const double p0 = r[k], m0 = r[-k];
    const double p1 = r[k * W], m1 = r[-k * W];
    d0 += Wt.d1[k] * (p0 - m0);
    d1 += Wt.d1[k] * (p1 - m1);
    e0 += Wt.d2[k] * (p0 + m0);
    e1 += Wt.d2[k] * (p1 + m1);
    e2 += Wt.d2[k] * (zp[k - 1] + zm[k - 1]);
  }
  const double w0 = Wt.d2[0];
  const double lap = f[0] * (e0 + w0 * uc) + f[1] * (e1 + w0 * uc) + f[2] * (e2 + w0 * uc) +
                     f[3] * d0 + f[4] * d1;
  const double p = psi + uc;
  const double p2 = p * p, p4 = p2 * p2, p7 = p4 * p2 * p;
  a.khu[idx] = (float)(v - a.eta * uc);
  a.khv[idx] = (float)(f[5] * (lap + ssrc / p7));
  a.pb[idx] = (float)p;
  a.sp7[idx] = (float)(ssrc / p7);
  a.eu[idx] = 0.0f;
  a.ev[idx] = 0.0f;
}

// The base evaluation at the face points (radiation condition in FP64).
template <int NG>
__global__ void __launch_bounds__(kBlock) k_cart_base_faces(BaseArgs a) {
  FacePoint<double> fp;
  if (!cart_face_point<double, NG>(a.d, a.zfac, blockIdx.x * kBlock + threadIdx.x, fp)) return;
  const bool bc4 = a.bc4 != 0;
  a.khu[fp.o] = (float)cart_face_slope(a.u, fp, bc4);
  a.khv[fp.o] = (float)cart_face_slope(a.v, fp, bc4);
  a.pb[fp.o] = (float)(a.psi[fp.o] + a.u[fp.o]);
  a.sp7[fp.o] = 0.0f;
  a.eu[fp.o] = 0.0f;
  a.ev[fp.o] = 0.0f;
}

// Residual H in FP64 on the interior of a Cartesian grid (state of storage
// type S), block sums of H^2 in the partial layout of k_residual.
template <typename S, int NG>
__global__ void __launch_bounds__(kTileThreads) k_cart_residual(ResidualArgs a) {
  constexpr Weights<NG> Wt{};
  const Dims& d = a.d;
  const S* U = static_cast<const S*>(a.u);
  const int i0 = blockIdx.x * TX + threadIdx.x, i1 = blockIdx.y * TY + threadIdx.y;
  const int i2 = blockIdx.z;
  double h2 = 0.0;
  if (i0 < d.N0 && i1 < d.N1) {
    const unsigned idx = sidx(d, i0, i1, i2);
    const unsigned st[3] = {1u, (unsigned)d.P0, (unsigned)d.P0 * (unsigned)d.R1};
    const unsigned n2d = (unsigned)d.N0 * (unsigned)d.N1;
    const unsigned k2 = (unsigned)i0 + (unsigned)d.N0 * (unsigned)i1;
    const double uc = (double)U[idx];
    double e[3] = {0, 0, 0};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int k = 1; k <= NG; ++k)
        e[ax] += Wt.d2[k] * ((double)U[idx + (unsigned)k * st[ax]] +
                             (double)U[idx - (unsigned)k * st[ax]]);
    const double w0 = Wt.d2[0];
    const double lap = a.fac[k2] * (e[0] + w0 * uc) + a.fac[n2d + k2] * (e[1] + w0 * uc) +
                       a.fac[2 * n2d + k2] * (e[2] + w0 * uc);
    const double Hv = lap + source<double>(a.ssrc[idx], a.psi[idx], uc);
    h2 = Hv * Hv;
  }
  const double tot = block_sum<kTileThreads>(h2);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    a.partial[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = tot;
}

// Sources psi_s and S_src at every stored point of a Cartesian grid.
__global__ void __launch_bounds__(kBlock) k_cart_sources(Dims d, const double* __restrict__ cx,
                                                         Punctures pz, double* __restrict__ psi64,
                                                         double* __restrict__ ssrc64,
                                                         float* __restrict__ psi32,
                                                         float* __restrict__ ssrc32) {
  const int next = d.P0 * d.R1 * planes_of(d);
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= next) return;
  const int j0 = t % d.P0, j1 = (t / d.P0) % d.R1, j2 = t / (d.P0 * d.R1);
  const double X[3] = {cx[j0], cx[d.P0 + j1], cx[d.P0 + d.R1 + j2]};
  double psi, src;
  bowen_york_point(pz, X, psi, src);
  psi64[t] = psi;
  ssrc64[t] = src;
  psi32[t] = (float)psi;
  ssrc32[t] = (float)src;
}

template <typename A, typename B>
__global__ void __launch_bounds__(kBlock) k_convert(const A* __restrict__ src,
                                                    B* __restrict__ dst, int n) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t < n) dst[t] = (B)src[t];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T* __restrict__ dst, T value, int n) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t < n) dst[t] = value;
}

// dst = a * src elementwise (n values).
__global__ void __launch_bounds__(kBlock) k_scale(double* __restrict__ dst,
                                                  const double* __restrict__ src, double a, int n) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t < n) dst[t] = a * src[t];
}

inline int nblocks(int n) { return (n + kBlock - 1) / kBlock; }

inline dim3 tile_grid(const Dims& d) {
  return dim3((d.N0 + TX - 1) / TX, (d.N1 + TY - 1) / TY, d.N2);
}

// Launches kernel k with the tile grid, optionally bracketed by timing events
// recorded in the same dispatch (hipExtLaunchKernelGGL).
template <typename K, typename A>
hipError_t tile_launch(K k, const A& args, const Dims& d, hipStream_t s, hipEvent_t t0,
                       hipEvent_t t1) {
  const dim3 grid = tile_grid(d), block(TX, TY, 1);
  if (t0 && t1)
    hipExtLaunchKernelGGL(k, grid, block, 0, s, t0, t1, 0, args);
  else
    k<<<grid, block, 0, s>>>(args);
  return hipGetLastError();
}

template <typename K, typename A>
hipError_t col_launch(K k, const A& args, int chunk, hipStream_t s, hipEvent_t t0,
                      hipEvent_t t1) {
  const Dims& d = args.d;
  // column tiles, then the outer-point blocks (k_stage_col)
  const dim3 grid(((d.N0 + TX - 1) / TX) * ((d.N1 + TY - 1) / TY) * ((d.N2 + chunk - 1) / chunk) +
                  outer_blocks(d));
  const dim3 block(TX, TY, 1);
  if (t0 && t1)
    hipExtLaunchKernelGGL(k, grid, block, 0, s, t0, t1, 0, args, chunk);
  else
    k<<<grid, block, 0, s>>>(args, chunk);
  return hipGetLastError();
}

template <typename T, int NG, bool NT, bool CORR, bool ZF>
hipError_t stage_dispatch_zf(int stage, const StageArgs<T>& a, hipStream_t s, hipEvent_t t0,
                             hipEvent_t t1) {
  switch (stage) {
    case 1: return tile_launch(k_stage<T, NG, 1, NT, CORR, ZF>, a, a.d, s, t0, t1);
    case 2: return tile_launch(k_stage<T, NG, 2, NT, CORR, ZF>, a, a.d, s, t0, t1);
    case 3: return tile_launch(k_stage<T, NG, 3, NT, CORR, ZF>, a, a.d, s, t0, t1);
    case 4: return tile_launch(k_stage<T, NG, 4, NT, CORR, ZF>, a, a.d, s, t0, t1);
    default: return hipErrorInvalidValue;
  }
}

// Plane-tile instance for grids with (ZF) or without stored z-face rows.
template <typename T, int NG, bool NT, bool CORR>
hipError_t stage_dispatch_nt(int stage, const StageArgs<T>& a, hipStream_t s, hipEvent_t t0,
                             hipEvent_t t1) {
  return a.d.zo ? stage_dispatch_zf<T, NG, NT, CORR, true>(stage, a, s, t0, t1)
                : stage_dispatch_zf<T, NG, NT, CORR, false>(stage, a, s, t0, t1);
}

template <typename T, int NG, bool CORR, bool ZF>
hipError_t col_dispatch_zf(int stage, const StageArgs<T>& a, int ch, hipStream_t s,
                           hipEvent_t t0, hipEvent_t t1) {
  switch (stage) {
    case 1: return col_launch(k_stage_col<T, NG, 1, CORR, ZF>, a, ch, s, t0, t1);
    case 2: return col_launch(k_stage_col<T, NG, 2, CORR, ZF>, a, ch, s, t0, t1);
    case 3: return col_launch(k_stage_col<T, NG, 3, CORR, ZF>, a, ch, s, t0, t1);
    case 4: return col_launch(k_stage_col<T, NG, 4, CORR, ZF>, a, ch, s, t0, t1);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int NG, bool CORR>
hipError_t col_dispatch(int stage, const StageArgs<T>& a, int ch, hipStream_t s, hipEvent_t t0,
                        hipEvent_t t1) {
  return a.d.zo ? col_dispatch_zf<T, NG, CORR, true>(stage, a, ch, s, t0, t1)
                : col_dispatch_zf<T, NG, CORR, false>(stage, a, ch, s, t0, t1);
}


// A Cartesian stage: the interior kernel, then the face kernel (timing events,
// when given, bracket both).
template <typename T, int NG, int STAGE, bool CORR>
hipError_t cart_stage_launch(const StageArgs<T>& a, hipStream_t s, hipEvent_t t0,
                             hipEvent_t t1) {
  const Dims& d = a.d;
  const dim3 block(TX, TY, 1);
  const int nf = 2 * d.NG * (d.N1 * d.N2 + d.N0 * d.N2 + d.N0 * d.N1);
  // interior: plane tiles (variant 1, then the face kernel) or z columns of
  // `chunk` planes (variant 2, the face points in blocks of the same launch)
  const bool cols = a.variant == 2;
  const int ch = a.chunk > 0 ? a.chunk : 1;
  if (cols) {
    const dim3 grid(((d.N0 + TX - 1) / TX) * ((d.N1 + TY - 1) / TY) * ((d.N2 + ch - 1) / ch) +
                    (nf + kTileThreads - 1) / kTileThreads);
    if (t0 && t1)
      hipExtLaunchKernelGGL(k_cart_col<T, NG, STAGE, CORR>, grid, block, 0, s, t0, t1, 0, a, ch);
    else
      k_cart_col<T, NG, STAGE, CORR><<<grid, block, 0, s>>>(a, ch);
    return hipGetLastError();
  }
  const dim3 grid = tile_grid(d);
  if (t0 && t1)
    hipExtLaunchKernelGGL(k_cart_stage<T, NG, STAGE, CORR>, grid, block, 0, s, t0, nullptr, 0, a);
  else
    k_cart_stage<T, NG, STAGE, CORR><<<grid, block, 0, s>>>(a);
  if (t0 && t1)
    hipExtLaunchKernelGGL(k_cart_faces<T, NG, STAGE, CORR>, dim3(nblocks(nf)), dim3(kBlock), 0, s,
                          nullptr, t1, 0, a);
  else
    k_cart_faces<T, NG, STAGE, CORR><<<nblocks(nf), kBlock, 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, int NG, bool CORR>
hipError_t cart_dispatch(int stage, const StageArgs<T>& a, hipStream_t s, hipEvent_t t0,
                         hipEvent_t t1) {
  switch (stage) {
    case 1: return cart_stage_launch<T, NG, 1, CORR>(a, s, t0, t1);
    case 2: return cart_stage_launch<T, NG, 2, CORR>(a, s, t0, t1);
    case 3: return cart_stage_launch<T, NG, 3, CORR>(a, s, t0, t1);
    case 4: return cart_stage_launch<T, NG, 4, CORR>(a, s, t0, t1);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int NG>
hipError_t stage_dispatch(int stage, const StageArgs<T>& a, hipStream_t s, hipEvent_t t0,
                          hipEvent_t t1) {
  if (a.d.cart) {
    if (a.corr) {
      // the split-state increment runs in single precision only
      if constexpr (std::is_same<T, float>::value) return cart_dispatch<T, NG, true>(stage, a, s, t0, t1);
      return hipErrorInvalidValue;
    }
    return cart_dispatch<T, NG, false>(stage, a, s, t0, t1);
  }
  const int ch = a.chunk > 0 ? a.chunk : 1;
  if constexpr (std::is_same<T, float>::value) {
    if (a.corr)
      return a.variant == 2 ? col_dispatch<T, NG, true>(stage, a, ch, s, t0, t1)
                            : stage_dispatch_nt<T, NG, false, true>(stage, a, s, t0, t1);
  }
  if (a.variant == 2) return col_dispatch<T, NG, false>(stage, a, ch, s, t0, t1);
  return a.streaming ? stage_dispatch_nt<T, NG, true, false>(stage, a, s, t0, t1)
                     : stage_dispatch_nt<T, NG, false, false>(stage, a, s, t0, t1);
}

template <typename T>
hipError_t stage_order(int order, int stage, const StageArgs<T>& a, hipStream_t s,
                       hipEvent_t t0, hipEvent_t t1) {
  switch (order) {
    case 2: return stage_dispatch<T, 1>(stage, a, s, t0, t1);
    case 4: return stage_dispatch<T, 2>(stage, a, s, t0, t1);
    case 6: return stage_dispatch<T, 3>(stage, a, s, t0, t1);
    case 8: return stage_dispatch<T, 4>(stage, a, s, t0, t1);
    case 10: return stage_dispatch<T, 5>(stage, a, s, t0, t1);
    default: return hipErrorInvalidValue;
  }
}

template <typename S, bool ZF>
hipError_t residual_order_zf(int order, const ResidualArgs& a, hipStream_t s) {
  switch (order) {
    case 2: return tile_launch(k_residual<S, 1, ZF>, a, a.d, s, nullptr, nullptr);
    case 4: return tile_launch(k_residual<S, 2, ZF>, a, a.d, s, nullptr, nullptr);
    case 6: return tile_launch(k_residual<S, 3, ZF>, a, a.d, s, nullptr, nullptr);
    case 8: return tile_launch(k_residual<S, 4, ZF>, a, a.d, s, nullptr, nullptr);
    case 10: return tile_launch(k_residual<S, 5, ZF>, a, a.d, s, nullptr, nullptr);
    default: return hipErrorInvalidValue;
  }
}

template <typename S>
hipError_t residual_order(int order, const ResidualArgs& a, hipStream_t s) {
  if (a.d.cart) {
    switch (order) {
      case 2: return tile_launch(k_cart_residual<S, 1>, a, a.d, s, nullptr, nullptr);
      case 4: return tile_launch(k_cart_residual<S, 2>, a, a.d, s, nullptr, nullptr);
      case 6: return tile_launch(k_cart_residual<S, 3>, a, a.d, s, nullptr, nullptr);
      case 8: return tile_launch(k_cart_residual<S, 4>, a, a.d, s, nullptr, nullptr);
      case 10: return tile_launch(k_cart_residual<S, 5>, a, a.d, s, nullptr, nullptr);
      default: return hipErrorInvalidValue;
    }
  }
  return a.d.zo ? residual_order_zf<S, true>(order, a, s) : residual_order_zf<S, false>(order, a, s);
}

template <bool ZF>
hipError_t base_order(int order, const BaseArgs& a, hipStream_t s) {
  switch (order) {
    case 2: return tile_launch(k_base<1, ZF>, a, a.d, s, nullptr, nullptr);
    case 4: return tile_launch(k_base<2, ZF>, a, a.d, s, nullptr, nullptr);
    case 6: return tile_launch(k_base<3, ZF>, a, a.d, s, nullptr, nullptr);
    case 8: return tile_launch(k_base<4, ZF>, a, a.d, s, nullptr, nullptr);
    case 10: return tile_launch(k_base<5, ZF>, a, a.d, s, nullptr, nullptr);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int residual_blocks(const Dims& d) {
  const dim3 g = tile_grid(d);
  return (int)(g.x * g.y * g.z);
}

hipError_t launch_stage(int order, int stage, const StageArgs<double>& a, hipStream_t s,
                        hipEvent_t t0, hipEvent_t t1) {
  return stage_order<double>(order, stage, a, s, t0, t1);
}
hipError_t launch_stage(int order, int stage, const StageArgs<float>& a, hipStream_t s,
                        hipEvent_t t0, hipEvent_t t1) {
  return stage_order<float>(order, stage, a, s, t0, t1);
}

hipError_t launch_residual(int order, bool fp32_state, const ResidualArgs& a, hipStream_t s) {
  return fp32_state ? residual_order<float>(order, a, s) : residual_order<double>(order, a, s);
}

hipError_t launch_finalize(const double* partial, int nparts, double divisor, double* out,
                           hipStream_t s) {
  k_finalize<<<1, kBlock, 0, s>>>(partial, nparts, divisor, out);
  return hipGetLastError();
}

hipError_t launch_sources(const Dims& d, const double* rho, const double* zc,
                          const double* cphi, const double* sphi, const Punctures& p,
                          double* psi64, double* ssrc64, float* psi32, float* ssrc32,
                          hipStream_t s) {
  const int next = d.P0 * d.R1 * d.N2;
  k_sources<<<nblocks(next), kBlock, 0, s>>>(d, rho, zc, cphi, sphi, p, psi64, ssrc64, psi32,
                                             ssrc32);
  return hipGetLastError();
}

hipError_t launch_cart_sources(const Dims& d, const double* cx, const Punctures& p,
                               double* psi64, double* ssrc64, float* psi32, float* ssrc32,
                               hipStream_t s) {
  const int next = d.P0 * d.R1 * planes_of(d);
  k_cart_sources<<<nblocks(next), kBlock, 0, s>>>(d, cx, p, psi64, ssrc64, psi32, ssrc32);
  return hipGetLastError();
}

template <int NG>
hipError_t cart_base(const BaseArgs& a, hipStream_t s) {
  const Dims& d = a.d;
  const int nf = 2 * d.NG * (d.N1 * d.N2 + d.N0 * d.N2 + d.N0 * d.N1);
  k_cart_base<NG><<<tile_grid(d), dim3(TX, TY, 1), 0, s>>>(a);
  k_cart_base_faces<NG><<<nblocks(nf), kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_base(int order, const BaseArgs& a, hipStream_t s) {
  if (a.d.cart) {
    switch (order) {
      case 2: return cart_base<1>(a, s);
      case 4: return cart_base<2>(a, s);
      case 6: return cart_base<3>(a, s);
      case 8: return cart_base<4>(a, s);
      case 10: return cart_base<5>(a, s);
      default: return hipErrorInvalidValue;
    }
  }
  return a.d.zo ? base_order<true>(order, a, s) : base_order<false>(order, a, s);
}

hipError_t launch_rebase(double* ub, double* vb, const float* eu, const float* ev, int n,
                         hipStream_t s) {
  k_rebase<<<nblocks(n), kBlock, 0, s>>>(ub, vb, eu, ev, n);
  return hipGetLastError();
}

template <int NG, bool ZF>
hipError_t batch_stage_ng(int stage, bool fp32_split, const void* descs, const int4* items,
                          const int* nitems, int nblocks_persistent, hipStream_t s) {
  const dim3 block(TX, TY, 1), grid(nblocks_persistent);
  if (fp32_split) {
    const StageArgs<float>* d = static_cast<const StageArgs<float>*>(descs);
    switch (stage) {
      case 1: k_batch_stage<float, NG, 1, true, ZF><<<grid, block, 0, s>>>(d, items, nitems); break;
      case 2: k_batch_stage<float, NG, 2, true, ZF><<<grid, block, 0, s>>>(d, items, nitems); break;
      case 3: k_batch_stage<float, NG, 3, true, ZF><<<grid, block, 0, s>>>(d, items, nitems); break;
      case 4: k_batch_stage<float, NG, 4, true, ZF><<<grid, block, 0, s>>>(d, items, nitems); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const StageArgs<double>* d = static_cast<const StageArgs<double>*>(descs);
    switch (stage) {
      case 1: k_batch_stage<double, NG, 1, false, ZF><<<grid, block, 0, s>>>(d, items, nitems); break;
      case 2: k_batch_stage<double, NG, 2, false, ZF><<<grid, block, 0, s>>>(d, items, nitems); break;
      case 3: k_batch_stage<double, NG, 3, false, ZF><<<grid, block, 0, s>>>(d, items, nitems); break;
      case 4: k_batch_stage<double, NG, 4, false, ZF><<<grid, block, 0, s>>>(d, items, nitems); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <bool ZF>
hipError_t batch_stage_order(int order, int stage, bool fp32_split, const void* descs,
                             const int4* items, const int* nitems, int nblocks_persistent,
                             hipStream_t s) {
  switch (order) {
    case 2: return batch_stage_ng<1, ZF>(stage, fp32_split, descs, items, nitems, nblocks_persistent, s);
    case 4: return batch_stage_ng<2, ZF>(stage, fp32_split, descs, items, nitems, nblocks_persistent, s);
    case 6: return batch_stage_ng<3, ZF>(stage, fp32_split, descs, items, nitems, nblocks_persistent, s);
    case 8: return batch_stage_ng<4, ZF>(stage, fp32_split, descs, items, nitems, nblocks_persistent, s);
    case 10: return batch_stage_ng<5, ZF>(stage, fp32_split, descs, items, nitems, nblocks_persistent, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_stage(int order, int stage, bool fp32_split, bool zfaces, const void* descs,
                              const int4* items, const int* nitems, int nblocks_persistent,
                              hipStream_t s) {
  return zfaces ? batch_stage_order<true>(order, stage, fp32_split, descs, items, nitems,
                                          nblocks_persistent, s)
                : batch_stage_order<false>(order, stage, fp32_split, descs, items, nitems,
                                           nblocks_persistent, s);
}

template <bool ZF>
hipError_t batch_residual_order(int order, const ResidualArgs* descs, const int4* items,
                                const int* nitems, double* partial, int nblocks_persistent,
                                hipStream_t s) {
  const dim3 block(TX, TY, 1), grid(nblocks_persistent);
  switch (order) {
    case 2: k_batch_residual<1, ZF><<<grid, block, 0, s>>>(descs, items, nitems, partial); break;
    case 4: k_batch_residual<2, ZF><<<grid, block, 0, s>>>(descs, items, nitems, partial); break;
    case 6: k_batch_residual<3, ZF><<<grid, block, 0, s>>>(descs, items, nitems, partial); break;
    case 8: k_batch_residual<4, ZF><<<grid, block, 0, s>>>(descs, items, nitems, partial); break;
    case 10: k_batch_residual<5, ZF><<<grid, block, 0, s>>>(descs, items, nitems, partial); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_residual(int order, bool zfaces, const ResidualArgs* descs,
                                 const int4* items, const int* nitems, double* partial,
                                 int nblocks_persistent, hipStream_t s) {
  return zfaces ? batch_residual_order<true>(order, descs, items, nitems, partial,
                                             nblocks_persistent, s)
                : batch_residual_order<false>(order, descs, items, nitems, partial,
                                              nblocks_persistent, s);
}

hipError_t launch_batch_finalize(const int4* ranges, const double* partial, double* out,
                                 int ngrids, hipStream_t s) {
  k_batch_finalize<<<ngrids, kBlock, 0, s>>>(ranges, partial, out);
  return hipGetLastError();
}

template <bool ZF>
hipError_t batch_base_order(int order, const BaseArgs* descs, const int4* items,
                            const int* nitems, int nblocks_persistent, hipStream_t s) {
  const dim3 block(TX, TY, 1), grid(nblocks_persistent);
  switch (order) {
    case 2: k_batch_base<1, ZF><<<grid, block, 0, s>>>(descs, items, nitems); break;
    case 4: k_batch_base<2, ZF><<<grid, block, 0, s>>>(descs, items, nitems); break;
    case 6: k_batch_base<3, ZF><<<grid, block, 0, s>>>(descs, items, nitems); break;
    case 8: k_batch_base<4, ZF><<<grid, block, 0, s>>>(descs, items, nitems); break;
    case 10: k_batch_base<5, ZF><<<grid, block, 0, s>>>(descs, items, nitems); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_base(int order, bool zfaces, const BaseArgs* descs, const int4* items,
                             const int* nitems, int nblocks_persistent, hipStream_t s) {
  return zfaces ? batch_base_order<true>(order, descs, items, nitems, nblocks_persistent, s)
                : batch_base_order<false>(order, descs, items, nitems, nblocks_persistent, s);
}

hipError_t launch_batch_rebase(const RebaseArgs* descs, const int2* items, const int* nitems,
                               int nblocks_persistent, hipStream_t s) {
  k_batch_rebase<<<nblocks_persistent, kBlock, 0, s>>>(descs, items, nitems);
  return hipGetLastError();
}

hipError_t launch_to_fp32(const double* src, float* dst, int n, hipStream_t s) {
  k_convert<double, float><<<nblocks(n), kBlock, 0, s>>>(src, dst, n);
  return hipGetLastError();
}
hipError_t launch_to_fp64(const float* src, double* dst, int n, hipStream_t s) {
  k_convert<float, double><<<nblocks(n), kBlock, 0, s>>>(src, dst, n);
  return hipGetLastError();
}
hipError_t launch_scale(double* dst, const double* src, double a, int n, hipStream_t s) {
  k_scale<<<nblocks(n), kBlock, 0, s>>>(dst, src, a, n);
  return hipGetLastError();
}

hipError_t launch_fill(double* dst, double value, int n, hipStream_t s) {
  k_fill<double><<<nblocks(n), kBlock, 0, s>>>(dst, value, n);
  return hipGetLastError();
}
hipError_t launch_fill(float* dst, float value, int n, hipStream_t s) {
  k_fill<float><<<nblocks(n), kBlock, 0, s>>>(dst, value, n);
  return hipGetLastError();
}

}  // namespace hr
