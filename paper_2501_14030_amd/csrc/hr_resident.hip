// Resident RK4 kernel for small grids (gfx950).
//
// At the paper's grid sizes (128 x 128 x 16) one RK4 stage moves ~22 MB and a
// stage kernel is bound by launch and memory latency, not bandwidth. Here one
// launch runs many whole RK4 steps (Algorithm 1, inner loop; RHS
// of Eq. 5 with the radiation condition at the outer points) and the state
// never leaves the chip:
//   * block b owns an 8 x 8 (or, for grids with few such patches, 8 x 4)
//     patch of (x0, x1) columns through all N2 phi planes (the last x0 patch
//     also the NG outer points of its rows); its threads are the patch's
//     (x0, x1) positions x up to 16 plane groups;
//   * y_n, the stage input v, the accumulator, psi_s and S_src of the block's
//     points sit in registers; the stage input u of the whole patch plus its
//     NG-deep rim (all planes) sits in LDS, so every stencil tap, phi included,
//     is an LDS read;
//   * after each stage the block writes its new stage input u to a global
//     exchange array (one per stage parity) and raises its stage counter; the
//     next stage waits only for the counters of its exchange partners (the
//     owners of its rim taps; the relation is symmetric), then loads its rim
//     from the exchange array. The exchange array is packed by patch
//     ([patch][plane][x1][x0], 512 contiguous bytes per 8 x 8 patch plane in
//     FP64), so a block's publish is whole cache lines and each rim strip
//     spans a few lines of one patch plane instead of one line per grid row;
//     the initial state is published the same way before the first stage.
//     Rim cells that are images of the patch's own points (inner-boundary
//     reflections onto itself) are copied within LDS, and the outer points,
//     read only by their own patch, stay in LDS;
//   * the image copies, the phi sums, the source term and the outer points'
//     radiation condition need only the patch's own cells and are computed
//     while the rim loads are in flight.
// All blocks are resident at once: each takes more than half of a compute
// unit's LDS, and the grid has at most as many blocks as the device has
// compute units (checked by occupancy before use).
// Exchange data and counters are written and read with agent-scope atomics,
// which are coherent across the XCDs' L2 caches without cache-wide
// write-back or invalidate; a full s_waitcnt before the block barrier orders
// the data stores before the counter store. Every wait is bounded: a poll
// count past spin_limit sets err, and the blocks leave their loops.
//
// The arithmetic per point is that of the stage kernels (in FP64 the same
// stencil summation order and stage combine; the single-precision instances
// fold the x0/x1 sums with the metric factors, see below), so results match
// them to rounding.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "hr_internal.h"
#include "hr_stencil.h"

namespace hr {
namespace {

constexpr int RB = kResPatch;

// Row stride (in elements) of an LDS tile of rows of n elements: the smallest
// w >= n with w = 8 (mod 16). For doubles, the two rows of 8 that one 16-lane
// group of a 64-bit LDS access reads fall on disjoint halves of the 32 banks;
// for floats, the four rows of 8 that one 32-lane group reads fall on four
// disjoint quarters.
constexpr int tile_row(int n) { return n + ((8 - n % 16) + 16) % 16; }
static_assert(tile_row(18) == 24 && tile_row(16) == 24 && tile_row(13) == 24, "tile rows");

template <typename T>
__device__ __forceinline__ void xstore(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T xload(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_zero_u32(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// A patch is RB = 8 columns (x0) by RY = 8 or 4 rows (x1), NP = RB RY
// positions. RT threads = NP positions x PG plane groups; plane group g holds
// planes g, g + PG, ... (NPT of them). T = double: the FP64 state; T = float
// with CORR: the split-state form's increment (slopes as in the stage kernels).
template <typename T, int NG, int NPT, int RT, bool CORR, int RY>
__device__ __forceinline__ void resident_body(const ResidentArgsT<T>& a, const int b) {
  constexpr int NP = RB * RY;                    // positions per plane
  constexpr int PG = RT / NP;
  constexpr int RW = tile_row(RB + 2 * NG);      // LDS tile row (x0) stride, padded
  constexpr int TP = RW * (RY + 2 * NG);         // tile cells per plane (corners unused)
  constexpr int VW = tile_row(RB + NG);          // v tile row: patch columns + outer
  constexpr int NRX = 2 * NG * RY;               // x0-side rim cells per plane
  constexpr int NRIM = NRX + 2 * NG * RB;        // rim cells per plane
  constexpr int NR = (NRIM * PG * NPT + RT - 1) / RT;
  constexpr int NQ = (NG * RY * PG * NPT + RT - 1) / RT;
  static_assert(NP * PG == RT && (NP & (NP - 1)) == 0, "block shape");
  constexpr Weights<NG> Wt{};
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  __shared__ int bad;

  const Dims& d = a.d;
  const int N2 = d.N2;
  T* ut = smem;                      // [N2][RY + 2 NG][RW]
  T* vt = smem + N2 * TP;            // [N2][RY][VW]
  const int t = threadIdx.x, pos = t & (NP - 1), x0l = pos & 7, x1l = pos >> 3, grp = t / NP;
  const int bx = b % a.nbx, by = b / a.nbx;
  const int x0b = bx * RB, x1b = by * RY;
  const int i0 = x0b + x0l, i1 = x1b + x1l;
  const bool last = bx == a.nbx - 1;
  const unsigned P0 = (unsigned)d.P0, N1 = (unsigned)d.N1;
  const unsigned n2d = (unsigned)d.N0 * N1;
  const unsigned o2d = (unsigned)NG * N1;

  // --- own points --------------------------------------------------------
  // The column's metric factors. The single-precision instances (the split
  // form's increment) fold the x0 and x1 sums into per-tap weights: f0 u,00 +
  // f3 u,0 = sum_k (cp0_k u(+k) + cm0_k u(-k)) + f0 w0 u with cp0_k = f0 d2_k +
  // f3 d1_k, cm0_k = f0 d2_k - f3 d1_k (likewise x1 with f1, f4), two FMAs per
  // tap pair instead of four operations; in FP64 the 20 weights would not fit
  // the 1024-thread block's 128 registers (they spill), so FP64 keeps the sums.
  constexpr bool kFold = sizeof(T) == 4;
  T f[6];
  T cp0[NG], cm0[NG], cp1[NG], cm1[NG], c0 = (T)0;
  {
    const unsigned k2 = (unsigned)i0 + (unsigned)d.N0 * (unsigned)i1;
#pragma unroll
    for (int q = 0; q < 6; ++q) f[q] = load_factor(a.fac, a.facb, q * n2d + k2);
    if constexpr (kFold) {
#pragma unroll
      for (int k = 1; k <= NG; ++k) {
        cp0[k - 1] = f[0] * (T)Wt.d2[k] + f[3] * (T)Wt.d1[k];
        cm0[k - 1] = f[0] * (T)Wt.d2[k] - f[3] * (T)Wt.d1[k];
        cp1[k - 1] = f[1] * (T)Wt.d2[k] + f[4] * (T)Wt.d1[k];
        cm1[k - 1] = f[1] * (T)Wt.d2[k] - f[4] * (T)Wt.d1[k];
      }
      c0 = (T)Wt.d2[0] * (f[0] + f[1] + f[2]);
    }
  }
  T yu[NPT], yv[NPT], su[NPT], sv[NPT], au[NPT], av[NPT], ps[NPT], ss[NPT];
  T hu[NPT], hv[NPT];   // split form: base slopes
  unsigned gidx[NPT];
  int lidx[NPT], vidx[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int i2 = grp + PG * j;
    const bool ok = i2 < N2;
    const int i2c = ok ? i2 : 0;
    gidx[j] = P0 * ((unsigned)i1 + N1 * (unsigned)i2c) + (unsigned)i0;
    lidx[j] = i2c * TP + (x1l + NG) * RW + (x0l + NG);
    vidx[j] = (i2c * RY + x1l) * VW + x0l;
    yu[j] = ok ? a.u[gidx[j]] : (T)0;
    yv[j] = ok ? a.v[gidx[j]] : (T)0;
    ps[j] = ok ? a.psi[gidx[j]] : (T)0;
    ss[j] = ok ? a.ssrc[gidx[j]] : (T)0;
    hu[j] = CORR && ok ? a.khu[gidx[j]] : (T)0;
    hv[j] = CORR && ok ? a.khv[gidx[j]] : (T)0;
    su[j] = yu[j];
    sv[j] = yv[j];
    au[j] = (T)0;
    av[j] = (T)0;
  }

  // --- outer points (last x0 patch only) ---------------------------------
  T oyu[NQ], oyv[NQ], osu[NQ], osv[NQ], oau[NQ], oav[NQ], oc[NQ], ori[NQ], oqd[NQ];
  T ohu[NQ], ohv[NQ];   // split form: base slopes of the outer points
  unsigned oidx[NQ];
  int otl[NQ], ovl[NQ];
  bool oval[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int o = t + RT * q;
    const int col = o % NG, rest = o / NG;
    const int r = rest % RY, pl = rest / RY;
    oval[q] = last && pl < N2;
    const int plc = oval[q] ? pl : 0;
    oidx[q] = P0 * ((unsigned)(x1b + r) + N1 * (unsigned)plc) + (unsigned)(d.N0 + col);
    otl[q] = plc * TP + (NG + r) * RW + (NG + RB + col);
    ovl[q] = (plc * RY + r) * VW + RB + col;
    const unsigned ko = (unsigned)col + (unsigned)NG * (unsigned)(x1b + r);
    oc[q] = oval[q] ? a.ofac[ko] : (T)0;
    ori[q] = oval[q] ? a.ofac[o2d + ko] : (T)0;
    oqd[q] = oval[q] ? a.ofac[2 * o2d + ko] : (T)0;
    oyu[q] = oval[q] ? a.u[oidx[q]] : (T)0;
    oyv[q] = oval[q] ? a.v[oidx[q]] : (T)0;
    ohu[q] = CORR && oval[q] ? a.khu[oidx[q]] : (T)0;
    ohv[q] = CORR && oval[q] ? a.khv[oidx[q]] : (T)0;
    osu[q] = oyu[q];
    osv[q] = oyv[q];
    oau[q] = (T)0;
    oav[q] = (T)0;
  }

  // --- rim cells: LDS slot and stored source (images resolved) ------------
  // kind 0: no cell (plane >= N2); 1: owned by another patch, read from the
  // exchange array; 2: an image of one of this patch's own points, copied
  // within LDS; 3: one of this patch's own outer points, stored into LDS by its
  // thread. Packed: LDS slot (15 bits), LDS source of a kind-2 cell (15 bits),
  // kind (2 bits); LDS indices stay below 16 planes x 18 rows x 24 < 2^15.
  unsigned rg[NR], rmeta[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int c = t + RT * q;
    const int pl = c / NRIM, w = c - pl * NRIM;
    const int plc = pl < N2 ? pl : 0;
    // sides 0/1: NG columns left/right of the patch (RY rows each); sides
    // 2/3: NG rows below/above (RB columns each)
    const int side = w < NRX ? w / (NG * RY) : 2 + (w - NRX) / (NG * RB);
    const int w2 = w < NRX ? w - side * (NG * RY) : w - NRX - (side - 2) * (NG * RB);
    int l0, l1;
    if (side == 0) { l0 = w2 % NG; l1 = NG + w2 / NG; }
    else if (side == 1) { l0 = NG + RB + w2 % NG; l1 = NG + w2 / NG; }
    else if (side == 2) { l0 = NG + w2 % RB; l1 = w2 / RB; }
    else { l0 = NG + w2 % RB; l1 = NG + RY + w2 / RB; }
    const int j0 = x0b + l0 - NG, j1 = x1b + l1 - NG;
    int s0 = j0, s1 = j1;
    bool flip = false;
    if (j0 < 0) {            // reflection through xx0 = 0
      s0 = -1 - j0;
      s1 = d.sph ? d.N1 - 1 - j1 : j1;
      flip = true;
    } else if (j1 < 0) {     // reflection through theta = 0
      s1 = -1 - j1;
      flip = true;
    } else if (j1 >= d.N1) { // reflection through theta = pi
      s1 = 2 * d.N1 - 1 - j1;
      flip = true;
    }
    const int sp = flip ? half_turn(plc, N2) : plc;
    // packed exchange slot of (s0, s1, sp); only read for cells of other
    // patches, which are interior points (outer points stay with their patch)
    const int ox = s0 / RB, oy = s1 / RY;
    rg[q] = ((unsigned)(ox + a.nbx * oy) * (unsigned)N2 + (unsigned)sp) * (unsigned)NP +
            (unsigned)((s1 - oy * RY) * RB + (s0 - ox * RB));
    const bool self = min(s0 / RB, a.nbx - 1) == bx && s1 / RY == by;
    const unsigned kind = pl >= N2 ? 0u : !self ? 1u : flip ? 2u : 3u;
    const unsigned rl = (unsigned)(plc * TP + l1 * RW + l0);
    const unsigned rs =
        kind == 2u ? (unsigned)(sp * TP + (s1 - x1b + NG) * RW + (s0 - x0b + NG)) : 0u;
    rmeta[q] = rl | (rs << 15) | (kind << 30);
  }

  // --- exchange partners --------------------------------------------------
  const int nw = a.waits[b * (kResMaxWait + 1)];
  const int wt = t < nw ? a.waits[b * (kResMaxWait + 1) + 1 + t] : 0;

  // packed exchange slot of this thread's point in plane 0
  const unsigned pslot = (unsigned)b * (unsigned)N2 * (unsigned)NP + (unsigned)pos;

  // publish the initial stage input (counter 1); stage e waits for counters
  // >= e and publishes its result with counter e + 1
#pragma unroll
  for (int j = 0; j < NPT; ++j)
    if (grp + PG * j < N2) xstore(a.x0 + pslot + (unsigned)NP * (unsigned)(grp + PG * j), su[j]);
  __builtin_amdgcn_s_waitcnt(0);
  if (t == 0) bad = 0;
  __syncthreads();
  if (t == 0)
    __hip_atomic_store(a.flags + b * kResFlagStride, 1u, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);

  const int nst = 4 * a.nsteps;
  for (int e = 1; e <= nst; ++e) {
    const int stage = (e - 1) & 3;
    // (1) stage input of the patch into LDS: own points and own outer points
    // from registers; v only where the outer points' radiation condition
    // reads it (the last four interior columns and the outer points)
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      if (grp + PG * j < N2) {
        ut[lidx[j]] = su[j];
        if (last && x0l >= RB - 4) vt[vidx[j]] = sv[j];
      }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (oval[q]) {
        ut[otl[q]] = osu[q];
        vt[ovl[q]] = osv[q];
      }
    // (2) wait until every exchange partner has published the previous stage
    // (one lane per partner; polling by every wave was measured slower); the
    // barrier also completes step 1
    if (t < nw) {
      const unsigned* fl = a.flags + wt * kResFlagStride;
      unsigned spin = 0;
      while (__hip_atomic_load(fl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)e) {
        if (++spin > a.spin_limit) {
          atomicOr(a.err, 1u);
          bad = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __syncthreads();
    if (bad) break;
    // (3) the rim: loads of the cells of other patches from the exchange array
    // are issued here and stored to LDS in step 6
    const T* src_x = ((e - 1) & 1) ? a.x1 : a.x0;
    T rv[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      rv[q] = (T)0;
      if ((rmeta[q] >> 30) == 1u) rv[q] = xload(src_x + rg[q]);
    }
    // rim cells that are images of the patch's own points: copied within LDS
    // while the loads are in flight
#pragma unroll
    for (int q = 0; q < NR; ++q)
      if ((rmeta[q] >> 30) == 2u) ut[rmeta[q] & 0x7fffu] = ut[(rmeta[q] >> 15) & 0x7fffu];
    // (4) the phi sums and the source term need only the patch's own planes:
    // computed while the rim loads are in flight
    T e2[NPT], src[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      e2[j] = (T)0;
      src[j] = (T)0;
      if (grp + PG * j >= N2) continue;
      const T* r = ut + lidx[j];
      const int i2 = grp + PG * j;
      int jp = i2, jm = i2;
#pragma unroll
      for (int k = 1; k <= NG; ++k) {
        jp = (jp + 1 == N2) ? 0 : jp + 1;
        jm = (jm == 0) ? N2 - 1 : jm - 1;
        e2[j] += (T)Wt.d2[k] * (r[(jp - i2) * TP] + r[(jm - i2) * TP]);
      }
      // the stage input of the own point is su[j] (step 1 stored it at r[0])
      if constexpr (CORR) {
        src[j] = source_delta(ss[j], ps[j], su[j]);
      } else {
        const T p = ps[j] + su[j];
        const T p2 = p * p;
        const T p4 = p2 * p2;
        src[j] = ss[j] / (p4 * p2 * p);
      }
    }
    // (5) the outer points' radiation condition needs only the patch's own
    // cells: also computed while the rim loads are in flight
    const T cy = a.cy[stage], ca = a.ca[stage];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if (!oval[q]) continue;
      // radiation condition with a one-sided xx0 derivative
      const T u0 = ut[otl[q]], u1 = ut[otl[q] - 1], u2 = ut[otl[q] - 2];
      const T v0 = osv[q], v1 = vt[ovl[q] - 1], v2 = vt[ovl[q] - 2];
      const bool bc4 = a.bc4 != 0;
      const T u3 = bc4 ? ut[otl[q] - 3] : (T)0, u4 = bc4 ? ut[otl[q] - 4] : (T)0;
      const T v3 = bc4 ? vt[ovl[q] - 3] : (T)0, v4 = bc4 ? vt[ovl[q] - 4] : (T)0;
      T kuo = -oc[q] * (u0 * ori[q] + outer_diff(u0, u1, u2, u3, u4, oqd[q], bc4));
      T kvo = -oc[q] * (v0 * ori[q] + outer_diff(v0, v1, v2, v3, v4, oqd[q], bc4));
      if constexpr (CORR) {
        kuo = ohu[q] + kuo;
        kvo = ohv[q] + kvo;
      }
      if (stage == 0) {
        oau[q] = u0 + ca * kuo;
        oav[q] = v0 + ca * kvo;
        osu[q] = u0 + cy * kuo;
        osv[q] = v0 + cy * kvo;
      } else if (stage == 3) {
        osu[q] = oau[q] + ca * kuo;
        osv[q] = oav[q] + ca * kvo;
        oyu[q] = osu[q];
        oyv[q] = osv[q];
      } else {
        osu[q] = oyu[q] + cy * kuo;
        osv[q] = oyv[q] + cy * kvo;
        oau[q] = oau[q] + ca * kuo;
        oav[q] = oav[q] + ca * kvo;
      }
    }

    // (6) loaded rim cells into LDS
#pragma unroll
    for (int q = 0; q < NR; ++q)
      if ((rmeta[q] >> 30) == 1u) ut[rmeta[q] & 0x7fffu] = rv[q];
    __syncthreads();

    // (7) x0/x1 sums, right-hand side and stage combine at the own points
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      if (grp + PG * j >= N2) continue;
      const T* r = ut + lidx[j];
      const T uc = su[j];
      T lap;
      if constexpr (kFold) {
        lap = c0 * uc + f[2] * e2[j];
#pragma unroll
        for (int k = 1; k <= NG; ++k) {
          lap += cp0[k - 1] * r[k] + cm0[k - 1] * r[-k];
          lap += cp1[k - 1] * r[k * RW] + cm1[k - 1] * r[-k * RW];
        }
      } else {
        T d0 = 0, d1 = 0, e0 = 0, e1 = 0;
#pragma unroll
        for (int k = 1; k <= NG; ++k) {
          const T p0 = r[k], m0 = r[-k];
          const T p1 = r[k * RW], m1 = r[-k * RW];
          d0 += (T)Wt.d1[k] * (p0 - m0);
          d1 += (T)Wt.d1[k] * (p1 - m1);
          e0 += (T)Wt.d2[k] * (p0 + m0);
          e1 += (T)Wt.d2[k] * (p1 + m1);
        }
        const T w0 = (T)Wt.d2[0];
        const T dd0 = e0 + w0 * uc, dd1 = e1 + w0 * uc, dd2 = e2[j] + w0 * uc;
        lap = f[0] * dd0 + f[1] * dd1 + f[2] * dd2 + f[3] * d0 + f[4] * d1;
      }
      T ku, kv;
      if constexpr (CORR) {
        ku = hu[j] + (sv[j] - a.eta * uc);
        kv = hv[j] + f[5] * (lap + src[j]);
      } else {
        ku = sv[j] - a.eta * uc;
        kv = f[5] * (lap + src[j]);
      }
      if (stage == 0) {
        au[j] = uc + ca * ku;
        av[j] = sv[j] + ca * kv;
        su[j] = uc + cy * ku;
        sv[j] = sv[j] + cy * kv;
      } else if (stage == 3) {
        su[j] = au[j] + ca * ku;
        sv[j] = av[j] + ca * kv;
        yu[j] = su[j];
        yv[j] = sv[j];
      } else {
        su[j] = yu[j] + cy * ku;
        sv[j] = yv[j] + cy * kv;
        au[j] = au[j] + ca * ku;
        av[j] = av[j] + ca * kv;
      }
    }
    if (e < nst) {
      // publish the next stage input u, then raise this block's counter
      T* dst = (e & 1) ? a.x1 : a.x0;
#pragma unroll
      for (int j = 0; j < NPT; ++j)
        if (grp + PG * j < N2)
          xstore(dst + pslot + (unsigned)NP * (unsigned)(grp + PG * j), su[j]);
      // (outer points are read only by their own patch, through LDS)
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (t == 0)
        __hip_atomic_store(a.flags + b * kResFlagStride, (unsigned)(e + 1), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    } else {
#pragma unroll
      for (int j = 0; j < NPT; ++j)
        if (grp + PG * j < N2) {
          a.u[gidx[j]] = yu[j];
          a.v[gidx[j]] = yv[j];
        }
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (oval[q]) {
          a.u[oidx[q]] = oyu[q];
          a.v[oidx[q]] = oyv[q];
        }
    }
  }
}

// One grid per launch: block b is patch b.
template <typename T, int NG, int NPT, int RT, bool CORR, int RY>
__global__ void __launch_bounds__(RT) k_resident(ResidentArgsT<T> a) {
  resident_body<T, NG, NPT, RT, CORR, RY>(a, (int)blockIdx.x);
}

// Several grids per launch (same order, plane group and patch rows): grid i
// owns blocks [tab[i].block0, tab[i].block0 + its patches); each grid has its
// own counters, exchange partners and exchange buffers, so the grids never
// wait for each other.
template <typename T, int NG, int NPT, int RT, bool CORR, int RY>
__global__ void __launch_bounds__(RT) k_resident_multi(const ResidentArgsT<T>* __restrict__ tab,
                                                       int n) {
  int gi = 0;
  while (gi + 1 < n && (int)blockIdx.x >= tab[gi + 1].block0) ++gi;
  // read in place (uniform scalar loads); a private copy would be indexed
  // with the runtime stage number and spill
  const ResidentArgsT<T>& a = tab[gi];
  resident_body<T, NG, NPT, RT, CORR, RY>(a, (int)blockIdx.x - a.block0);
}

// Threads by N2: one plane per thread (for 8 x 8 patches 1024 threads when
// N2 > 8: four waves per SIMD to hide LDS and exchange latency). Deeper grids
// would need several planes per thread and more registers than a 1024-thread
// block has.
struct ResShape {
  const void* kernel;   // one grid per launch
  const void* multi;    // several grids per launch
  int threads;
};

template <typename T, int NG, bool CORR, int RY>
ResShape shape_for(int N2) {
  constexpr int NP = kResPatch * RY;
  if (N2 <= 4)
    return {(const void*)k_resident<T, NG, 1, 4 * NP, CORR, RY>,
            (const void*)k_resident_multi<T, NG, 1, 4 * NP, CORR, RY>, 4 * NP};
  if (N2 <= 8)
    return {(const void*)k_resident<T, NG, 1, 8 * NP, CORR, RY>,
            (const void*)k_resident_multi<T, NG, 1, 8 * NP, CORR, RY>, 8 * NP};
  if (N2 <= 16)
    return {(const void*)k_resident<T, NG, 1, 16 * NP, CORR, RY>,
            (const void*)k_resident_multi<T, NG, 1, 16 * NP, CORR, RY>, 16 * NP};
  return {nullptr, nullptr, 0};
}

template <typename T, bool CORR>
ResShape resident_kernel(int order, int N2, int ry) {
  if (ry != 8 && ry != 4) return {nullptr, nullptr, 0};
  switch (order) {
    case 8: return ry == 8 ? shape_for<T, 4, CORR, 8>(N2) : shape_for<T, 4, CORR, 4>(N2);
    case 10: return ry == 8 ? shape_for<T, 5, CORR, 8>(N2) : shape_for<T, 5, CORR, 4>(N2);
    default: return {nullptr, nullptr, 0};
  }
}

template <typename T, bool CORR>
hipError_t launch_resident_t(int order, const ResidentArgsT<T>& a, hipStream_t s, hipEvent_t t0,
                             hipEvent_t t1) {
  const ResShape rs = resident_kernel<T, CORR>(order, a.d.N2, a.ry);
  const void* k = rs.kernel;
  if (!k) return hipErrorInvalidValue;
  const int nb = a.nbx * a.nby;
  if (nb <= 0 || nb > kResMaxBlocks || a.nsteps <= 0) return hipErrorInvalidValue;
  const int nflags = nb * kResFlagStride;
  k_zero_u32<<<(nflags + 255) / 256, 256, 0, s>>>(a.flags, nflags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = resident_lds_bytes(a.d, sizeof(T), a.ry);
  e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  ResidentArgsT<T> arg = a;
  void* args[] = {&arg};
  // The caller has checked that every block fits at once (one per compute unit,
  // resident_capacity); the blocks synchronise only through their bounded
  // counter waits, so a plain launch suffices. If the device were shared and a
  // block could not start, its partners' waits would time out (err) instead
  // of hanging.
  return hipExtLaunchKernel(k, dim3(nb), dim3(rs.threads), args, lds, s, t0, t1, 0);
}

// Raises the dynamic-LDS limit of kernel k to at least lds bytes, never
// lowering it: a captured interval holds launches of one kernel instance with
// different LDS sizes, each of which must stay within the limit.
std::mutex g_lds_mu;
std::map<const void*, size_t> g_lds_set;

hipError_t raise_lds_limit(const void* k, size_t lds) {
  std::lock_guard<std::mutex> lk(g_lds_mu);
  size_t& cur = g_lds_set[k];
  if (lds <= cur) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) cur = lds;
  return e;
}

// Several grids in one launch; see launch_resident_multi.
template <typename T, bool CORR>
hipError_t launch_resident_multi_t(int order, const ResidentArgsT<T>* dev_tab,
                                   const ResidentArgsT<T>* host_tab, int n, hipStream_t s) {
  if (n <= 0 || !dev_tab || !host_tab) return hipErrorInvalidValue;
  const int ry = host_tab[0].ry;
  const ResShape r0 = resident_kernel<T, CORR>(order, host_tab[0].d.N2, ry);
  if (!r0.multi) return hipErrorInvalidValue;
  int total = 0;
  size_t lds = 0;
  for (int i = 0; i < n; ++i) {
    const ResidentArgsT<T>& a = host_tab[i];
    const int nb = a.nbx * a.nby;
    // every grid runs the same kernel instance, its blocks follow the
    // previous grid's
    if (a.ry != ry || resident_kernel<T, CORR>(order, a.d.N2, ry).multi != r0.multi ||
        nb <= 0 || a.block0 != total || a.nsteps <= 0)
      return hipErrorInvalidValue;
    total += nb;
    lds = std::max(lds, resident_lds_bytes(a.d, sizeof(T), ry));
    const int nflags = nb * kResFlagStride;
    k_zero_u32<<<(nflags + 255) / 256, 256, 0, s>>>(a.flags, nflags);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (total > kResMaxBlocks) return hipErrorInvalidValue;
  const hipError_t e = raise_lds_limit(r0.multi, lds);
  if (e != hipSuccess) return e;
  const ResidentArgsT<T>* tab = dev_tab;
  int cnt = n;
  void* args[] = {&tab, &cnt};
  // the caller has checked that all blocks fit at once (resident_multi_capacity)
  return hipExtLaunchKernel(r0.multi, dim3(total), dim3(r0.threads), args, lds, s, nullptr,
                            nullptr, 0);
}

}  // namespace

size_t resident_lds_bytes(const Dims& d, size_t elem, int ry) {
  const int RH = ry + 2 * d.NG, RW = tile_row(RB + 2 * d.NG), VW = tile_row(RB + d.NG);
  const size_t need = (size_t)d.N2 * (RW * RH + ry * VW) * elem;
  // more than half of the 160 KiB of LDS per compute unit: one block per CU
  return std::max<size_t>(need, 82 * 1024);
}

int resident_capacity(int order, const Dims& d, bool split, int ry) {
  const ResShape rs = split ? resident_kernel<float, true>(order, d.N2, ry)
                            : resident_kernel<double, false>(order, d.N2, ry);
  const void* k = rs.kernel;
  if (!k) return 0;
  const size_t lds = resident_lds_bytes(d, split ? sizeof(float) : sizeof(double), ry);
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  int per = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, rs.threads, lds) != hipSuccess)
    return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per * cus;
}

hipError_t launch_resident(int order, const ResidentArgsT<double>& a, hipStream_t s,
                           hipEvent_t t0, hipEvent_t t1) {
  return launch_resident_t<double, false>(order, a, s, t0, t1);
}

hipError_t launch_resident(int order, const ResidentArgsT<float>& a, hipStream_t s,
                           hipEvent_t t0, hipEvent_t t1) {
  return launch_resident_t<float, true>(order, a, s, t0, t1);
}

hipError_t launch_resident_multi(int order, const ResidentArgsT<double>* dev_tab,
                                 const ResidentArgsT<double>* host_tab, int n, hipStream_t s) {
  return launch_resident_multi_t<double, false>(order, dev_tab, host_tab, n, s);
}

hipError_t launch_resident_multi(int order, const ResidentArgsT<float>* dev_tab,
                                 const ResidentArgsT<float>* host_tab, int n, hipStream_t s) {
  return launch_resident_multi_t<float, true>(order, dev_tab, host_tab, n, s);
}

const void* resident_kernel_key(int order, int N2, bool split, int ry) {
  return split ? resident_kernel<float, true>(order, N2, ry).multi
               : resident_kernel<double, false>(order, N2, ry).multi;
}

int resident_multi_capacity(int order, int N2, bool split, int ry, size_t lds) {
  const ResShape rs = split ? resident_kernel<float, true>(order, N2, ry)
                            : resident_kernel<double, false>(order, N2, ry);
  if (!rs.multi) return 0;
  if (raise_lds_limit(rs.multi, lds) != hipSuccess) return 0;
  int per = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, rs.multi, rs.threads, lds) != hipSuccess)
    return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per * cus;
}

}  // namespace hr
