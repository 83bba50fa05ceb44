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

#include "hr_internal.h"

namespace hr {
namespace {

// ---------------------------------------------------------------------------
// Centred finite-difference weights of order 2*NG, from the closed forms for
// equispaced centred stencils (m = NG):
//   first derivative   w_k = (-1)^(k+1) (m!)^2 / ( k (m-k)! (m+k)! )
//   second derivative  w_k = 2 (-1)^(k+1) (m!)^2 / ( k^2 (m-k)! (m+k)! ),
//                      w_0 = -2 sum_{k=1..m} 1/k^2
// evaluated at compile time as one rounding of an exact integer ratio.
constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }
constexpr long long gcdll(long long a, long long b) { return b == 0 ? a : gcdll(b, a % b); }
constexpr long long lcm_upto(int m) {
  long long l = 1;
  for (int k = 2; k <= m; ++k) l = l / gcdll(l, k) * k;
  return l;
}
constexpr double w1(int m, int k) {
  return ((k % 2) ? 1.0 : -1.0) * fact(m) * fact(m) / (k * fact(m - k) * fact(m + k));
}
constexpr double w2(int m, int k) {
  if (k == 0) {
    const long long L = lcm_upto(m), D = L * L;
    long long num = 0;
    for (int j = 1; j <= m; ++j) num += D / ((long long)j * j);
    return -2.0 * (double)num / (double)D;
  }
  return ((k % 2) ? 2.0 : -2.0) * fact(m) * fact(m) / ((double)k * k * fact(m - k) * fact(m + k));
}
static_assert(w2(4, 0) == -205.0 / 72.0, "8th-order centre weight");
static_assert(w2(5, 0) == -5269.0 / 1800.0, "10th-order centre weight");

template <int NG>
struct Weights {
  double d1[NG + 1];
  double d2[NG + 1];
  constexpr Weights() : d1(), d2() {
    for (int k = 0; k <= NG; ++k) {
      d1[k] = k == 0 ? 0.0 : w1(NG, k);
      d2[k] = w2(NG, k);
    }
  }
};

// ---------------------------------------------------------------------------
// Neighbour addressing in the extended layout with virtual inner ghosts.
struct Addr {
  int i0, i1, i2;
  int s1, s2;      // strides of x1 and x2
  int base;        // flat index of the centre
  int refl0;       // row base of the xx0 = 0 reflection (i1', i2 + N2/2)
  int i2h;         // i2 + N2/2 (mod N2)
  int N1, N2;

  __device__ __forceinline__ Addr(const Dims& d, int a0, int a1, int a2)
      : i0(a0), i1(a1), i2(a2), s1(d.P0), s2(d.P0 * d.N1), N1(d.N1), N2(d.N2) {
    base = i0 + s1 * i1 + s2 * i2;
    i2h = i2 + (N2 >> 1);
    i2h -= (i2h >= N2) ? N2 : 0;
    const int i1r = d.sph ? (N1 - 1 - i1) : i1;
    refl0 = s1 * i1r + s2 * i2h;
  }
  // x0 - k (k >= 1): interior, or reflected through xx0 = 0
  __device__ __forceinline__ int x0m(int k) const {
    const int j = i0 - k;
    return (j >= 0) ? base - k : refl0 + (-1 - j);
  }
  // x0 + k never leaves the stored range for interior centres.
  __device__ __forceinline__ int x0p(int k) const { return base + k; }
  __device__ __forceinline__ int x1m(int k) const {
    const int j = i1 - k;
    return (j >= 0) ? base - k * s1 : i0 + s1 * (-1 - j) + s2 * i2h;
  }
  __device__ __forceinline__ int x1p(int k) const {
    const int j = i1 + k;
    return (j < N1) ? base + k * s1 : i0 + s1 * (2 * N1 - 1 - j) + s2 * i2h;
  }
  __device__ __forceinline__ int wrap2(int j) const {
    j %= N2;
    return j < 0 ? j + N2 : j;
  }
  __device__ __forceinline__ int x2m(int k) const { return i0 + s1 * i1 + s2 * wrap2(i2 - k); }
  __device__ __forceinline__ int x2p(int k) const { return i0 + s1 * i1 + s2 * wrap2(i2 + k); }
};

// Un-normalised centred sums along the three directions; C is the compute
// type, S the storage type of the field.
template <int NG, typename C, typename S>
struct Sums {
  C d0, d1, dd0, dd1, dd2, uc;
};

template <int NG, typename C, typename S>
__device__ __forceinline__ Sums<NG, C, S> stencil(const S* __restrict__ U, const Addr& a) {
  constexpr Weights<NG> W{};
  Sums<NG, C, S> r;
  const C uc = (C)U[a.base];
  r.uc = uc;
  C d0 = 0, d1 = 0, e0 = 0, e1 = 0, e2 = 0;
#pragma unroll
  for (int k = 1; k <= NG; ++k) {
    const C p0 = (C)U[a.x0p(k)], m0 = (C)U[a.x0m(k)];
    const C p1 = (C)U[a.x1p(k)], m1 = (C)U[a.x1m(k)];
    const C p2 = (C)U[a.x2p(k)], m2 = (C)U[a.x2m(k)];
    d0 += (C)W.d1[k] * (p0 - m0);
    d1 += (C)W.d1[k] * (p1 - m1);
    e0 += (C)W.d2[k] * (p0 + m0);
    e1 += (C)W.d2[k] * (p1 + m1);
    e2 += (C)W.d2[k] * (p2 + m2);
  }
  const C w0 = (C)W.d2[0];
  r.d0 = d0;
  r.d1 = d1;
  r.dd0 = e0 + w0 * uc;
  r.dd1 = e1 + w0 * uc;
  r.dd2 = e2 + w0 * uc;
  return r;
}

// (psi + u)^-7 times the source, in the compute type.
template <typename C>
__device__ __forceinline__ C source(C ssrc, C psi, C u) {
  const C p = psi + u;
  const C p2 = p * p;
  const C p4 = p2 * p2;
  return ssrc / (p4 * p2 * p);
}

// RK4 stage combine for one point, given the stage slopes.
template <int STAGE, typename T>
__device__ __forceinline__ void combine(const StageArgs<T>& a, int idx, T uin, T vin, T ku,
                                        T kv) {
  if constexpr (STAGE == 1) {
    a.uout[idx] = uin + a.cy * ku;
    a.vout[idx] = vin + a.cy * kv;
    a.au[idx] = uin + a.ca * ku;
    a.av[idx] = vin + a.ca * kv;
  } else if constexpr (STAGE == 4) {
    a.uout[idx] = a.au[idx] + a.ca * ku;
    a.vout[idx] = a.av[idx] + a.ca * kv;
  } else {
    const T un = a.un[idx], vn = a.vn[idx];
    a.uout[idx] = un + a.cy * ku;
    a.vout[idx] = vn + a.cy * kv;
    a.au[idx] = a.au[idx] + a.ca * ku;
    a.av[idx] = a.av[idx] + a.ca * kv;
  }
}

template <typename T, int NG, int STAGE>
__global__ void __launch_bounds__(kBlock) k_stage(StageArgs<T> a) {
  const Dims& d = a.d;
  const int nblk_int = (d.nint + kBlock - 1) / kBlock;
  if ((int)blockIdx.x < nblk_int) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= d.nint) return;
    const int i0 = t % d.N0;
    const int r = t / d.N0;
    const int i1 = r % d.N1;
    const int i2 = r / d.N1;
    const Addr ad(d, i0, i1, i2);
    const Sums<NG, T, T> s = stencil<NG, T, T>(a.uin, ad);
    const int n2d = d.N0 * d.N1;
    const int k2 = i0 + d.N0 * i1;
    const T* F = a.fac;
    const T lap = F[k2] * s.dd0 + F[n2d + k2] * s.dd1 + F[2 * n2d + k2] * s.dd2 +
                  F[3 * n2d + k2] * s.d0 + F[4 * n2d + k2] * s.d1;
    const T c2 = F[5 * n2d + k2];
    const int idx = ad.base;
    const T u = s.uc;
    const T v = a.vin[idx];
    const T ku = v - a.eta * u;
    const T kv = c2 * (lap + source<T>(a.ssrc[idx], a.psi[idx], u));
    combine<STAGE, T>(a, idx, u, v, ku, kv);
  } else {
    const int t = (blockIdx.x - nblk_int) * kBlock + threadIdx.x;
    if (t >= d.nout) return;
    const int q = t % NG;
    const int r = t / NG;
    const int i1 = r % d.N1;
    const int i2 = r / d.N1;
    const int idx = d.N0 + q + d.P0 * (i1 + d.N1 * i2);
    const int o2d = NG * d.N1;
    const int ko = q + NG * i1;
    const T c = a.ofac[ko], rinv = a.ofac[o2d + ko], qd = a.ofac[2 * o2d + ko];
    const T u0 = a.uin[idx], u1 = a.uin[idx - 1], u2 = a.uin[idx - 2];
    const T v0 = a.vin[idx], v1 = a.vin[idx - 1], v2 = a.vin[idx - 2];
    const T ku = -c * (u0 * rinv + ((T)3 * u0 - (T)4 * u1 + u2) * qd);
    const T kv = -c * (v0 * rinv + ((T)3 * v0 - (T)4 * v1 + v2) * qd);
    combine<STAGE, T>(a, idx, u0, v0, ku, kv);
  }
}

// Sum over a 64-wide wavefront, then over the block's wavefronts in a fixed
// order. Returns the block total in thread 0.
__device__ __forceinline__ double block_sum(double x) {
  __shared__ double wsum[kBlock / 64];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) wsum[wid] = x;
  __syncthreads();
  double tot = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / 64; ++w) tot += wsum[w];
  return tot;
}

template <typename S, int NG>
__global__ void __launch_bounds__(kBlock) k_residual(ResidualArgs a) {
  const Dims& d = a.d;
  const int t = blockIdx.x * kBlock + threadIdx.x;
  double h2 = 0.0;
  if (t < d.nint) {
    const int i0 = t % d.N0;
    const int r = t / d.N0;
    const int i1 = r % d.N1;
    const int i2 = r / d.N1;
    const Addr ad(d, i0, i1, i2);
    const S* U = static_cast<const S*>(a.u);
    const Sums<NG, double, S> s = stencil<NG, double, S>(U, ad);
    const int n2d = d.N0 * d.N1;
    const int k2 = i0 + d.N0 * i1;
    const double* F = a.fac;
    const double lap = F[k2] * s.dd0 + F[n2d + k2] * s.dd1 + F[2 * n2d + k2] * s.dd2 +
                       F[3 * n2d + k2] * s.d0 + F[4 * n2d + k2] * s.d1;
    const double H = lap + source<double>(a.ssrc[ad.base], a.psi[ad.base], s.uc);
    h2 = H * H;
  }
  const double tot = block_sum(h2);
  if (threadIdx.x == 0) a.partial[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock) k_finalize(const double* __restrict__ partial,
                                                     int nparts, int nint,
                                                     double* __restrict__ out) {
  double s = 0.0;
  for (int j = threadIdx.x; j < nparts; j += kBlock) s += partial[j];
  const double tot = block_sum(s);
  if (threadIdx.x == 0) {
    out[0] = sqrt(tot / (double)nint);
    out[1] = tot;
  }
}

// psi_singular and (1/8) A_ij A^ij at every stored point (interior and outer).
__global__ void __launch_bounds__(kBlock) k_sources(Dims d, const double* __restrict__ rho,
                                                    const double* __restrict__ zc,
                                                    const double* __restrict__ cphi,
                                                    const double* __restrict__ sphi,
                                                    Punctures pz, double* __restrict__ psi64,
                                                    double* __restrict__ ssrc64,
                                                    float* __restrict__ psi32,
                                                    float* __restrict__ ssrc32) {
  const int next = d.P0 * d.N1 * d.N2;
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= next) return;
  const int e = t % (d.P0 * d.N1);
  const int i2 = t / (d.P0 * d.N1);
  const double X[3] = {rho[e] * cphi[i2], rho[e] * sphi[i2], zc[e]};
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
  const double src = aa / 8.0;
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

inline int nblocks(int n) { return (n + kBlock - 1) / kBlock; }

template <typename T, int NG>
hipError_t stage_dispatch(int stage, const StageArgs<T>& a, hipStream_t s) {
  const int nb = nblocks(a.d.nint) + nblocks(a.d.nout);
  switch (stage) {
    case 1: k_stage<T, NG, 1><<<nb, kBlock, 0, s>>>(a); break;
    case 2: k_stage<T, NG, 2><<<nb, kBlock, 0, s>>>(a); break;
    case 3: k_stage<T, NG, 3><<<nb, kBlock, 0, s>>>(a); break;
    case 4: k_stage<T, NG, 4><<<nb, kBlock, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t stage_order(int order, int stage, const StageArgs<T>& a, hipStream_t s) {
  switch (order) {
    case 2: return stage_dispatch<T, 1>(stage, a, s);
    case 4: return stage_dispatch<T, 2>(stage, a, s);
    case 6: return stage_dispatch<T, 3>(stage, a, s);
    case 8: return stage_dispatch<T, 4>(stage, a, s);
    case 10: return stage_dispatch<T, 5>(stage, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename S>
hipError_t residual_order(int order, const ResidualArgs& a, int nb, hipStream_t s) {
  switch (order) {
    case 2: k_residual<S, 1><<<nb, kBlock, 0, s>>>(a); break;
    case 4: k_residual<S, 2><<<nb, kBlock, 0, s>>>(a); break;
    case 6: k_residual<S, 3><<<nb, kBlock, 0, s>>>(a); break;
    case 8: k_residual<S, 4><<<nb, kBlock, 0, s>>>(a); break;
    case 10: k_residual<S, 5><<<nb, kBlock, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_stage(int order, int stage, const StageArgs<double>& a, hipStream_t s) {
  return stage_order<double>(order, stage, a, s);
}
hipError_t launch_stage(int order, int stage, const StageArgs<float>& a, hipStream_t s) {
  return stage_order<float>(order, stage, a, s);
}

hipError_t launch_residual(int order, bool fp32_state, const ResidualArgs& a, int nb,
                           hipStream_t s) {
  return fp32_state ? residual_order<float>(order, a, nb, s)
                    : residual_order<double>(order, a, nb, s);
}

hipError_t launch_finalize(const double* partial, int nparts, int nint, double* out,
                           hipStream_t s) {
  k_finalize<<<1, kBlock, 0, s>>>(partial, nparts, nint, out);
  return hipGetLastError();
}

hipError_t launch_sources(const Dims& d, const double* rho, const double* zc,
                          const double* cphi, const double* sphi, const Punctures& p,
                          double* psi64, double* ssrc64, float* psi32, float* ssrc32,
                          hipStream_t s) {
  const int next = d.P0 * d.N1 * d.N2;
  k_sources<<<nblocks(next), kBlock, 0, s>>>(d, rho, zc, cphi, sphi, p, psi64, ssrc64, psi32,
                                             ssrc32);
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
hipError_t launch_fill(double* dst, double value, int n, hipStream_t s) {
  k_fill<double><<<nblocks(n), kBlock, 0, s>>>(dst, value, n);
  return hipGetLastError();
}
hipError_t launch_fill(float* dst, float value, int n, hipStream_t s) {
  k_fill<float><<<nblocks(n), kBlock, 0, s>>>(dst, value, n);
  return hipGetLastError();
}

}  // namespace hr
