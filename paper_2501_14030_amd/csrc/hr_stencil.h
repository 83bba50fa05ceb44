// Device helpers shared by the stage kernels: centred finite-difference
// weights, the split-state source difference and the phi + pi plane map of
// the inner-boundary images.
#pragma once

#include <hip/hip_runtime.h>

namespace hr {

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

// Source difference of the split-state form: S p^-7 [(1 + x)^-7 - 1], x = e/p.
// With q = p + e and y = p/q = 1/(1 + x): (1 + x)^-7 - 1 = y^7 - 1 =
// (y - 1)(1 + y + ... + y^6) and y - 1 = -e/q, so the small difference is
// formed without cancellation from one division, two products and a
// six-step Horner sum (FP32 relative error within a few ulp).
__device__ __forceinline__ float source_delta(float sp7, float pb, float e) {
  const float r = 1.0f / (pb + e);
  const float y = pb * r;
  float s = 1.0f;
#pragma unroll
  for (int k = 0; k < 6; ++k) s = s * y + 1.0f;
  return -sp7 * (e * r) * s;
}

// Radial-derivative term of the outer radiation condition, qd x (one-sided
// xx0 difference of f at an outer point, times 2 dxx0), with qd = 1 /
// (2 dxx0 dr/dxx0) and f0 the point itself, f1 ... its inner neighbours along
// xx0: second order (3 f0 - 4 f1 + f2) / 2, or with bc4 fourth order
// (25 f0 - 48 f1 + 36 f2 - 16 f3 + 3 f4) / 12, the derivative at f0 of the
// quartic through the five values.
template <typename T>
__device__ __forceinline__ T outer_diff(T f0, T f1, T f2, T f3, T f4, T qd, bool bc4) {
  if (bc4)
    return ((T)25 * f0 - (T)48 * f1 + (T)36 * f2 - (T)16 * f3 + (T)3 * f4) *
           (qd * (T)(1.0 / 6.0));
  return ((T)3 * f0 - (T)4 * f1 + f2) * qd;
}

// One metric factor: from the bfloat16 planes when given (single precision
// only; the 16 stored bits are the high half of the FP32 value), else from the
// table of the stage's own type.
template <typename T>
__device__ __forceinline__ T load_factor(const T* fac, const unsigned short* facb,
                                         unsigned i) {
  if constexpr (sizeof(T) == 4) {
    if (facb) return __uint_as_float((unsigned)facb[i] << 16);
  }
  return fac[i];
}

// Plane index of phi + pi (N2 even).
__device__ __forceinline__ int half_turn(int i2, int N2) {
  const int h = i2 + (N2 >> 1);
  return h >= N2 ? h - N2 : h;
}

}  // namespace hr
