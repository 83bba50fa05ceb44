// Learned warm start: a small MLP predicting the puncture correction u from the
// configuration and the grid coordinates, trained on relaxation solves, whose
// prediction becomes the initial state of the relaxation (which still judges
// the result by its residual).
//
// Network (FP32): x (F features) -> W1,b1 -> GELU -> W2,b2 -> GELU -> W3,b3 -> y,
// with log u = out_scale * y + out_shift. Dense layers run on MFMA
// (v_mfma_f32_32x32x2f32) in an LDS-tiled GEMM with a fused bias / GELU
// epilogue; backward uses the same GEMM in its transposed forms, deterministic
// column sums for the biases, and Adam.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "hr_internal.h"

using namespace hr;

namespace {

constexpr int kFeat = 15;   // 9 configuration + 4 coordinate + 2 puncture-distance features

// ---------------------------------------------------------------------------
// GEMM C[M x N] = A[M x K] B[K x N] (+ bias[n]) with optional GELU, FP32, on
// MFMA. A(m,k) = TA ? A[k*lda + m] : A[m*lda + k];
// B(k,n) = TB ? B[n*ldb + k] : B[k*ldb + n].
// Block: 256 threads (4 wavefronts in 2 x 2), tile 64 x 64, K step 16; each
// wavefront owns a 32 x 32 sub-tile accumulated by v_mfma_f32_32x32x2f32:
//   operand A: lane l holds A[l % 32][l / 32], operand B: B[l / 32][l % 32],
//   result register r of lane l is row 8 (r / 4) + 4 (l / 32) + r % 4,
//   column l % 32.
constexpr int GBM = 64, GBN = 64, GBK = 16;
constexpr int kMaxSlices = 32;   // split-K slices of a weight gradient, at most

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
  return cdf + z * pdf;
}

//
// Split K (grid z > 1): block z sums k in [z kc, min(K, (z + 1) kc)) and writes
// its partial product to C + z * cz (no bias, no activation); k_sum_slices
// then adds the slices in a fixed order. Used for the weight gradients,
// whose M x N is one layer's weights but whose K is the batch.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256)
    k_gemm(int M, int N, int K, const float* __restrict__ A, int lda,
           const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
           const float* __restrict__ bias, float* __restrict__ Zout, int act, int kc,
           size_t cz) {
  __shared__ float As[GBK][GBM + 4];
  __shared__ float Bs[GBK][GBN + 4];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
  const int kb = blockIdx.z * kc;
  const int ke = min(K, kb + kc);
  C += blockIdx.z * cz;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  for (int k0 = kb; k0 < ke; k0 += GBK) {
    // stage A (64 x 16) and B (16 x 64) tiles, zero outside the matrices
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;   // 0..1023
      // consecutive threads walk the contiguous dimension of each operand
      const int akk = TA ? e / GBM : e % GBK;
      const int amm = TA ? e % GBM : e / GBK;
      const int gm = m0 + amm, gak = k0 + akk;
      float va = 0.0f;
      if (gm < M && gak < ke) va = TA ? A[(size_t)gak * lda + gm] : A[(size_t)gm * lda + gak];
      As[akk][amm] = va;
      const int bkk = TB ? e % GBK : e / GBN;
      const int bnn = TB ? e / GBK : e % GBN;
      const int gn = n0 + bnn, gbk = k0 + bkk;
      float vb = 0.0f;
      if (gn < N && gbk < ke) vb = TB ? B[(size_t)gn * ldb + gbk] : B[(size_t)gbk * ldb + gn];
      Bs[bkk][bnn] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 2) {
      const float a = As[kk + (lane >> 5)][wm * 32 + (lane & 31)];
      const float b = Bs[kk + (lane >> 5)][wn * 32 + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int col = n0 + wn * 32 + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (row < M && col < N) {
      float z = acc[r];
      if (bias) z += bias[col];
      if (Zout) Zout[(size_t)row * ldc + col] = z;
      C[(size_t)row * ldc + col] = act ? gelu(z) : z;
    }
  }
}

// C[i] = sum over z < nz of P[z n + i], i < n, in the order z = 0, 1, ...
__global__ void __launch_bounds__(256) k_sum_slices(const float* __restrict__ P, int nz, long n,
                                                    float* __restrict__ C) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
  for (int z = 0; z < nz; ++z) s += P[(size_t)z * n + i];
  C[i] = s;
}

// out[j] = sum_i X[i*ld + j], i < M, j < N: per-block partial sums over row
// chunks, then a fixed-order second pass (deterministic).
__global__ void __launch_bounds__(256) k_colsum_partial(const float* __restrict__ X, int M, int N,
                                                        int ld, int rows_per_block,
                                                        float* __restrict__ part) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  const int r0 = blockIdx.y * rows_per_block;
  const int r1 = min(M, r0 + rows_per_block);
  float s = 0.0f;
  for (int i = r0; i < r1; ++i) s += X[(size_t)i * ld + j];
  part[(size_t)blockIdx.y * N + j] = s;
}

__global__ void __launch_bounds__(256) k_colsum_final(const float* __restrict__ part, int nparts,
                                                      int N, float* __restrict__ out) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  float s = 0.0f;
  for (int p = 0; p < nparts; ++p) s += part[(size_t)p * N + j];
  out[j] = s;
}

// dZ = dH * GELU'(Z), elementwise.
__global__ void __launch_bounds__(256) k_gelu_back(const float* __restrict__ dH,
                                                   const float* __restrict__ Z,
                                                   float* __restrict__ dZ, long n) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t < n) dZ[t] = dH[t] * gelu_grad(Z[t]);
}

// Mean squared error: dY = 2 (Y - T) / B, per-block partial sums of (Y - T)^2.
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                             int B, float* __restrict__ dY,
                                             float* __restrict__ part) {
  __shared__ float ws[4];
  const int t = blockIdx.x * 256 + threadIdx.x;
  float e = 0.0f;
  if (t < B) {
    const float d = Y[t] - T[t];
    dY[t] = 2.0f * d / (float)B;
    e = d * d;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) e += __shfl_xor(e, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Adam step on n parameters (bias-corrected learning rate lr_t).
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              long n, float lr_t, float b1, float b2, float eps) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const float gi = g[t];
  const float mi = b1 * m[t] + (1.0f - b1) * gi;
  const float vi = b2 * v[t] + (1.0f - b2) * gi * gi;
  m[t] = mi;
  v[t] = vi;
  p[t] = p[t] - lr_t * mi / (sqrtf(vi) + eps);
}

// Input features of every stored point of a grid (extended layout order):
// 9 normalised configuration values, 4 coordinate values (2 xx0/xx0_max - 1,
// cos xx1, sin xx1 cos xx2, sin xx1 sin xx2) and the logarithm of the distance
// to each of the first two punctures, divided by 5.
struct FeatArgs {
  Dims d;
  double x0max;
  float cfg[9];
  const double* rho;   // cylindrical radius and z over the (i0, i1) plane
  const double* zc;
  const double* cphi;
  const double* sphi;
  double px[2][3];     // puncture positions (the second repeats the first if n = 1)
  int row0;    // first stored point (extended-layout index) of this launch
  int nrows;   // points in this launch; row t of X is point row0 + t
  float* X;
};

__global__ void __launch_bounds__(256) k_features(FeatArgs a) {
  const int tl = blockIdx.x * 256 + threadIdx.x;
  if (tl >= a.nrows) return;
  const int t = a.row0 + tl;
  const int i0 = t % a.d.P0;
  const int r = t / a.d.P0;
  const int i1 = r % a.d.N1;
  const int i2 = r / a.d.N1;
  const double pi = 3.14159265358979323846;
  const double xx0 = (i0 + 0.5) * (a.x0max / a.d.N0);
  const double xx1 = (i1 + 0.5) * (pi / a.d.N1);
  const double xx2 = -pi + (i2 + 0.5) * (2.0 * pi / a.d.N2);
  float* x = a.X + (size_t)tl * kFeat;
#pragma unroll
  for (int k = 0; k < 9; ++k) x[k] = a.cfg[k];
  x[9] = (float)(2.0 * xx0 / a.x0max - 1.0);
  x[10] = (float)cos(xx1);
  x[11] = (float)(sin(xx1) * cos(xx2));
  x[12] = (float)(sin(xx1) * sin(xx2));
  const int e = i0 + a.d.P0 * i1;
  const double X0 = a.rho[e] * a.cphi[i2], Y0 = a.rho[e] * a.sphi[i2], Z0 = a.zc[e];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const double dx = X0 - a.px[p][0], dy = Y0 - a.px[p][1], dz = Z0 - a.px[p][2];
    x[13 + p] = (float)(0.1 * log(dx * dx + dy * dy + dz * dz));
  }
}

// u = exp(scale y + shift) into the FP64 state, v = eta u.
__global__ void __launch_bounds__(256) k_write_state(const float* __restrict__ y, int n,
                                                     float scale, float shift, double eta,
                                                     double* __restrict__ u,
                                                     double* __restrict__ v) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const double uu = exp((double)scale * (double)y[t] + (double)shift);
  u[t] = uu;
  v[t] = eta * uu;
}

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

struct hr_mlp {
  int F = kFeat, Wd = 256;
  long np = 0;                    // parameter count
  std::vector<float> host;        // initial parameters
  float out_scale = 1.0f, out_shift = 0.0f;
  bool bound = false;
  int device = 0;
  int max_batch = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  float *X = nullptr, *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *Y = nullptr;
  float *dY = nullptr, *dH = nullptr, *dZ = nullptr, *part = nullptr, *T = nullptr;
  float* kpart = nullptr;         // split-K slices of the weight gradients
  float* host_part = nullptr;
  long adam_t = 0;
  // parameter offsets
  long oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
};

namespace {

hr_status mfail(hr_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

#define HR_HIPM(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return mfail(HR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

size_t mlp_layout(hr_mlp* n, int B, char* base) {
  size_t off = 0;
  auto take = [&](size_t floats) -> float* {
    float* q = base ? (float*)(base + off) : nullptr;
    off = (off + floats * sizeof(float) + 255) / 256 * 256;
    return q;
  };
  n->p = take(n->np);
  n->g = take(n->np);
  n->m = take(n->np);
  n->v = take(n->np);
  n->X = take((size_t)B * n->F);
  n->Z1 = take((size_t)B * n->Wd);
  n->H1 = take((size_t)B * n->Wd);
  n->Z2 = take((size_t)B * n->Wd);
  n->H2 = take((size_t)B * n->Wd);
  n->Y = take((size_t)B);
  n->T = take((size_t)B);
  n->dY = take((size_t)B);
  n->dH = take((size_t)B * n->Wd);
  n->dZ = take((size_t)B * n->Wd);
  n->part = take((size_t)(B / 64 + 8) * n->Wd + 1024);
  n->kpart = take((size_t)kMaxSlices * n->Wd * n->Wd);
  return off;
}

template <bool TA, bool TB>
hipError_t gemm(hipStream_t s, int M, int N, int K, const float* A, int lda, const float* B,
                int ldb, float* C, int ldc, const float* bias, float* Z, int act) {
  const dim3 grid(cdiv(N, GBN), cdiv(M, GBM));
  k_gemm<TA, TB><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, bias, Z, act, K, 0);
  return hipGetLastError();
}

// Weight gradient C[M x N] (ldc = N) = A^T B summed over the batch K, split
// into slices of K so that the launch has ~512 blocks (at most kMaxSlices,
// each at least 256 rows of the batch), then the slices added in order.
hipError_t gemm_wgrad(hipStream_t s, int M, int N, int K, const float* A, int lda, const float* B,
                      int ldb, float* C, float* slices) {
  const int tiles = (int)(cdiv(N, GBN) * cdiv(M, GBM));
  int nz = std::max(1, std::min({kMaxSlices, 512 / tiles, K / 256}));
  const int kc = (int)cdiv(cdiv(K, nz), GBK) * GBK;   // whole K steps per slice
  nz = (int)cdiv(K, kc);
  if (nz == 1) return gemm<true, false>(s, M, N, K, A, lda, B, ldb, C, N, nullptr, nullptr, 0);
  const size_t cz = (size_t)M * N;
  const dim3 grid(cdiv(N, GBN), cdiv(M, GBM), nz);
  k_gemm<true, false><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, slices, N, nullptr, nullptr,
                                           0, kc, cz);
  k_sum_slices<<<cdiv((long)cz, 256), 256, 0, s>>>(slices, nz, (long)cz, C);
  return hipGetLastError();
}

hipError_t colsum(hipStream_t s, const float* X, int M, int N, float* part, float* out) {
  const int rows = 64;
  const int nb = (int)cdiv(M, rows);
  k_colsum_partial<<<dim3(cdiv(N, 256), nb), 256, 0, s>>>(X, M, N, N, rows, part);
  k_colsum_final<<<cdiv(N, 256), 256, 0, s>>>(part, nb, N, out);
  return hipGetLastError();
}

// Forward pass on the first B rows of n->X into n->Y (keeps Z1, H1, Z2, H2).
hipError_t forward(hr_mlp* n, int B) {
  hipError_t e;
  e = gemm<false, true>(n->stream, B, n->Wd, n->F, n->X, n->F, n->p + n->oW1, n->F, n->H1, n->Wd,
                        n->p + n->ob1, n->Z1, 1);
  if (e != hipSuccess) return e;
  e = gemm<false, true>(n->stream, B, n->Wd, n->Wd, n->H1, n->Wd, n->p + n->oW2, n->Wd, n->H2,
                        n->Wd, n->p + n->ob2, n->Z2, 1);
  if (e != hipSuccess) return e;
  return gemm<false, true>(n->stream, B, 1, n->Wd, n->H2, n->Wd, n->p + n->oW3, n->Wd, n->Y, 1,
                           n->p + n->ob3, nullptr, 0);
}

// Loss and gradients into n->g for the first B rows of X and T; returns the
// mean squared error through *loss (synchronises).
hr_status loss_and_grad(hr_mlp* n, int B, float* loss) {
  HR_HIPM(forward(n, B));
  const int nb = (int)cdiv(B, 256);
  k_mse<<<nb, 256, 0, n->stream>>>(n->Y, n->T, B, n->dY, n->part);
  HR_HIPM(hipGetLastError());
  HR_HIPM(hipMemcpyAsync(n->host_part, n->part, nb * sizeof(float), hipMemcpyDeviceToHost,
                         n->stream));
  const int W = n->Wd, F = n->F;
  float* g = n->g;
  // layer 3: dW3 = dY^T H2 (1 x W), db3 = sum dY, dH2 = dY W3
  HR_HIPM(gemm_wgrad(n->stream, 1, W, B, n->dY, 1, n->H2, W, g + n->oW3, n->kpart));
  HR_HIPM(colsum(n->stream, n->dY, B, 1, n->part + 1024, g + n->ob3));
  HR_HIPM((gemm<false, false>(n->stream, B, W, 1, n->dY, 1, n->p + n->oW3, W, n->dH, W, nullptr,
                              nullptr, 0)));
  k_gelu_back<<<cdiv((long)B * W, 256), 256, 0, n->stream>>>(n->dH, n->Z2, n->dZ, (long)B * W);
  HR_HIPM(hipGetLastError());
  // layer 2: dW2 = dZ2^T H1, db2 = colsum dZ2, dH1 = dZ2 W2
  HR_HIPM(gemm_wgrad(n->stream, W, W, B, n->dZ, W, n->H1, W, g + n->oW2, n->kpart));
  HR_HIPM(colsum(n->stream, n->dZ, B, W, n->part + 1024, g + n->ob2));
  HR_HIPM((gemm<false, false>(n->stream, B, W, W, n->dZ, W, n->p + n->oW2, W, n->dH, W, nullptr,
                              nullptr, 0)));
  k_gelu_back<<<cdiv((long)B * W, 256), 256, 0, n->stream>>>(n->dH, n->Z1, n->dZ, (long)B * W);
  HR_HIPM(hipGetLastError());
  // layer 1: dW1 = dZ1^T X, db1 = colsum dZ1
  HR_HIPM(gemm_wgrad(n->stream, W, F, B, n->dZ, W, n->X, F, g + n->oW1, n->kpart));
  HR_HIPM(colsum(n->stream, n->dZ, B, W, n->part + 1024, g + n->ob1));
  HR_HIPM(hipStreamSynchronize(n->stream));
  double s = 0.0;
  for (int i = 0; i < nb; ++i) s += n->host_part[i];
  *loss = (float)(s / B);
  return HR_OK;
}

hr_status check_mlp(const hr_mlp* n, int B) {
  if (!n) return mfail(HR_EINVAL, "null network");
  if (!n->bound) return mfail(HR_ESTATE, "network has no bound workspace");
  if (B < 1 || B > n->max_batch) return mfail(HR_EINVAL, "batch size out of range");
  return HR_OK;
}

}  // namespace

extern "C" {

hr_status hr_mlp_create(int width, unsigned long long seed, hr_mlp** out) {
  if (!out) return mfail(HR_EINVAL, "null output pointer");
  *out = nullptr;
  if (width < 8 || width > 1024 || width % 8) return mfail(HR_EINVAL, "width must be 8..1024, a multiple of 8");
  hr_mlp* n = new (std::nothrow) hr_mlp();
  if (!n) return mfail(HR_ENOMEM, "host allocation failed");
  n->Wd = width;
  const long F = n->F, W = width;
  n->oW1 = 0;
  n->ob1 = n->oW1 + W * F;
  n->oW2 = n->ob1 + W;
  n->ob2 = n->oW2 + W * W;
  n->oW3 = n->ob2 + W;
  n->ob3 = n->oW3 + W;
  n->np = n->ob3 + 1;
  n->host.assign(n->np, 0.0f);
  std::mt19937_64 rng(seed);
  auto fill = [&](long off, long count, long fan_in) {
    std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / (double)fan_in));
    for (long i = 0; i < count; ++i) n->host[off + i] = (float)nd(rng);
  };
  fill(n->oW1, W * F, F);
  fill(n->oW2, W * W, W);
  fill(n->oW3, W, W);
  *out = n;
  return HR_OK;
}

size_t hr_mlp_param_count(const hr_mlp* n) { return n ? (size_t)n->np : 0; }

size_t hr_mlp_workspace_bytes(const hr_mlp* n, int max_batch) {
  if (!n || max_batch < 1) return 0;
  return mlp_layout(const_cast<hr_mlp*>(n), max_batch, nullptr);
}

hr_status hr_mlp_bind(hr_mlp* n, void* dev_ptr, size_t bytes, int max_batch, void* hip_stream) {
  if (!n) return mfail(HR_EINVAL, "null network");
  if (n->bound) return mfail(HR_ESTATE, "network already bound");
  if (max_batch < 1 || max_batch > 262144) return mfail(HR_EINVAL, "max_batch must be 1..262144");
  if (!dev_ptr || ((uintptr_t)dev_ptr % 256) != 0)
    return mfail(HR_EINVAL, "workspace pointer must be non-null and 256-byte aligned");
  if (bytes < mlp_layout(n, max_batch, nullptr)) return mfail(HR_ENOMEM, "workspace too small");
  HR_HIPM(hipGetDevice(&n->device));
  if (hip_stream) {
    n->stream = (hipStream_t)hip_stream;
  } else {
    HR_HIPM(hipStreamCreate(&n->stream));
    n->own_stream = true;
  }
  HR_HIPM(hipHostMalloc((void**)&n->host_part, ((size_t)max_batch / 256 + 8) * sizeof(float),
                        hipHostMallocDefault));
  mlp_layout(n, max_batch, (char*)dev_ptr);
  n->max_batch = max_batch;
  HR_HIPM(hipMemcpyAsync(n->p, n->host.data(), n->np * sizeof(float), hipMemcpyHostToDevice,
                         n->stream));
  HR_HIPM(hipMemsetAsync(n->m, 0, n->np * sizeof(float), n->stream));
  HR_HIPM(hipMemsetAsync(n->v, 0, n->np * sizeof(float), n->stream));
  HR_HIPM(hipStreamSynchronize(n->stream));
  n->bound = true;
  return HR_OK;
}

void hr_mlp_destroy(hr_mlp* n) {
  if (!n) return;
  if (n->bound) {
    (void)hipSetDevice(n->device);
    (void)hipStreamSynchronize(n->stream);
    if (n->host_part) (void)hipHostFree(n->host_part);
    if (n->own_stream) (void)hipStreamDestroy(n->stream);
  }
  delete n;
}

hr_status hr_mlp_get_params(const hr_mlp* n, float* host, size_t count) {
  if (!n || !host || count != (size_t)n->np) return mfail(HR_EINVAL, "count must equal the parameter count");
  if (!n->bound) {
    std::memcpy(host, n->host.data(), count * sizeof(float));
    return HR_OK;
  }
  HR_HIPM(hipMemcpyAsync(host, n->p, count * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  HR_HIPM(hipStreamSynchronize(n->stream));
  return HR_OK;
}

hr_status hr_mlp_set_params(hr_mlp* n, const float* host, size_t count) {
  if (!n || !host || count != (size_t)n->np) return mfail(HR_EINVAL, "count must equal the parameter count");
  std::memcpy(n->host.data(), host, count * sizeof(float));
  if (n->bound) {
    HR_HIPM(hipMemcpyAsync(n->p, host, count * sizeof(float), hipMemcpyHostToDevice, n->stream));
    HR_HIPM(hipStreamSynchronize(n->stream));
  }
  return HR_OK;
}

hr_status hr_mlp_set_output_map(hr_mlp* n, float scale, float shift) {
  if (!n || !(scale != 0.0f) || !std::isfinite(scale) || !std::isfinite(shift))
    return mfail(HR_EINVAL, "finite non-zero scale and finite shift required");
  n->out_scale = scale;
  n->out_shift = shift;
  return HR_OK;
}

hr_status hr_mlp_forward(hr_mlp* n, const float* host_x, int B, float* host_y) {
  hr_status st = check_mlp(n, B);
  if (st != HR_OK) return st;
  if (!host_x || !host_y) return mfail(HR_EINVAL, "null input or output");
  HR_HIPM(hipSetDevice(n->device));
  HR_HIPM(hipMemcpyAsync(n->X, host_x, (size_t)B * n->F * sizeof(float), hipMemcpyHostToDevice,
                         n->stream));
  HR_HIPM(forward(n, B));
  HR_HIPM(hipMemcpyAsync(host_y, n->Y, (size_t)B * sizeof(float), hipMemcpyDeviceToHost,
                         n->stream));
  HR_HIPM(hipStreamSynchronize(n->stream));
  return HR_OK;
}

hr_status hr_mlp_gradients(hr_mlp* n, const float* host_x, const float* host_t, int B,
                           float* host_grad, float* loss) {
  hr_status st = check_mlp(n, B);
  if (st != HR_OK) return st;
  if (!host_x || !host_t || !host_grad || !loss) return mfail(HR_EINVAL, "null argument");
  HR_HIPM(hipSetDevice(n->device));
  HR_HIPM(hipMemcpyAsync(n->X, host_x, (size_t)B * n->F * sizeof(float), hipMemcpyHostToDevice,
                         n->stream));
  HR_HIPM(hipMemcpyAsync(n->T, host_t, (size_t)B * sizeof(float), hipMemcpyHostToDevice,
                         n->stream));
  st = loss_and_grad(n, B, loss);
  if (st != HR_OK) return st;
  HR_HIPM(hipMemcpyAsync(host_grad, n->g, n->np * sizeof(float), hipMemcpyDeviceToHost,
                         n->stream));
  HR_HIPM(hipStreamSynchronize(n->stream));
  return HR_OK;
}

hr_status hr_mlp_train_step(hr_mlp* n, const float* dev_x, const float* dev_t, int B, float lr,
                            float* loss) {
  hr_status st = check_mlp(n, B);
  if (st != HR_OK) return st;
  if (!dev_x || !dev_t || !loss || !(lr > 0)) return mfail(HR_EINVAL, "need inputs, targets, lr > 0");
  HR_HIPM(hipSetDevice(n->device));
  HR_HIPM(hipMemcpyAsync(n->X, dev_x, (size_t)B * n->F * sizeof(float), hipMemcpyDeviceToDevice,
                         n->stream));
  HR_HIPM(hipMemcpyAsync(n->T, dev_t, (size_t)B * sizeof(float), hipMemcpyDeviceToDevice,
                         n->stream));
  st = loss_and_grad(n, B, loss);
  if (st != HR_OK) return st;
  n->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float lr_t = lr * (float)(std::sqrt(1.0 - std::pow(b2, (double)n->adam_t)) /
                                  (1.0 - std::pow(b1, (double)n->adam_t)));
  k_adam<<<cdiv(n->np, 256), 256, 0, n->stream>>>(n->p, n->g, n->m, n->v, n->np, lr_t, b1, b2,
                                                   1e-8f);
  HR_HIPM(hipGetLastError());
  return HR_OK;
}

hr_status hr_mlp_grid_features(hr_mlp* n, const hr_grid* g, const double* cfg9, float* dev_out) {
  if (!n || !g || !cfg9 || !dev_out) return mfail(HR_EINVAL, "null argument");
  (void)n;
  if (!g->bound) return mfail(HR_ESTATE, "grid not bound");
  if (!g->have_sources) return mfail(HR_ESTATE, "punctures not set");
  if (g->d.zo)
    return mfail(HR_EINVAL, "the warm-start features do not cover SinhCylindrical or Cartesian grids");
  FeatArgs a{};
  a.d = g->d;
  a.x0max = g->coords == HR_SPHERICAL ? g->prm.rmax : 1.0;
  for (int k = 0; k < 9; ++k) a.cfg[k] = (float)cfg9[k];
  a.rho = g->rho;
  a.zc = g->zc;
  a.cphi = g->cphi;
  a.sphi = g->sphi;
  for (int p = 0; p < 2; ++p)
    for (int k = 0; k < 3; ++k) a.px[p][k] = g->pz.x[p < g->pz.n ? p : 0][k];
  a.X = dev_out;
  a.row0 = 0;
  a.nrows = g->d.P0 * g->d.N1 * g->d.N2;
  k_features<<<cdiv(a.nrows, 256), 256, 0, g->stream>>>(a);
  HR_HIPM(hipGetLastError());
  HR_HIPM(hipStreamSynchronize(g->stream));
  return HR_OK;
}

hr_status hr_warm_start(hr_grid* g, hr_mlp* n, const double* cfg9, double eta) {
  if (!g || !n || !cfg9) return mfail(HR_EINVAL, "null argument");
  if (!g->bound || !n->bound) return mfail(HR_ESTATE, "grid and network must be bound");
  if (!g->have_sources) return mfail(HR_ESTATE, "punctures not set");
  if (!(eta > 0)) return mfail(HR_EINVAL, "eta must be > 0");
  if (g->d.zo)
    return mfail(HR_EINVAL, "the warm-start features do not cover SinhCylindrical or Cartesian grids");
  HR_HIPM(hipSetDevice(g->device));
  HR_HIPM(hipStreamSynchronize(g->stream));
  FeatArgs a{};
  a.d = g->d;
  a.x0max = g->coords == HR_SPHERICAL ? g->prm.rmax : 1.0;
  for (int k = 0; k < 9; ++k) a.cfg[k] = (float)cfg9[k];
  a.rho = g->rho;
  a.zc = g->zc;
  a.cphi = g->cphi;
  a.sphi = g->sphi;
  for (int p = 0; p < 2; ++p)
    for (int k = 0; k < 3; ++k) a.px[p][k] = g->pz.x[p < g->pz.n ? p : 0][k];
  const int next = g->d.P0 * g->d.N1 * g->d.N2;
  // the grid's stored points go through the network in max_batch chunks
  for (int start = 0; start < next; start += n->max_batch) {
    const int B = std::min(n->max_batch, next - start);
    a.X = n->X;
    a.row0 = start;
    a.nrows = B;
    k_features<<<cdiv(B, 256), 256, 0, n->stream>>>(a);
    HR_HIPM(hipGetLastError());
    HR_HIPM(forward(n, B));
    k_write_state<<<cdiv(B, 256), 256, 0, n->stream>>>(n->Y, B, n->out_scale, n->out_shift, eta,
                                                       g->f64.un + start, g->f64.vn + start);
    HR_HIPM(hipGetLastError());
  }
  HR_HIPM(hipStreamSynchronize(n->stream));
  return HR_OK;
}

}  // extern "C"
