/*
 * hrelax.h -- C ABI of the MI355X hyperbolic-relaxation solver for
 * conformally flat binary-black-hole puncture initial data.
 *
 * The method (arXiv:2501.14030, "Basic equations" section):
 *   Eq. (4)  lap(u) + (1/8) A_ij A^ij (psi_s + u)^-7 = 0
 *            for the regular part u of the conformal factor psi = psi_s + u,
 *            lap = flat-space Laplacian in curvilinear coordinates,
 *            A_ij  = Bowen-York puncture extrinsic curvature.
 *   Eq. (5)  d_t u = v - eta u,   d_t v = c^2 [ lap(u) + (1/8) A A (psi_s+u)^-7 ]
 *            a damped wave system whose steady state solves Eq. (4); it is
 *            integrated by the method of lines with classic RK4, with a wave
 *            speed proportional to the local grid spacing (end of the same
 *            section). The driver follows the paper's Algorithm 1: per RK
 *            stage RHS, boundary conditions and the RK substep; periodically
 *            the residual H (left-hand side of Eq. 4) and its grid L2 norm,
 *            then a stop test on that norm.
 *
 * Conventions shared by every entry point:
 *   * Return value: hr_status; 0 is success, negative values are errors. No
 *     function aborts, throws or exits. hr_last_error() returns a
 *     thread-local message for the last failing call on that thread.
 *   * A handle is not thread-safe; use one handle per host thread / stream.
 *   * Grid functions are cell-centred. "Interior" arrays hold N0*N1*N2
 *     doubles, index i0 + N0*(i1 + N1*i2) (x0 fastest). "Extended" arrays
 *     also hold the NG outer-boundary points beyond xx0's maximum:
 *     (N0+NG)*N1*N2 doubles, index i0 + (N0+NG)*(i1 + N1*i2). NG = fd_order/2.
 *     All other ghost points are images of stored points (parity +1) and are
 *     never stored.
 *   * Host pointers are only read or written during the call; the caller
 *     keeps ownership. Device memory is owned by the caller (hr_grid_bind).
 */
#ifndef HRELAX_H
#define HRELAX_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hr_grid hr_grid;

typedef enum {
  HR_OK = 0,
  HR_EINVAL = -1,      /* invalid argument */
  HR_ENOMEM = -2,      /* workspace too small / host allocation failed */
  HR_EDEVICE = -3,     /* a HIP runtime call failed */
  HR_ENOTCONV = -4,    /* tolerance not reached within n_steps */
  HR_ENONFINITE = -5,  /* residual became NaN or Inf (e.g. dt above the RK4 limit) */
  HR_ESTATE = -6       /* call out of order (e.g. relax before bind/set_punctures) */
} hr_status;

typedef enum {
  HR_SINHSYMTP = 0, /* prolate-spheroidal, sinh-stretched radial coordinate */
  HR_SPHERICAL = 1  /* uniform r in [0, rmax], theta, phi */
} hr_coords;

typedef enum {
  HR_FP64 = 0,            /* every step in double precision */
  HR_FP32 = 1,            /* bulk steps in single precision only */
  HR_FP32_FP64FINISH = 2  /* single precision until the switch, then double */
} hr_precision;

/*
 * Coordinate parameters. SinhSymTP (companion-paper coordinates; the exact
 * map is a reading, listed with the design notes):
 *   A(xx0) = amax sinh(xx0/sinhwaa)/sinh(1/sinhwaa), xx0 in [0,1],
 *   x = A sin(xx1) cos(xx2), y = A sin(xx1) sin(xx2),
 *   z = sqrt(A^2 + bscale^2) cos(xx1); foci (0,0,+-bscale).
 * Spherical: r = xx0 in [0, rmax].
 * cfl: dt = cfl * ds_g when hr_relax receives dt <= 0, ds_g = smallest proper
 * cell width over the interior.
 */
typedef struct {
  double amax;    /* default 1e6 */
  double sinhwaa; /* default 0.07 */
  double bscale;  /* default 1.0 */
  double rmax;    /* default 100 */
  double cfl;     /* default 0.5 */
} hr_grid_params;

/* Fills p with the defaults above. */
void hr_default_params(hr_grid_params* p);

/*
 * Creates a grid (host side only; no device memory yet).
 *   coords   HR_SINHSYMTP or HR_SPHERICAL
 *   N0,N1,N2 interior points along xx0, xx1 (theta), xx2 (phi);
 *            N0 >= NG, N1 >= NG, N2 even and >= 2 (phi + pi parity images),
 *            total stored points below 2^31.
 *   fd_order centred finite-difference order: 2, 4, 6, 8 or 10
 *   p        coordinate parameters, NULL for defaults (copied)
 *   out      receives the handle; free it with hr_grid_destroy.
 * Errors: HR_EINVAL.
 */
hr_status hr_grid_create(hr_coords coords, int N0, int N1, int N2, int fd_order,
                         const hr_grid_params* p, hr_grid** out);

/* Frees the handle and its host resources (never the caller's device memory).
 * NULL is accepted. */
void hr_grid_destroy(hr_grid* g);

/* Interior and extended point counts (either pointer may be NULL). */
hr_status hr_grid_sizes(const hr_grid* g, size_t* n_interior, size_t* n_extended);

/* Device workspace the grid needs (all precisions), in bytes. The paper sizes
 * the whole footprint up front ("Memory Management" subsection). */
size_t hr_workspace_bytes(const hr_grid* g);

/*
 * Binds caller-owned device memory and a HIP stream (hipStream_t passed as
 * void*; NULL = the library creates and owns a stream of default priority).
 * dev_ptr must be 256-byte aligned and at least hr_workspace_bytes() long; it
 * stays owned by the caller and must outlive the handle's device work.
 * Uploads the coordinate tables and zeroes the state. Synchronous.
 * Errors: HR_EINVAL (NULL/misaligned), HR_ENOMEM (too small), HR_EDEVICE.
 */
hr_status hr_grid_bind(hr_grid* g, void* dev_ptr, size_t bytes, void* hip_stream);

/*
 * Sets the punctures (paper "Basic equations": Brandt-Bruegmann punctures with
 * the Bowen-York extrinsic curvature) and computes on the device
 *   psi_s = 1 + sum_n m_n/(2 r_n),
 *   S_src = (1/8) A_ij A^ij,
 *   A^ij = sum_n 3/(2 r_n^2)[P^i n^j + P^j n^i - (delta^ij - n^i n^j) P.n]
 *          + 3/r_n^3 [(S x n)^i n^j + (S x n)^j n^i],
 * then resets u = v = 0.
 *   n  number of punctures, 1..4
 *   m  n bare masses (> 0); x, P, S: 3n doubles each (position, linear
 *      momentum, spin), host memory.
 * Errors: HR_EINVAL, HR_ESTATE (not bound), HR_EDEVICE.
 */
hr_status hr_set_punctures(hr_grid* g, int n, const double* m, const double* x,
                           const double* P, const double* S);

/* Report filled by hr_relax. history (optional, caller-owned, history_cap
 * doubles) receives the residual after every check. */
typedef struct {
  long steps_taken;   /* RK4 steps done by this call */
  long fp32_steps;    /* of which in single precision */
  double residual;    /* last residual checked (FP64), NaN if none */
  double dt_used;
  double* history;
  long history_cap;
  long n_history;     /* checks done (may exceed history_cap) */
} hr_relax_report;

/*
 * Relaxes Eq. (5) from the current state with classic RK4.
 *   eta         damping factor (> 0)
 *   c           wave-speed scale kappa: c(x) = kappa ds_min(x)/ds_g (> 0)
 *   dt          time step; <= 0 means cfl * ds_g
 *   n_steps     maximum number of RK4 steps (>= 0)
 *   tol         > 0: stop at the first check whose residual is below tol;
 *               <= 0: run exactly n_steps
 *   check_every residual check every this many steps (> 0)
 *   prec        HR_FP64, HR_FP32 or HR_FP32_FP64FINISH (see
 *               hr_set_fp32_switch)
 *   rep         optional report
 * Residuals are always computed in FP64 (FP32 states are promoted).
 * Returns HR_OK, HR_ENOTCONV (tol > 0 not reached), HR_ENONFINITE,
 * HR_EINVAL, HR_ESTATE or HR_EDEVICE. Blocks until the last residual readback.
 */
hr_status hr_relax(hr_grid* g, double eta, double c, double dt, long n_steps,
                   double tol, int check_every, hr_precision prec,
                   hr_relax_report* rep);

/*
 * Switch rule for HR_FP32_FP64FINISH: the single-precision phase ends at the
 * first check whose residual is below switch_residual, or after stall_checks
 * consecutive checks without a new minimum, or after max_fp32_steps steps
 * (<= 0: no cap). Defaults: 1e-6, 2, no cap.
 */
hr_status hr_set_fp32_switch(hr_grid* g, double switch_residual, int stall_checks,
                             long max_fp32_steps);

/* Copies u or v (FP64 state) to host memory; n must be the interior or the
 * extended count, which selects the layout. */
hr_status hr_get_u(const hr_grid* g, double* host_out, size_t n);
hr_status hr_get_v(const hr_grid* g, double* host_out, size_t n);

/* Sets u or v from host memory (warm start, resume). n = extended count sets
 * every stored point; n = interior count sets the interior and fills each
 * outer point by the 1/r continuation f(i0) = f(N0-1) r(N0-1)/r(i0). */
hr_status hr_set_u(hr_grid* g, const double* host_in, size_t n);
hr_status hr_set_v(hr_grid* g, const double* host_in, size_t n);

/* Grid L2 norm of the Hamiltonian-constraint residual of the current state,
 * sqrt(sum_interior H^2 / N_interior), in FP64. */
hr_status hr_residual_l2(hr_grid* g, double* out);

/* cfl * ds_g. */
hr_status hr_suggest_dt(const hr_grid* g, double cfl, double* dt);

/*
 * Kernel configuration of a grid (performance only; results are identical up
 * to floating-point rounding order, and bitwise identical for the streaming
 * switch, which changes cache policy only).
 *   variant    0 = automatic, 1 = plane tiles (one phi plane per block),
 *              2 = phi-marching columns (a block walks `chunk` phi planes)
 *   streaming  -1 = automatic (by grid size), 0 = cached, 1 = non-temporal
 *              loads/stores for fields touched once per stage
 *   chunk      phi planes per block for variant 2 (0 = automatic)
 * Errors: HR_EINVAL.
 */
typedef struct {
  int variant;
  int streaming;
  int chunk;
} hr_kernel_config;

hr_status hr_set_kernel_config(hr_grid* g, const hr_kernel_config* cfg);
hr_status hr_get_kernel_config(const hr_grid* g, hr_kernel_config* cfg);

/*
 * Measurement: runs n_steps RK4 steps of the current state in precision prec
 * (HR_FP64 or HR_FP32), bracketing every stage-kernel launch with hipEvents
 * recorded on the grid's stream, and returns in avg_us[0..3] the mean duration
 * of the stage-1..4 kernels in microseconds (avg_us[4]: mean over all four).
 * The state advances by n_steps. Errors: HR_EINVAL, HR_ESTATE, HR_EDEVICE.
 */
hr_status hr_time_stage_kernels(hr_grid* g, double eta, double c, double dt, long n_steps,
                                hr_precision prec, double* avg_us);

/* Message of the last failing call on this thread ("" if none). */
const char* hr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HRELAX_H */
