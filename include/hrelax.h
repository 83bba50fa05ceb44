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
 *     SinhCylindrical grids also hold the NG outer rows beyond each z face:
 *     (N0+NG)*(N1+2NG)*N2 doubles, index i0 + (N0+NG)*(i1 + NG + (N1+2NG)*i2)
 *     for i1 in [-NG, N1+NG). All other ghost points are images of stored
 *     points (parity +1) and are never stored.
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
  HR_SINHSYMTP = 0,    /* prolate-spheroidal, sinh-stretched radial coordinate */
  HR_SPHERICAL = 1,    /* uniform r in [0, rmax], theta, phi */
  HR_SINHSPHERICAL = 2, /* r = amax sinh(xx0/w)/sinh(1/w), xx0 in [0,1], theta, phi */
  HR_SINHCYLINDRICAL = 3, /* rho = A(xx0), z = A(xx1), xx1 in [-1,1], phi; the
                            same sinh stretching A for rho and z; both z faces
                            are outer boundaries */
  HR_CARTESIAN = 4        /* x, y, z in the cube [-rmax, rmax]^3; all six faces
                             are outer boundaries, no parity images */
} hr_coords;

typedef enum {
  HR_FP64 = 0,            /* every step in double precision */
  HR_FP32 = 1,            /* every step in single precision (state rounded to FP32;
                             the residual floor is set by single precision) */
  HR_FP32_FP64FINISH = 2  /* split state: FP64 base + FP32 increment integrated in
                             single precision, FP64 rebase/residual/stop test every
                             check, then plain FP64 steps to the tolerance */
} hr_precision;

/*
 * Coordinate parameters. SinhSymTP (companion-paper coordinates; the exact
 * map is a reading, listed with the design notes):
 *   A(xx0) = amax sinh(xx0/sinhwaa)/sinh(1/sinhwaa), xx0 in [0,1],
 *   x = A sin(xx1) cos(xx2), y = A sin(xx1) sin(xx2),
 *   z = sqrt(A^2 + bscale^2) cos(xx1); foci (0,0,+-bscale).
 * Spherical: r = xx0 in [0, rmax]. Cartesian: rmax is the cube's half side.
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
 * Creates a grid (host side only; no device memory yet): the setup steps of
 * Algorithm 1 that sample the coordinates xx^i and precompute the reference
 * metric (here the Laplacian factors of Eq. 4 per (xx0, xx1), the wave speed
 * and the outer-boundary geometry), on the SinhSymTP grids of the "Basic
 * equations" section or the spherical-like, cylindrical-like and
 * Cartesian-like families the conclusions name.
 *   coords   HR_SINHSYMTP, HR_SPHERICAL, HR_SINHSPHERICAL, HR_SINHCYLINDRICAL or
 *            HR_CARTESIAN
 *   N0,N1,N2 interior points along xx0, xx1 (theta, or z for SinhCylindrical),
 *            xx2 (phi); N0 >= NG, N1 >= NG, N2 even and >= 2 (phi + pi parity
 *            images), total stored points below 2^31. SinhCylindrical also
 *            stores NG outer rows beyond each z face, so its extended layout
 *            (hr_get_u) is (N0 + NG) x (N1 + 2 NG) x N2; the warm-start
 *            network does not take these grids. Cartesian grids (x, y, z
 *            along xx0, xx1, xx2; each N_d >= max(NG, 2), any parity) store NG
 *            outer layers beyond every face: the extended layout is the padded
 *            box (N0 + 2 NG) x (N1 + 2 NG) x (N2 + 2 NG), whose edge and corner
 *            points are never read and stay zero. They relax in HR_FP64,
 *            HR_FP32 or HR_FP32_FP64FINISH on the stage kernels (no resident
 *            kernel, batch, volume norm or warm start: those calls return
 *            HR_EINVAL for them).
 *   fd_order centred finite-difference order: 2, 4, 6, 8 or 10
 *   p        coordinate parameters, NULL for defaults (copied)
 *   out      receives the handle; free it with hr_grid_destroy.
 * Errors: HR_EINVAL.
 */
hr_status hr_grid_create(hr_coords coords, int N0, int N1, int N2, int fd_order,
                         const hr_grid_params* p, hr_grid** out);

/* Frees the handle and its host resources (the "free storage" step at the end
 * of Algorithm 1; never the caller's device memory, which the caller frees).
 * Waits for the grid's outstanding device work first. NULL is accepted. */
void hr_grid_destroy(hr_grid* g);

/* Interior and extended point counts (either pointer may be NULL); they size
 * the arrays of hr_get_u/v and hr_set_u/v. Errors: HR_EINVAL (null grid). */
hr_status hr_grid_sizes(const hr_grid* g, size_t* n_interior, size_t* n_extended);

/* Device workspace the grid needs (all precisions), in bytes. The paper sizes
 * the whole footprint up front ("Memory Management" subsection). */
size_t hr_workspace_bytes(const hr_grid* g);

/*
 * Binds caller-owned device memory and a HIP stream (hipStream_t passed as
 * void*; NULL = the library creates and owns a stream of default priority).
 * This is the allocation step of Algorithm 1: the whole device footprint
 * (Runge-Kutta stage storage, source terms, coefficient tables) is one block
 * sized up front, as the "Memory Management" subsection of Sec. 4 does.
 * dev_ptr must be 256-byte aligned and at least hr_workspace_bytes() long; it
 * stays owned by the caller and must outlive the handle's device work.
 * Uploads the coordinate tables and zeroes the state. Synchronous.
 * Errors: HR_EINVAL (NULL/misaligned), HR_ENOMEM (too small), HR_EDEVICE.
 */
hr_status hr_grid_bind(hr_grid* g, void* dev_ptr, size_t bytes, void* hip_stream);

/*
 * Sets the punctures (paper "Basic equations": Brandt-Bruegmann punctures with
 * the Bowen-York extrinsic curvature; Algorithm 1's "compute constant source
 * terms" step) and computes on the device
 *   psi_s = 1 + sum_n m_n/(2 r_n),
 *   S_src = (1/8) A_ij A^ij,
 *   A^ij = sum_n 3/(2 r_n^2)[P^i n^j + P^j n^i - (delta^ij - n^i n^j) P.n]
 *          + 3/r_n^3 [(S x n)^i n^j + (S x n)^j n^i],
 * then resets u = v = 0.
 *   n  number of punctures, 1..4
 *   m  n bare masses (> 0); x, P, S: 3n doubles each (position, linear
 *      momentum, spin), host memory.
 * On a SinhSymTP grid every puncture must lie at one of the two foci
 * (0, 0, +-bscale), each coordinate within 1e-12 bscale: the coordinates put
 * their finest cells there (the paper's binary punctures sit at the foci).
 * On a Cartesian grid a puncture may not sit on a cell centre (all three
 * coordinates within 1e-9 cell widths of -rmax + (j + 1/2) dx), where r = 0.
 * Arguments are checked before the grid's state, so an invalid argument is
 * HR_EINVAL even on an unbound grid.
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
  long resident_fallbacks;  /* check intervals (or the final unchecked tail)
                               rerun on the stage kernels because a resident
                               launch's exchange wait timed out; the call then
                               continues on the stage kernels */
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
 * A resident launch whose exchange wait times out is undone and its interval
 * rerun on the stage kernels (see hr_set_wait_limit).
 */
hr_status hr_relax(hr_grid* g, double eta, double c, double dt, long n_steps,
                   double tol, int check_every, hr_precision prec,
                   hr_relax_report* rep);

/*
 * For callers that cannot allocate device memory (code between graph
 * captures, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * form of hr_relax, same arguments and results (prec is HR_FP64), whose
 * scratch -- the RK4 stage buffers and accumulators, the resident kernel's
 * exchange buffers and stage counters, the residual partial sums -- lives in
 * a static device array of the library (64 MiB, one per GPU, held until the
 * process ends) instead of the grid's bound workspace. The state, sources and
 * tables stay in the workspace. The call allocates nothing: no hipMalloc or
 * hipFree, no graph instantiation, no events; it launches the same kernels
 * as hr_relax, eagerly, and waits for its stream before returning.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (other threads, other streams) race
 * and must be serialised by the caller.
 * Errors: those of hr_relax; HR_ENOMEM when the grid's scratch exceeds 64 MiB
 * (six FP64 fields of the extended layout plus partial sums: up to about 1.3
 * million stored points, e.g. 128x128x16 and 256x128x32 fit, 256x256x32 does
 * not); HR_ESTATE when c differs from the wave-speed scale whose planes are
 * loaded (1 after hr_grid_bind, else the c of the last hr_relax).
 */
hr_status hr_relax_noalloc(hr_grid* g, double eta, double c, double dt,
                           long n_steps, double tol, int check_every,
                           hr_relax_report* rep);

/*
 * HR_FP32_FP64FINISH, the single-precision bulk with a double-precision finish
 * (paper: strongly typed single-precision builds, "Roofline Analysis"
 * subsection). The state is split into an FP64 base y_b and an FP32 increment
 * e. Every check_every steps: the FP64 slopes k(y_b) are evaluated once, e
 * starts from 0 and is integrated with RK4 in FP32 using the slope
 * k(y_b) + L e + S_src[(psi_s + u_b + e_u)^-7 - (psi_s + u_b)^-7] (L the linear
 * part of Eq. 5 with its boundary conditions), then y_b += e in FP64 and the
 * FP64 residual of y_b is checked. In exact arithmetic this is the FP64 RK4
 * trajectory; rounding is relative to the increment, not to u. The phase
 * ends, and plain FP64 steps continue to the tolerance, at the first check
 * whose residual is below switch_residual (0: ten times tol), after
 * stall_checks consecutive checks without a new minimum, or after
 * max_fp32_steps steps (<= 0: no cap). Defaults: 0, 8, no cap.
 */
hr_status hr_set_fp32_switch(hr_grid* g, double switch_residual, int stall_checks,
                             long max_fp32_steps);

/* Copies u or v (FP64 state) to host memory -- the solution transfer from
 * device to host of the "Data Transfer Optimization" subsection; n must be
 * the interior or the extended count, which selects the layout. Waits for the
 * grid's stream. Errors: HR_EINVAL (null pointer, other n), HR_ESTATE (not
 * bound), HR_EDEVICE. */
hr_status hr_get_u(const hr_grid* g, double* host_out, size_t n);
hr_status hr_get_v(const hr_grid* g, double* host_out, size_t n);

/* Sets u or v from host memory: Algorithm 1's "set initial conditions" step
 * with a caller-given state (warm start, resume; u = v = 0 is what
 * hr_set_punctures leaves). n = extended count sets every stored point; n =
 * interior count sets the interior and fills each outer point by the 1/r
 * continuation f(i0) = f(N0-1) r(N0-1)/r(i0) (SinhCylindrical's z-face rows
 * then continue the nearest interior row the same way along xx1).
 * Synchronous. Errors: HR_EINVAL
 * (null pointer, other n), HR_ESTATE (not bound), HR_EDEVICE. */
hr_status hr_set_u(hr_grid* g, const double* host_in, size_t n);
hr_status hr_set_v(hr_grid* g, const double* host_in, size_t n);

/* Sets v = eta u at every stored point of the FP64 state: the relation that
 * the steady state of Eq. (5) obeys for damping eta (u_t = v - eta u = 0).
 * Lets a relaxation continue with another damping factor from a state relaxed
 * with the first (e.g. after a heavily damped smoothing phase of a warm
 * start), u unchanged. Synchronous. Errors: HR_EINVAL (null grid, eta not
 * finite and > 0), HR_ESTATE (not bound), HR_EDEVICE. */
hr_status hr_reset_v(hr_grid* g, double eta);

/* L2 norm of the Hamiltonian-constraint residual of the current state, in
 * FP64: by default the grid norm over points, sqrt(sum_interior H^2 /
 * N_interior) (the grid L2 norm of the constraint violations that the paper's
 * stop test uses, Data Transfer Optimization subsection); with
 * hr_set_residual_norm(g, HR_NORM_VOLUME, radius) the volume-weighted norm
 * sqrt(sum H^2 dV / sum dV), dV = |h0 h1 h2| dxx0 dxx1 dxx2 the proper cell
 * volume, optionally over the cells within an integration radius. */
hr_status hr_residual_l2(hr_grid* g, double* out);

typedef enum {
  HR_NORM_POINTS = 0,  /* mean of H^2 over interior points (default) */
  HR_NORM_VOLUME = 1   /* H^2 weighted by the proper cell volume */
} hr_norm;

/*
 * Selects the residual norm for hr_residual_l2 and for the stop test of
 * hr_relax (the tolerance is then compared with the volume-weighted norm).
 * The volume norm takes every interior cell at its proper volume, so the fine
 * cells near the punctures count less and the large outer cells more than in
 * the point norm. radius > 0 restricts the volume norm to the cells whose
 * centre lies at a Cartesian distance below radius from the origin (both sums,
 * H^2 dV and dV, run over those cells); radius <= 0 takes the whole grid.
 * Called on a bound grid, it waits for the grid's stream before updating the
 * weights on the device. Grids in a batch must use HR_NORM_POINTS
 * (hr_batch_relax returns HR_EINVAL otherwise). Errors: HR_EINVAL (null grid,
 * unknown norm, non-finite radius, radius > 0 with HR_NORM_POINTS, no cell
 * centre within the radius, HR_NORM_VOLUME on a Cartesian grid, whose cells are
 * all equal), HR_EDEVICE.
 */
hr_status hr_set_residual_norm(hr_grid* g, hr_norm norm, double radius);

/* dt = cfl * ds_g, ds_g the smallest proper cell width over the interior: the
 * time step that keeps the CFL condition everywhere with the wave speed
 * proportional to the local grid spacing (end of the "Basic equations"
 * section; Algorithm 1's "compute timestep"). Host only. Errors: HR_EINVAL
 * (null pointer, cfl <= 0). */
hr_status hr_suggest_dt(const hr_grid* g, double cfl, double* dt);

/*
 * Kernel configuration of a grid (performance only; results are identical up
 * to floating-point rounding order, and bitwise identical for the streaming
 * switch, which changes cache policy only).
 *   variant    0 = automatic (3 where it applies, else 1 or 2 by size),
 *              1 = plane tiles (one phi plane per block),
 *              2 = phi-marching columns (a block walks `chunk` phi planes;
 *              on Cartesian grids `chunk` z planes),
 *              3 = resident (FP64 steps, and the FP32 increment steps of
 *              HR_FP32_FP64FINISH): one kernel launch runs up to
 *              1000 whole RK4 steps with the state of every 8 x 8 (or
 *              8 x 4, see chunk) (x0, x1) patch (all phi planes) on one
 *              compute unit; the patches exchange their stage input through
 *              the grid's stage buffers. Needs a bound grid with N0 a
 *              multiple of 8 and N1 of the patch rows, N2 <= 16, fd_order 8
 *              or 10 and no more patches than the device holds at once (256
 *              on MI355X: up to 128 x 128 (x0, x1) with 8 x 8 patches), else
 *              HR_EINVAL. Plain HR_FP32 stages run plane tiles instead.
 *              A timed-out exchange wait (not expected) is reported as
 *              HR_EDEVICE by the relaxing call.
 *   streaming  -1 = automatic (by grid size), 0 = cached, 1 = non-temporal
 *              loads/stores for fields touched once per stage
 *   chunk      phi (Cartesian: z) planes per block for variant 2 (0 =
 *              automatic: 16 for FP64 stages, 8 for single-precision ones and
 *              on Cartesian grids); for variant 3 the patch rows along x1, 8 or 4
 *              (0 = automatic: 8 x 4 patches where 8 x 8 ones would leave
 *              more than half of the compute units idle and 8 x 4 ones fit,
 *              else 8 x 8)
 *   graph      -1 = automatic (on), 0 = off, 1 = on: hr_relax captures the
 *              launches of one check interval (RK stages, residual) in a HIP
 *              graph once per (precision form, check_every, eta, dt, c,
 *              configuration) and replays it
 * Errors: HR_EINVAL.
 */
typedef struct {
  int variant;
  int streaming;
  int chunk;
  int graph;
} hr_kernel_config;

hr_status hr_set_kernel_config(hr_grid* g, const hr_kernel_config* cfg);
hr_status hr_get_kernel_config(const hr_grid* g, hr_kernel_config* cfg);

/*
 * Order of the one-sided xx0 difference in the outer radiation condition
 * k_f = -c (f/r + d_r f), with d_r f = (d f / d xx0) / (dr / d xx0) at each
 * outer point (the outer-boundary step of the paper's Algorithm 1; the
 * condition itself comes from the companion paper): 2 (default) takes the
 * point and two inner neighbours along xx0, 4 the point and four. The steady
 * state depends on the choice through the boundary only. Applies to every
 * precision, kernel variant and to batches. On the z faces of SinhCylindrical
 * and every face of a Cartesian grid the difference runs along that face's
 * direction (see hr_grid_create) with the same order. Errors: HR_EINVAL (null
 * grid, order not 2 or 4, N0 < order, or N1 (SinhCylindrical, Cartesian) or N2
 * (Cartesian) < order).
 */
hr_status hr_set_outer_bc_order(hr_grid* g, int order);

/*
 * Storage of the metric-factor planes (the five Laplacian coefficients and
 * c^2 per (xx0, xx1)) read by the single-precision stages (HR_FP32 and the
 * FP32 increment of HR_FP32_FP64FINISH): bits = 32 (default) reads FP32
 * copies, bits = 16 reads bfloat16 copies (the FP32 values rounded to the
 * nearest 8-bit-mantissa value, widened in the kernel). IEEE half precision
 * cannot hold the range of these factors (near the axis and the origin they
 * exceed 65504), hence bfloat16. FP64 stages, residuals, base slopes and the
 * outer-boundary factors always use their own FP64 or FP32 tables.
 * Errors: HR_EINVAL (null grid, bits not 32 or 16).
 */
hr_status hr_set_factor_storage(hr_grid* g, int bits);

/*
 * Bound on the resident kernel's exchange waits: a block gives up after this
 * many polls of one partner's stage counter (each poll is one memory round
 * trip, ~1-2 us), sets an error word, and every block leaves its loop. A
 * timeout means the device could not hold every block at once (other work
 * occupied compute units). hr_relax and hr_relax_noalloc then restore the
 * state of the interval's start (copied before every resident launch) and
 * rerun the interval on the stage kernels, which the rest of the call uses
 * (counted in hr_relax_report.resident_fallbacks); the timing utilities
 * (hr_time_stage_kernels, hr_autotune) return HR_EDEVICE; hr_batch_relax
 * returns HR_EDEVICE and the resident grids' states are unspecified until set
 * again (hr_set_punctures, hr_set_u/v). polls = 0 restores the default, 2^19
 * (about a second). Small values force the timeout path. Errors: HR_EINVAL.
 */
hr_status hr_set_wait_limit(hr_grid* g, unsigned polls);

/*
 * The configuration the relaxation actually runs for precision prec, with the
 * automatic choices resolved (variant 0 becomes 3 where the resident kernel
 * applies and prec is HR_FP64 or HR_FP32_FP64FINISH, else 2 or 1 by size;
 * graph 0 for the resident kernel, whose check interval is a single launch).
 * Errors: HR_EINVAL.
 */
hr_status hr_resolved_kernel(const hr_grid* g, hr_precision prec, hr_kernel_config* cfg);

/*
 * Autotuner: times the stage kernels of this grid in precision prec (HR_FP64
 * or HR_FP32) for every candidate configuration -- plane tiles, phi columns
 * with chunk 1, 2, 4, ... up to N2, and (FP64, where they apply) the resident
 * kernel on 8 x 8 and on 8 x 4 patches -- over n_steps (>= 1) rounds of
 * stages 1-3 (which never write the
 * state y_n; the resident kernel runs whole steps on a copy of the state that
 * is put back afterwards, so the state is unchanged),
 * keeps the fastest in the grid (as hr_set_kernel_config would) and in a
 * process-wide cache keyed by (N0, N1, N2, fd_order, prec); a cached shape is
 * not timed again. best and best_us (optional) receive the choice and its mean
 * stage time in microseconds. Errors: HR_EINVAL, HR_ESTATE, HR_EDEVICE.
 */
hr_status hr_autotune(hr_grid* g, hr_precision prec, int n_steps, hr_kernel_config* best,
                      double* best_us);

/*
 * Measurement: runs n_steps RK4 steps of the current state in precision prec
 * (HR_FP64, HR_FP32, or HR_FP32_FP64FINISH: the split form's FP32 increment
 * steps after one FP64 base evaluation, added into the base at the end),
 * bracketing every stage-kernel launch with hipEvents
 * recorded on the grid's stream, and returns in avg_us[0..3] the mean duration
 * of the stage-1..4 kernels in microseconds (avg_us[4]: mean over all four).
 * With the resident variant (FP64) the n_steps (at most 100000) run in one
 * launch and every entry is its duration / (4 n_steps).
 * The state advances by n_steps. Errors: HR_EINVAL, HR_ESTATE, HR_EDEVICE.
 */
hr_status hr_time_stage_kernels(hr_grid* g, double eta, double c, double dt, long n_steps,
                                hr_precision prec, double* avg_us);

/*
 * Measurement of the relaxation's own launches: with on != 0, each resident
 * kernel launch that later hr_relax calls on this grid issue (its FP64 steps,
 * and the FP32 increment steps of HR_FP32_FP64FINISH where the resident
 * kernel runs them) is bracketed by a pair of HIP events recorded inside the
 * dispatch on the grid's stream, and read after the check interval's own
 * synchronisation (no extra synchronisation). hr_set_launch_timing resets the
 * totals; hr_get_launch_timing returns the summed launch durations in
 * microseconds, the number of launches timed and the RK stages they ran (any
 * pointer may be NULL). Launches of the stage kernels (graph-captured check
 * intervals) are not timed here; hr_time_stage_kernels times those. Errors:
 * HR_EINVAL (null grid), HR_EDEVICE.
 */
hr_status hr_set_launch_timing(hr_grid* g, int on);
hr_status hr_get_launch_timing(const hr_grid* g, double* total_us, long* launches, long* stages);

/*
 * Batched relaxation (catalogs of configurations; the paper relaxes several
 * independent patches with one CUDA stream each, "Multiple, Independent
 * Patches" subsection). A batch groups n bound grids of the same fd_order on
 * one device; the grids stay owned by the caller and must outlive the batch.
 * Every RK stage is one persistent kernel launch over all grids still
 * relaxing; the launches of one check interval are captured once in a HIP
 * graph and replayed. Each grid keeps its own dt (cfl * ds_g), eta and
 * wave-speed scale, and stops at its own first check below tol.
 *   hr_batch_create     n >= 1 distinct bound grids (array copied), none of
 *                       them Cartesian. Errors: HR_EINVAL, HR_ESTATE (a grid
 *                       not bound).
 *   hr_batch_workspace_bytes / hr_batch_bind
 *                       device memory for descriptors and work lists, owned
 *                       by the caller, 256-byte aligned; hip_stream NULL = the
 *                       library creates one (default priority).
 *   hr_batch_relax      eta[n], c[n] per grid; n_steps is rounded up to a
 *                       multiple of check_every; prec HR_FP64 or
 *                       HR_FP32_FP64FINISH (each grid switches to FP64 by its
 *                       own rule, see hr_set_fp32_switch); reps: optional array
 *                       of n reports. Returns HR_OK when every grid converged
 *                       (or, with tol <= 0, ran n_steps), else HR_ENONFINITE /
 *                       HR_ENOTCONV; HR_EINVAL, HR_ESTATE, HR_EDEVICE.
 *   hr_batch_destroy    frees host resources (never the caller's memory).
 */
typedef struct hr_batch hr_batch;

hr_status hr_batch_create(int n, hr_grid* const* grids, hr_batch** out);
size_t hr_batch_workspace_bytes(const hr_batch* b);
hr_status hr_batch_bind(hr_batch* b, void* dev_ptr, size_t bytes, void* hip_stream);
hr_status hr_batch_relax(hr_batch* b, const double* eta, const double* c, long n_steps,
                         double tol, int check_every, hr_precision prec,
                         hr_relax_report* reps);
void hr_batch_destroy(hr_batch* b);

/*
 * Learned warm start. An MLP (FP32) maps 15 features -- 9 configuration
 * values (caller-normalised: mass ratio, spins chi1 and chi2, momentum
 * magnitude, separation), 4 coordinate values of a grid point
 * (2 xx0/xx0_max - 1, cos xx1, sin xx1 cos xx2, sin xx1 sin xx2) and
 * 0.1 log(r_n^2) for the distance r_n to each of the first two punctures --
 * through
 * two hidden layers of `width` GELU units to y, with log u = scale y + shift.
 * Trained on the relaxation's own solves; its prediction is only an initial
 * state, which the relaxation then drives to the residual tolerance.
 *   hr_mlp_create          width (multiple of 8, 8..1024); He-normal
 *                          weights from seed, zero biases (host side).
 *   hr_mlp_param_count     parameters, laid out W1[width x 15], b1, W2[width x
 *                          width], b2, W3[1 x width], b3 (row-major, FP32).
 *   hr_mlp_workspace_bytes / hr_mlp_bind
 *                          caller-owned device memory for parameters, Adam
 *                          moments and activations of up to max_batch rows
 *                          (1..262144); 256-byte aligned; stream NULL = own.
 *   hr_mlp_get/set_params  host copies (count = hr_mlp_param_count).
 *   hr_mlp_set_output_map  scale (non-zero) and shift of log u.
 *   hr_mlp_forward         host x[B x 15] -> host y[B] (network output y).
 *   hr_mlp_gradients       host x, host targets t[B] -> loss = mean (y-t)^2
 *                          and its gradient w.r.t. every parameter (host).
 *   hr_mlp_train_step      device x[B x 15], device t[B]: loss, gradient and
 *                          one Adam step (beta1 0.9, beta2 0.999, eps 1e-8).
 *                          x and t are read on the network's stream: work
 *                          that writes them on another stream must be
 *                          ordered before the call (event wait or sync).
 *   hr_mlp_grid_features   device out[n_extended x 15] for a bound grid with
 *                          punctures set, written on the grid's stream
 *                          (same ordering rule for earlier users of out).
 *   hr_warm_start          sets u = exp(scale y + shift) and v = eta u at every
 *                          stored point of the grid (punctures must be set).
 * Errors: HR_EINVAL, HR_ESTATE, HR_ENOMEM, HR_EDEVICE.
 */
typedef struct hr_mlp hr_mlp;

hr_status hr_mlp_create(int width, unsigned long long seed, hr_mlp** out);
size_t hr_mlp_param_count(const hr_mlp* n);
size_t hr_mlp_workspace_bytes(const hr_mlp* n, int max_batch);
hr_status hr_mlp_bind(hr_mlp* n, void* dev_ptr, size_t bytes, int max_batch, void* hip_stream);
void hr_mlp_destroy(hr_mlp* n);
hr_status hr_mlp_get_params(const hr_mlp* n, float* host, size_t count);
hr_status hr_mlp_set_params(hr_mlp* n, const float* host, size_t count);
hr_status hr_mlp_set_output_map(hr_mlp* n, float scale, float shift);
hr_status hr_mlp_forward(hr_mlp* n, const float* host_x, int batch, float* host_y);
hr_status hr_mlp_gradients(hr_mlp* n, const float* host_x, const float* host_t, int batch,
                           float* host_grad, float* loss);
hr_status hr_mlp_train_step(hr_mlp* n, const float* dev_x, const float* dev_t, int batch,
                            float lr, float* loss);
hr_status hr_mlp_grid_features(hr_mlp* n, const hr_grid* g, const double* cfg9, float* dev_out);
hr_status hr_warm_start(hr_grid* g, hr_mlp* n, const double* cfg9, double eta);

/* Message of the last failing call on this thread ("" if none). */
const char* hr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HRELAX_H */
