/*
 * hgks.h - C ABI of the MI355X library for the per-stage finite-volume update of
 * the high-order gas-kinetic scheme (HGKS) of Cao, Pan & Xu, "High-order
 * gas-kinetic scheme with parallel computation for direct numerical simulation of
 * turbulent flows", arXiv:2005.08736.
 *
 * The library advances the conservative cell averages
 *     Q = (rho, rho U, rho V, rho W, rho E)
 * on a structured 3-D box with the two-stage fourth-order scheme of Sec. 2.1,
 * Eq. (two-stage), whose operator L(Q) = -(1/|Omega|) sum_p F_p (Eq. (finite))
 * uses 2x2 Gauss points per face and the gas-kinetic flux of Eq. (flux) (the
 * smooth simplified form of the first Remark of Sec. 2.1 in HGKS_MODE_SMOOTH).
 *
 * Conventions
 *  - State layout: double q[5][nz][ny][nx] (x fastest), device memory, owned by
 *    the caller, updated in place.
 *  - Every device buffer (state, workspace, outputs) is allocated by the caller;
 *    the library never allocates or frees device memory.  The handle itself is
 *    host memory owned by the library until hgks_destroy.
 *  - All work is enqueued on the caller's HIP stream (hipStream_t passed as
 *    void*; NULL = the default stream).  One handle per stream; calls on one
 *    handle must not overlap.
 *  - Nondimensional gas: R = 1, T = p / rho, internal degrees of freedom
 *    K = (5 - 3 gamma)/(gamma - 1), viscosity mu(T) = mu_ref (T/T_ref)^mu_exp,
 *    collision time tau = mu/p (start of Sec. 3).
 *  - Every function returns an int status (HGKS_OK or a negative code); no C++
 *    exception crosses the boundary.
 */
#ifndef HGKS_H
#define HGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HGKS_OK = 0,
  HGKS_E_INVALID_ARG = -1, /* bad parameter, pointer, size or grid */
  HGKS_E_DEVICE = -2,      /* a HIP runtime call failed */
  HGKS_E_NONPHYSICAL = -3, /* rho <= 0, p <= 0 or a non-finite value appeared */
  HGKS_E_UNSUPPORTED = -4, /* valid but not implemented combination */
  HGKS_E_WORKSPACE = -5    /* workspace missing, too small or misaligned */
};

/* HGKS_MODE_SMOOTH: linear-weight WENO5 normal reconstruction, fourth-order
 *   tangential polynomials and the smooth second-order gas-kinetic flux
 *   (Remark 1 of Sec. 2.1; the Taylor-Green and channel cases).
 * HGKS_MODE_WENOZ: WENO-Z reconstruction (weights of the Z type with exponent
 *   weno_p in 1..4 and epsilon weno_eps > 0) in the normal direction and along
 *   both tangential axes, and the full flux of Eq. (flux) integrated in time, with
 *   the artificial collision time of Sec. 3 (c_art >= 0; isotropic turbulence).
 * HGKS_MODE_WENOZ_CHAR: as HGKS_MODE_WENOZ, with the WENO-Z reconstruction done
 *   on characteristic variables omega = R^{-1} Q (the Remark of Sec. 2.1 on
 *   non-smooth flows), R the right eigenvectors of the Jacobian of the
 *   face-normal Euler flux: in the normal direction at the mean of the face's two
 *   cells, in the tangential directions at the face's equilibrium state Q0 (all
 *   four Gauss points and all reconstructed fields of the face).  More robust on
 *   under-resolved shocklets (Ma_t around 1); no adjoint (HGKS_E_UNSUPPORTED from
 *   hgks_step_vjp). */
enum { HGKS_MODE_SMOOTH = 0, HGKS_MODE_WENOZ = 1, HGKS_MODE_WENOZ_CHAR = 2 };
/* HGKS_PREC_F64: all arithmetic in FP64.
 * HGKS_PREC_F32FLUX: reconstruction and flux arithmetic in FP32 around FP64
 *   anchors, FP64 state and compensated accumulation of the flux divergence. */
enum { HGKS_PREC_F64 = 0, HGKS_PREC_F32FLUX = 1 };
/* HGKS_BC_WALL_ISOTHERMAL: no-slip isothermal walls at both ends of y (the
 * channel of Sec. 3.3), closed by ghost cells mirroring the first three rows:
 * velocity reversed, equal pressure, temperature 2 T_wall - T (at least
 * T_wall / 2).  Smooth mode only (HGKS_E_UNSUPPORTED in mode Z). */
enum { HGKS_BC_PERIODIC = 0, HGKS_BC_WALL_ISOTHERMAL = 1 /* y only */ };

/* Number of doubles written by hgks_diagnostics. */
#define HGKS_NDIAG 34

typedef struct {
  int32_t nx, ny, nz;      /* cells per axis; >= 6 on every periodic axis */
  double lx, ly, lz;       /* box lengths (channel: ly = 2, y in [-1, 1]) */
  int32_t bc_y;            /* HGKS_BC_* for the y axis; x and z are periodic */
  double stretch_b;        /* 0: uniform y; > 0: tanh map y = tanh(b (eta/(1.5 pi) - 1))/tanh b,
                              eta uniform on [0, 3 pi] (Sec. 3.3; needs walls; ly unused) */
  double gamma, prandtl;   /* specific-heat ratio (> 1) and Prandtl number (> 0) */
  double mu_ref, T_ref, mu_exp; /* mu(T) = mu_ref (T/T_ref)^mu_exp (Sec. 3.4) */
  int32_t mode;            /* HGKS_MODE_* */
  double cfl;              /* dt = cfl * min_cells min_d dx_d / (|U_d| + c) */
  double c_art, weno_eps;  /* artificial collision-time constant C (Sec. 3), WENO-Z epsilon */
  int32_t weno_p;          /* WENO-Z exponent */
  double T_wall, body_force_x; /* wall temperature (> 0 with walls); constant streamwise body
                                  force f_x added after each step by the trapezoidal rule
                                  (Sec. 3.3): (rho U) += dt/2 (rho^{n+1} + rho^n) f_x,
                                  (rho E) += dt/2 ((rho U)^{n+1} + (rho U)^n) f_x */
  int32_t precision;       /* HGKS_PREC_* */
  double bulk_momentum;    /* 0: off.  > 0: constant bulk momentum (Sec. 3.3): each step's
                              force f_x, applied by the same trapezoidal rule, is the value
                              that makes the box integral of (rho U)^{n+1} equal
                              bulk_momentum |Omega|, i.e. f_x = (bulk_momentum |Omega| -
                              int (rho U)~ dOmega) / (dt/2 int (rho^n + rho~) dOmega) with ~
                              the unforced update; excludes body_force_x != 0 */
} hgks_params;

typedef struct hgks_handle hgks_handle;

/* Bytes of device workspace hgks_init needs for these parameters (0 if the
 * parameters are invalid).  The workspace must be 256-byte aligned. */
size_t hgks_workspace_bytes(const hgks_params* p);

/* Validate the parameters, bind the caller's state q (device) and workspace
 * (device, ws_bytes >= hgks_workspace_bytes(p)) and stream.  No device memory is
 * allocated.  Errors: HGKS_E_INVALID_ARG (bad parameters, NULL pointers),
 * HGKS_E_WORKSPACE, HGKS_E_UNSUPPORTED, HGKS_E_DEVICE. */
int hgks_init(const hgks_params* p, double* q, void* workspace, size_t ws_bytes, void* hip_stream,
              hgks_handle** out);

/* Advance the bound state by nsteps two-stage steps (Eq. (two-stage)).  dt > 0:
 * fixed time step; dt <= 0: each step takes dt from the CFL rule above, computed
 * on the device from the current state.  dt_taken (host, nsteps doubles) receives
 * the time steps when not NULL.  The call synchronizes the stream once at the
 * end.  On HGKS_E_NONPHYSICAL the state holds the last good step and
 * hgks_failed_step reports the index (0-based, counted over the handle's
 * lifetime) of the step that produced the bad state. */
int hgks_step(hgks_handle* h, int32_t nsteps, double dt, double* dt_taken);

/* Operator of Eq. (finite) and its time derivative at an arbitrary state:
 * L = L(q_in), dL = dL/dt(q_in), all device [5][nz][ny][nx].  dt enters only
 * mode-Z terms (artificial collision time, time integrals) and must be > 0 in
 * that mode (HGKS_E_INVALID_ARG otherwise).  Enqueued on the handle's stream,
 * no synchronization. */
int hgks_operator(hgks_handle* h, const double* q_in, double dt, double* L, double* dL);

/* Face fluxes of direction dir (0 = x, 1 = y, 2 = z) of the state q_in: F^n and
 * dF^n/dt averaged over the face (divide-by-area form: 1/4 sum over the Gauss
 * points; with a stretched y, faces having y as a tangential axis weight their
 * Gauss points by their share of the row height), global frame, face n+1/2
 * stored at the index of cell n (with walls, the bottom wall face of row -1/2 is
 * not exported).  Device [5][nz][ny][nx] each.  dt as for hgks_operator.  A parity aid; no
 * synchronization. */
int hgks_face_flux(hgks_handle* h, int32_t dir, const double* q_in, double dt, double* F, double* dF);

/* Face fluxes of the two wall faces of the channel (Sec. 3.3; isothermal walls
 * in y): the y-face fluxes F^n and dF^n/dt of the state q_in at the bottom wall
 * y = -1 (face -1/2) and the top wall y = +1 (face ny-1/2) of every (x, z)
 * column, face averages in the global frame as hgks_face_flux gives them.  F and
 * dF are device [2][5][nz][nx] (entry 0 bottom, 1 top).  With the interior faces
 * telescoping in Eq. (finite), these are the only fluxes that change the box's
 * momentum and energy besides the body force.  A parity aid; no synchronization.
 * Errors: HGKS_E_INVALID_ARG for NULL pointers, HGKS_E_UNSUPPORTED without walls. */
int hgks_wall_flux(hgks_handle* h, const double* q_in, double* F, double* dF);

/* Adjoint of one two-stage step (Eq. (two-stage)) with the time step dt frozen
 * (dt > 0): given the state q_n the step starts from and the cotangent lam_np1 of
 * the state after the step, writes lam_n = (dQ^{n+1}/dQ^n)^T lam_np1.  All three
 * are device [5][nz][ny][nx] and lam_n must not overlap q_n or lam_np1.  The
 * first stage is recomputed from q_n; the reverse sweep runs the hand-written
 * adjoint of the face-flux kernels (Gauss-point flux, tangential and normal
 * reconstruction, compatibility state) and of the stage formulas.  Device
 * atomics accumulate the cell cotangents, so repeated calls agree to rounding,
 * not bitwise.  Smooth mode: constant viscosity, FP64 or the FP32-flux form
 * (whose recomputed forward and reverse run in FP32, the cotangents and their
 * accumulation in FP64).  Mode Z (WENO-Z with its smooth nonlinear weights and
 * the full flux integrated over dt, Eq. (flux)): FP64, constant viscosity or
 * mu(T); |b0 - b2| in the Z weights and |p_l - p_r| in the collision time take
 * the derivative sign(x) with sign(0) = +1.  HGKS_E_UNSUPPORTED otherwise (mode
 * Z with the FP32-flux form, mu(T) in smooth mode, walls, stretching, body
 * force).  Enqueued on the handle's stream, no synchronization; the bound state
 * is not touched.  Uses the workspace: the smooth mode keeps its face-field
 * cotangents (10 N doubles) in the face-flux arrays, so after the call those
 * arrays hold zeros, not the step's face fluxes. */
int hgks_step_vjp(hgks_handle* h, const double* q_n, double dt, const double* lam_np1, double* lam_n);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): hgks_init + hgks_step +
 * hgks_destroy in one call, with the workspace taken from a static device array
 * of the library instead of the caller.  Arguments as for hgks_init (p, q,
 * hip_stream) and hgks_step (nsteps, dt, dt_taken); the results are those of
 * that sequence.  The array holds HGKS_STATIC_WORKSPACE_BYTES; parameters whose
 * hgks_workspace_bytes exceeds it (about 400 bytes per cell in FP64, 280 in the
 * FP32-flux form: up to ~160k cells) return HGKS_E_WORKSPACE before any device
 * work.  Each device holds its own copy of the array from the first call made
 * with that device current until the process ends; the call allocates and frees
 * no device memory.  Every call on a device shares that device's copy, which
 * keeps the last call's contents (each call resets the control block and writes
 * every other part before reading it): calls that overlap on one device, from
 * several threads or on several streams, race and must not be made.
 * Synchronizes the stream. */
#define HGKS_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int hgks_step_static(const hgks_params* p, double* q, int32_t nsteps, double dt, double* dt_taken,
                     void* hip_stream);

/* Global FP64 diagnostics of the bound state (Sec. 3.1, 3.4): out (host) receives
 * HGKS_NDIAG doubles in this order:
 *   0..4 totals sum Q_k |Omega_i|; 5 E_k; 6 enstrophy zeta; 7 eps1; 8 eps2;
 *   9 eps3; 10 rho_rms; 11 u_rms; 12 Ma_t; 13 min rho; 14 min p; 15 K;
 *   16 eps_s; 17 eps_d; 18 <p theta>; 19 mean rho; 20..22 <(d_i U_i)^2>;
 *   23..25 <(d_i U_i)^3>; 26..28 <(d_i U_i)^4>; 29 S_u; 30 F_u; 31 mean c;
 *   32 volume; 33 max over cells and axes of (|U_d| + c)/dx_d.
 * Derivatives use the sixth-order central difference of Sec. 3.1.  Reductions
 * run in a fixed order, so repeated calls give bitwise-identical results.
 * Synchronizes the stream. */
int hgks_diagnostics(hgks_handle* h, double* out);

/* Histogram of the normalized dilatation r = theta / theta_rms over the cells of
 * the bound state, the quantity whose contours Sec. 3.4 shows for the isotropic
 * cases (shocklets where r <= -3, strong expansion where r >= 2).  theta = div U
 * with U = (rho U)/rho by the sixth-order central difference of Sec. 3.1 (wall
 * ghosts within reach of a wall, as in hgks_diagnostics); theta_rms is the square
 * root of the mean of theta^2 over the cells (uniform mesh), and r = 0 everywhere
 * when theta_rms = 0.  nbins uniform bins of width (hi - lo) / nbins cover
 * [lo, hi): counts (host, nbins + 2 entries) receives in slot 0 the cells with
 * r < lo, in slot 1 + b those with b = floor((r - lo) * (nbins / (hi - lo))),
 * clamped to nbins - 1 (the rounding of values just below hi), and in slot
 * nbins + 1 those with r >= hi or r not finite.  theta_rms (host) receives
 * theta_rms.  Both evaluate r and the bin in FP64.
 * Errors: HGKS_E_INVALID_ARG for NULL pointers, nbins outside
 * [1, HGKS_PDF_MAX_BINS], lo >= hi or lo, hi or hi - lo not finite;
 * HGKS_E_UNSUPPORTED on a stretched mesh.  Uses the diagnostics' block-partial
 * workspace; enqueued on the handle's stream, which it synchronizes. */
#define HGKS_PDF_MAX_BINS 4096
int hgks_dilatation_pdf(hgks_handle* h, int32_t nbins, double lo, double hi, int64_t* counts, double* theta_rms);

/* The normalized dilatation r = theta / theta_rms (defined as for
 * hgks_dilatation_pdf) on one plane of cells, the data of the slice contours of
 * Sec. 3.4: the cells whose index along axis (0 x, 1 y, 2 z) is index.  out (host)
 * receives the plane's cells with the two remaining axes in the state's order,
 * the slower one first: [nz][ny] for axis 0, [nz][nx] for axis 1, [ny][nx] for
 * axis 2.  theta_rms (host) receives theta_rms over the whole box.  Errors:
 * HGKS_E_INVALID_ARG for NULL pointers, axis outside 0..2 or index outside the
 * axis; HGKS_E_UNSUPPORTED on a stretched mesh.  Uses the diagnostics' block
 * partials and the face-flux arrays of the workspace as scratch; enqueued on the
 * handle's stream, which it synchronizes. */
int hgks_dilatation_slice(hgks_handle* h, int32_t axis, int32_t index, double* out, double* theta_rms);

/* Plane-averaged profiles of the bound state per y row, the statistics of the
 * channel in Sec. 3.3 (mean velocity, velocity fluctuations, Reynolds stress, and
 * the total-stress balance built from them): Reynolds averages <.> over the
 * nx * nz cells of each row, with U = (rho U)/rho, p = (gamma - 1)(rho E -
 * rho |U|^2 / 2) and T = p / rho per cell, the second moments about the row
 * means (u' = U - <U>).  out (host, ny * HGKS_NPROFILE doubles, row j at
 * out + j * HGKS_NPROFILE) receives
 *   0 <rho>, 1 <U>, 2 <V>, 3 <W>, 4 <p>, 5 <T>, 6 <u'u'>, 7 <v'v'>, 8 <w'w'>,
 *   9 <u'v'>, 10 <rho U>.
 * Any mesh and boundary.  Fixed reduction order, so repeated calls are bitwise
 * identical.  Uses the face-flux arrays of the workspace as scratch (like
 * hgks_step_vjp, so they no longer hold the step's face fluxes afterwards);
 * enqueued on the handle's stream, which it synchronizes.  Errors:
 * HGKS_E_INVALID_ARG for NULL pointers, HGKS_E_DEVICE. */
#define HGKS_NPROFILE 11
int hgks_plane_profiles(hgks_handle* h, double* out);

/* Per-kernel timing.  While enabled, hgks_step brackets every kernel launch with
 * HIP events recorded on the handle's stream and accumulates the elapsed times
 * per kernel class (see HGKS_KCLASS_*); hgks_step_vjp does the same for its
 * kernels.  Enabling creates HIP events (host runtime objects, no workspace use);
 * disabling releases them.  hgks_profile_read synchronizes the stream, copies the
 * accumulated milliseconds and launch counts of the first n classes (ms and counts
 * are host arrays of n entries) and resets the accumulators. */
enum {
  HGKS_KCLASS_DT = 0,           /* time step from the CFL block maxima */
  HGKS_KCLASS_FLUX_STAGE1 = 1,  /* fused face flux of one direction, stage 1 (F and dF/dt) */
  HGKS_KCLASS_FLUX_STAGE2 = 2,  /* the same, stage 2 (dF/dt only) */
  HGKS_KCLASS_STAGE1 = 3,       /* divergence + Q*, R */
  HGKS_KCLASS_STAGE2 = 4,       /* divergence + Q^{n+1} + CFL block maxima */
  HGKS_KCLASS_OPERATOR_VJP = 5, /* adjoint of the face fluxes of one direction (hgks_step_vjp) */
  HGKS_KCLASS_COUNT = 6
};
int hgks_profile_enable(hgks_handle* h, int enable);
int hgks_profile_read(hgks_handle* h, double* ms, int64_t* counts, int n);

/* Index of the step that produced a non-physical state (-1 if none). */
int hgks_failed_step(const hgks_handle* h);

/* Release the handle (host memory only). */
void hgks_destroy(hgks_handle* h);

/* Static string for a status code. */
const char* hgks_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* HGKS_H */
