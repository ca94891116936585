/*
 * gbr.h -- C ABI of the MI355X (gfx950) implementation of the MEG7
 * gradient-based reconstruction hot path (Chamarthi, arXiv 2305.00762):
 * the conservative residual of the 2D compressible Navier-Stokes equations
 * and the SSP Runge-Kutta stage update, on device-resident
 * structure-of-arrays state.
 *
 * Conventions shared by every call
 *   - State arrays Q, Res, Qn, Qk, Qout are device pointers to float64 SoA
 *     [4][ny][nx], x fastest: Q = (rho, rho u, rho v, E) (paper Sec. 1,
 *     eq. CNS-base).  They are owned by the caller, must not overlap unless
 *     stated, and are only accessed during the call's stream work.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All calls are asynchronous and stream ordered; argument errors are
 *     reported before anything is enqueued.
 *   - Every call returns GBR_OK (0) or a negative GBR_E* code; no exception
 *     or abort crosses the ABI.  A context is used by one host thread at a
 *     time; contexts are independent.
 *   - Device faults cannot be reported asynchronously: gbr_check()
 *     synchronises the stream and reports GBR_ESTATE if a kernel saw a
 *     non-finite value or a non-positive density or pressure.
 */
#ifndef GBR_H
#define GBR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GBR_OK = 0,
    GBR_EINVAL = -1,       /* bad argument                                   */
    GBR_ENOMEM = -2,       /* device allocation failed                       */
    GBR_EDEVICE = -3,      /* HIP runtime error                              */
    GBR_ESTATE = -4,       /* non-finite / non-positive rho or p seen        */
    GBR_EUNSUPPORTED = -5  /* option not available in the library            */
};

enum { GBR_BC_PERIODIC = 0, GBR_BC_TRANSMISSIVE = 1, GBR_BC_REFLECT = 2, GBR_BC_NOSLIP = 3,
       GBR_BC_INFLOW = 4 };
enum { GBR_RIEMANN_HLLC = 0, GBR_RIEMANN_HLLC_SS = 1 };

/* One side of the domain for gbr_set_sides.  The side is split into two
 * segments: segment 0 where the cell-centre coordinate along the side is
 * below split0 + split_speed * t (t: the context's device time), segment 1
 * elsewhere (split0 = +inf: one segment).  kind[g] is one of GBR_BC_*;
 * state[g] = (rho, u, v, p) is the fixed primitive state of a GBR_BC_INFLOW
 * segment (ignored otherwise). */
typedef struct {
    int kind[2];
    double state[2][4];
    double split0, split_speed;
} gbr_side;
enum { GBR_RECON_PRIM = 0, GBR_RECON_CONS = 1 };
enum { GBR_MP_FLAGGED = 0, GBR_MP_EVERYWHERE = 1 };
enum { GBR_PREC_FP64 = 0, GBR_PREC_FP32_BULK = 1 };
enum { GBR_DET_PLAIN = 0, GBR_DET_MLP = 1 };

typedef struct gbr_ctx gbr_ctx;

/* Human-readable text of a status code (static storage). */
const char *gbr_strerror(int status);

/* Version string of the library (static storage). */
const char *gbr_version(void);

/* Create a context for an nx x ny grid (paper Sec. 1: uniform Cartesian
 * cells, values at cell centres) with ratio of specific heats gamma
 * (eq. eqn:pressure), constant dynamic viscosity mu (mu = 0: Euler) and
 * Prandtl number Pr (eq. eqn:visc).  Requires nx, ny >= 12 (twice the
 * 6-cell stencil reach), gamma > 1, mu >= 0, Pr > 0.  Allocates only
 * context scratch on the current HIP device; the default geometry is
 * [0,1]^2, periodic, and the default scheme is primitive reconstruction,
 * MP limiting at flagged interfaces, FP64, plain detector.  *out receives
 * the context (NULL on error). */
int gbr_init(int nx, int ny, double gamma, double mu, double Pr, gbr_ctx **out);

/* Release a context and its scratch (NULL is accepted). */
int gbr_destroy(gbr_ctx *ctx);

/* Domain [x0,x1] x [y0,y1] (cell sizes dx = (x1-x0)/nx, dy = (y1-y0)/ny) and
 * boundary type per direction: GBR_BC_PERIODIC, or GBR_BC_TRANSMISSIVE
 * (ghost cells copy the nearest interior cell).  Clears any side table set
 * by gbr_set_sides. */
int gbr_set_geometry(gbr_ctx *ctx, double x0, double x1, double y0, double y1,
                     int bc_x, int bc_y);

/* Scheme options: recon = GBR_RECON_PRIM (MEG7-prim, Sec. 2.2: GRB and the
 * MP procedure on the primitive variables) or GBR_RECON_CONS (MEG7-cons,
 * Secs. 2.2-2.3 and Table 2: GRB and the MP procedure on the conservative
 * variables and their sixth-order gradients, characteristic projection with
 * the eigenvectors of the conservative flux Jacobian at the mean of the two
 * cells beside the interface, velocity gradients of the viscous flux by the
 * chain rule; FP64 with the plain detector only, on the 31x15 and 15x15
 * tilings), mp_mode = GBR_MP_FLAGGED (MP limiter in characteristic variables
 * at interfaces the detector flags, Secs. 2.3-2.4) or GBR_MP_EVERYWHERE (the
 * MEG7 states -- characteristic projection and MP test -- at every
 * interface, while smooth interfaces keep the reconstructed cell fluxes of
 * eqs. flux-full, flux-right; FP64, plain detector, seventh order, HLLC, on
 * the 31x15 and 15x15 tilings), precision = GBR_PREC_FP64
 * or GBR_PREC_FP32_BULK (gradients, reconstruction and fluxes in float32 with
 * FP64 state, stage update and flux differencing), detector = GBR_DET_PLAIN
 * (density detector, Sec. 2.4) or GBR_DET_MLP (learned detector, needs
 * gbr_mlp_set_weights).  Unsupported combinations return GBR_EUNSUPPORTED
 * and leave the scheme unchanged. */
int gbr_set_scheme(gbr_ctx *ctx, int recon, int mp_mode, int precision, int detector);

/* Boundaries by side, for the paper's wall-bounded test cases (the double
 * Mach reflection and the viscous shock tube of Sec. 3).  sides: host array
 * of four gbr_side, in the order left (x0), right (x1), bottom (y0), top
 * (y1), copied before return; NULL returns to the per-direction types of
 * gbr_set_geometry.  Kinds: GBR_BC_PERIODIC (both segments of both sides of
 * an axis, or none), GBR_BC_TRANSMISSIVE (nearest interior cell),
 * GBR_BC_REFLECT (slip wall: the six ghost layers mirror the interior about
 * the wall with the normal momentum negated), GBR_BC_NOSLIP (adiabatic
 * no-slip wall: mirrored, both momentum components negated), GBR_BC_INFLOW
 * (the fixed state in every ghost layer).  In a corner ghost cell the mirror
 * and sign rules of both sides compose; a fixed state of the x side takes
 * precedence over one of the y side.  Runge-Kutta stage k evaluates the
 * boundary at t + c_k dt, c = (0, 1, 1/2).  FP64 with the plain detector only
 * (GBR_EUNSUPPORTED otherwise); GBR_EINVAL for an unknown kind, a periodic
 * kind on only part of an axis, a non-positive or non-finite inflow state, or
 * a NaN split. */
int gbr_set_sides(gbr_ctx *ctx, const gbr_side *sides);

/* Riemann solver: GBR_RIEMANN_HLLC (default; eq. eqn:Riemann with Einfeldt
 * bounds) or GBR_RIEMANN_HLLC_SS, the shock-stable HLLC the paper uses for
 * the double Mach reflection, in its low-Mach-limited form: the two acoustic
 * wave terms of the HLLC dissipation scaled by
 * phi = sin(pi/2 min(1, Ma/0.1)), Ma = max(|u_L|/c_L, |u_R|/c_R) of the
 * normal velocities.  FP64 with the plain detector and the seventh-order GRB,
 * in either variable set, on the 31x15 and 15x15 tilings (GBR_EUNSUPPORTED
 * otherwise). */
int gbr_set_riemann(gbr_ctx *ctx, int kind);

/* The context's device time, read by boundary segments that move
 * (split_speed != 0).  gbr_set_time and gbr_get_time are synchronous;
 * gbr_advance_time enqueues t += *dt_dev on the stream (call it once per
 * step, after the third stage, with the step's device time step). */
int gbr_set_time(gbr_ctx *ctx, double t);
int gbr_get_time(gbr_ctx *ctx, double *t);
int gbr_advance_time(gbr_ctx *ctx, const double *dt_dev, void *stream);

/* GRB order: 7 (default; eq. eqn:grb and the flux reconstruction of eqs.
 * flux-full, flux-right) or 4, the fourth-order subset alpha = 4, beta = 0 of
 * eqs. (good_6tth-order_scheme_flux), (alpha-beta) with the same sixth-order
 * gradients (Sec. 2.2 remark on the fourth-order scheme; the flux
 * reconstruction of eq. (fourth) and its mirror image).  The order replaces
 * the GRB states wherever they enter (smooth branch and the value the MP
 * procedure starts from) and the flux reconstruction; detector, MP bounds,
 * HLLC and viscous flux are unchanged.  Order 4 runs in FP64 with the plain
 * detector and HLLC, in either variable set, on the 31x15 and 15x15 tilings; otherwise
 * GBR_EUNSUPPORTED (the scheme is left unchanged).  GBR_EINVAL for an order
 * other than 7 or 4. */
int gbr_set_order(gbr_ctx *ctx, int order);

/* Res = Res(Q), the semi-discrete right-hand side of eq.
 * (eqn-differencing_residual) with the flux differences of eq. (deriv).
 * Q and Res: device [4][ny][nx]; must not overlap. */
int gbr_residual(gbr_ctx *ctx, const double *Q, double *Res, void *stream);

/* One stage of the third-order TVD Runge-Kutta scheme, eq. (rk):
 *   stage 1: Qout = Qn + dt Res(Qn)                      (pass Qk == Qn)
 *   stage 2: Qout = 3/4 Qn + 1/4 Qk + 1/4 dt Res(Qk)
 *   stage 3: Qout = 1/3 Qn + 2/3 Qk + 2/3 dt Res(Qk)
 * dt_dev: device pointer to one double (e.g. written by gbr_compute_dt), read
 * on the device, so a whole step needs no host synchronisation.
 * Qout must not overlap Qn or Qk. */
int gbr_rk_stage(gbr_ctx *ctx, int stage, const double *dt_dev, const double *Qn,
                 const double *Qk, double *Qout, void *stream);

/* The time step of Sec. 2.5:
 *   dt = cfl * min( (1/alpha_v) min(dx^2/nu, dy^2/nu), min(dx/(|u|+c), dy/(|v|+c)) )
 * over all cells of Q, alpha_v = 4, nu = mu/rho, c = sqrt(gamma p/rho);
 * written to the device double *dt_dev.  cfl > 0. */
int gbr_compute_dt(gbr_ctx *ctx, const double *Q, double cfl, double *dt_dev,
                   void *stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the time
 * step of gbr_compute_dt without a context and without any allocation.  The
 * grid is nx x ny cells (1 <= nx, ny; nx ny <= GBR_NOALLOC_MAX_CELLS) of size
 * dx x dy (> 0), gamma > 1, mu >= 0, cfl > 0; Q and dt_dev as for
 * gbr_compute_dt (caller-owned device memory).  The reduction's scratch --
 * partial minima of at most 1024 first-pass workgroups and a status word,
 * 16.5 KB -- is a file-scope device array of the library, one per GPU, held
 * until the process ends; its address is looked up once per device (on the
 * first call there, or by gbr_init).  A bad state (non-finite, rho <= 0,
 * p <= 0) makes *dt_dev NaN, since there is no context to report it to; the
 * status word is cleared again by the call.  Calls that overlap on one GPU
 * (on different streams) share that scratch and race: serialise them.
 * Returns GBR_EINVAL for sizes beyond the limits. */
#define GBR_NOALLOC_MAX_CELLS (1 << 29)
int gbr_compute_dt_noalloc(int nx, int ny, double dx, double dy, double gamma, double mu,
                           const double *Q, double cfl, double *dt_dev, void *stream);

/* The same time step (Sec. 2.5) of the state the last stage-3 call wrote,
 * without another pass over it: every stage-3 call (gbr_rk_stage with
 * stage = 3) reduces, while it writes Q^(n+1), the extrema the time step
 * needs -- max(|u|+c), max(|v|+c) and min(rho) over the grid, per cell with
 * the arithmetic of gbr_compute_dt -- into context words.  Since fl(a/x) is
 * monotone in x, dt from the extrema equals gbr_compute_dt on that state bit
 * for bit, provided the state was not modified after the stage-3 call.  The
 * call reads and clears the words (a single small kernel on `stream`), so
 * each stage-3 output serves one call; it returns GBR_EINVAL when no stage-3
 * call came since the last one (or since gbr_init).  cfl > 0; dt_dev: device
 * double. */
int gbr_stage_dt(gbr_ctx *ctx, double cfl, double *dt_dev, void *stream);

/* Flag export (debugging and parity): when enabled, every residual or stage
 * call records the detector outcome sigma (1 = smooth, 0 = flagged) of each
 * interface in context buffers.  gbr_get_flags copies the last call's flags
 * to sig_x [ny][nx+1] (x-interface j+1/2 of row i at [i][j+1]) and sig_y
 * [ny+1][nx] (y-interface i+1/2 of column j at [i+1][j]); each may be a host
 * or a device pointer, or NULL. */
int gbr_export_flags(gbr_ctx *ctx, int enable);
int gbr_get_flags(gbr_ctx *ctx, uint8_t *sig_x, uint8_t *sig_y, void *stream);

/* Kernel timing.  With timing enabled, every residual or stage call records
 * three HIP events on its stream: before the learned detector's flag-map
 * kernel (detector = MLP; otherwise no kernel runs there), before the stage
 * kernel and after it.  gbr_timing_read waits for the last recorded event and
 * returns the summed durations (milliseconds) of the flag-map and stage
 * kernels and the number of calls since timing was enabled or last read,
 * then starts a new count.  Events are created by the context as needed and
 * reused; gbr_timing(ctx, 0) stops recording. */
int gbr_timing(gbr_ctx *ctx, int enable);
int gbr_timing_read(gbr_ctx *ctx, double *detector_ms, double *stage_ms, uint64_t *launches);

/* Tile shapes of the stage kernel.  gbr_tiling_count() is the number of
 * compiled shapes; gbr_set_tiling selects one (0 = default 31x15 cells per
 * workgroup); gbr_get_tiling reports the shape in use (the viscous form falls
 * back to variant 0 where a shape has no viscous build).  gbr_autotune times
 * every shape on the residual of the device state Q (reps launches each,
 * enqueued on `stream` and synchronised) and keeps the fastest; it allocates
 * and frees one scratch array of the size of Q. */
int gbr_tiling_count(void);
int gbr_set_tiling(gbr_ctx *ctx, int variant);
int gbr_get_tiling(gbr_ctx *ctx, int *variant, int *tile_x, int *tile_y);
int gbr_autotune(gbr_ctx *ctx, const double *Q, int reps, void *stream);

/* ---- Learned discontinuity detector ------------------------------------
 * A small network stands in for the density detector of Sec. 2.4 (which
 * supplies its training labels and remains the fallback for low-margin cells):
 * features per cell = four 7-point stencils (rho and p along x and along y),
 * each normalised as (s - mean) / ((max - min) + 1e-3) in float32 and rounded
 * to bfloat16 (28 values, padded to 32); MLP 28 -> 32 -> 32 -> 1 with ReLU,
 * bf16 weights, float32 accumulation on the matrix cores; output a logit,
 * chi = [logit > 0].
 *
 * Parameters (float32, host arrays): w[1952] = W1 [32 out][28 in] row-major,
 * then W2 [32][32], then w3 [32]; b[65] = b1 [32], b2 [32], b3. */
typedef struct gbr_mlp gbr_mlp;

/* Create / destroy a network object (parameters, Adam moments, scratch for
 * batches of up to 65536 cells) on the current device. */
int gbr_mlp_create(gbr_mlp **out);
int gbr_mlp_destroy(gbr_mlp *m);

/* Upload parameters (host w[1952], b[65]; resets the Adam state) / download
 * the float32 master parameters (either pointer may be NULL).  Synchronous. */
int gbr_mlp_set_params(gbr_mlp *m, const float *w, const float *b);
int gbr_mlp_get_params(gbr_mlp *m, float *w, float *b);

/* Features of every cell of the device state Q of `ctx`'s grid, for the
 * network's evaluation along x and along y (Sec. 2.4 works dimension by
 * dimension): feat = device [2][ny*nx][32] bf16 bit patterns, rows
 * [0, n) along x and [n, 2n) along y (row = cell i*nx + j); and, if chi is not
 * NULL, the directional plain labels chi = device [2][ny*nx]:
 * [psi_x < psi_c] then [psi_y < psi_c]. */
int gbr_mlp_features(gbr_ctx *ctx, const double *Q, uint16_t *feat, uint8_t *chi,
                     void *stream);

/* Logits of n feature rows (device feat [n][32] -> device logits [n]). */
int gbr_mlp_forward(gbr_mlp *m, const uint16_t *feat, int n, float *logits, void *stream);

/* Gradient of the mean binary cross-entropy over the batch cells idx[batch]
 * (device int32 indices into feat/labels; 1 <= batch <= 65536): grad = device
 * float32 [2018] = d/dw [1952], d/db [65], then the summed (not averaged)
 * loss.  Deterministic (fixed-order reduction). */
int gbr_mlp_grad(gbr_mlp *m, const uint16_t *feat, const uint8_t *labels, const int *idx,
                 int batch, float *grad, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * gradient of the batch, learning rate lr; loss (device or host float, may be
 * NULL) receives the batch's summed loss. */
int gbr_mlp_train_step(gbr_mlp *m, const uint16_t *feat, const uint8_t *labels, const int *idx,
                       int batch, float lr, float *loss, void *stream);

/* Use the network's current weights as the detector of `ctx` (copied), with
 * plain-detector fallback where |logit| < margin; select it with
 * gbr_set_scheme(..., GBR_DET_MLP).  With it selected, every residual or
 * stage call first evaluates the network once per cell of the grid into a
 * per-cell flag map owned by the context (nx*ny bytes, allocated here), which
 * the stage kernel's sigma buffers read (the network is evaluated along x
 * and along y, each flag feeding the buffer of its direction).
 * gbr_mlp_stats reports the network evaluations since the last reset (two
 * per cell and call: along x and along y) and how many of them fell back to
 * the plain detector (synchronises the device; optionally resets both
 * counts). */
int gbr_set_mlp_detector(gbr_ctx *ctx, const gbr_mlp *m, float margin, void *stream);
int gbr_mlp_stats(gbr_ctx *ctx, uint64_t *evaluated, uint64_t *fallbacks, int reset);

/* Per-step evaluation of the learned detector (a change of the method, off
 * by default): with per_step = 1 the flag map is evaluated only by residual
 * calls and stage-1 calls, i.e. on Q^n, and stages 2 and 3 reuse it, so the
 * detector sees Q^n for all three stages of a step instead of each stage's
 * input.  The caller must run the stages of a step in order on one context;
 * a stage-2 or stage-3 call with no flag map evaluated before it returns
 * GBR_EINVAL.  With per_step = 1 every stage-3 call also stores the density
 * and pressure of its output, rounded to float32, in a context buffer
 * (8*nx*ny bytes, allocated by the first call with per_step = 1;
 * GBR_ENOMEM if that fails).  Like the time-step extrema of gbr_stage_dt
 * they describe the output as that call wrote it: when gbr_stage_dt takes
 * the next step's time step from those extrema, the next flag map whose
 * input is that same output buffer reads the stored values instead of the
 * state (the values it would compute from it, so the flags are unchanged).
 * A step begun otherwise -- gbr_compute_dt, a time step of the caller's, a
 * state the caller wrote -- evaluates the flag map from the state; a caller
 * that writes the output buffer and then calls gbr_stage_dt breaks both
 * contracts alike.  GBR_EINVAL if per_step is not 0 or 1. */
int gbr_set_mlp_reuse(gbr_ctx *ctx, int per_step);

/* Copy the learned detector's per-cell flag map of the last evaluation
 * (nx*ny bytes, row-major [ny][nx]: bit 0 chi^x, bit 1 chi^y; the network's
 * sign where |logit| >= margin, else the plain label) to chi, a host or
 * device pointer; synchronises `stream`.  GBR_EINVAL if the context has no
 * flag map (gbr_set_mlp_detector was never called). */
int gbr_mlp_get_flagmap(gbr_ctx *ctx, uint8_t *chi, void *stream);

/* Self-test of the reciprocal the detector features use (the hardware
 * estimate refined by one fused Newton step in place of IEEE division; the
 * features of the learned detector take one reciprocal per stencil): compares
 * it with IEEE float32 division over every float with bit pattern in
 * [lo, hi), on the current device, and writes the number of differing results
 * to *mismatches (host pointer).  Synchronises the device.  The features use
 * it for normal x below 2^126, i.e. bit patterns [0x00800000, 0x7E800000),
 * where the answer is 0.  Returns GBR_EINVAL if mismatches is NULL or lo > hi. */
int gbr_selftest_reciprocal(uint32_t lo, uint32_t hi, uint64_t *mismatches);

/* Self-test of the division inside the time-step extrema of stage 3 (one
 * reciprocal of rho refined by two Newton steps shared by three quotients,
 * each with one fused correction -- the steps of the hardware's IEEE
 * division when its scaling step is idle): compares it with IEEE division on
 * `count` operand pairs drawn by a counter-based hash from `seed`
 * (magnitudes log-uniform over [2^-300, 2^300], random signs, every 16th
 * numerator zero, where only the sign of a zero quotient may differ) on the
 * current device, and writes the number of differing quotients to
 * *mismatches (host pointer); 0 is the expected answer.  Synchronises the
 * device.  GBR_EINVAL if mismatches is NULL. */
int gbr_selftest_division(uint64_t seed, uint64_t count, uint64_t *mismatches);

/* Synchronise `stream`, return GBR_ESTATE if any kernel since the last check
 * saw a non-finite value or rho <= 0 or p <= 0 in an interior cell, and
 * clear that record. */
int gbr_check(gbr_ctx *ctx, void *stream);

/* ------------------------------------------------------------------------
 * Batched grids: many independent grids advanced together, each stage of
 * every grid in ONE launch over the tiles of all grids (persistent or one
 * workgroup per tile, see below), with a per-grid time step (Sec. 2.5) and the
 * whole step [dt, stage 1, stage 2, stage 3] (eq. rk) replayed as a captured
 * HIP graph.  A grid of the batch runs the same tile function as the
 * single-grid calls with the same tile shape and precision (results agree to
 * rounding: the compiler may contract multiply-adds differently in the two
 * kernels).  Grids with mu > 0 take the viscous form of the tile function.
 *
 * gbr_batch_init: nprob grids; per grid p: nx[p], ny[p] (>= 12),
 * geom[4p..4p+3] = x0, x1, y0, y1, bc[2p], bc[2p+1] = boundary types in x and
 * y, gamma[p] > 1, mu[p] >= 0, Pr[p] > 0, cfl[p] > 0 (host arrays, copied);
 * precision GBR_PREC_FP64 or GBR_PREC_FP32_BULK.  Allocates the batch's
 * device tables (per grid: about 200 bytes plus 64 doubles of time-step
 * partials).  The detector is the plain one. */
typedef struct gbr_batch gbr_batch;
int gbr_batch_init(int nprob, const int *nx, const int *ny, const double *geom, const int *bc,
                   const double *gamma, const double *mu, const double *Pr, const double *cfl,
                   int precision, gbr_batch **out);
int gbr_batch_destroy(gbr_batch *b);

/* Register the grids' state arrays: three device arrays per grid (host arrays
 * X, Y, Z of nprob device pointers, each a SoA [4][ny][nx] FP64 array, all
 * distinct).  The caller owns them and keeps them alive while the batch
 * steps.  The state is read from X first; steps rotate the roles, and
 * gbr_batch_current tells which set (0 = X, 1 = Y, 2 = Z) holds the state.
 * Registering again resets that to X and drops captured graphs. */
int gbr_batch_set_arrays(gbr_batch *b, double *const *X, double *const *Y, double *const *Z);
int gbr_batch_current(gbr_batch *b, int *which);

/* One SSP-RK3 step of every grid, enqueued on `stream`.  With graphs enabled
 * (the default) and a non-NULL stream, the first step from each of the three
 * array roles is captured into a graph and later steps replay it; with a
 * NULL stream or graphs disabled the kernels are launched directly. */
int gbr_batch_step(gbr_batch *b, void *stream);
int gbr_batch_use_graph(gbr_batch *b, int enable);

/* Launch forms: 0 = 31x15 and 1 = 15x15 cells per workgroup with a
 * persistent tile loop (as many workgroups as fit on the chip at once), 2 =
 * 31x15 and 3 = 15x15 with one workgroup per tile.  gbr_batch_autotune times
 * the first stage of a step from the current state for each form (`reps`
 * launches, writing into the next array set, which a step overwrites anyway)
 * and keeps the fastest.  gbr_batch_info reports the form, its tile shape,
 * the tile count and the number of workgroups of a stage launch. */
int gbr_batch_tiling_count(void);
int gbr_batch_set_tiling(gbr_batch *b, int variant);
int gbr_batch_autotune(gbr_batch *b, int reps, void *stream);
int gbr_batch_info(gbr_batch *b, int *tiling, int *tile_x, int *tile_y, int *total_tiles,
                   int *workgroups);

/* Kernel timing of batched steps: with timing enabled, gbr_batch_step
 * launches its kernels directly (no graph) and records a HIP event pair on
 * its stream around every stage launch; gbr_batch_timing_read waits for the
 * last one and returns the summed stage-launch durations (milliseconds) and
 * the number of stage launches since timing was enabled or last read. */
int gbr_batch_timing(gbr_batch *b, int enable);
int gbr_batch_timing_read(gbr_batch *b, double *stage_ms, uint64_t *launches);

/* Per-grid time steps of the last step (host dt[nprob]; synchronises
 * `stream`), and the device status as gbr_check reports it. */
int gbr_batch_get_dt(gbr_batch *b, double *dt, void *stream);
int gbr_batch_check(gbr_batch *b, void *stream);

/* ---------------------------------------------------------------------------
 * Three dimensions: the inviscid 3D extension the paper tests with the
 * Taylor-Green vortex (Sec. 3, comparison of fourth- and seventh-order GRB).
 * The scheme is applied dimension by dimension: per direction, the rotated
 * primitives (rho, u_n, u_t1, u_t2, p) with the tangential components taken
 * cyclically (x: v, w; y: w, u; z: u, v), the same detector, GRB states, flux
 * reconstruction, characteristic MP limiting (plus an identity row for the
 * second tangential velocity) and HLLC as in 2D.  State Q: device FP64
 * [5][nz][ny][nx] = (rho, rho u, rho v, rho w, E), x fastest, caller-owned.
 * Each residual or stage call accumulates -dF/dx - dG/dy - dH/dz into
 * context scratch and the last kernel stores the residual or the stage: by
 * default three line-sweep kernels, x, y, z (gbr3_set_sweeps selects
 * another launch form).  Errors as for the 2D entry points.
 * ------------------------------------------------------------------------- */
typedef struct gbr3_ctx gbr3_ctx;

/* Context for an nx x ny x nz grid (each >= 12), ratio of specific heats
 * gamma > 1; default domain [0,1]^3, periodic, order 7.  Allocates the 5n
 * FP64 residual accumulator and the time-step scratch on the current device. */
int gbr3_init(int nx, int ny, int nz, double gamma, gbr3_ctx **out);
int gbr3_destroy(gbr3_ctx *ctx);

/* Domain and boundary type per axis (GBR_BC_PERIODIC or GBR_BC_TRANSMISSIVE). */
int gbr3_set_geometry(gbr3_ctx *ctx, double x0, double x1, double y0, double y1, double z0,
                      double z1, int bc_x, int bc_y, int bc_z);

/* GRB order 7 (default) or 4 (the subset alpha = 4, beta = 0, eq. fourth). */
int gbr3_set_order(gbr3_ctx *ctx, int order);

/* How a residual or stage call is launched (the same scheme; the residuals
 * agree to rounding, the flags exactly):
 *   GBR3_SWEEPS_LINES (default): three line-sweep kernels, x, y, z, each
 *     reading Q and the accumulator (32 positions x 8 lines per workgroup);
 *   GBR3_SWEEPS_XY_FUSED: the x and y sweeps in one kernel over
 *     15x15 tiles of each z plane (the tile staged once, the residual kept
 *     in registers), then the z line sweep;
 *   GBR3_SWEEPS_XY_FUSED_HALF: as the fused form, sweeping 8 lines of the
 *     tile at a time (less LDS per workgroup).
 * GBR_EINVAL for another value. */
enum { GBR3_SWEEPS_LINES = 0, GBR3_SWEEPS_XY_FUSED = 1, GBR3_SWEEPS_XY_FUSED_HALF = 2 };
int gbr3_set_sweeps(gbr3_ctx *ctx, int form);

/* Res = Res(Q) (eqs. eqn-differencing_residual, deriv in 3D).  Q and Res must
 * not overlap. */
int gbr3_residual(gbr3_ctx *ctx, const double *Q, double *Res, void *stream);

/* SSP-RK3 stage (eq. rk), as gbr_rk_stage. */
int gbr3_rk_stage(gbr3_ctx *ctx, int stage, const double *dt_dev, const double *Qn,
                  const double *Qk, double *Qout, void *stream);

/* dt = cfl min(dx/(|u|+c), dy/(|v|+c), dz/(|w|+c)) over the grid (Sec. 2.5,
 * inviscid), to a device scalar; deterministic. */
int gbr3_compute_dt(gbr3_ctx *ctx, const double *Q, double cfl, double *dt_dev, void *stream);

/* The same time step of the state the last stage-3 call wrote, from the
 * extrema max(|u|+c), max(|v|+c), max(|w|+c) its z sweep reduced while
 * writing it (as gbr_stage_dt in 2D): equal to gbr3_compute_dt on that state
 * bit for bit, provided the state was not modified after the stage-3 call.
 * Each stage-3 output serves one call; GBR_EINVAL when no stage-3 call came
 * since the last one (or since gbr3_init).  cfl > 0; dt_dev: device double. */
int gbr3_stage_dt(gbr3_ctx *ctx, double cfl, double *dt_dev, void *stream);

/* Interface flags of the last residual or stage (after gbr3_export_flags(ctx,
 * 1)): host arrays [nz][ny][nx+1], [nz][ny+1][nx], [nz+1][ny][nx]; any may be
 * NULL.  Synchronous. */
int gbr3_export_flags(gbr3_ctx *ctx, int enable);
int gbr3_get_flags(gbr3_ctx *ctx, uint8_t *sig_x, uint8_t *sig_y, uint8_t *sig_z,
                   void *stream);

/* Status (non-finite or non-positive rho or p seen), as gbr_check. */
int gbr3_check(gbr3_ctx *ctx, void *stream);

/* Timing of residual and stage calls: two HIP events per call on the caller's
 * stream; gbr3_timing_read returns the summed milliseconds of the three sweep
 * kernels and the number of calls, and resets. */
int gbr3_timing(gbr3_ctx *ctx, int enable);
int gbr3_timing_read(gbr3_ctx *ctx, double *sweeps_ms, uint64_t *calls);

#ifdef __cplusplus
}
#endif
#endif /* GBR_H */
