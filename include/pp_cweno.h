/*
 * pp_cweno.h - C ABI of the MI355X (gfx950) library for the positivity-
 * preserving fifth-order finite-volume compact-WENO scheme for the Euler
 * equations (Guo, Xiong & Shi, arXiv 1402.5618).
 *
 * The library advances cell averages of the conserved variables
 *   1D: U = (rho, rho u, E)            (Sec. 1, eq. (1DEuler))
 *   2D: U = (rho, rho u, rho v, E)     (dimension-by-dimension extension)
 * on a uniform grid (Sec. 2.2, h = (b - a) / N) with the per-stage spatial
 * operator L(U) of eq. (1DEulerFV-b): component-wise compact-WENO
 * reconstruction (eqs. (CWENO-FV), (weight) and their mirror), the
 * positivity-preserving limiter (Sec. 2.4, steps 1-4), the HLLC flux
 * (eqs. (HLLC), (contact-v), (star-l), (acoustic ws)), and the SSP-RK3
 * stage update of eq. (RK3).
 *
 * Conventions for every entry point:
 *  - All state/output pointers are DEVICE pointers to float64 arrays owned
 *    by the caller; the library never frees them.  Layouts:
 *      1D        [3][n]            component-major, contiguous
 *      2D        [4][ny][nx]       component-major, x fastest
 *      batched   [3][sum_i n_i]    problems back to back in config order
 *  - Calls enqueue work on the stream given in the config and return
 *    without synchronising, except pp_cweno_init, pp_cweno_status,
 *    pp_cweno_run and pp_cweno_destroy, which synchronise that stream.
 *  - Every call returns PP_OK (0) or a negative PP_E* code.  Argument
 *    errors (PP_EINVAL / PP_EUNSUPPORTED) are detected on the host before
 *    anything is launched and leave the context usable.  PP_EDEVICE means a
 *    HIP runtime error; the context must then be destroyed.
 *    pp_cweno_last_error() gives a message for the last failure.
 *  - One context per host thread / stream; calls on one context are not
 *    thread-safe.
 */
#ifndef PP_CWENO_H
#define PP_CWENO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pp_cweno_ctx pp_cweno_ctx; /* opaque, library-owned */

enum {
    PP_OK = 0,
    PP_EINVAL = -1,        /* invalid argument (checked before any launch)          */
    PP_ENOMEM = -2,        /* device or host allocation failed                      */
    PP_EDEVICE = -3,       /* HIP runtime error                                     */
    PP_ESTATE = -4,        /* a stage produced a non-finite value or left the set G */
    PP_EUNSUPPORTED = -5   /* valid but not supported by this build (e.g. size)     */
};

/* Boundary conditions (Sec. 3: periodic, Neumann/transmissive, reflective). */
enum { PP_BC_PERIODIC = 0, PP_BC_TRANSMISSIVE = 1, PP_BC_REFLECTIVE = 2 };

/* Arithmetic of the reconstruction, solves and HLLC.  PP_FP64: all double.
 * PP_MIXED: weights, rows, tridiagonal solves (plus one FP64-residual
 * refinement sweep) and HLLC in float; limiter, flux difference and stage
 * accumulation in double.  Inputs and outputs are float64 in both cases. */
enum { PP_FP64 = 0, PP_MIXED = 1 };

/* Time-step rules (readings of condition (CFL-CD) of the theorem in Sec. 2.4);
 * in every rule the last step is shortened to land on t_end:
 *  PP_DT_CFL     : dt = cfl * h / S (1D), cfl / (Sx/dx + Sy/dy) (2D), with
 *                  S = max(|u|+a) over the cell averages at the start of
 *                  each step.
 *  PP_DT_H53     : dt = cfl * h^(5/3) / S  (Example 3.1, Table 1; 1D only).
 *  PP_DT_PP      : dt = cfl * h / S (1D), cfl / (Sx/dx + Sy/dy) (2D) with S
 *                  over the cell averages AND the limited interface states
 *                  (2D Gauss-node operator: the limited node states) of the
 *                  step's input, the states the theorem's proof advances by
 *                  first-order HLLC steps.  The inputs of stages 2 and 3 are
 *                  checked against dt * S_s / h <= gl_w1 (2D: dt (Sx_s/dx +
 *                  Sy_s/dy) <= gl_w1) with the same dt; a stage that breaks it
 *                  sets status bit 2 (informative: not PP_ESTATE).  Near
 *                  vacuum the density-limited interface states keep their
 *                  pressure, so S can become huge and dt tiny.  Every
 *                  reconstruction; 2D in FP64.
 *  PP_DT_RESTART : PP_DT_CFL's dt; a step in which any stage output leaves
 *                  the admissible set (rho <= 0, p <= 0 or not finite) is
 *                  discarded and redone from U^n with half the dt, up to 60
 *                  times; the run stops with PP_ESTATE after that, or as soon
 *                  as half the dt no longer changes t in FP64 (a stall).  The
 *                  next step starts again from the averages' dt.  1D and 2D,
 *                  every reconstruction (in 2D and for the explicit and
 *                  characteristic schemes the step tried is kept in the
 *                  stage-1 buffers and copied to U when it stands). */
enum { PP_DT_CFL = 0, PP_DT_H53 = 1, PP_DT_PP = 2, PP_DT_RESTART = 3 };

/* Numerical flux at the faces.  PP_FLUX_HLLC: eq. (HLLC) with the acoustic
 * wave speeds (acoustic ws), the default and the paper's scheme.
 * PP_FLUX_LF: the Lax-Friedrichs flux the paper names as a more dissipative
 * alternative for the low-density example (Example 3.6; not defined there),
 * taken in its local form F = (f(U-) + f(U+))/2 - alpha (U+ - U-)/2 with
 * alpha = max(|u| + a) of the two interface states; evaluated in double in
 * both precisions. */
enum { PP_FLUX_HLLC = 0, PP_FLUX_LF = 1 };

/* Interface reconstruction (Secs. 2.2, 2.3 and the comparisons of Sec. 3).
 * PP_RECON_CWENO: the compact scheme on the conserved variables,
 * solution-dependent tridiagonal systems per component (the default).
 * PP_RECON_CHAR: the compact scheme along characteristic fields (Sec. 2.3,
 * eqs. (cha-1), (1DEuler-FVC)): per node the rows of each field from the
 * characteristic variables of the Roe average's left eigenvectors, a 3x3
 * block tridiagonal system in the conserved nodal values per side (the
 * paper's choice for discontinuous problems).  In 2D each line takes the
 * eigenvectors of the flux Jacobian along it: 4x4 blocks (acoustic,
 * entropy, shear and acoustic fields).  FP64, the line operator
 * (PP_FV_LINE), also for batched 1D ensembles; the block rows live in
 * device scratch allocated at init: per line of a 2D sweep (about 1.35 MB
 * per 2048-cell line) or per workgroup of a batched launch (one per CU).
 * PP_RECON_WENOJS / PP_RECON_WENOZ:
 * the classical explicit fifth-order finite-volume WENO the paper compares
 * against, with Jiang-Shu weights (eps 1e-6, a reading; the paper gives
 * none) or WENO-Z weights (weno_eps), each face value from its own five
 * averages.  The limiter, flux and stage update are shared.  The explicit
 * and characteristic schemes run in FP64 (else PP_EUNSUPPORTED at init),
 * single lines, 2D grids and batched ensembles alike. */
enum { PP_RECON_CWENO = 0, PP_RECON_WENOJS = 1, PP_RECON_WENOZ = 2, PP_RECON_CHAR = 3 };

/* 2D face fluxes.  PP_FV_LINE: one state pair per face from the line's
 * reconstruction, dimension by dimension (the default; fifth order for the
 * density wave, second order for general nonlinear 2D flows).
 * PP_FV_GAUSS: a multi-dimensional finite-volume operator (the paper leaves
 * multi-D schemes to future work, Sec. 4): each face flux is the average over
 * the face by three-point Gauss-Legendre quadrature.  The compact
 * reconstruction along each line gives face values averaged over the cell's
 * transverse extent; across the lines, the quartic through the averages of
 * five neighbouring face values gives the values at the Gauss nodes; the
 * limiter steps of Sec. 2.4 act on each cell's six node states with the
 * Gauss-weighted middle state; the numerical flux is taken per node.  Fifth
 * order on nonlinear smooth 2D data.  2D, FP64, PP_RECON_CWENO, unbatched
 * (else PP_EUNSUPPORTED at init); 8 more doubles per cell of scratch. */
enum { PP_FV_LINE = 0, PP_FV_GAUSS = 1 };

typedef struct {
    int ndim;            /* 1, or 2 (dimension-by-dimension sweeps)                    */
    int64_t nx, ny;      /* cells (ny = 1 in 1D); nx <= 4096 in 1D, nx, ny <= 2048 in 2D */
    double dx, dy;       /* uniform spacing h > 0 (dy ignored in 1D)                     */
    double gamma;        /* ratio of specific heats > 1 (1.4 for air)                   */
    int bc[4];           /* x_lo, x_hi, y_lo, y_hi: PP_BC_*; periodic on both ends of an
                            axis or on neither                                          */
    int precision;       /* PP_FP64 or PP_MIXED                                         */
    double weno_eps;     /* epsilon of the WENO-Z weights, eq. (weight): 1e-13          */
    double pp_eps_cap;   /* cap of the limiter's epsilon, step 1: 1e-13                 */
    double gl_w1;        /* Gauss-Lobatto end weight w^_1 in (0, 1/2): 1/12 (M = 4)      */
    int64_t nbatch;      /* 0: single grid.  > 0: batched 1D ensemble of nbatch lines   */
    const int64_t *lengths; /* host [nbatch] cells per problem (batched only; 3..4096)  */
    const double *dxs;      /* host [nbatch] spacing per problem (batched only)         */
    const int *bcs;         /* host [nbatch][2] boundary codes (batched; non-periodic)  */
    void *stream;        /* hipStream_t to enqueue on (NULL: the null stream)           */
    int flux;            /* PP_FLUX_HLLC (default) or PP_FLUX_LF                        */
    int recon;           /* PP_RECON_CWENO (default), _WENOJS, _WENOZ or _CHAR           */
    int batch_rule;      /* time-step rule of the batched driver, per problem:
                            PP_DT_CFL (default), PP_DT_PP or PP_DT_RESTART              */
    int fv;              /* 2D face fluxes: PP_FV_LINE (default) or PP_FV_GAUSS          */
} pp_cweno_config;

/* Fill *cfg with defaults: ndim 1, gamma 1.4, epsilons 1e-13, gl_w1 1/12, FP64,
 * HLLC, compact reconstruction, periodic, no batch, null stream.  Sizes and
 * spacings are left zero. */
void pp_cweno_config_defaults(pp_cweno_config *cfg);

/* Validate cfg, allocate device scratch, and return a context in *out
 * (caller frees it with pp_cweno_destroy).  Host arrays of the config are
 * copied.  Synchronises the stream. */
int pp_cweno_init(const pp_cweno_config *cfg, pp_cweno_ctx **out);

/* L = L(U): the limited spatial operator of eq. (1DEuler-FVCW) (2D: L_x + L_y)
 * for the state U, with the limiter's epsilon computed from U (step 1).
 * U and L are distinct device arrays in the grid layout. */
int pp_cweno_rhs(pp_cweno_ctx *ctx, const double *U, double *L);

/* One stage of eq. (RK3): Uout = a*U0 + b*(Us + dt*L(Us)) with
 * (a, b) = (0, 1), (3/4, 1/4), (1/3, 2/3) for stage = 1, 2, 3.
 * Uout must not alias U0 or Us. */
int pp_cweno_stage(pp_cweno_ctx *ctx, const double *U0, const double *Us, double *Uout,
                   int stage, double dt);

/* One SSP-RK3 step of size dt, in place on U (device). */
int pp_cweno_step(pp_cweno_ctx *ctx, double *U, double dt);

/* pp_cweno_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * one SSP-RK3 step of size dt, in place on the 1D line U ([3][nx], device),
 * for the configuration *cfg (ndim 1, no batch, compact reconstruction, FP64
 * or mixed, nx <= 4096; validated on the host as pp_cweno_init does), with
 * no context.  Results equal pp_cweno_step's for the same configuration.
 * Its stage buffers and scalars live in a fixed device array of the library
 * (192 KiB + 256 bytes per GPU, held until the process ends); the first call
 * on a device looks up that device's copy and sets the kernels' LDS limits.
 * It calls no hipMalloc / hipFree and allocates nothing.  Enqueued on
 * cfg->stream; not synchronised.  Every call on a GPU shares that GPU's
 * array, so calls that overlap on one GPU (two streams, two threads) race;
 * serialise them.  The stage checks of the status word are not reported.
 * Errors as pp_cweno_init (message via pp_cweno_last_error(NULL)); larger
 * lines give PP_EUNSUPPORTED. */
int pp_cweno_step_static(const pp_cweno_config *cfg, double *U, double dt);

/* Advance U (in place) from t = 0 until t_end or nsteps_max steps, whichever
 * comes first, with the time-step rule `rule` (PP_DT_*) and factor cfl; dt is
 * computed on the device every step.  Writes the time reached and the number
 * of steps taken to *t_out, *steps_out (host; either may be NULL).  A 1D run
 * of the compact scheme loops inside one kernel; the other runs replay a
 * captured hipGraph of 16 steps on a private stream ordered after the
 * config's stream (kernel timing on: launched directly).  Synchronises;
 * returns PP_ESTATE if a stage left the admissible set. */
int pp_cweno_run(pp_cweno_ctx *ctx, double *U, double t_end, int64_t nsteps_max, double cfl,
                 int rule, double *t_out, int64_t *steps_out);

/* Batched ensemble: one SSP-RK3 step of every problem of the packed state
 * Upacked, problem i with its own dt_dev[i] (device array); problems with
 * dt_dev[i] <= 0 are left unchanged.  Per stage, one persistent launch per
 * length class of the launch plan (a single launch under plans 0 and 3). */
int pp_cweno_batch_step(pp_cweno_ctx *ctx, double *Upacked, const double *dt_dev);

/* Batched ensemble driver: advance every problem to t_end with per-problem
 * dt = cfl * dx_i / S_i under the config's batch_rule (PP_DT_CFL: S_i from
 * problem i's averages; PP_DT_PP: from its averages and limited interface
 * states; PP_DT_RESTART: PP_DT_CFL with the step redone at half dt when a
 * stage output of that problem leaves G), nsteps_max steps at most (redone
 * steps not counted); steps_out (host [nbatch], may be NULL) receives each
 * problem's step count.  Synchronises. */
int pp_cweno_batch_run(pp_cweno_ctx *ctx, double *Upacked, double t_end, int64_t nsteps_max,
                       double cfl, int64_t *steps_out);

/* Continue the last pp_cweno_batch_run on the same context and state: every
 * problem with t < t_end and fewer than nsteps_max steps (the total over the
 * run and its continuations) resumes from its stored t and step count with
 * the dt of its current averages; with the same t_end this is exactly what
 * the uninterrupted run would do (a later t_end also works, but the steps
 * already clipped to the earlier one stay clipped).  Lets a long run advance
 * in bounded pieces.  steps_out and t_out (host
 * [nbatch], may be NULL) receive each problem's step count and time.  The
 * status of the run is kept across continuations (PP_ESTATE once any stage
 * has left the admissible set).  PP_EINVAL if no run was started on the
 * context, or after a timed pp_cweno_batch_tune (force_plan < 0: it steps a
 * copy of the state and resets the per-problem times; a forced plan does not).
 * Synchronises. */
int pp_cweno_batch_continue(pp_cweno_ctx *ctx, double *Upacked, double t_end, int64_t nsteps_max,
                            double cfl, int64_t *steps_out, double *t_out);

/* Batched ensembles: choose the launch plan used by pp_cweno_batch_step and
 * pp_cweno_batch_run.  The problems, sorted by length, are cut into length
 * classes, each processed by one persistent launch per stage with the LDS of
 * its longest problem and a kernel shape: how many lanes share one
 * tridiagonal system of eq. (CWENO-FV) (64 w for w waves per system), and so
 * how many rows each lane chases serially (n / (64 w)) and how large the
 * separator system solved by parallel cyclic reduction is.
 *   plan p % 3 = 0: one class;  1: > 2048 cells | the rest;
 *                2: > 2048 | 1025..2048 | <= 1024 cells;
 *   plan p / 3 = 0: classes of lines <= 2048 cells take one wave per system;
 *                1: two waves per system (lines > 2048 always take two).
 * force_plan in [0, 5] sets that plan without timing.  force_plan < 0 times
 * one step of every plan on a device copy of Upacked (per-problem dt from cfl
 * and the initial averages; Upacked is left unchanged) and keeps the fastest.
 * *plan_out (may be NULL) receives the plan; ms_out (host [6], may be NULL)
 * the measured ms per step of each plan (force_plan < 0 only).  The plan
 * changes results only by the rounding of the chunk partition, since the
 * problems are independent.  Synchronises; allocates a device copy of the
 * state on first use.  Not to be called while a batched run is in flight on
 * the same context. */
int pp_cweno_batch_tune(pp_cweno_ctx *ctx, const double *Upacked, double cfl, int force_plan,
                        int *plan_out, double *ms_out);

/* Steps redone with half the dt under PP_DT_RESTART since the last
 * pp_cweno_run or pp_cweno_batch_run on ctx (batched: summed over the
 * problems; a continuation adds to it) into *out (host).  Synchronises. */
int pp_cweno_restarts(pp_cweno_ctx *ctx, int64_t *out);

/* out_dev[0] = max(|u|+a) (2D: also out_dev[1] = max(|v|+a)) over the cell
 * averages of U (device pointers). */
int pp_cweno_max_speed(pp_cweno_ctx *ctx, const double *U, double *out_dev);

/* Synchronise the stream and return the sticky status: *flags (may be NULL)
 * receives bit 0 = non-finite value seen, bit 1 = rho <= 0 or p <= 0 seen in a
 * stage output, bit 2 = (PP_DT_PP only) a stage-2 or stage-3 input broke
 * condition (CFL-CD) under its step's dt.  Returns PP_ESTATE if bit 0 or 1 is
 * set; clears all bits. */
int pp_cweno_status(pp_cweno_ctx *ctx, uint32_t *flags);

/* Test hook: reconstructed interface states and face fluxes of the operator
 * for state U (FP64 or mixed, as configured): um, up [ncomp][cells] are
 * U-_{i+1/2} and U+_{i-1/2} before limiting; flux [ncomp][lines][n+1].
 * 1D only (lines = 1).  Any pointer may be NULL. */
int pp_cweno_debug_line(pp_cweno_ctx *ctx, const double *U, double *um, double *up,
                        double *flux);

/* Test hook: solve one tridiagonal system a_i x_{i-1} + b_i x_i + c_i x_{i+1}
 * = r_i, i = 0..n-1 (cyclic != 0: indices mod n; otherwise a_0 and c_{n-1}
 * are ignored), 3 <= n <= 4096, with the device's chunked chasing and
 * parallel cyclic reduction of the separators (the solver of eq. (CWENO-FV)
 * in the mixed form and on FP64 lines of more than 2048 cells; here in
 * FP64, 64 lanes for n <= 2048, 128 above).  a, b, c, r, x: device arrays
 * [n] owned by the caller (x may not alias the others).  Pivot-free, as the
 * paper's chasing method.  Enqueued on the context's stream. */
int pp_cweno_tridiag_solve_debug(pp_cweno_ctx *ctx, int64_t n, int cyclic, const double *a,
                                 const double *b, const double *c, const double *r, double *x);

/* Kernel timing for measurement: with on != 0, every later launch of the
 * line kernel (x and y lines) and of the 2D combine kernel is bracketed by
 * HIP events on the context's stream.  pp_cweno_get_timing synchronises and
 * writes out[0..5] = {x-line ms total, x-line launches, y-line ms total,
 * y-line launches, combine ms total, combine launches} since the last
 * pp_cweno_set_timing call.  At most 4096 launches per class are timed. */
int pp_cweno_set_timing(pp_cweno_ctx *ctx, int on);
int pp_cweno_get_timing(pp_cweno_ctx *ctx, double *out);

/* Message for the last error on ctx (or for init failures when ctx is NULL). */
const char *pp_cweno_last_error(const pp_cweno_ctx *ctx);

/* Release the context and its device scratch (synchronises).  NULL is a no-op. */
void pp_cweno_destroy(pp_cweno_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* PP_CWENO_H */
