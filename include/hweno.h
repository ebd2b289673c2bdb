/*
 * libhweno -- MI355X (gfx950) implementation of the fifth-order finite volume
 * derivative-based Hermite WENO scheme with unified stencils (Chen & Zhao)
 * and its SSP-RK3 time stepping, for u_t + div F(u) = 0, u(x,0) = u0(x)
 * (Sec. 1, eq. hyperbolic-conservation-laws) on uniform 1D and 2D meshes.
 *
 * The library evolves, per cell, the average u-bar and the derivative
 * averages of every conserved component (Sec. 2.1: v-bar = mean of u_x;
 * Sec. 2.2: scaled averages v-bar = (1/dy) int u_x, w-bar = (1/dx) int u_y).
 * One handle holds one or many independent problems (same dimension, flux
 * family and configuration; any sizes, domains, boundaries and end times);
 * every RK stage of every problem of a handle is one kernel launch.
 *
 * Conventions for every call:
 *   - Returns HWENO_OK (0) or a negative HWENO_ERR_* status; never aborts.
 *     hweno_last_error() then describes the failure.
 *   - All work is ordered on the HIP stream given to hweno_create.  Calls
 *     marked "synchronising" wait for that stream before returning; the
 *     others only enqueue, and device-side failures (non-admissible states)
 *     surface at the next synchronising call.
 *   - Host pointers are plain C arrays owned by the caller; "on_device"
 *     arguments select device pointers (also owned by the caller) instead.
 *   - State arrays at the boundary are always double precision with the
 *     layout  state[((var*K + comp)*ny + j)*nx + i],  var 0 = u-bar,
 *     1 = v-bar, 2 = w-bar (2D); K = 1 (scalar), 3 (1D Euler: rho, rho*mu, E)
 *     or 4 (2D Euler: rho, rho*mu, rho*nu, E); ny = 1 in 1D.
 */
#ifndef HWENO_H
#define HWENO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hweno_handle hweno_handle; /* opaque; owns what it allocates */

enum {
    HWENO_OK = 0,
    HWENO_ERR_ARG = -1,       /* invalid argument or configuration            */
    HWENO_ERR_NONFINITE = -2, /* non-finite value, or rho <= 0 / p <= 0        */
    HWENO_ERR_HIP = -3,       /* a HIP runtime call failed                     */
    HWENO_ERR_STATE = -4,     /* call out of order (e.g. step before set_state)*/
    HWENO_ERR_OOM = -5        /* device memory or workspace too small          */
};

/* Flux families (Sec. 3: Burgers, Examples 1 and 3; Euler, Examples 2 and 4;
 * linear advection f = a u, g = b u). */
enum { HWENO_ADVECTION = 0, HWENO_BURGERS = 1, HWENO_EULER = 2 };

/* Boundary treatment per axis: periodic wrap; transmissive (every unknown
 * of the ghost cells copied from the nearest interior cell; the inflow and
 * outflow ends of Sec. 3.2's tubes); reflective, a solid wall (Euler only:
 * the ghost cells hold the mirror image of the interior, with the normal
 * momentum and the derivative means along the wall normal of the other
 * quantities negated; the blast-wave problem of Sec. 3.2). */
enum { HWENO_PERIODIC = 0, HWENO_TRANSMISSIVE = 1, HWENO_REFLECTIVE = 2 };

/* Arithmetic of the path:
 *   F64       everything in double precision;
 *   F32       state and arithmetic in single precision (time step in double);
 *   F32_ACC64 single-precision reconstruction and fluxes, cell averages kept
 *             and updated in double, flux differences taken in double;
 *   F32_KAHAN single-precision everything, cell averages kept as a
 *             compensated (hi, lo) single-precision pair. */
enum { HWENO_F64 = 0, HWENO_F32 = 1, HWENO_F32_ACC64 = 2, HWENO_F32_KAHAN = 3 };

/* Nonlinear weights w~_m = gamma_m (1 + tau^2 / D_m), w = w~ / sum w~:
 *   W_PAPER  D_m = beta_m + eps in 1D (eq. nonlinear-weights) and
 *            beta_m^2 + eps in 2D (eq. nonlinear-weights-2D), as printed;
 *   W_BETA   D_m = beta_m + eps in both dimensions (the default: the form
 *            that reproduces the paper's Tables 1 and 3);
 *   W_BETA2  D_m = beta_m^2 + eps in both dimensions;
 *   W_LINEAR w_m = gamma_m (the linear scheme; for tests). */
enum { HWENO_W_PAPER = 0, HWENO_W_BETA = 1, HWENO_W_BETA2 = 2, HWENO_W_LINEAR = 3 };

typedef struct {
    int32_t dim;          /* 1 or 2                                        */
    int32_t flux;         /* HWENO_ADVECTION / HWENO_BURGERS / HWENO_EULER */
    int32_t nx, ny;       /* cells; nx >= 4, ny >= 4 in 2D, ny = 1 in 1D    */
    double xlo, xhi, ylo, yhi; /* domain [xlo,xhi] x [ylo,yhi]             */
    int32_t bc_x, bc_y;   /* HWENO_PERIODIC / _TRANSMISSIVE / _REFLECTIVE  */
    double gas_gamma;     /* ratio of specific heats (Euler), e.g. 1.4      */
    double adv[2];        /* advection velocity (a, b)                      */
    double t_end;         /* final time used by hweno_run_to_time           */
} hweno_problem;

typedef struct {
    int32_t precision;    /* HWENO_F64 ... HWENO_F32_KAHAN                 */
    int32_t gauss_q;      /* Gauss points per edge in 2D: 2 or 3           */
    int32_t weights;      /* HWENO_W_*                                      */
    double gamma_lin[5];  /* linear weights gamma_0..gamma_M, M = 2 (1D) or
                             4 (2D); positive, summing to one (eq. rewrite,
                             eq. rewrite-2D)                                */
    double eps;           /* epsilon of the weights (1e-8 in the paper)    */
    double cfl;           /* CFL number (0.6 in the paper's tests)         */
    double dt_exponent;   /* 1: dt = cfl*dx/alpha (1D), cfl/(ax/dx+ay/dy)
                             (2D); e != 1 uses dx^e, dy^e (5/3 for the
                             accuracy runs of Sec. 3.1)                    */
    int32_t characteristic; /* Euler only: 1 = reconstruction and derivative
                             modification in the local characteristic
                             variables of each cell's own average (remark
                             closing Sec. 2.2), 0 = per conserved
                             component; scalar laws ignore it             */
    int32_t smoothness;   /* indicator beta_0 of p0: HWENO_BETA_MOMENT (the
                             paper's, eq. smoothness-indicator: squared
                             scaled derivatives at the cell centre) or
                             HWENO_BETA_CLASSICAL (the integral form it is
                             compared with, eq. smoothness-indicator-
                             typical and its 2D form)                     */
    int32_t alpha_stage;  /* 1: the Lax-Friedrichs speeds of stages 2 and 3
                             are those of their own input states U^(1),
                             U^(2) (dt still from U^n); 0: U^n's speeds in
                             all three stages (the paper's, Sec. 2.1)      */
    int32_t reserved_;    /* zero                                           */
} hweno_config;

enum { HWENO_BETA_MOMENT = 0, HWENO_BETA_CLASSICAL = 1 };

/* Fills cfg with the paper's settings for dimension dim: gamma = 1/400 per
 * linear polynomial and the rest on p0 (Sec. 3), eps = 1e-8, CFL 0.6, Q = 3,
 * W_BETA, F64, dt_exponent 1, component-wise reconstruction, the moment
 * smoothness indicator, one set of speeds per step. */
void hweno_default_config(int32_t dim, hweno_config* cfg);

/* Bytes of device memory hweno_create needs for these problems, so that a
 * caller can provide them as one workspace (e.g. a torch uint8 tensor).
 * Returns 0 on invalid arguments. */
size_t hweno_workspace_bytes(const hweno_problem* probs, int32_t nprob,
                             const hweno_config* cfg);

/* Creates a handle for nprob problems (all of the same dim and flux), each
 * an instance of u_t + div F(u) = 0 on a uniform Cartesian mesh (Sec. 1,
 * eq. hyperbolic-conservation-laws; the meshes of Sec. 2.1 and 2.2) with the
 * scheme parameters of Sec. 2 (linear weights of eq. rewrite /
 * eq. rewrite-2D, eps of the nonlinear weights, Gauss points per edge) and
 * the CFL number of Sec. 3.
 * workspace: device memory of at least hweno_workspace_bytes() bytes that the
 * handle uses for all its buffers (it stays owned by the caller and must
 * outlive the handle), or NULL to let the handle allocate its own.
 * hip_stream: the hipStream_t every call is ordered on; NULL makes the
 * handle create a private blocking stream of its own (a stream that HIP
 * graphs can be captured on), destroyed with the handle.
 * Errors: ERR_ARG (mismatched dims or flux, nx/ny out of range, gauss_q not
 * 2 or 3, linear weights not all positive or |sum - 1| > 1e-12, eps <= 0,
 * cfl <= 0), ERR_OOM, ERR_HIP. */
int hweno_create(const hweno_problem* probs, int32_t nprob, const hweno_config* cfg,
                 void* workspace, size_t ws_bytes, void* hip_stream, hweno_handle** out);

/* Uploads the state of problem prob (layout above, double) and sets its time
 * to t: the initial data u(x, 0) = u0(x) of Sec. 1 as the cell averages and
 * derivative averages the scheme evolves (Sec. 2.1: u-bar and v-bar;
 * Sec. 2.2: u-bar, v-bar, w-bar), or any later state.  The wave speeds of
 * the state are reduced afresh by the next step.  Synchronising.
 * Errors: ERR_ARG (bad prob index or NULL src). */
int hweno_set_state(hweno_handle* h, int32_t prob, const double* src,
                    int32_t src_on_device, double t);

/* Downloads the state of problem prob (layout above, double) and its time.
 * Synchronising; reports a pending ERR_NONFINITE first. */
int hweno_get_state(hweno_handle* h, int32_t prob, double* dst, int32_t dst_on_device,
                    double* t);

/* The semi-discrete operator of eq. semi-discrete-scheme (1D) or
 * eq. 2D-semi-discrete-scheme-uniform (2D), L(U) = (L^u, L^v[, L^w]), and the
 * modified state U-hat = (u-bar, v-hat[, w-hat]) of Step 3, for the current
 * state of problem prob, with the global Lax-Friedrichs speeds taken from its
 * current cell averages.  Both outputs have the state layout (double).
 * Either may be NULL.  Synchronising.  Does not change the state. */
int hweno_rhs(hweno_handle* h, int32_t prob, double* L_out, double* Uhat_out,
              int32_t on_device);

/* Lax-Friedrichs speeds (alpha_x, alpha_y) of the current cell averages of
 * problem prob: max |f'(u)| over its cells, the speed of the global
 * Lax-Friedrichs flux (Sec. 2.1, the flux of the semi-discrete scheme;
 * Sec. 2.2, separate speeds for the x- and y-fluxes); for Euler the
 * spectral radius |velocity| + sound speed of the flux Jacobian.
 * Synchronising.  Errors: ERR_NONFINITE if a cell is not admissible. */
int hweno_alpha(hweno_handle* h, int32_t prob, double* ax, double* ay);

/* One SSP-RK3 step (Sec. 2.1 Step 4, Sec. 2.2 Step 4) of every problem that
 * has not reached its t_end.  dt_in: NULL for the CFL rule (alpha from the
 * step's initial cell averages, last step clipped onto t_end), or a host
 * array of nprob time steps (a problem's step is still clipped onto t_end;
 * a value <= 0 skips the problem).  dt_out: NULL, or a host array of nprob
 * doubles receiving the steps taken (then the call synchronises).
 * Otherwise the call only enqueues. Errors: ERR_STATE before set_state.
 * The speeds of a state are reduced from its cell averages by the first
 * step after set_state; later steps use the speeds stage 3 gathered from
 * the state it wrote (the same bits as a fresh reduction). */
int hweno_step(hweno_handle* h, const double* dt_in, double* dt_out);

/* nsteps steps (Sec. 2.1 Step 4, Sec. 2.2 Step 4) with the CFL rule, each
 * as hweno_step(h, NULL, NULL) would take it (problems at their t_end do not
 * move).  Only enqueues.  In graph mode, runs of 8 steps are replayed as one
 * graph, which spares the launch gaps between graphs.  Errors: ERR_ARG for
 * nsteps < 0, ERR_STATE before set_state. */
int hweno_steps(hweno_handle* h, int32_t nsteps);

/* Advances every problem to its t_end with SSP-RK3 steps (Sec. 2.1 Step 4,
 * Sec. 2.2 Step 4) whose length follows the CFL rule of Sec. 3 (dt = CFL
 * dx / alpha in 1D, CFL / (alpha_x/dx + alpha_y/dy) in 2D, dx^e with the
 * configured exponent), the last step clipped onto t_end.  Synchronising.
 * steps_out (may be NULL) receives the number of steps of the longest run.
 * Errors: ERR_NONFINITE (names the problem and cell), ERR_STATE. */
int hweno_run_to_time(hweno_handle* h, int64_t* steps_out);

/* Waits for the handle's stream and reports a pending device-side error. */
int hweno_sync(hweno_handle* h);

/* Launch configuration of the stage kernels.  tile_rows: rows one
 * workgroup marches through in 2D (8..1024) or cells per tile in 1D (fixed
 * by the kernel, ignored); grid_blocks: workgroups of the persistent launch
 * (0 = one per tile); use_graph: capture steps as HIP graphs (1) or launch
 * eagerly (0); variant: register allocation of the 2D Euler stage kernels
 * (0: for the occupancy their face arrays comfortably allow; 1: for one
 * workgroup more per CU, with fewer registers; ignored elsewhere); source
 * (read only): where the configuration came from (HWENO_TUNED_*).  Changing
 * any of these never changes a result bit. */
typedef struct {
    int32_t tile_rows;
    int32_t grid_blocks;
    int32_t use_graph;
    int32_t variant;
    int32_t source;
    int32_t reserved;
} hweno_tuning;

enum { HWENO_TUNED_DEFAULT = 0, HWENO_TUNED_BY_CALLER = 1, HWENO_TUNED_BY_TIMING = 2,
       HWENO_TUNED_FROM_CACHE = 3 };

int hweno_get_tuning(const hweno_handle* h, hweno_tuning* t);
/* Errors: ERR_ARG for values out of range. */
int hweno_set_tuning(hweno_handle* h, const hweno_tuning* t);

/* Times candidate launch configurations (segment heights 16-64 and those
 * whose tile count just fits two or three rounds of the GPU's workgroup
 * slots, persistent grid sizes, register variants; the caller's use_graph
 * is kept) on a few steps
 * of the handle's current state, which it restores: after at least 50 ms of
 * warm-up steps, every candidate on three steps, then the four fastest and
 * the configuration in use on six steps, twice; the configuration in use is
 * kept unless another is more than 1% faster.
 * If the environment variable HWENO_TUNING_CACHE names a file, a
 * configuration stored there for the same device, dimension, flux,
 * precision, Gauss points, reconstruction and size class (problems and
 * cells to the nearest power of two) is applied without timing, and a newly
 * timed winner is appended (one JSON object per line).  Synchronising.
 * best (may be NULL) receives the configuration in use afterwards. */
int hweno_autotune(hweno_handle* h, hweno_tuning* best);
int hweno_autotune(hweno_handle* h, hweno_tuning* best);

/* The candidate launch configurations hweno_autotune times for this handle
 * (its problems, flux, precision and device), in the order it times them,
 * with the handle's use_graph.  *count receives their number; the first
 * min(count, cap) are written to out (out may be NULL when cap is 0).
 * Errors: ERR_ARG for a NULL handle or count, cap < 0, or out NULL with
 * cap > 0. */
int hweno_tuning_candidates(hweno_handle* h, hweno_tuning* out, int32_t cap, int32_t* count);

/* Per-kernel timing of nsteps steps (CFL rule), launched eagerly on the
 * handle's stream with a HIP event pair around every kernel.  Synchronising.
 * total_ms: first to last event; stage_ms: sum of the fused stage kernels;
 * alpha_ms: wave-speed reductions (none once stage 3 has gathered the
 * speeds); other_ms: dt and time-update kernels. */
typedef struct {
    double total_ms;
    double stage_ms;
    double alpha_ms;
    double other_ms;
    int64_t steps;        /* steps in which some problem advanced */
    int64_t stage_launches;
} hweno_timing;

int hweno_timed_steps(hweno_handle* h, int32_t nsteps, hweno_timing* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): one step
 * of one problem as hweno_step takes it (same kernels, same bits), on a
 * state the caller holds in device memory, with no handle.
 *   prob, cfg   as for hweno_create (one problem); the step is clipped onto
 *               prob->t_end, and none is taken when t >= t_end;
 *   state_in    device, the boundary layout above (double), read only;
 *   state_out   device, same layout; receives the new state (when no step
 *               is taken, the input as stored in the configured precision);
 *               may equal state_in;
 *   t           the state's time;
 *   dt_in       > 0: the step to take (still clipped); otherwise the CFL
 *               rule on the state's own wave speeds;
 *   dt_out      device double or NULL: the step taken, 0 if none;
 *   bad_out     device int64 or NULL: -1, or the first cell (j*nx + i) of
 *               the input that is not admissible (then no step is taken);
 *   hip_stream  the stream every launch is ordered on (NULL: null stream).
 * Every intermediate buffer (three stage states, saved hats, problem table,
 * work lists) lives in one fixed device array of HWENO_NOALLOC_SCRATCH_BYTES
 * per GPU, which each GPU the library runs on holds until the process ends;
 * its address is looked up once per device, on the first call there.  The
 * call allocates nothing and copies nothing between host and device: it only
 * enqueues kernels.  A problem needs, per cell, 3 K (su + D sd) + K D sd
 * bytes (K components, D = dim, su = 8 except 4 for F32, sd = 8 for F64 and
 * 4 otherwise) plus a few KB: e.g. at most about 190 000 cells of 2D Euler
 * in F64, 299 000 in F32_ACC64.
 * Every call on a GPU shares that GPU's array and leaves its contents behind
 * (each call rewrites what it reads first): calls that overlap on one GPU,
 * on different streams or threads, race and give undefined results.
 * Errors (hweno_last_error(NULL)): ERR_ARG as hweno_create, NULL states, or a
 * problem larger than the array; ERR_HIP. */
#define HWENO_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int hweno_step_noalloc(const hweno_problem* prob, const hweno_config* cfg,
                       const double* state_in, double* state_out, double t, double dt_in,
                       double* dt_out, int64_t* bad_out, void* hip_stream);

int hweno_destroy(hweno_handle* h);

/* Text of the last error on h, or of the last failed hweno_create on this
 * thread when h is NULL.  Never NULL. */
const char* hweno_last_error(const hweno_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* HWENO_H */
