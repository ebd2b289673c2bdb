/*
 * Plain FP64 CPU oracle for the fifth-order derivative-based finite volume
 * HWENO scheme with unified stencils (Chen & Zhao), and its SSP-RK3 time
 * stepping, in 1D and 2D.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a slow, obviously correct implementation written straight from the
 * paper.  It shares no code, header, table or helper with the GPU library and
 * must never be called on the product path.  Only the test suite, the smoke
 * check and the CPU baseline leg of the benchmark load it.
 *
 * Every routine works on double precision host arrays.  State layout (the same
 * convention as the GPU library's boundary, restated here on purpose):
 *     state[((var*K + comp)*ny + j)*nx + i]
 * var 0 = cell average u-bar, var 1 = v-bar, var 2 = w-bar (2D only).
 * 1D: v-bar is the cell mean of u_x (Sec. 2.1).  2D: v-bar = (1/dy)*integral
 * of u_x over the cell and w-bar = (1/dx)*integral of u_y (scaled averages,
 * Sec. 2.2).  K = 1 for scalar laws, 3 for 1D Euler, 4 for 2D Euler.
 */
#ifndef HWENO_ORACLE_H
#define HWENO_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_ADVECTION = 0, ORC_BURGERS = 1, ORC_EULER = 2 };
enum { ORC_PERIODIC = 0, ORC_TRANSMISSIVE = 1, ORC_REFLECTIVE = 2 };
enum { ORC_W_PAPER = 0, ORC_W_BETA = 1, ORC_W_BETA2 = 2, ORC_W_LINEAR = 3 };
enum { ORC_BETA_MOMENT = 0, ORC_BETA_CLASSICAL = 1 };

typedef struct {
    int dim;               /* 1 or 2 */
    int flux;              /* ORC_ADVECTION / ORC_BURGERS / ORC_EULER */
    int nx, ny;            /* ny must be 1 in 1D */
    double xlo, xhi, ylo, yhi;
    int bc_x, bc_y;        /* ORC_PERIODIC / ORC_TRANSMISSIVE / ORC_REFLECTIVE
                              (solid wall, Euler only: ghosts mirror the
                              interior, the normal momentum and the
                              derivative along the axis change sign) */
    double gas_gamma;      /* ideal gas ratio of specific heats (Euler) */
    double adv[2];         /* advection velocity (a, b) */
    int gauss_q;           /* Gauss points per edge in 2D: 1, 2 or 3 */
    int weights;           /* ORC_W_* */
    double gamma_lin[5];   /* linear weights gamma_0..gamma_M (M=2 in 1D, 4 in 2D) */
    double eps;            /* epsilon of the nonlinear weights */
    int charwise;          /* Euler: 1 = reconstruct and modify in local
                              characteristic variables, 0 = per component */
    int smoothness;        /* indicator of p0: ORC_BETA_MOMENT (the paper's,
                              eq. smoothness-indicator) or ORC_BETA_CLASSICAL
                              (eq. smoothness-indicator-typical, -2D) */
    int alpha_stage;       /* 1: the Lax-Friedrichs speeds of stages 2 and 3
                              come from their input states U^(1), U^(2)
                              (whole-grid stepping only); 0: all three stages
                              use those of U^n.  dt always uses U^n's. */
} orc_problem;

/* Number of conserved components K of the problem. */
int orc_ncomp(const orc_problem* p);

/* --- single-cell reconstruction, exposed for the pins ------------------- */

/* 1D: ub = (u_{i-1}, u_i, u_{i+1}); vb = (v_{i-1}, v_{i+1}) (physical means of
 * u_x).  out (length 25): c0[5] c1[2] c2[2] beta[3] omega[3] C[5]
 *   u(+1/2) u(-1/2) u_x(+1/2) u_x(-1/2) vhat.  Returns 0. */
int orc_recon_1d(const orc_problem* p, const double ub[3], const double vb[2],
                 double dx, double* out);

/* 2D: q[17] in the order of Appendix A (9 averages row by row from (i-1,j-1),
 * then v-bar of W,E,S,N face neighbours, then w-bar of W,E,S,N).
 * out (length 15+12+5+5+15+2 = 54): c0[15] lin[4][3] beta[5] omega[5] C[15]
 *   vhat what.  Basis order 1, xi, eta, xi^2, xi*eta, eta^2, xi^3, xi^2 eta,
 * xi eta^2, eta^3, xi^4, xi^3 eta, xi^2 eta^2, xi eta^3, eta^4. */
int orc_recon_2d(const orc_problem* p, const double q[17], double* out);

/* Classical smoothness indicator of a polynomial given by its monomial
 * coefficients in cell units (1D: c[5] of 1, xi, .., xi^4; 2D: c[15] in the
 * basis order above): the sum over all derivative orders >= 1 of the
 * integral over the cell of the squared derivative. */
double orc_smoothness_classical_1d(const double c[5]);
double orc_smoothness_classical_2d(const double c[15]);

/* Evaluate a 2D combined polynomial C[15] at local (xi, eta):
 * out = (U, dU/dxi, dU/deta). */
void orc_poly2d_eval(const double C[15], double xi, double eta, double out[3]);

/* Eigen-decomposition of the Euler flux Jacobian dF/dU in direction dir
 * (0 = x, 1 = y) at the state U: R (K x K, row-major, columns = right
 * eigenvectors), L = R^-1 (rows = left eigenvectors), lam = eigenvalues in
 * the order (v_n - c, v_n, [v_n,] v_n + c).  Returns -1 unless Euler. */
int orc_euler_eigen(const orc_problem* p, int dir, const double* U, double* R, double* L,
                    double* lam);

/* Reconstruction of one cell in local characteristic variables (the remark
 * closing Sec. 2.2): the stencil is projected with the left eigenvectors of
 * the cell's own average state, every characteristic field goes through the
 * scalar reconstruction, and the polynomial is mapped back with R.
 * 1D: ub[3*K] = averages of cells i-1, i, i+1 (cell-major: ub[j*K + c]),
 *     vb[2*K] = derivative means of cells i-1, i+1; out: C[K][5] then vhat[K].
 * 2D: q[17*K] = the 17 stencil values of orc_recon_2d, each a K-vector
 *     (q[s*K + c]); dir picks the x (0) or y (1) eigenvectors; out: C[K][15]
 *     then vhat[K], what[K].  Returns 0. */
int orc_recon_char_1d(const orc_problem* p, const double* ub, const double* vb, double dx,
                      double* out);
int orc_recon_char_2d(const orc_problem* p, const double* q, int dir, double* out);

/* Physical flux pieces, for the Euler pins.  dir 0 = x, 1 = y.
 * f_out = F(U) (K values); jv_out = (dF/dU) * V (K values). */
int orc_flux(const orc_problem* p, int dir, const double* U, const double* V,
             double* f_out, double* jv_out);

/* --- whole-grid operators ---------------------------------------------- */

/* Global Lax-Friedrichs speeds from the cell averages of `state` (interior
 * cells).  Returns 0, or -2 if a value is non-finite or, for Euler, a density
 * or pressure is not positive; *bad_cell then holds the flat cell index. */
int orc_alpha(const orc_problem* p, const double* state, double* ax, double* ay,
              long long* bad_cell);

/* Time step from the CFL rule: 1D cfl*dx^e/ax; 2D cfl/(ax/dx^e + ay/dy^e). */
double orc_dt(const orc_problem* p, double ax, double ay, double cfl, double dt_exponent);

/* Semi-discrete operator L(U) and the modified state U-hat = (u, vhat[, what]),
 * both in the state layout, for given Lax-Friedrichs speeds. */
int orc_rhs(const orc_problem* p, const double* state, double ax, double ay,
            double* L_out, double* Uhat_out);

/* One SSP-RK3 step with the derivative modification, in place.  Returns
 * -2 if, with alpha_stage, an intermediate stage is not admissible. */
int orc_step(const orc_problem* p, double* state, double ax, double ay, double dt);

/* Advance from t0 to t_end: per step alpha from U^n, dt from the CFL rule,
 * last step clipped so that t lands on t_end.  *steps_out = steps taken. */
int orc_run(const orc_problem* p, double* state, double t0, double t_end,
            double cfl, double dt_exponent, long long* steps_out);

/* One SSP-RK3 step (given alpha and dt) evaluated only for the cells of the
 * window [i0,i0+wi) x [j0,j0+wj) of the full-grid state (not with
 * alpha_stage, whose speeds need the whole intermediate states: -1).  The result equals
 * the window of orc_step's result; out has the state layout of the window
 * (nx -> wi, ny -> wj).  Used to check single cells of very large grids. */
int orc_step_window(const orc_problem* p, const double* state, double ax, double ay,
                    double dt, int i0, int j0, int wi, int wj, double* out);

/* L and U-hat on a window, as orc_step_window does for a step. */
int orc_rhs_window(const orc_problem* p, const double* state, double ax, double ay,
                   int i0, int j0, int wi, int wj, double* L_out, double* Uhat_out);

/* Number of threads the whole-grid loops may use (OpenMP); 0 = library default. */
void orc_set_threads(int n);
int orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
