/*
 * Plain FP64 CPU oracle of the derivative-based FV-HWENO scheme (Chen & Zhao).
 * TEST INFRASTRUCTURE ONLY: see hweno_oracle.h.  Written for readability and
 * checkability against the paper, not for speed: every cell is reconstructed
 * with the Appendix A coefficients, polynomials are evaluated monomial by
 * monomial, and fluxes are computed directly from their definitions.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA contraction,
 * so every result is a plain sequence of IEEE double operations).
 */
#include "hweno_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 0;
/* Loops over fewer work items than this run on one thread: the fork and
 * join of a parallel region would cost more than the loop (every result is
 * the same either way; iterations are independent). */
#define OMP_MIN_WORK 4096

void orc_set_threads(int n) { g_threads = n; }

int orc_get_threads(void) {
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_ncomp(const orc_problem* p) {
    if (p->flux != ORC_EULER) return 1;
    return p->dim == 1 ? 3 : 4;
}

static int nvars(const orc_problem* p) { return p->dim == 1 ? 2 : 3; }

/* ======================================================================
 * Physical fluxes (Sec. 2.1 derivative system; Sec. 2.2 eq. 2D-uvw;
 * Euler systems of Examples 2 and 4)
 * ====================================================================== */

/* F(U) in direction dir (0 = x, 1 = y). */
static void phys_flux(const orc_problem* p, int dir, const double* U, double* F) {
    if (p->flux == ORC_ADVECTION) {
        F[0] = p->adv[dir] * U[0];
    } else if (p->flux == ORC_BURGERS) {
        F[0] = 0.5 * U[0] * U[0];
    } else if (p->dim == 1) {
        /* 1D Euler: (rho, rho*mu, E) -> (rho*mu, rho*mu^2 + p, mu*(E+p)) */
        double g = p->gas_gamma;
        double rho = U[0], m = U[1], E = U[2];
        double u = m / rho;
        double pr = (g - 1.0) * (E - 0.5 * rho * u * u);
        F[0] = m;
        F[1] = m * u + pr;
        F[2] = u * (E + pr);
    } else {
        /* 2D Euler: (rho, rho*mu, rho*nu, E) */
        double g = p->gas_gamma;
        double rho = U[0], m = U[1], n = U[2], E = U[3];
        double u = m / rho, v = n / rho;
        double pr = (g - 1.0) * (E - 0.5 * rho * (u * u + v * v));
        if (dir == 0) {
            F[0] = m;
            F[1] = m * u + pr;
            F[2] = m * v;
            F[3] = u * (E + pr);
        } else {
            F[0] = n;
            F[1] = n * u;
            F[2] = n * v + pr;
            F[3] = v * (E + pr);
        }
    }
}

/* (dF/dU)(U) * V: the derivative fluxes h = f'(u) v (1D) and f^v, f^w, g^v, g^w
 * (2D) of the differentiated system; for systems this is the Jacobian-vector
 * product obtained with the chain rule. */
static void flux_jvp(const orc_problem* p, int dir, const double* U, const double* V,
                     double* JV) {
    if (p->flux == ORC_ADVECTION) {
        JV[0] = p->adv[dir] * V[0];
    } else if (p->flux == ORC_BURGERS) {
        JV[0] = U[0] * V[0];
    } else if (p->dim == 1) {
        double g = p->gas_gamma;
        double rho = U[0], m = U[1], E = U[2];
        double u = m / rho;
        double pr = (g - 1.0) * (E - 0.5 * rho * u * u);
        double H = (E + pr) / rho;
        double drho = V[0], dm = V[1], dE = V[2];
        double dp = (g - 1.0) * (dE - u * dm + 0.5 * u * u * drho);
        JV[0] = dm;
        JV[1] = 2.0 * u * dm - u * u * drho + dp;
        JV[2] = H * dm + u * (dE + dp) - u * H * drho;
    } else {
        double g = p->gas_gamma;
        double rho = U[0], m = U[1], n = U[2], E = U[3];
        double u = m / rho, v = n / rho;
        double pr = (g - 1.0) * (E - 0.5 * rho * (u * u + v * v));
        double H = (E + pr) / rho;
        double drho = V[0], dm = V[1], dn = V[2], dE = V[3];
        double dp = (g - 1.0) * (dE - u * dm - v * dn + 0.5 * (u * u + v * v) * drho);
        if (dir == 0) {
            JV[0] = dm;
            JV[1] = 2.0 * u * dm - u * u * drho + dp;
            JV[2] = v * dm + u * dn - u * v * drho;
            JV[3] = H * dm + u * (dE + dp) - u * H * drho;
        } else {
            JV[0] = dn;
            JV[1] = v * dm + u * dn - u * v * drho;
            JV[2] = 2.0 * v * dn - v * v * drho + dp;
            JV[3] = H * dn + v * (dE + dp) - v * H * drho;
        }
    }
}

int orc_flux(const orc_problem* p, int dir, const double* U, const double* V,
             double* f_out, double* jv_out) {
    if (f_out) phys_flux(p, dir, U, f_out);
    if (jv_out) flux_jvp(p, dir, U, V, jv_out);
    return 0;
}

/* Largest |eigenvalue| of dF/dU in direction dir at state U; returns 0 if the
 * state is admissible, -2 if not (non-finite, or rho <= 0 / p <= 0). */
static int max_speed(const orc_problem* p, int dir, const double* U, double* s) {
    int K = orc_ncomp(p);
    for (int k = 0; k < K; ++k)
        if (!isfinite(U[k])) return -2;
    if (p->flux == ORC_ADVECTION) {
        *s = fabs(p->adv[dir]);
    } else if (p->flux == ORC_BURGERS) {
        *s = fabs(U[0]);
    } else {
        double g = p->gas_gamma;
        double rho = U[0];
        double ke, vel;
        if (p->dim == 1) {
            double u = U[1] / rho;
            ke = 0.5 * rho * u * u;
            vel = u;
        } else {
            double u = U[1] / rho, v = U[2] / rho;
            ke = 0.5 * rho * (u * u + v * v);
            vel = dir == 0 ? u : v;
        }
        double pr = (g - 1.0) * (U[K - 1] - ke);
        if (!(rho > 0.0) || !(pr > 0.0)) return -2;
        *s = fabs(vel) + sqrt(g * pr / rho);
    }
    return 0;
}

/* ======================================================================
 * 1D reconstruction (Sec. 2.1, Steps 1-3; Appendix A)
 * ====================================================================== */

/* Linear weights gamma_m must be positive and sum to one (eq. rewrite). */

typedef struct {
    double c0[5], c1[2], c2[2];
    double beta[3], omega[3];
    double C[5];   /* u_i(x) = sum_l C[l] xi^l, xi = (x - x_i)/dx */
    double vhat;
} recon1d_t;

/* Nonlinear weights from the smoothness indicators (eq. nonlinear-weights for
 * 1D, eq. nonlinear-weights-2D for 2D).  M = number of linear polynomials. */
static void nonlinear_weights(const orc_problem* p, int M, const double* beta,
                              double* omega) {
    const double* gam = p->gamma_lin;
    if (p->weights == ORC_W_LINEAR) {
        for (int m = 0; m <= M; ++m) omega[m] = gam[m];
        return;
    }
    /* tau: average distance of beta_1..beta_M from beta_0 */
    double tau = 0.0;
    for (int m = 1; m <= M; ++m) tau += fabs(beta[0] - beta[m]);
    tau = tau / (double)M;
    int squared;
    if (p->weights == ORC_W_PAPER)
        squared = (p->dim == 2); /* 1D prints beta + eps, 2D prints beta^2 + eps */
    else
        squared = (p->weights == ORC_W_BETA2);
    double wt[5], sum = 0.0;
    for (int m = 0; m <= M; ++m) {
        double den = squared ? beta[m] * beta[m] + p->eps : beta[m] + p->eps;
        wt[m] = gam[m] * (1.0 + tau * tau / den);
        sum += wt[m];
    }
    for (int m = 0; m <= M; ++m) omega[m] = wt[m] / sum;
}

/* Classical smoothness indicator (eq. smoothness-indicator-typical and its 2D
 * form eq. smoothness-indicator-typical-2D), in cell units xi = (x - x_i)/dx:
 * the powers of dx cancel, leaving the sum over derivative orders of the
 * integrals of the squared derivatives over [-1/2, 1/2] (per variable).  The
 * integrals use the 4-point Gauss-Legendre rule per variable, exact for the
 * squared derivatives of a quartic (degree <= 6). */
static const double GL4_X[4] = {-0.43056815579702629, -0.16999052179242813,
                                0.16999052179242813, 0.43056815579702629};
static const double GL4_W[4] = {0.17392742256872693, 0.32607257743127307,
                                0.32607257743127307, 0.17392742256872693};

/* k (k-1) ... (k-m+1): the factor that the m-th derivative puts on xi^k */
static double falling(int k, int m) {
    double r = 1.0;
    for (int i = 0; i < m; ++i) r *= (double)(k - i);
    return r;
}

double orc_smoothness_classical_1d(const double c[5]) {
    double b = 0.0;
    for (int l = 1; l <= 4; ++l)
        for (int q = 0; q < 4; ++q) {
            double d = 0.0;
            for (int k = l; k <= 4; ++k) d += c[k] * falling(k, l) * pow(GL4_X[q], k - l);
            b += GL4_W[q] * d * d;
        }
    return b;
}

static void recon_1d(const orc_problem* p, const double ub[3], double vm, double vp,
                     double dx, recon1d_t* r) {
    /* Appendix A: p0 matches the three cell averages and the derivative means
     * of the two neighbours (the target cell's own derivative is left out). */
    double dvm = dx * vm, dvp = dx * vp;
    double um = ub[0], u0 = ub[1], up = ub[2];
    r->c0[0] = -47.0 / 480.0 * um + 287.0 / 240.0 * u0 - 47.0 / 480.0 * up
               - 9.0 / 320.0 * dvm + 9.0 / 320.0 * dvp;
    r->c0[1] = -13.0 / 16.0 * um + 13.0 / 16.0 * up - 5.0 / 16.0 * dvm - 5.0 / 16.0 * dvp;
    r->c0[2] = 5.0 / 4.0 * um - 5.0 / 2.0 * u0 + 5.0 / 4.0 * up + 3.0 / 8.0 * dvm
               - 3.0 / 8.0 * dvp;
    r->c0[3] = 1.0 / 4.0 * um - 1.0 / 4.0 * up + 1.0 / 4.0 * dvm + 1.0 / 4.0 * dvp;
    r->c0[4] = -1.0 / 2.0 * um + u0 - 1.0 / 2.0 * up - 1.0 / 4.0 * dvm + 1.0 / 4.0 * dvp;
    r->c1[0] = u0;
    r->c1[1] = u0 - um;
    r->c2[0] = u0;
    r->c2[1] = up - u0;

    /* Step 2: beta = sum_{l>=1} (l! c_l)^2, the squared scaled derivatives at
     * the cell centre. */
    static const double fact[5] = {1.0, 1.0, 2.0, 6.0, 24.0};
    double b0 = 0.0;
    for (int l = 1; l <= 4; ++l) b0 += (fact[l] * r->c0[l]) * (fact[l] * r->c0[l]);
    r->beta[0] = p->smoothness == ORC_BETA_CLASSICAL ? orc_smoothness_classical_1d(r->c0) : b0;
    r->beta[1] = r->c1[1] * r->c1[1];
    r->beta[2] = r->c2[1] * r->c2[1];

    /* Step 3: nonlinear weights and the HWENO polynomial
     *   u_i = w0 (p0/g0 - sum_m g_m/g0 p_m) + sum_m w_m p_m. */
    nonlinear_weights(p, 2, r->beta, r->omega);
    const double* g = p->gamma_lin;
    const double* w = r->omega;
    for (int l = 0; l < 5; ++l) {
        double pm1 = l < 2 ? r->c1[l] : 0.0;
        double pm2 = l < 2 ? r->c2[l] : 0.0;
        r->C[l] = w[0] * (r->c0[l] / g[0] - g[1] / g[0] * pm1 - g[2] / g[0] * pm2)
                  + w[1] * pm1 + w[2] * pm2;
    }
    /* modified derivative: (u_i(x_{i+1/2}) - u_i(x_{i-1/2})) / dx */
    double up_ = 0.0, um_ = 0.0;
    for (int l = 0; l < 5; ++l) {
        up_ += r->C[l] * pow(0.5, l);
        um_ += r->C[l] * pow(-0.5, l);
    }
    r->vhat = (up_ - um_) / dx;
}

/* value and x-derivative of sum_l C[l] xi^l at xi */
static void poly1d_eval(const double C[5], double xi, double dx, double* u, double* ux) {
    double a = 0.0, b = 0.0;
    for (int l = 0; l < 5; ++l) a += C[l] * pow(xi, l);
    for (int l = 1; l < 5; ++l) b += (double)l * C[l] * pow(xi, l - 1);
    *u = a;
    *ux = b / dx;
}

int orc_recon_1d(const orc_problem* p, const double ub[3], const double vb[2], double dx,
                 double* out) {
    recon1d_t r;
    recon_1d(p, ub, vb[0], vb[1], dx, &r);
    int k = 0;
    for (int l = 0; l < 5; ++l) out[k++] = r.c0[l];
    for (int l = 0; l < 2; ++l) out[k++] = r.c1[l];
    for (int l = 0; l < 2; ++l) out[k++] = r.c2[l];
    for (int l = 0; l < 3; ++l) out[k++] = r.beta[l];
    for (int l = 0; l < 3; ++l) out[k++] = r.omega[l];
    for (int l = 0; l < 5; ++l) out[k++] = r.C[l];
    double u, ux;
    poly1d_eval(r.C, 0.5, dx, &u, &ux);
    out[k++] = u;
    double u2, ux2;
    poly1d_eval(r.C, -0.5, dx, &u2, &ux2);
    out[k++] = u2;
    out[k++] = ux;
    out[k++] = ux2;
    out[k++] = r.vhat;
    return 0;
}

/* ======================================================================
 * 2D reconstruction (Sec. 2.2, Steps 1-3; Appendix A)
 * ====================================================================== */

/* exponents (m, n) of the basis monomial xi^m eta^n, in the order in which
 * Appendix A lists the coefficients c_{0,1..15} */
static const int MEXP[15] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0, 4, 3, 2, 1, 0};
static const int NEXP[15] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4};

double orc_smoothness_classical_2d(const double c[15]) {
    double b = 0.0;
    for (int m = 0; m <= 4; ++m)
        for (int n = 0; m + n <= 4; ++n) {
            if (m + n == 0) continue;
            for (int q = 0; q < 4; ++q)
                for (int s = 0; s < 4; ++s) {
                    double d = 0.0;
                    for (int k = 0; k < 15; ++k) {
                        if (MEXP[k] < m || NEXP[k] < n) continue;
                        d += c[k] * falling(MEXP[k], m) * falling(NEXP[k], n) *
                             pow(GL4_X[q], MEXP[k] - m) * pow(GL4_X[s], NEXP[k] - n);
                    }
                    b += GL4_W[q] * GL4_W[s] * d * d;
                }
        }
    return b;
}

typedef struct {
    double c0[15];
    double lin[4][3]; /* p_1..p_4: constant, xi, eta coefficients */
    double beta[5], omega[5];
    double C[15];
    double vhat, what;
} recon2d_t;

static void coeffs_2d(const double* qq, double c0[15], double lin[4][3]) {
    /* q_1..q_17 of Appendix A (1-based, as printed) */
    const double* q = qq - 1;
    c0[0] = (5 * q[1] - 292 * q[2] + 5 * q[3] - 292 * q[4] + 4028 * q[5] - 292 * q[6]
             + 5 * q[7] - 292 * q[8] + 5 * q[9] - 81 * q[10] + 81 * q[11] - 81 * q[16]
             + 81 * q[17]) / 2880.0;
    c0[1] = (2 * q[1] - 2 * q[3] - 19 * q[4] + 19 * q[6] + 2 * q[7] - 2 * q[9] - 6 * q[10]
             - 6 * q[11] + 3 * q[12] + 3 * q[13]) / 24.0;
    c0[2] = (2 * q[1] - 19 * q[2] + 2 * q[3] - 2 * q[7] + 19 * q[8] - 2 * q[9] + 3 * q[14]
             + 3 * q[15] - 6 * q[16] - 6 * q[17]) / 24.0;
    c0[3] = (-q[1] + 2 * q[2] - q[3] + 62 * q[4] - 124 * q[5] + 62 * q[6] - q[7] + 2 * q[8]
             - q[9] + 18 * q[10] - 18 * q[11]) / 48.0;
    c0[4] = (-3 * q[1] + 3 * q[3] + 3 * q[7] - 3 * q[9] - 5 * q[12] + 5 * q[13] - 5 * q[14]
             + 5 * q[15]) / 8.0;
    c0[5] = (-q[1] + 62 * q[2] - q[3] + 2 * q[4] - 124 * q[5] + 2 * q[6] - q[7] + 62 * q[8]
             - q[9] + 18 * q[16] - 18 * q[17]) / 48.0;
    c0[6] = (-q[1] + q[3] + 4 * q[4] - 4 * q[6] - q[7] + q[9] + 4 * q[10] + 4 * q[11]
             - 2 * q[12] - 2 * q[13]) / 20.0;
    c0[7] = (-q[1] + 2 * q[2] - q[3] + q[7] - 2 * q[8] + q[9]) / 4.0;
    c0[8] = (-q[1] + q[3] + 2 * q[4] - 2 * q[6] - q[7] + q[9]) / 4.0;
    c0[9] = (-q[1] + 4 * q[2] - q[3] + q[7] - 4 * q[8] + q[9] - 2 * q[14] - 2 * q[15]
             + 4 * q[16] + 4 * q[17]) / 20.0;
    c0[10] = (-2 * q[4] + 4 * q[5] - 2 * q[6] - q[10] + q[11]) / 4.0;
    c0[11] = (q[1] - q[3] - q[7] + q[9] + 2 * q[12] - 2 * q[13]) / 4.0;
    c0[12] = (q[1] - 2 * q[2] + q[3] - 2 * q[4] + 4 * q[5] - 2 * q[6] + q[7] - 2 * q[8]
              + q[9]) / 4.0;
    c0[13] = (q[1] - q[3] - q[7] + q[9] + 2 * q[14] - 2 * q[15]) / 4.0;
    c0[14] = (-2 * q[2] + 4 * q[5] - 2 * q[8] - q[16] + q[17]) / 4.0;

    double uc = q[5];
    /* p_1 on {ij, i-1 j, i j-1}, p_2 on {ij, i+1 j, i j-1},
     * p_3 on {ij, i+1 j, i j+1}, p_4 on {ij, i-1 j, i j+1} */
    lin[0][0] = uc; lin[0][1] = uc - q[4]; lin[0][2] = uc - q[2];
    lin[1][0] = uc; lin[1][1] = q[6] - uc; lin[1][2] = uc - q[2];
    lin[2][0] = uc; lin[2][1] = q[6] - uc; lin[2][2] = q[8] - uc;
    lin[3][0] = uc; lin[3][1] = uc - q[4]; lin[3][2] = q[8] - uc;
}

/* integral of t^k over [-1/2, 1/2] */
static double mono_int(int k) {
    return (pow(0.5, k + 1) - pow(-0.5, k + 1)) / (double)(k + 1);
}

static void recon_2d(const orc_problem* p, const double* q, recon2d_t* r) {
    coeffs_2d(q, r->c0, r->lin);

    /* Step 2: beta = sum over monomials of degree >= 1 of (m! n! c_mn)^2 */
    static const double fact[5] = {1.0, 1.0, 2.0, 6.0, 24.0};
    double b0 = 0.0;
    for (int l = 1; l < 15; ++l) {
        double s = fact[MEXP[l]] * fact[NEXP[l]] * r->c0[l];
        b0 += s * s;
    }
    r->beta[0] = p->smoothness == ORC_BETA_CLASSICAL ? orc_smoothness_classical_2d(r->c0) : b0;
    for (int m = 0; m < 4; ++m)
        r->beta[m + 1] = r->lin[m][1] * r->lin[m][1] + r->lin[m][2] * r->lin[m][2];

    /* Step 3: nonlinear weights and the combined polynomial */
    nonlinear_weights(p, 4, r->beta, r->omega);
    const double* g = p->gamma_lin;
    const double* w = r->omega;
    for (int l = 0; l < 15; ++l) {
        double inner = r->c0[l] / g[0];
        double outer = 0.0;
        for (int m = 0; m < 4; ++m) {
            double cml = l < 3 ? r->lin[m][l] : 0.0;
            inner -= g[m + 1] / g[0] * cml;
            outer += w[m + 1] * cml;
        }
        r->C[l] = w[0] * inner + outer;
    }

    /* modified derivatives: cell integrals of the partial derivatives of the
     * HWENO polynomial, in the scaled units of v-bar and w-bar:
     *   vhat = (1/dy) int u_x dOmega = int_{unit square} dU/dxi,
     *   what = (1/dx) int u_y dOmega = int_{unit square} dU/deta. */
    double vh = 0.0, wh = 0.0;
    for (int l = 0; l < 15; ++l) {
        int m = MEXP[l], n = NEXP[l];
        if (m > 0) vh += r->C[l] * (double)m * mono_int(m - 1) * mono_int(n);
        if (n > 0) wh += r->C[l] * (double)n * mono_int(m) * mono_int(n - 1);
    }
    r->vhat = vh;
    r->what = wh;
}

void orc_poly2d_eval(const double C[15], double xi, double eta, double out[3]) {
    double u = 0.0, ux = 0.0, uy = 0.0;
    for (int l = 0; l < 15; ++l) {
        int m = MEXP[l], n = NEXP[l];
        u += C[l] * pow(xi, m) * pow(eta, n);
        if (m > 0) ux += C[l] * (double)m * pow(xi, m - 1) * pow(eta, n);
        if (n > 0) uy += C[l] * (double)n * pow(xi, m) * pow(eta, n - 1);
    }
    out[0] = u;
    out[1] = ux;
    out[2] = uy;
}

int orc_recon_2d(const orc_problem* p, const double q[17], double* out) {
    recon2d_t r;
    recon_2d(p, q, &r);
    int k = 0;
    for (int l = 0; l < 15; ++l) out[k++] = r.c0[l];
    for (int m = 0; m < 4; ++m)
        for (int l = 0; l < 3; ++l) out[k++] = r.lin[m][l];
    for (int m = 0; m < 5; ++m) out[k++] = r.beta[m];
    for (int m = 0; m < 5; ++m) out[k++] = r.omega[m];
    for (int l = 0; l < 15; ++l) out[k++] = r.C[l];
    out[k++] = r.vhat;
    out[k++] = r.what;
    return 0;
}

/* ======================================================================
 * Local characteristic variables for the Euler equations (the remark that
 * closes Sec. 2.2: for systems, reconstruction and modification run in the
 * local characteristic directions)
 * ====================================================================== */

int orc_euler_eigen(const orc_problem* p, int dir, const double* U, double* R, double* L,
                    double* lam) {
    if (p->flux != ORC_EULER) return -1;
    double g = p->gas_gamma;
    int K = orc_ncomp(p);
    double rho = U[0];
    /* normal and tangential velocity; in 2D the normal momentum is component
     * 1 + dir and the tangential one 2 - dir */
    int in = 1, it = 2;
    if (K == 4 && dir == 1) { in = 2; it = 1; }
    double vn = U[in] / rho;
    double vt = K == 4 ? U[it] / rho : 0.0;
    double q2 = vn * vn + vt * vt;
    double pr = (g - 1.0) * (U[K - 1] - 0.5 * rho * q2);
    double c = sqrt(g * pr / rho);
    double H = (U[K - 1] + pr) / rho;
    double b1 = (g - 1.0) / (c * c);
    double b2 = 0.5 * b1 * q2;
    for (int k = 0; k < K * K; ++k) R[k] = L[k] = 0.0;
    if (K == 3) {
        /* columns: v - c, v, v + c */
        double r[3][3] = {{1.0, 1.0, 1.0}, {vn - c, vn, vn + c}, {H - vn * c, 0.5 * q2, H + vn * c}};
        double l[3][3] = {{0.5 * (b2 + vn / c), -0.5 * (b1 * vn + 1.0 / c), 0.5 * b1},
                          {1.0 - b2, b1 * vn, -b1},
                          {0.5 * (b2 - vn / c), -0.5 * (b1 * vn - 1.0 / c), 0.5 * b1}};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                R[a * 3 + b] = r[a][b];
                L[a * 3 + b] = l[a][b];
            }
        lam[0] = vn - c; lam[1] = vn; lam[2] = vn + c;
        return 0;
    }
    /* 2D, in the component order (rho, normal momentum, tangential momentum,
     * E); columns: v_n - c, entropy v_n, shear v_n, v_n + c */
    double r[4][4] = {{1.0, 1.0, 0.0, 1.0},
                      {vn - c, vn, 0.0, vn + c},
                      {vt, vt, 1.0, vt},
                      {H - vn * c, 0.5 * q2, vt, H + vn * c}};
    double l[4][4] = {{0.5 * (b2 + vn / c), -0.5 * (b1 * vn + 1.0 / c), -0.5 * b1 * vt, 0.5 * b1},
                      {1.0 - b2, b1 * vn, b1 * vt, -b1},
                      {-vt, 0.0, 1.0, 0.0},
                      {0.5 * (b2 - vn / c), -0.5 * (b1 * vn - 1.0 / c), -0.5 * b1 * vt, 0.5 * b1}};
    /* (rho, normal, tangential, E) -> storage component index */
    int map[4] = {0, in, it, 3};
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            R[map[a] * 4 + b] = r[a][b];   /* rows of R are components */
            L[a * 4 + map[b]] = l[a][b];   /* columns of L are components */
        }
    lam[0] = vn - c; lam[1] = vn; lam[2] = vn; lam[3] = vn + c;
    return 0;
}

static double dotk(const double* a, const double* b, int K) {
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += a[k] * b[k];
    return s;
}

/* 1D cell in characteristic variables: C[c][l] physical coefficients and
 * vh[c] the physical modified derivative.  Scalar laws: per component. */
static void char_recon_1d(const orc_problem* p, const double* ub, const double* vb, double dx,
                          double C[4][5], double vh[4]) {
    int K = orc_ncomp(p);
    if (p->flux != ORC_EULER || !p->charwise) {
        for (int c = 0; c < K; ++c) {
            double s[3] = {ub[c], ub[K + c], ub[2 * K + c]};
            recon1d_t r;
            recon_1d(p, s, vb[c], vb[K + c], dx, &r);
            memcpy(C[c], r.C, sizeof(r.C));
            vh[c] = r.vhat;
        }
        return;
    }
    double R[16], L[16], lam[4];
    orc_euler_eigen(p, 0, ub + K, R, L, lam);   /* the cell's own average */
    double Cw[4][5], vw[4];
    for (int k = 0; k < K; ++k) {
        const double* lk = L + k * K;
        double s[3] = {dotk(lk, ub, K), dotk(lk, ub + K, K), dotk(lk, ub + 2 * K, K)};
        recon1d_t r;
        recon_1d(p, s, dotk(lk, vb, K), dotk(lk, vb + K, K), dx, &r);
        memcpy(Cw[k], r.C, sizeof(r.C));
        vw[k] = r.vhat;
    }
    for (int c = 0; c < K; ++c) {
        for (int l = 0; l < 5; ++l) {
            double a = 0.0;
            for (int k = 0; k < K; ++k) a += R[c * K + k] * Cw[k][l];
            C[c][l] = a;
        }
        double a = 0.0;
        for (int k = 0; k < K; ++k) a += R[c * K + k] * vw[k];
        vh[c] = a;
    }
}

int orc_recon_char_1d(const orc_problem* p, const double* ub, const double* vb, double dx,
                      double* out) {
    int K = orc_ncomp(p);
    double C[4][5], vh[4];
    char_recon_1d(p, ub, vb, dx, C, vh);
    for (int c = 0; c < K; ++c)
        for (int l = 0; l < 5; ++l) out[c * 5 + l] = C[c][l];
    for (int c = 0; c < K; ++c) out[5 * K + c] = vh[c];
    return 0;
}

/* 2D cell in the characteristic variables of direction dir (scalar laws and
 * charwise = 0: per component, dir ignored).  q[s*K + c]. */
static void char_recon_2d(const orc_problem* p, const double* q, int dir, double C[4][15],
                          double vh[4], double wh[4]) {
    int K = orc_ncomp(p);
    int ch = p->flux == ORC_EULER && p->charwise;
    double R[16], L[16], lam[4];
    if (ch) orc_euler_eigen(p, dir, q + 4 * K, R, L, lam);   /* stencil entry 5: the cell */
    double Cw[4][15], vw[4], ww[4];
    for (int k = 0; k < K; ++k) {
        double s[17];
        for (int e = 0; e < 17; ++e) s[e] = ch ? dotk(L + k * K, q + e * K, K) : q[e * K + k];
        recon2d_t r;
        recon_2d(p, s, &r);
        memcpy(Cw[k], r.C, sizeof(r.C));
        vw[k] = r.vhat;
        ww[k] = r.what;
    }
    for (int c = 0; c < K; ++c) {
        if (!ch) {
            memcpy(C[c], Cw[c], sizeof(Cw[c]));
            vh[c] = vw[c];
            wh[c] = ww[c];
            continue;
        }
        for (int l = 0; l < 15; ++l) {
            double a = 0.0;
            for (int k = 0; k < K; ++k) a += R[c * K + k] * Cw[k][l];
            C[c][l] = a;
        }
        double a = 0.0, b = 0.0;
        for (int k = 0; k < K; ++k) {
            a += R[c * K + k] * vw[k];
            b += R[c * K + k] * ww[k];
        }
        vh[c] = a;
        wh[c] = b;
    }
}

int orc_recon_char_2d(const orc_problem* p, const double* q, int dir, double* out) {
    int K = orc_ncomp(p);
    double C[4][15], vh[4], wh[4];
    char_recon_2d(p, q, dir, C, vh, wh);
    for (int c = 0; c < K; ++c)
        for (int l = 0; l < 15; ++l) out[c * 15 + l] = C[c][l];
    for (int c = 0; c < K; ++c) {
        out[15 * K + c] = vh[c];
        out[16 * K + c] = wh[c];
    }
    return 0;
}


/* Gauss-Legendre nodes on [-1/2, 1/2] with weights summing to one */
static int gauss_rule(int Q, double* node, double* wt) {
    if (Q == 1) {
        node[0] = 0.0; wt[0] = 1.0;
    } else if (Q == 2) {
        double a = 0.5 / sqrt(3.0);
        node[0] = -a; node[1] = a;
        wt[0] = 0.5; wt[1] = 0.5;
    } else if (Q == 3) {
        double a = 0.5 * sqrt(0.6);
        node[0] = -a; node[1] = 0.0; node[2] = a;
        wt[0] = 5.0 / 18.0; wt[1] = 8.0 / 18.0; wt[2] = 5.0 / 18.0;
    } else {
        return -1;
    }
    return 0;
}

/* ======================================================================
 * Extended grids with ghost margins and the boundary index maps
 * ====================================================================== */

typedef struct {
    int K, nv;
    int nxe, nye; /* extended sizes */
    double* a;    /* plane (var*K + comp), row-major nye x nxe */
} ext_t;

static double* ext_at(ext_t* e, int var, int comp) {
    return e->a + (size_t)(var * e->K + comp) * e->nxe * e->nye;
}

static int ext_alloc(ext_t* e, int K, int nv, int nxe, int nye) {
    e->K = K;
    e->nv = nv;
    e->nxe = nxe;
    e->nye = nye;
    e->a = (double*)calloc((size_t)nv * K * nxe * nye, sizeof(double));
    return e->a ? 0 : -1;
}

static void ext_free(ext_t* e) { free(e->a); e->a = NULL; }

/* ghost index maps: periodic wraps, transmissive copies the nearest interior
 * cell (all unknowns, the averages and the derivative averages alike) */
static int bc_map(int i, int n, int bc) {
    if (bc == ORC_PERIODIC) {
        int r = i % n;
        return r < 0 ? r + n : r;
    }
    if (bc == ORC_REFLECTIVE) {
        /* mirror images across both walls: period 2n, folded */
        int r = i % (2 * n);
        if (r < 0) r += 2 * n;
        return r < n ? r : 2 * n - 1 - r;
    }
    if (i < 0) return 0;
    if (i >= n) return n - 1;
    return i;
}

/* Sign with which the unknown (var v, component c) of a cell is taken into
 * the ghost position i of an axis (0 = x, 1 = y).  Across a solid wall the
 * mirror image of the flow has the normal velocity reversed: the normal
 * momentum is odd and every other conserved quantity even, and the mean of
 * the derivative along the axis (v-bar for x, w-bar for y) has the opposite
 * parity of its quantity.  An odd number of reflections applies the sign. */
static double bc_sign(const orc_problem* p, int axis, int i, int n, int v, int c) {
    int bc = axis == 0 ? p->bc_x : p->bc_y;
    if (bc != ORC_REFLECTIVE) return 1.0;
    int r = i % (2 * n);
    if (r < 0) r += 2 * n;
    if (r < n) return 1.0;
    double s = (p->flux == ORC_EULER && c == 1 + axis) ? -1.0 : 1.0;
    return v == 1 + axis ? -s : s;
}

/* fill ext (margins gx, gy) from the full-grid state: window origin (i0, j0) */
static void fill_from_state(const orc_problem* p, const double* st, ext_t* e, int i0,
                            int j0, int gx, int gy) {
    int nx = p->nx, ny = p->ny;
    for (int v = 0; v < e->nv; ++v)
        for (int c = 0; c < e->K; ++c) {
            double* dst = ext_at(e, v, c);
            const double* src = st + (size_t)(v * e->K + c) * nx * ny;
            for (int jj = 0; jj < e->nye; ++jj) {
                int j = p->dim == 1 ? 0 : bc_map(j0 + jj - gy, ny, p->bc_y);
                double sy = p->dim == 1 ? 1.0 : bc_sign(p, 1, j0 + jj - gy, ny, v, c);
                for (int ii = 0; ii < e->nxe; ++ii) {
                    int i = bc_map(i0 + ii - gx, nx, p->bc_x);
                    double sx = bc_sign(p, 0, i0 + ii - gx, nx, v, c);
                    dst[(size_t)jj * e->nxe + ii] = sx * sy * src[(size_t)j * nx + i];
                }
            }
        }
}

/* ghost fill of a margin-(gx,gy) extended copy of the whole grid from its own
 * interior */
static void ghost_fill(const orc_problem* p, ext_t* e, int gx, int gy) {
    int nx = p->nx, ny = p->ny;
    for (int v = 0; v < e->nv; ++v)
        for (int c = 0; c < e->K; ++c) {
            double* a = ext_at(e, v, c);
            for (int jj = 0; jj < e->nye; ++jj) {
                int j = p->dim == 1 ? 0 : bc_map(jj - gy, ny, p->bc_y);
                double sy = p->dim == 1 ? 1.0 : bc_sign(p, 1, jj - gy, ny, v, c);
                for (int ii = 0; ii < e->nxe; ++ii) {
                    int i = bc_map(ii - gx, nx, p->bc_x);
                    int inside = (ii - gx == i) && (p->dim == 1 || jj - gy == j);
                    if (!inside)
                        a[(size_t)jj * e->nxe + ii] = bc_sign(p, 0, ii - gx, nx, v, c) * sy *
                                                      a[(size_t)(j + gy) * e->nxe + (i + gx)];
                }
            }
        }
}

/* ======================================================================
 * One evaluation of L(U) and U-hat on a rectangle of an extended grid
 * ====================================================================== */

/* Computes, for every cell of [xa,xb) x [ya,yb) (ext coordinates), the
 * semi-discrete operator L (eq. semi-discrete-scheme, eq. 2D-semi-discrete-
 * scheme-uniform) and U-hat; U must be valid two cells around the rectangle.
 * L and Uh are ext-shaped. */
static int eval_operator(const orc_problem* p, ext_t* U, double ax, double ay, int xa,
                         int xb, int ya, int yb, ext_t* L, ext_t* Uh) {
    int K = U->K, nxe = U->nxe, nye = U->nye;
    double dx = (p->xhi - p->xlo) / p->nx;
    int nthreads = orc_get_threads();
    (void)nthreads;

    if (p->dim == 1) {
        /* reconstruct cells xa-1 .. xb (those touching the rectangle's interfaces) */
        int nc = xb - xa + 2;
        double* um = (double*)malloc(sizeof(double) * nc * K * 4); /* u(+1/2),u(-1/2),ux(+),ux(-) */
        double* vh = (double*)malloc(sizeof(double) * nc * K);
        if (!um || !vh) { free(um); free(vh); return -5; }
#pragma omp parallel for num_threads(nthreads) schedule(static) if (nc * K >= OMP_MIN_WORK)
        for (int t = 0; t < nc; ++t) {
            int i = xa - 1 + t;
            double s[12], w[8];
            for (int c = 0; c < K; ++c) {
                const double* ub = ext_at(U, 0, c);
                const double* vb = ext_at(U, 1, c);
                s[c] = ub[i - 1];
                s[K + c] = ub[i];
                s[2 * K + c] = ub[i + 1];
                w[c] = vb[i - 1];
                w[K + c] = vb[i + 1];
            }
            double Cc[4][5], vc[4];
            char_recon_1d(p, s, w, dx, Cc, vc);
            for (int c = 0; c < K; ++c) {
                double* o = um + ((size_t)t * K + c) * 4;
                poly1d_eval(Cc[c], 0.5, dx, &o[0], &o[2]);
                poly1d_eval(Cc[c], -0.5, dx, &o[1], &o[3]);
                vh[(size_t)t * K + c] = vc[c];
            }
        }
        /* interface fluxes (global Lax-Friedrichs) at x_{i+1/2}, i = xa-1 .. xb-1 */
        int ne = xb - xa + 1;
        double* fl = (double*)malloc(sizeof(double) * ne * K * 2);
        if (!fl) { free(um); free(vh); return -5; }
        for (int e = 0; e < ne; ++e) {
            double uL[4], uR[4], vL[4], vR[4], fL[4], fR[4], hL[4], hR[4];
            for (int c = 0; c < K; ++c) {
                const double* oL = um + ((size_t)e * K + c) * 4;       /* cell xa-1+e */
                const double* oR = um + ((size_t)(e + 1) * K + c) * 4; /* cell xa+e */
                uL[c] = oL[0]; vL[c] = oL[2];
                uR[c] = oR[1]; vR[c] = oR[3];
            }
            phys_flux(p, 0, uL, fL);
            phys_flux(p, 0, uR, fR);
            flux_jvp(p, 0, uL, vL, hL);
            flux_jvp(p, 0, uR, vR, hR);
            for (int c = 0; c < K; ++c) {
                fl[((size_t)e * K + c) * 2 + 0] = 0.5 * (fL[c] + fR[c]) - 0.5 * ax * (uR[c] - uL[c]);
                fl[((size_t)e * K + c) * 2 + 1] = 0.5 * (hL[c] + hR[c]) - 0.5 * ax * (vR[c] - vL[c]);
            }
        }
        for (int i = xa; i < xb; ++i) {
            int e = i - xa; /* flux at i-1/2 is e, at i+1/2 is e+1 */
            for (int c = 0; c < K; ++c) {
                double fm = fl[((size_t)e * K + c) * 2], fp = fl[((size_t)(e + 1) * K + c) * 2];
                double hm = fl[((size_t)e * K + c) * 2 + 1], hp = fl[((size_t)(e + 1) * K + c) * 2 + 1];
                ext_at(L, 0, c)[i] = -(fp - fm) / dx;
                ext_at(L, 1, c)[i] = -(hp - hm) / dx;
                ext_at(Uh, 0, c)[i] = ext_at(U, 0, c)[i];
                ext_at(Uh, 1, c)[i] = vh[(size_t)(i - xa + 1) * K + c];
            }
        }
        free(um); free(vh); free(fl);
        return 0;
    }

    /* ---- 2D ---- */
    double dy = (p->yhi - p->ylo) / p->ny;
    int Q = p->gauss_q;
    double gn[3], gw[3];
    if (gauss_rule(Q, gn, gw)) return -1;
    /* reconstruct the cells of the rectangle grown by one (corners unused);
     * in characteristic variables the x-edges take the polynomial built with
     * the x eigenvectors and the y-edges the one built with the y
     * eigenvectors, and v-hat (w-hat) comes from the x (y) polynomial */
    int ch = p->flux == ORC_EULER && p->charwise;
    int rw = xb - xa + 2, rh = yb - ya + 2;
    double* poly = (double*)malloc(sizeof(double) * (size_t)rw * rh * K * 15 * 2);
    double* hat = (double*)malloc(sizeof(double) * (size_t)rw * rh * K * 2);
    if (!poly || !hat) { free(poly); free(hat); return -5; }
    double* polyY = poly + (size_t)rw * rh * K * 15;
#pragma omp parallel for num_threads(nthreads) schedule(static) if (rw * rh >= OMP_MIN_WORK)
    for (int tj = 0; tj < rh; ++tj) {
        int j = ya - 1 + tj;
        for (int ti = 0; ti < rw; ++ti) {
            int i = xa - 1 + ti;
            int corner = (ti == 0 || ti == rw - 1) && (tj == 0 || tj == rh - 1);
            if (corner) continue;
            double q[17 * 4];
            for (int c = 0; c < K; ++c) {
                const double* ub = ext_at(U, 0, c);
                const double* vb = ext_at(U, 1, c);
                const double* wb = ext_at(U, 2, c);
#define AT(a, ii, jj) (a)[(size_t)(jj) * nxe + (ii)]
                double qc[17] = {
                    AT(ub, i - 1, j - 1), AT(ub, i, j - 1), AT(ub, i + 1, j - 1),
                    AT(ub, i - 1, j),     AT(ub, i, j),     AT(ub, i + 1, j),
                    AT(ub, i - 1, j + 1), AT(ub, i, j + 1), AT(ub, i + 1, j + 1),
                    AT(vb, i - 1, j), AT(vb, i + 1, j), AT(vb, i, j - 1), AT(vb, i, j + 1),
                    AT(wb, i - 1, j), AT(wb, i + 1, j), AT(wb, i, j - 1), AT(wb, i, j + 1)};
#undef AT
                for (int e = 0; e < 17; ++e) q[e * K + c] = qc[e];
            }
            double Cx[4][15], vx[4], wx[4];
            char_recon_2d(p, q, 0, Cx, vx, wx);
            double Cy[4][15], vy[4], wy[4];
            if (ch) char_recon_2d(p, q, 1, Cy, vy, wy);
            for (int c = 0; c < K; ++c) {
                size_t o = ((size_t)tj * rw + ti) * K + c;
                memcpy(poly + o * 15, Cx[c], sizeof(double) * 15);
                memcpy(polyY + o * 15, ch ? Cy[c] : Cx[c], sizeof(double) * 15);
                hat[o * 2 + 0] = vx[c];
                hat[o * 2 + 1] = ch ? wy[c] : wx[c];
            }
        }
    }
    (void)nye;

    /* edge fluxes: x-edges between rectangle-grown columns, y-edges between rows */
    int nxe_edges = xb - xa + 1, nye_edges = yb - ya + 1;
    size_t nfx = (size_t)nxe_edges * (yb - ya) * K * 3;
    size_t nfy = (size_t)(xb - xa) * nye_edges * K * 3;
    double* FX = (double*)calloc(nfx, sizeof(double));
    double* FY = (double*)calloc(nfy, sizeof(double));
    if (!FX || !FY) { free(poly); free(hat); free(FX); free(FY); return -5; }

#pragma omp parallel for num_threads(nthreads) schedule(static) if (rw * rh >= OMP_MIN_WORK)
    for (int tj = 1; tj < rh - 1; ++tj) {
        for (int e = 0; e < nxe_edges; ++e) {
            /* edge between grown-rect columns e and e+1, row tj */
            const double* PL = poly + (((size_t)tj * rw + e) * K) * 15;
            const double* PR = poly + (((size_t)tj * rw + e + 1) * K) * 15;
            double acc[3][4] = {{0}};
            for (int mu = 0; mu < Q; ++mu) {
                double UL[4], UR[4], VL[4], VR[4], WL[4], WR[4];
                for (int c = 0; c < K; ++c) {
                    double o[3];
                    orc_poly2d_eval(PL + c * 15, 0.5, gn[mu], o);
                    UL[c] = o[0]; VL[c] = o[1] / dx; WL[c] = o[2] / dy;
                    orc_poly2d_eval(PR + c * 15, -0.5, gn[mu], o);
                    UR[c] = o[0]; VR[c] = o[1] / dx; WR[c] = o[2] / dy;
                }
                double fL[4], fR[4], fvL[4], fvR[4], fwL[4], fwR[4];
                phys_flux(p, 0, UL, fL);
                phys_flux(p, 0, UR, fR);
                flux_jvp(p, 0, UL, VL, fvL);
                flux_jvp(p, 0, UR, VR, fvR);
                flux_jvp(p, 0, UL, WL, fwL);
                flux_jvp(p, 0, UR, WR, fwR);
                for (int c = 0; c < K; ++c) {
                    double f = 0.5 * (fL[c] + fR[c]) - 0.5 * ax * (UR[c] - UL[c]);
                    double fv = 0.5 * (fvL[c] + fvR[c]) - 0.5 * ax * (VR[c] - VL[c]);
                    double fw = 0.5 * (fwL[c] + fwR[c]) - 0.5 * ax * (WR[c] - WL[c]);
                    acc[0][c] += gw[mu] * f;
                    acc[1][c] += gw[mu] * fv;
                    acc[2][c] += gw[mu] * fw;
                }
            }
            for (int c = 0; c < K; ++c)
                for (int s = 0; s < 3; ++s)
                    FX[(((size_t)(tj - 1) * nxe_edges + e) * K + c) * 3 + s] = dy * acc[s][c];
        }
    }
#pragma omp parallel for num_threads(nthreads) schedule(static) if (rw * rh >= OMP_MIN_WORK)
    for (int e = 0; e < nye_edges; ++e) {
        for (int ti = 1; ti < rw - 1; ++ti) {
            const double* PB = polyY + (((size_t)e * rw + ti) * K) * 15;       /* below */
            const double* PT = polyY + (((size_t)(e + 1) * rw + ti) * K) * 15; /* above */
            double acc[3][4] = {{0}};
            for (int mu = 0; mu < Q; ++mu) {
                double UL[4], UR[4], VL[4], VR[4], WL[4], WR[4];
                for (int c = 0; c < K; ++c) {
                    double o[3];
                    orc_poly2d_eval(PB + c * 15, gn[mu], 0.5, o);
                    UL[c] = o[0]; VL[c] = o[1] / dx; WL[c] = o[2] / dy;
                    orc_poly2d_eval(PT + c * 15, gn[mu], -0.5, o);
                    UR[c] = o[0]; VR[c] = o[1] / dx; WR[c] = o[2] / dy;
                }
                double gL[4], gR[4], gvL[4], gvR[4], gwL[4], gwR[4];
                phys_flux(p, 1, UL, gL);
                phys_flux(p, 1, UR, gR);
                flux_jvp(p, 1, UL, VL, gvL);
                flux_jvp(p, 1, UR, VR, gvR);
                flux_jvp(p, 1, UL, WL, gwL);
                flux_jvp(p, 1, UR, WR, gwR);
                for (int c = 0; c < K; ++c) {
                    double g = 0.5 * (gL[c] + gR[c]) - 0.5 * ay * (UR[c] - UL[c]);
                    double gv = 0.5 * (gvL[c] + gvR[c]) - 0.5 * ay * (VR[c] - VL[c]);
                    double gw_ = 0.5 * (gwL[c] + gwR[c]) - 0.5 * ay * (WR[c] - WL[c]);
                    acc[0][c] += gw[mu] * g;
                    acc[1][c] += gw[mu] * gv;
                    acc[2][c] += gw[mu] * gw_;
                }
            }
            for (int c = 0; c < K; ++c)
                for (int s = 0; s < 3; ++s)
                    FY[(((size_t)e * (xb - xa) + (ti - 1)) * K + c) * 3 + s] = dx * acc[s][c];
        }
    }

    for (int j = ya; j < yb; ++j)
        for (int i = xa; i < xb; ++i)
            for (int c = 0; c < K; ++c) {
                int ei = i - xa, ej = j - ya;
                const double* fm = FX + (((size_t)ej * nxe_edges + ei) * K + c) * 3;
                const double* fp = FX + (((size_t)ej * nxe_edges + ei + 1) * K + c) * 3;
                const double* gm = FY + (((size_t)ej * (xb - xa) + ei) * K + c) * 3;
                const double* gp = FY + (((size_t)(ej + 1) * (xb - xa) + ei) * K + c) * 3;
                size_t at = (size_t)j * nxe + i;
                ext_at(L, 0, c)[at] = -(fp[0] - fm[0] + gp[0] - gm[0]) / (dx * dy);
                ext_at(L, 1, c)[at] = -(fp[1] - fm[1] + gp[1] - gm[1]) / dy;
                ext_at(L, 2, c)[at] = -(fp[2] - fm[2] + gp[2] - gm[2]) / dx;
                size_t o = ((size_t)(ej + 1) * rw + (ei + 1)) * K + c;
                ext_at(Uh, 0, c)[at] = ext_at(U, 0, c)[at];
                ext_at(Uh, 1, c)[at] = hat[o * 2 + 0];
                ext_at(Uh, 2, c)[at] = hat[o * 2 + 1];
            }
    free(poly); free(hat); free(FX); free(FY);
    return 0;
}

/* ======================================================================
 * SSP-RK3 with the derivative modification (Sec. 2.1 Step 4, Sec. 2.2 Step 4)
 * ====================================================================== */

/* Runs the three stages on an extended grid whose margins are gx (and gy):
 * if refill is set, the ghosts of each stage's input are refilled from its
 * interior (whole-grid stepping); otherwise each stage shrinks the valid
 * region by two cells (window stepping, margins of six).  On return the
 * stage-3 result is in E over the final rectangle. */
/* Window stepping: after a stage, the cells of the window's margin that lie
 * outside the domain across a transmissive boundary get the value of the
 * nearest boundary cell of the same stage, as the whole-grid ghost fill does.
 * (Across periodic boundaries the computed margin values already equal those
 * of the wrapped cells.)  (i0, j0) is the window origin. */
static void window_refill(const orc_problem* p, ext_t* e, int i0, int j0, int gx, int gy,
                          int xa, int xb, int ya, int yb) {
    int tx = p->bc_x != ORC_PERIODIC;
    int ty = p->dim == 2 && p->bc_y != ORC_PERIODIC;
    if (!tx && !ty) return;
    for (int v = 0; v < e->nv; ++v)
        for (int c = 0; c < e->K; ++c) {
            double* a = ext_at(e, v, c);
            for (int jj = ya; jj < yb; ++jj)
                for (int ii = xa; ii < xb; ++ii) {
                    int gi = i0 + ii - gx, gj = j0 + jj - gy;
                    int si = tx ? bc_map(gi, p->nx, p->bc_x) : gi;
                    int sj = ty ? bc_map(gj, p->ny, p->bc_y) : gj;
                    if (si == gi && sj == gj) continue;
                    double sg = (tx ? bc_sign(p, 0, gi, p->nx, v, c) : 1.0) *
                                (ty ? bc_sign(p, 1, gj, p->ny, v, c) : 1.0);
                    a[(size_t)jj * e->nxe + ii] =
                        sg * a[(size_t)(sj - j0 + gy) * e->nxe + (si - i0 + gx)];
                }
        }
}

/* Lax-Friedrichs speeds of an extended whole-grid state (interior cells);
 * -2 if a cell is not admissible. */
static int ext_alpha(const orc_problem* p, ext_t* e, int gx, int gy, double* ax, double* ay) {
    int K = e->K;
    double mx = 0.0, my = 0.0;
    for (int j = gy; j < e->nye - gy; ++j)
        for (int i = gx; i < e->nxe - gx; ++i) {
            double U[4];
            for (int c = 0; c < K; ++c) U[c] = ext_at(e, 0, c)[(size_t)j * e->nxe + i];
            double s;
            if (max_speed(p, 0, U, &s)) return -2;
            if (s > mx) mx = s;
            if (p->dim == 2) {
                if (max_speed(p, 1, U, &s)) return -2;
                if (s > my) my = s;
            }
        }
    *ax = mx;
    *ay = my;
    return 0;
}

static int ssprk3_ext(const orc_problem* p, ext_t* E, double ax, double ay, double dt,
                      int gx, int gy, int refill, int i0, int j0) {
    int K = E->K, nv = E->nv, nxe = E->nxe, nye = E->nye;
    ext_t U1, U2, L, Uh, Uhn;
    int rc = 0;
    if (ext_alloc(&U1, K, nv, nxe, nye) || ext_alloc(&U2, K, nv, nxe, nye) ||
        ext_alloc(&L, K, nv, nxe, nye) || ext_alloc(&Uh, K, nv, nxe, nye) ||
        ext_alloc(&Uhn, K, nv, nxe, nye))
        return -5;
    size_t plane = (size_t)nxe * nye;
    int two_d = p->dim == 2;
    /* rectangle of stage s */
    int xa[3], xb[3], ya[3], yb[3];
    for (int s = 0; s < 3; ++s) {
        int sh = refill ? 2 : 2 * (s + 1);
        if (refill) sh = gx;
        xa[s] = sh; xb[s] = nxe - sh;
        int shy = refill ? gy : (two_d ? 2 * (s + 1) : 0);
        ya[s] = two_d ? shy : 0;
        yb[s] = two_d ? nye - shy : 1;
    }
    ext_t* stage_in[3] = {E, &U1, &U2};
    for (int s = 0; s < 3 && rc == 0; ++s) {
        ext_t* Us = stage_in[s];
        if (refill && s > 0) ghost_fill(p, Us, gx, gy);
        double sax = ax, say = ay;
        if (p->alpha_stage && s > 0) {
            /* speeds of this stage's input over the interior cells */
            if (!refill) { rc = -1; break; }
            rc = ext_alpha(p, Us, gx, gy, &sax, &say);
            if (rc) break;
        }
        rc = eval_operator(p, Us, sax, say, xa[s], xb[s], ya[s], yb[s], &L, &Uh);
        if (rc) break;
        for (int v = 0; v < nv; ++v)
            for (int c = 0; c < K; ++c) {
                double* uh = ext_at(&Uh, v, c);
                double* l = ext_at(&L, v, c);
                double* uhn = ext_at(&Uhn, v, c);
                for (int j = ya[s]; j < yb[s]; ++j)
                    for (int i = xa[s]; i < xb[s]; ++i) {
                        size_t at = (size_t)j * nxe + i;
                        if (s == 0) {
                            uhn[at] = uh[at];
                            ext_at(&U1, v, c)[at] = uh[at] + dt * l[at];
                        } else if (s == 1) {
                            ext_at(&U2, v, c)[at] =
                                3.0 / 4.0 * uhn[at] + 1.0 / 4.0 * (uh[at] + dt * l[at]);
                        } else {
                            ext_at(E, v, c)[at] =
                                1.0 / 3.0 * uhn[at] + 2.0 / 3.0 * (uh[at] + dt * l[at]);
                        }
                    }
            }
        if (!refill && s < 2)
            window_refill(p, s == 0 ? &U1 : &U2, i0, j0, gx, gy, xa[s], xb[s], ya[s], yb[s]);
    }
    (void)plane;
    ext_free(&U1); ext_free(&U2); ext_free(&L); ext_free(&Uh); ext_free(&Uhn);
    return rc;
}

static int check_problem(const orc_problem* p) {
    if (p->dim != 1 && p->dim != 2) return -1;
    if (p->dim == 1 && p->ny != 1) return -1;
    if (p->nx < 4 || (p->dim == 2 && p->ny < 4)) return -1;
    if (p->dim == 2 && gauss_rule(p->gauss_q, (double[3]){0}, (double[3]){0})) return -1;
    if (p->smoothness != ORC_BETA_MOMENT && p->smoothness != ORC_BETA_CLASSICAL) return -1;
    if (p->bc_x < ORC_PERIODIC || p->bc_x > ORC_REFLECTIVE) return -1;
    if (p->dim == 2 && (p->bc_y < ORC_PERIODIC || p->bc_y > ORC_REFLECTIVE)) return -1;
    if (p->flux != ORC_EULER && (p->bc_x == ORC_REFLECTIVE ||
                                 (p->dim == 2 && p->bc_y == ORC_REFLECTIVE)))
        return -1;
    int M = p->dim == 1 ? 2 : 4;
    double s = 0.0;
    for (int m = 0; m <= M; ++m) {
        if (!(p->gamma_lin[m] > 0.0)) return -1;
        s += p->gamma_lin[m];
    }
    if (fabs(s - 1.0) > 1e-12) return -1;
    return 0;
}

static void ext_to_state(const orc_problem* p, ext_t* e, int gx, int gy, double* st, int wi,
                         int wj) {
    for (int v = 0; v < e->nv; ++v)
        for (int c = 0; c < e->K; ++c) {
            double* a = ext_at(e, v, c);
            double* d = st + (size_t)(v * e->K + c) * wi * wj;
            for (int j = 0; j < wj; ++j)
                for (int i = 0; i < wi; ++i)
                    d[(size_t)j * wi + i] = a[(size_t)(j + (p->dim == 2 ? gy : 0)) * e->nxe + i + gx];
        }
}

int orc_alpha(const orc_problem* p, const double* st, double* ax, double* ay,
              long long* bad_cell) {
    int K = orc_ncomp(p);
    size_t ncell = (size_t)p->nx * p->ny;
    double sx = 0.0, sy = 0.0;
    for (size_t idx = 0; idx < ncell; ++idx) {
        double U[4], s;
        for (int c = 0; c < K; ++c) U[c] = st[(size_t)c * ncell + idx];
        if (max_speed(p, 0, U, &s)) {
            if (bad_cell) *bad_cell = (long long)idx;
            return -2;
        }
        if (s > sx) sx = s;
        if (p->dim == 2) {
            max_speed(p, 1, U, &s);
            if (s > sy) sy = s;
        }
    }
    *ax = sx;
    *ay = sy;
    return 0;
}

double orc_dt(const orc_problem* p, double ax, double ay, double cfl, double e) {
    double dx = (p->xhi - p->xlo) / p->nx;
    if (p->dim == 1) return cfl * pow(dx, e) / ax;
    double dy = (p->yhi - p->ylo) / p->ny;
    return cfl / (ax / pow(dx, e) + ay / pow(dy, e));
}

int orc_rhs(const orc_problem* p, const double* st, double ax, double ay, double* L_out,
            double* Uhat_out) {
    return orc_rhs_window(p, st, ax, ay, 0, 0, p->nx, p->ny, L_out, Uhat_out);
}

int orc_rhs_window(const orc_problem* p, const double* st, double ax, double ay, int i0,
                   int j0, int wi, int wj, double* L_out, double* Uhat_out) {
    if (check_problem(p)) return -1;
    int K = orc_ncomp(p), nv = nvars(p);
    int g = 2, gy = p->dim == 2 ? 2 : 0;
    ext_t E, L, Uh;
    if (ext_alloc(&E, K, nv, wi + 2 * g, p->dim == 2 ? wj + 2 * gy : 1) ||
        ext_alloc(&L, K, nv, E.nxe, E.nye) || ext_alloc(&Uh, K, nv, E.nxe, E.nye))
        return -5;
    fill_from_state(p, st, &E, i0, j0, g, gy);
    int rc = eval_operator(p, &E, ax, ay, g, g + wi, gy, gy + (p->dim == 2 ? wj : 1), &L, &Uh);
    if (rc == 0) {
        if (L_out) ext_to_state(p, &L, g, gy, L_out, wi, p->dim == 2 ? wj : 1);
        if (Uhat_out) ext_to_state(p, &Uh, g, gy, Uhat_out, wi, p->dim == 2 ? wj : 1);
    }
    ext_free(&E); ext_free(&L); ext_free(&Uh);
    return rc;
}

int orc_step(const orc_problem* p, double* st, double ax, double ay, double dt) {
    if (check_problem(p)) return -1;
    int K = orc_ncomp(p), nv = nvars(p);
    int g = 2, gy = p->dim == 2 ? 2 : 0;
    ext_t E;
    if (ext_alloc(&E, K, nv, p->nx + 2 * g, p->dim == 2 ? p->ny + 2 * gy : 1)) return -5;
    fill_from_state(p, st, &E, 0, 0, g, gy);
    int rc = ssprk3_ext(p, &E, ax, ay, dt, g, gy, 1, 0, 0);
    if (rc == 0) ext_to_state(p, &E, g, gy, st, p->nx, p->ny);
    ext_free(&E);
    return rc;
}

int orc_step_window(const orc_problem* p, const double* st, double ax, double ay, double dt,
                    int i0, int j0, int wi, int wj, double* out) {
    if (check_problem(p)) return -1;
    int K = orc_ncomp(p), nv = nvars(p);
    int g = 6, gy = p->dim == 2 ? 6 : 0;
    int wjj = p->dim == 2 ? wj : 1;
    ext_t E;
    if (ext_alloc(&E, K, nv, wi + 2 * g, p->dim == 2 ? wj + 2 * gy : 1)) return -5;
    fill_from_state(p, st, &E, i0, j0, g, gy);
    int rc = ssprk3_ext(p, &E, ax, ay, dt, g, gy, 0, i0, j0);
    if (rc == 0) ext_to_state(p, &E, g, gy, out, wi, wjj);
    ext_free(&E);
    return rc;
}

int orc_run(const orc_problem* p, double* st, double t0, double t_end, double cfl,
            double dt_exponent, long long* steps_out) {
    double t = t0;
    long long n = 0;
    while (t < t_end) {
        double ax, ay;
        int rc = orc_alpha(p, st, &ax, &ay, NULL);
        if (rc) { if (steps_out) *steps_out = n; return rc; }
        double dt = orc_dt(p, ax, ay, cfl, dt_exponent);
        double rem = t_end - t;
        int last = !(dt < rem);
        if (last) dt = rem;
        rc = orc_step(p, st, ax, ay, dt);
        if (rc) { if (steps_out) *steps_out = n; return rc; }
        ++n;
        t = last ? t_end : t + dt;
    }
    if (steps_out) *steps_out = n;
    return 0;
}
