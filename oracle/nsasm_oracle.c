/*
 * nsasm CPU oracle -- TEST INFRASTRUCTURE, not part of the product.
 *
 * Plain, slow, FP64 implementation of the element-by-element assembly of the
 * incompressible Navier-Stokes momentum right-hand side over linear tetrahedra
 * (the RHS assembly of Sec. II, specialised to P1 tetrahedra with four Gauss
 * points, constant density and viscosity and an eddy viscosity computed once per
 * element as in Sec. V-B).  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no source with the GPU library.
 *
 * The paper does not print the discrete equations (it defers them to the Alya
 * formulation paper), so the weak form below is the standard Galerkin one; the
 * readings taken where the paper is silent are:
 *   convective term  advective form  -rho (u . grad) u
 *   pressure term    gradient form   -grad p (no integration by parts)
 *   viscous term     Laplacian form  -(mu + mu_t) grad N_a . grad u_i
 *   eddy viscosity   Smagorinsky, Delta = V^(1/3), |S| = sqrt(2 S:S)
 *   body force       +rho f, constant acceleration
 *   orientation      V = |det J| / 6
 *   no boundary conditions, no stabilisation, one time level.
 *
 * For element e with vertices a = 0..3:
 *   J = [x1-x0 | x2-x0 | x3-x0], D = det J, V = |D|/6,
 *   grad N_a = row a of J^-1 (a = 1..3), grad N_0 = -(grad N_1 + grad N_2 + grad N_3),
 *   G = grad u, q = grad p, mu_e = mu + mu_t,
 *   Gauss points g = 0..3: N_a(g) = alpha if a == g else beta, weight V/4,
 *   u^g = sum_a N_a(g) u_a,  r^g = -rho G u^g - q + rho f,
 *   R^e_a = sum_g (V/4) N_a(g) r^g - mu_e V G grad N_a,
 *   R_n = sum over (e, a) with node(e, a) = n of R^e_a.
 *
 * The convective term may instead take the divergence, skew-symmetric,
 * rotational or EMAC form (convective() in element_body.inc); the default is
 * the advective form above.
 *
 * Velocity vector-Jacobian product g = (dR/du)^T lambda (not in the paper; the
 * adjoint form of the same assembly), per element with lambda^g, Lambda =
 * grad lambda, Phi = Lambda : G, for the advective form:
 *   g_b = -rho sum_g (V/4) [ N_b(g) G^T lambda^g + lambda^g (u^g . grad N_b) ]
 *         - mu_e V Lambda grad N_b - V Phi d mu_t / d u_b,
 * (the other forms add their terms by the chain rule in element_vjp),
 *   d mu_t / d u_{b,k} = rho (cs Delta)^2 (2/|S|) sum_j S_kj d_j N_b  (0 if |S| = 0).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double rho, mu, cs;
    double f[3];
    int model; /* eddy viscosity: 0 Smagorinsky, 1 Vreman; none when cs == 0 */
    int form;  /* convective form: 0 advective, 1 divergence, 2 skew-symmetric,
                  3 rotational, 4 EMAC (see convective() in element_body.inc) */
} oracle_params;

/* Symmetric 4-point rule on the tetrahedron, exact for degree 2. */
#define GAUSS_ALPHA ((5.0 + 3.0 * sqrt(5.0)) / 20.0)
#define GAUSS_BETA ((5.0 - sqrt(5.0)) / 20.0)

enum { ORACLE_OK = 0, ORACLE_BAD_INDEX = 1, ORACLE_DEGENERATE = 2, ORACLE_NOMEM = 3 };

/* ---------------------------------------------------------------- geometry */

/* Jacobian of the map from the reference tetrahedron, its determinant, the
 * volume and the constant shape-function gradients.  Returns 0 when D == 0. */
static int element_geometry(const double xe[4][3], double gradN[4][3], double *vol, double *det) {
    double J[3][3];
    for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c) J[i][c] = xe[c + 1][i] - xe[0][i]; /* column c = x_{c+1} - x_0 */
    double D = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
             - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
             + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    *det = D;
    if (D == 0.0 || !isfinite(D)) return 0;
    /* inverse = adjugate / D; adj[r][c] = cofactor[c][r] */
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / D;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / D;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / D;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / D;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / D;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / D;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / D;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / D;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / D;
    for (int a = 1; a < 4; ++a)
        for (int j = 0; j < 3; ++j) gradN[a][j] = inv[a - 1][j];
    for (int j = 0; j < 3; ++j) gradN[0][j] = -(gradN[1][j] + gradN[2][j] + gradN[3][j]);
    *vol = fabs(D) / 6.0;
    return 1;
}

/* ------------------------------------------- real and complex element bodies */

#define SCALAR double
#define SQRT_S sqrt
#define RE_S(x) (x)
#define FN(name) name##_r
#include "element_body.inc"
#undef SCALAR
#undef SQRT_S
#undef RE_S
#undef FN

#define SCALAR double complex
#define SQRT_S csqrt
#define RE_S(x) creal(x)
#define FN(name) name##_c
#include "element_body.inc"
#undef SCALAR
#undef SQRT_S
#undef RE_S
#undef FN

/* --------------------------------------------------------------- helpers */

static int gather_element(int64_t nn, const double *x, const int32_t *conn, int64_t e,
                          int32_t ids[4], double xe[4][3]) {
    for (int a = 0; a < 4; ++a) {
        int32_t n = conn[4 * e + a];
        if (n < 0 || (int64_t)n >= nn) return 0;
        ids[a] = n;
        for (int i = 0; i < 3; ++i) xe[a][i] = x[3 * (int64_t)n + i];
    }
    return 1;
}

static void set_params(oracle_params *prm, double rho, double mu, double cs, const double *f, int model,
                       int form) {
    prm->rho = rho;
    prm->mu = mu;
    prm->cs = cs;
    for (int i = 0; i < 3; ++i) prm->f[i] = f[i];
    prm->model = model;
    prm->form = form;
}

/* Each convective form of convective() written as
 *   c = G u + alpha (tr G) u + beta G^T u,
 * using div(u (x) u) = (u . grad) u + (div u) u and
 * (curl u) x u = (u . grad) u - grad(|u|^2 / 2) = G u - G^T u.
 * Used only by the VJP's chain rule; the forward evaluates the definitions. */
static void form_coefficients(int form, double *alpha, double *beta) {
    static const double tab[5][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.5, 0.0}, {0.0, -1.0}, {1.0, 1.0}};
    const int k = (form >= 0 && form < 5) ? form : 0;
    *alpha = tab[k][0];
    *beta = tab[k][1];
}

/* D = d mu_t / d G (D_ij = d mu_t / d G_ij) at velocity gradient G, for the
 * selected model; 0 where the model is not differentiable (|S| = 0 for
 * Smagorinsky, B <= 0 or alpha:alpha = 0 for Vreman). */
static void eddy_derivative(const double G[3][3], double vol, const oracle_params *prm, double D[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) D[i][j] = 0.0;
    if (prm->cs <= 0.0) return;
    const double delta = cbrt(vol);
    if (prm->model != 1) {
        /* mu_t = rho (cs Delta)^2 |S|, d|S|/dG = 2 S / |S| */
        double S[3][3], smag;
        (void)smagorinsky_r(G, vol, prm, S, &smag);
        if (smag == 0.0) return;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                D[i][j] = prm->rho * (prm->cs * delta) * (prm->cs * delta) * 2.0 * S[i][j] / smag;
        return;
    }
    /* Vreman: nu = c sqrt(B/aa); chain rule through beta(alpha) and B(beta) */
    const double c = 2.5 * prm->cs * prm->cs;
    double alpha[3][3], beta[3][3], aa = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            alpha[i][j] = G[j][i];
            aa += alpha[i][j] * alpha[i][j];
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double b = 0;
            for (int m = 0; m < 3; ++m) b += delta * delta * alpha[m][i] * alpha[m][j];
            beta[i][j] = b;
        }
    const double B = beta[0][0] * beta[1][1] - beta[0][1] * beta[0][1] + beta[0][0] * beta[2][2] -
                     beta[0][2] * beta[0][2] + beta[1][1] * beta[2][2] - beta[1][2] * beta[1][2];
    if (aa == 0.0 || B <= 0.0) return;
    /* dB/dbeta for the six independent entries (upper triangle) */
    double dB[3][3] = {{beta[1][1] + beta[2][2], -2.0 * beta[0][1], -2.0 * beta[0][2]},
                       {0.0, beta[0][0] + beta[2][2], -2.0 * beta[1][2]},
                       {0.0, 0.0, beta[0][0] + beta[1][1]}};
    const double root = sqrt(B / aa);
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
            /* d beta_ij / d alpha_kl = Delta^2 (delta_il alpha_kj + delta_jl alpha_ki), i <= j */
            double dBda = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = i; j < 3; ++j) {
                    const double dbeta = delta * delta * ((i == l ? alpha[k][j] : 0.0) + (j == l ? alpha[k][i] : 0.0));
                    dBda += dB[i][j] * dbeta;
                }
            const double dnu = c / (2.0 * root) * (dBda / aa - B * 2.0 * alpha[k][l] / (aa * aa));
            D[l][k] = prm->rho * dnu; /* alpha_kl = G_lk */
        }
}

static int n_threads_or_default(int nthreads) {
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* ------------------------------------------------------------ public API */

/* Number of OpenMP threads a call with nthreads = 0 would use. */
int oracle_default_threads(void) { return n_threads_or_default(0); }

/* Per-element volume V_e and shape-function gradients gradN (ne x 4 x 3). */
int oracle_geometry(int64_t nn, const double *x, int64_t ne, const int32_t *conn, double *vol,
                    double *gradN) {
    for (int64_t e = 0; e < ne; ++e) {
        int32_t ids[4];
        double xe[4][3], gN[4][3], V, D;
        if (!gather_element(nn, x, conn, e, ids, xe)) return ORACLE_BAD_INDEX;
        if (!element_geometry(xe, gN, &V, &D)) return ORACLE_DEGENERATE;
        vol[e] = V;
        memcpy(gradN + 12 * e, gN, sizeof gN);
    }
    return ORACLE_OK;
}

/* Per-element eddy viscosity mu_t (ne values). */
int oracle_eddy(int64_t nn, const double *x, int64_t ne, const int32_t *conn, const double *u,
                double rho, double mu, double cs, const double *f, int model, int form, double *mu_t) {
    oracle_params prm;
    set_params(&prm, rho, mu, cs, f, model, form);
    for (int64_t e = 0; e < ne; ++e) {
        int32_t ids[4];
        double xe[4][3], gN[4][3], V, D, ue[4][3], pe[4] = {0, 0, 0, 0}, G[3][3], S[3][3], q[3], sm;
        if (!gather_element(nn, x, conn, e, ids, xe)) return ORACLE_BAD_INDEX;
        if (!element_geometry(xe, gN, &V, &D)) return ORACLE_DEGENERATE;
        for (int a = 0; a < 4; ++a)
            for (int i = 0; i < 3; ++i) ue[a][i] = u[3 * (int64_t)ids[a] + i];
        gradients_r(gN, ue, pe, G, q);
        mu_t[e] = eddy_viscosity_r(G, V, &prm, S, &sm);
    }
    return ORACLE_OK;
}

/* Assembled right-hand side rhs (nn x 3), FP64.  OpenMP over elements; each
 * thread sums into a private copy of rhs, the copies are added at the end in
 * thread order (deterministic for a fixed thread count). */
int oracle_rhs(int64_t nn, const double *x, int64_t ne, const int32_t *conn, const double *u,
               const double *p, double rho, double mu, double cs, const double *f, int model, int form, double *rhs,
               int nthreads) {
    oracle_params prm;
    set_params(&prm, rho, mu, cs, f, model, form);
    const int nt = n_threads_or_default(nthreads);
    double *part = (double *)calloc((size_t)nt * (size_t)nn * 3, sizeof(double));
    if (!part) return ORACLE_NOMEM;
    int status = ORACLE_OK;
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        const int t = omp_get_thread_num();
#else
        const int t = 0;
#endif
        double *mine = part + (size_t)t * (size_t)nn * 3;
#pragma omp for schedule(static)
        for (int64_t e = 0; e < ne; ++e) {
            int32_t ids[4];
            double xe[4][3], gN[4][3], V, D, ue[4][3], pe[4], re[4][3];
            if (!gather_element(nn, x, conn, e, ids, xe)) {
#pragma omp atomic write
                status = ORACLE_BAD_INDEX;
                continue;
            }
            if (!element_geometry(xe, gN, &V, &D)) {
#pragma omp atomic write
                status = ORACLE_DEGENERATE;
                continue;
            }
            for (int a = 0; a < 4; ++a) {
                for (int i = 0; i < 3; ++i) ue[a][i] = u[3 * (int64_t)ids[a] + i];
                pe[a] = p[ids[a]];
            }
            element_rhs_r(gN, V, ue, pe, &prm, re);
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) mine[3 * (int64_t)ids[a] + i] += re[a][i];
        }
#pragma omp for schedule(static)
        for (int64_t k = 0; k < nn * 3; ++k) {
            double s = 0;
            for (int tt = 0; tt < nt; ++tt) s += part[(size_t)tt * (size_t)nn * 3 + k];
            rhs[k] = s;
        }
    }
    free(part);
    return status;
}

/* Complex-step form: velocity u_re + i u_im and pressure p_re + i p_im, real x;
 * serial. */
int oracle_rhs_complex(int64_t nn, const double *x, int64_t ne, const int32_t *conn,
                       const double *u_re, const double *u_im, const double *p_re, const double *p_im,
                       double rho, double mu, double cs, const double *f, int model, int form, double *r_re,
                       double *r_im) {
    oracle_params prm;
    set_params(&prm, rho, mu, cs, f, model, form);
    double complex *acc = (double complex *)calloc((size_t)nn * 3, sizeof(double complex));
    if (!acc) return ORACLE_NOMEM;
    for (int64_t e = 0; e < ne; ++e) {
        int32_t ids[4];
        double xe[4][3], gN[4][3], V, D;
        double complex ue[4][3], pe[4], re[4][3];
        if (!gather_element(nn, x, conn, e, ids, xe)) { free(acc); return ORACLE_BAD_INDEX; }
        if (!element_geometry(xe, gN, &V, &D)) { free(acc); return ORACLE_DEGENERATE; }
        for (int a = 0; a < 4; ++a) {
            for (int i = 0; i < 3; ++i) {
                int64_t k = 3 * (int64_t)ids[a] + i;
                ue[a][i] = u_re[k] + I * u_im[k];
            }
            pe[a] = p_re[ids[a]] + I * p_im[ids[a]];
        }
        element_rhs_c(gN, V, ue, pe, &prm, re);
        for (int a = 0; a < 4; ++a)
            for (int i = 0; i < 3; ++i) acc[3 * (int64_t)ids[a] + i] += re[a][i];
    }
    for (int64_t k = 0; k < nn * 3; ++k) {
        r_re[k] = creal(acc[k]);
        r_im[k] = cimag(acc[k]);
    }
    free(acc);
    return ORACLE_OK;
}

/* One element's velocity VJP contribution ge[b][k]. */
static void element_vjp(const double gN[4][3], double V, const double ue[4][3],
                        const double le[4][3], const oracle_params *prm, double ge[4][3]) {
    const double pe[4] = {0, 0, 0, 0};
    double G[3][3], S[3][3], q[3], smag;
    gradients_r(gN, ue, pe, G, q);
    const double mu_e = prm->mu + eddy_viscosity_r(G, V, prm, S, &smag);

    double Lam[3][3]; /* Lambda_kj = sum_a lambda_{a,k} d_j N_a */
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int a = 0; a < 4; ++a) s += le[a][k] * gN[a][j];
            Lam[k][j] = s;
        }
    double Phi = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Phi += Lam[i][j] * G[i][j];

    for (int b = 0; b < 4; ++b)
        for (int k = 0; k < 3; ++k) ge[b][k] = 0;

    double alpha, beta;
    form_coefficients(prm->form, &alpha, &beta);
    const double w = V / 4.0;
    for (int g = 0; g < 4; ++g) {
        double N[4], ug[3], lg[3];
        for (int a = 0; a < 4; ++a) N[a] = (a == g) ? GAUSS_ALPHA : GAUSS_BETA;
        for (int j = 0; j < 3; ++j) {
            ug[j] = 0;
            lg[j] = 0;
            for (int a = 0; a < 4; ++a) {
                ug[j] += N[a] * ue[a][j];
                lg[j] += N[a] * le[a][j];
            }
        }
        /* lambda^g . c(u^g) with c = K u^g, K = G + alpha tr(G) I + beta G^T.
         * d/du_{b,k} = N_b (K^T lambda^g)_k + sum_n d_n N_b d(lambda^g . c)/dG_kn,
         * d(lambda^g . c)/dG_kn = lambda^g_k u^g_n + alpha delta_kn (lambda^g . u^g)
         *                         + beta u^g_k lambda^g_n. */
        const double trG = G[0][0] + G[1][1] + G[2][2];
        double lu = 0;
        for (int j = 0; j < 3; ++j) lu += lg[j] * ug[j];
        for (int b = 0; b < 4; ++b) {
            double udn = 0, ldn = 0;
            for (int j = 0; j < 3; ++j) {
                udn += ug[j] * gN[b][j];
                ldn += lg[j] * gN[b][j];
            }
            for (int k = 0; k < 3; ++k) {
                double gtl = 0, gl = 0;
                for (int i = 0; i < 3; ++i) {
                    gtl += lg[i] * G[i][k];
                    gl += G[k][i] * lg[i];
                }
                const double ktl = gtl + alpha * trG * lg[k] + beta * gl;
                const double dg = lg[k] * udn + alpha * lu * gN[b][k] + beta * ug[k] * ldn;
                ge[b][k] += -prm->rho * w * (N[b] * ktl + dg);
            }
        }
    }
    double D[3][3]; /* d mu_t / d G */
    eddy_derivative(G, V, prm, D);
    for (int b = 0; b < 4; ++b)
        for (int k = 0; k < 3; ++k) {
            double lv = 0, dv = 0;
            for (int j = 0; j < 3; ++j) {
                lv += gN[b][j] * Lam[k][j];
                dv += D[k][j] * gN[b][j];
            }
            ge[b][k] += -mu_e * V * lv - V * Phi * dv;
        }
}

/* Velocity vector-Jacobian product g = (dR/du)^T lam (nn x 3), FP64, OpenMP as
 * in oracle_rhs. */
int oracle_vjp(int64_t nn, const double *x, int64_t ne, const int32_t *conn, const double *u,
               const double *lam, double rho, double mu, double cs, const double *f, int model, int form, double *grad,
               int nthreads) {
    oracle_params prm;
    set_params(&prm, rho, mu, cs, f, model, form);
    const int nt = n_threads_or_default(nthreads);
    double *part = (double *)calloc((size_t)nt * (size_t)nn * 3, sizeof(double));
    if (!part) return ORACLE_NOMEM;
    int status = ORACLE_OK;
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        const int t = omp_get_thread_num();
#else
        const int t = 0;
#endif
        double *mine = part + (size_t)t * (size_t)nn * 3;
#pragma omp for schedule(static)
        for (int64_t e = 0; e < ne; ++e) {
            int32_t ids[4];
            double xe[4][3], gN[4][3], V, D, ue[4][3], le[4][3], ge[4][3];
            if (!gather_element(nn, x, conn, e, ids, xe)) {
#pragma omp atomic write
                status = ORACLE_BAD_INDEX;
                continue;
            }
            if (!element_geometry(xe, gN, &V, &D)) {
#pragma omp atomic write
                status = ORACLE_DEGENERATE;
                continue;
            }
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) {
                    ue[a][i] = u[3 * (int64_t)ids[a] + i];
                    le[a][i] = lam[3 * (int64_t)ids[a] + i];
                }
            element_vjp(gN, V, ue, le, &prm, ge);
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) mine[3 * (int64_t)ids[a] + i] += ge[a][i];
        }
#pragma omp for schedule(static)
        for (int64_t k = 0; k < nn * 3; ++k) {
            double s = 0;
            for (int tt = 0; tt < nt; ++tt) s += part[(size_t)tt * (size_t)nn * 3 + k];
            grad[k] = s;
        }
    }
    free(part);
    return status;
}

/* Pressure vector-Jacobian product g_p = (dR/dp)^T lam (nn values).  The
 * pressure enters only through -sum_g (V/4) N_a(g) q with q = grad p, so per
 * element g_p[b] = -sum_g (V/4) lambda^g . grad N_b.  OpenMP as oracle_rhs. */
int oracle_vjp_p(int64_t nn, const double *x, int64_t ne, const int32_t *conn, const double *lam,
                 double *grad_p, int nthreads) {
    const int nt = n_threads_or_default(nthreads);
    double *part = (double *)calloc((size_t)nt * (size_t)nn, sizeof(double));
    if (!part) return ORACLE_NOMEM;
    int status = ORACLE_OK;
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        const int t = omp_get_thread_num();
#else
        const int t = 0;
#endif
        double *mine = part + (size_t)t * (size_t)nn;
#pragma omp for schedule(static)
        for (int64_t e = 0; e < ne; ++e) {
            int32_t ids[4];
            double xe[4][3], gN[4][3], V, D, le[4][3];
            if (!gather_element(nn, x, conn, e, ids, xe)) {
#pragma omp atomic write
                status = ORACLE_BAD_INDEX;
                continue;
            }
            if (!element_geometry(xe, gN, &V, &D)) {
#pragma omp atomic write
                status = ORACLE_DEGENERATE;
                continue;
            }
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) le[a][i] = lam[3 * (int64_t)ids[a] + i];
            for (int g = 0; g < 4; ++g) {
                double N[4], lg[3];
                for (int a = 0; a < 4; ++a) N[a] = (a == g) ? GAUSS_ALPHA : GAUSS_BETA;
                for (int i = 0; i < 3; ++i) {
                    lg[i] = 0;
                    for (int a = 0; a < 4; ++a) lg[i] += N[a] * le[a][i];
                }
                for (int b = 0; b < 4; ++b) {
                    double dot = 0;
                    for (int i = 0; i < 3; ++i) dot += lg[i] * gN[b][i];
                    mine[ids[b]] -= (V / 4.0) * dot;
                }
            }
        }
#pragma omp for schedule(static)
        for (int64_t k = 0; k < nn; ++k) {
            double s = 0;
            for (int tt = 0; tt < nt; ++tt) s += part[(size_t)tt * (size_t)nn + k];
            grad_p[k] = s;
        }
    }
    free(part);
    return status;
}
