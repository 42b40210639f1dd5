/*
 * hrm_oracle.c -- plain double-precision CPU reference for the hot path of the
 * positivity-preserving fractional algorithm for the four-equation HRM
 * (Wong, Angel & Kiris, arXiv:2208.04488): one hyperbolic SSP-RK stage of the
 * five-equation model with PP-WCNS-IS, followed by the algebraic
 * infinite-rate thermal relaxation.
 *
 * TEST INFRASTRUCTURE.  This library is the oracle of the HIP library, not
 * part of it.  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no source, header, table or helper
 * with the HIP code and imports nothing from it.
 *
 * It is written to be checked against the paper by eye, not to be fast:
 *   - every face recomputes the primitive state of its six stencil nodes;
 *   - ghost nodes come from an index map (copy for transmissive ends, wrap
 *     for periodic ends), never from a padded copy of the array;
 *   - the characteristic projection uses the dense matrices of App. D;
 *   - all arithmetic is IEEE double; the build disables FMA contraction.
 * Readings of passages that are silent or ambiguous are marked "reading:".
 *
 * State layout: W[c * ncell + cell], cell = (z * ny + y) * nx + x, with the
 * component order of the conservative vector of Sec. 2:
 *   alpha_k rho_k (k = 0..N-1), rho u_d (d = 0..D-1), E, alpha_k (k = 0..N-2).
 * Primitive vector V of App. D, same slots:
 *   alpha_k rho_k, u_d, p, alpha_k (k = 0..N-2).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXN 8
#define ORC_MAXM (2 * ORC_MAXN + 3)

#define ORC_TRANSMISSIVE 0
#define ORC_PERIODIC 1
#define ORC_DIRICHLET 2 /* ghost nodes take a given state per line (Sec. 5.9 inflow) */

#define ORC_NO_LIMITERS 1  /* skip the PP interpolation and flux limiters */
#define ORC_NO_BLEND 2     /* sigma^s = 0: pure HCS flux (App. B ablation) */
#define ORC_FIRST_ORDER 4  /* first-order HLLC fluxes only (Sec. 4.1.1) */
#define ORC_FOUR_EQ 32    /* the four-equation HRM solved directly with first-order HLLC */

/* diagnostic counters */
#define ORC_C_ALG1 0      /* interpolation limiter, partial density limited */
#define ORC_C_ALG2 1      /* interpolation limiter, volume fractions limited */
#define ORC_C_IHS 2       /* interpolation hard switch */
#define ORC_C_ALG3 3      /* flux limiter, theta < 1 in Alg. 3 */
#define ORC_C_ALG4 4      /* flux limiter, theta < 1 in Alg. 4 */
#define ORC_C_FHS 5       /* flux hard switch */
#define ORC_C_RELAX_BAD 6 /* relaxation input outside script-G (cell left as is) */
#define ORC_NCOUNT 8

typedef struct {
    int N, D;
    int n[3];
    double dx[3];
    int bc_lo[3], bc_hi[3];
    double gamma[ORC_MAXN], cv[ORC_MAXN], pinf[ORC_MAXN], q[ORC_MAXN];
    double eps_weno;                  /* App. C: 1e-15 */
    double eps_i_ar, eps_i_a;         /* Sec. 4.3.2 interpolation limiter: 1e-10, 1e-10 */
    double hs_i_ar, hs_i_a, hs_i_rc2; /* interpolation hard switch: 1e-11, 1e-11, 1e-9 */
    double eps_f_ar, eps_f_a, eps_f_re; /* flux limiter: 1e-10, 1e-10, 1e-8 */
    double hs_f_ar, hs_f_a, hs_f_re;  /* flux hard switch: 1e-11, 1e-11, 1e-9 */
    double Cs, qexp, psi;             /* sensor C_s = 1e12, q = 2; HCS psi = 256/175 */
    int flags;
    int weights;                      /* ORC_W_IS (App. C) or ORC_W_MLP (learned weights) */
    const double *mlp;                /* ORC_W_MLP: the 1347 network parameters */
    const double *bnd[3][2];          /* ORC_DIRICHLET sides: ghost states, M x (n_a n_b) */
} orc_setup;

#define ORC_W_IS 0
#define ORC_W_MLP 1

/* one node (or interpolated face state) with the quantities of Sec. 2 */
typedef struct {
    double W[ORC_MAXM];     /* conservative vector */
    double V[ORC_MAXM];     /* primitive vector of App. D */
    double alpha[ORC_MAXN]; /* all N volume fractions, alpha_N = 1 - sum of the others */
    double rho, rhoe_t, gbar, pbar, rhoc2, c;
} orc_state;

static int IMOM(const orc_setup *s, int d) { return s->N + d; }
static int IE(const orc_setup *s) { return s->N + s->D; }
static int IAL(const orc_setup *s, int k) { return s->N + s->D + 1 + k; }
static int NCOMP(const orc_setup *s) { return 2 * s->N + s->D; }
static long NCELL(const orc_setup *s) { return (long)s->n[0] * s->n[1] * s->n[2]; }

/* ------------------------------------------------------------------------ */
/* Sec. 2: mixture equation of state under pressure equilibrium.              */
/*   1/(gbar-1)            = sum_k alpha_k/(gamma_k-1)                         */
/*   gbar pbar/(gbar-1)    = sum_k alpha_k gamma_k pinf_k/(gamma_k-1)          */
/*   p/(gbar-1) + gbar pbar/(gbar-1) = rho (e - qbar)                           */
/*   rho c^2 = gbar (p + pbar)                                                 */
/*   rho (e - qbar) = E - |rho u|^2/(2 rho) - sum_k alpha_k rho_k q_k          */
/* ------------------------------------------------------------------------ */
static void mixture_gamma(const orc_setup *s, const double *alpha, double *gbar, double *pbar)
{
    double inv = 0.0, gp = 0.0;
    for (int k = 0; k < s->N; ++k) {
        inv += alpha[k] / (s->gamma[k] - 1.0);
        gp += alpha[k] * s->gamma[k] * s->pinf[k] / (s->gamma[k] - 1.0);
    }
    *gbar = 1.0 + 1.0 / inv;
    *pbar = gp * (*gbar - 1.0) / *gbar;
}

/* W -> primitive state (hot-path step a1) */
static void state_from_cons(const orc_setup *s, const double *W, orc_state *st)
{
    const int N = s->N, D = s->D, M = NCOMP(s);
    for (int c = 0; c < M; ++c) st->W[c] = W[c];
    double rho = 0.0;
    for (int k = 0; k < N; ++k) rho += W[k];
    st->rho = rho;
    double asum = 0.0;
    for (int k = 0; k < N - 1; ++k) {
        st->alpha[k] = W[IAL(s, k)];
        asum += W[IAL(s, k)];
    }
    st->alpha[N - 1] = 1.0 - asum;
    mixture_gamma(s, st->alpha, &st->gbar, &st->pbar);
    double mom2 = 0.0, rq = 0.0;
    for (int d = 0; d < D; ++d) mom2 += W[IMOM(s, d)] * W[IMOM(s, d)];
    for (int k = 0; k < N; ++k) rq += W[k] * s->q[k];
    st->rhoe_t = W[IE(s)] - 0.5 * mom2 / rho - rq;
    double p = (st->gbar - 1.0) * st->rhoe_t - st->gbar * st->pbar;
    st->rhoc2 = st->gbar * (p + st->pbar);
    st->c = sqrt(st->rhoc2 / rho);
    for (int k = 0; k < N; ++k) st->V[k] = W[k];
    for (int d = 0; d < D; ++d) st->V[IMOM(s, d)] = W[IMOM(s, d)] / rho;
    st->V[IE(s)] = p;
    for (int k = 0; k < N - 1; ++k) st->V[IAL(s, k)] = W[IAL(s, k)];
}

/* primitive -> conservative (the same EOS read the other way) */
static void state_from_prim(const orc_setup *s, const double *V, orc_state *st)
{
    const int N = s->N, D = s->D, M = NCOMP(s);
    for (int c = 0; c < M; ++c) st->V[c] = V[c];
    double rho = 0.0;
    for (int k = 0; k < N; ++k) rho += V[k];
    st->rho = rho;
    double asum = 0.0;
    for (int k = 0; k < N - 1; ++k) {
        st->alpha[k] = V[IAL(s, k)];
        asum += V[IAL(s, k)];
    }
    st->alpha[N - 1] = 1.0 - asum;
    mixture_gamma(s, st->alpha, &st->gbar, &st->pbar);
    const double p = V[IE(s)];
    st->rhoe_t = p / (st->gbar - 1.0) + st->gbar * st->pbar / (st->gbar - 1.0);
    st->rhoc2 = st->gbar * (p + st->pbar);
    st->c = sqrt(st->rhoc2 / rho);
    double u2 = 0.0, rq = 0.0;
    for (int d = 0; d < D; ++d) u2 += V[IMOM(s, d)] * V[IMOM(s, d)];
    for (int k = 0; k < N; ++k) rq += V[k] * s->q[k];
    for (int k = 0; k < N; ++k) st->W[k] = V[k];
    for (int d = 0; d < D; ++d) st->W[IMOM(s, d)] = rho * V[IMOM(s, d)];
    st->W[IE(s)] = st->rhoe_t + 0.5 * rho * u2 + rq;
    for (int k = 0; k < N - 1; ++k) st->W[IAL(s, k)] = V[IAL(s, k)];
}

/* rho (e - qbar) of a conservative vector (equation below the set script-G) */
static double rhoe_tilde(const orc_setup *s, const double *W)
{
    double rho = 0.0, mom2 = 0.0, rq = 0.0;
    for (int k = 0; k < s->N; ++k) {
        rho += W[k];
        rq += W[k] * s->q[k];
    }
    for (int d = 0; d < s->D; ++d) mom2 += W[IMOM(s, d)] * W[IMOM(s, d)];
    return W[IE(s)] - 0.5 * mom2 / rho - rq;
}

/* all N volume fractions of a conservative vector */
static void alphas_of(const orc_setup *s, const double *W, double *alpha)
{
    double asum = 0.0;
    for (int k = 0; k < s->N - 1; ++k) {
        alpha[k] = W[IAL(s, k)];
        asum += alpha[k];
    }
    alpha[s->N - 1] = 1.0 - asum;
}

/* Sec. 4.1: flux vectors in direction n.  G has alpha_k u_n in the last N-1
 * slots (eq:W_G_eqn); F has zeros there (eq:F_x_F_y_def). */
static void flux_vec(const orc_setup *s, int n, const orc_state *st, int with_alpha, double *out)
{
    const int N = s->N, D = s->D;
    const double un = st->V[IMOM(s, n)], p = st->V[IE(s)];
    for (int k = 0; k < N; ++k) out[k] = st->W[k] * un;
    for (int d = 0; d < D; ++d) out[IMOM(s, d)] = st->W[IMOM(s, d)] * un + (d == n ? p : 0.0);
    out[IE(s)] = (st->W[IE(s)] + p) * un;
    for (int k = 0; k < N - 1; ++k) out[IAL(s, k)] = with_alpha ? st->alpha[k] * un : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.1.1: HLLC solver for the five-equation model.                      */
/* Returns s_* (the face velocity u-hat of the first-order scheme) and       */
/* writes G^HLLC = F^HLLC + (0, ..., f_alpha) into G.                         */
/* ------------------------------------------------------------------------ */
static double hllc(const orc_setup *s, int n, const orc_state *L, const orc_state *R, double *G)
{
    const int N = s->N, D = s->D, M = NCOMP(s);
    const double uL = L->V[IMOM(s, n)], uR = R->V[IMOM(s, n)];
    const double pL = L->V[IE(s)], pR = R->V[IE(s)];
    /* wave speeds of Einfeldt / Batten et al.; ubar, cbar arithmetic means */
    const double ubar = 0.5 * (uL + uR), cbar = 0.5 * (L->c + R->c);
    const double sL = fmin(ubar - cbar, uL - L->c);
    const double sR = fmax(ubar + cbar, uR + R->c);
    const double sstar = (pR - pL + L->rho * uL * (sL - uL) - R->rho * uR * (sR - uR)) /
                         (L->rho * (sL - uL) - R->rho * (sR - uR));
    double WsL[ORC_MAXM], WsR[ORC_MAXM], FL[ORC_MAXM], FR[ORC_MAXM];
    for (int side = 0; side < 2; ++side) {
        const orc_state *K = side == 0 ? L : R;
        const double sK = side == 0 ? sL : sR;
        const double uK = K->V[IMOM(s, n)], pK = K->V[IE(s)];
        double *Ws = side == 0 ? WsL : WsR;
        const double chi = (sK - uK) / (sK - sstar);
        for (int k = 0; k < N; ++k) Ws[k] = chi * K->W[k];
        for (int d = 0; d < D; ++d)
            Ws[IMOM(s, d)] = d == n ? chi * K->rho * sstar : chi * K->rho * K->V[IMOM(s, d)];
        Ws[IE(s)] = chi * (K->W[IE(s)] + (sstar - uK) * (K->rho * sstar + pK / (sK - uK)));
        for (int k = 0; k < N - 1; ++k) Ws[IAL(s, k)] = K->alpha[k];
    }
    flux_vec(s, n, L, 0, FL);
    flux_vec(s, n, R, 0, FR);
    const double sm = fmin(0.0, sL), sp = fmax(0.0, sR);
    /* reading: sign(0) = 0, i.e. the average of the two star fluxes */
    const double sg = sstar > 0.0 ? 1.0 : (sstar < 0.0 ? -1.0 : 0.0);
    for (int c = 0; c < M; ++c)
        G[c] = 0.5 * (1.0 + sg) * (FL[c] + sm * (WsL[c] - L->W[c])) +
               0.5 * (1.0 - sg) * (FR[c] + sp * (WsR[c] - R->W[c]));
    /* upwind volume-fraction flux f_alpha_k */
    for (int k = 0; k < N - 1; ++k)
        G[IAL(s, k)] = 0.5 * (1.0 + sg) * (L->alpha[k] * sstar) + 0.5 * (1.0 - sg) * (R->alpha[k] * sstar);
    return sstar;
}

/* ------------------------------------------------------------------------ */
/* Learned nonlinear weights (an extension of the method, not in the paper).  */
/* The interpolant at i+1/2 is a convex combination of the three 3-point      */
/* candidates of the fifth-order interpolation from u_{i-2..i+2}:             */
/*   S_l = (3u_{i-2} - 10u_{i-1} + 15u_i)/8,  S_c = (-u_{i-1} + 6u_i + 3u_{i+1})/8, */
/*   S_r = (3u_i + 6u_{i+1} - u_{i+2})/8,                                      */
/* whose linear weights d = (1/16, 10/16, 5/16) give the fifth-order value;  */
/* the value is formed as S_c + omega_l (S_l - S_c) + omega_r (S_r - S_c).    */
/* A perceptron 5-32-32-3 (ReLU) maps the normalised stencil                 */
/*   x_j = (u_j - u_i) r,  r = 1 / max_j |u_j - u_i|   (x = 0 if the max is 0) */
/* to logits z that rescale the classical WENO5 weights of x (Jiang & Shu):   */
/*   omega_k = d_k e^{tanh z_k} / (eps + beta_k)^2, normalised, eps = 1e-6,   */
/* so each weight moves by at most a factor e either way; the indicators     */
/* beta_k are those of x rounded to float; r is formed once and multiplies    */
/* each difference.  A zero last layer gives the classical weights.  1347     */
/* parameters, in this order:                                                 */
/* W1[5][32], b1[32], W2[32][32], b2[32], W3[32][3], b3[3] (row = input unit). */
/* The number formats are those of a bfloat16 matrix-core evaluation with     */
/* float accumulation: inputs, W1, b1, W2, W3 and both hidden activations     */
/* (after the ReLU) are rounded to bfloat16 (through float, to nearest even); */
/* b2 and b3 are float; the sums themselves are taken in double here.         */
/* ------------------------------------------------------------------------ */
#define ORC_MLP_NPARAM 1347

/* round to float, then to bfloat16 (8 significant bits), ties to even */
static double bf16_round(double x)
{
    float f = (float)x;
    unsigned int u;
    memcpy(&u, &f, sizeof(u));
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf, NaN */
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    memcpy(&f, &u, sizeof(f));
    return (double)f;
}

static double to_float(double x) { return (double)(float)x; }

#define MLP_EPS 1e-6
#define MLP_BOUND 1.0 /* each classical weight is rescaled by at most e^{+-1} */

/* smoothness indicators of the three candidates (Jiang & Shu) */
static void weno5_beta(const double *x, double *beta)
{
    const double a0 = x[0] - 2.0 * x[1] + x[2], b0 = x[0] - 4.0 * x[1] + 3.0 * x[2];
    const double a1 = x[1] - 2.0 * x[2] + x[3], b1 = x[1] - x[3];
    const double a2 = x[2] - 2.0 * x[3] + x[4], b2 = 3.0 * x[2] - 4.0 * x[3] + x[4];
    beta[0] = 13.0 / 12.0 * a0 * a0 + 0.25 * b0 * b0;
    beta[1] = 13.0 / 12.0 * a1 * a1 + 0.25 * b1 * b1;
    beta[2] = 13.0 / 12.0 * a2 * a2 + 0.25 * b2 * b2;
}

/* omega[3] for the normalised stencil x[5] */
static void mlp_weights(const double *P, const double *x, double *omega)
{
    const double *W1 = P, *b1 = P + 160, *W2 = P + 192, *b2 = P + 1216, *W3 = P + 1248, *b3 = P + 1344;
    double xb[5], h1[32], h2[32], z[3];
    for (int j = 0; j < 5; ++j) xb[j] = bf16_round(x[j]);
    for (int h = 0; h < 32; ++h) {
        double a = bf16_round(b1[h]);
        for (int j = 0; j < 5; ++j) a += xb[j] * bf16_round(W1[j * 32 + h]);
        h1[h] = bf16_round(a > 0.0 ? a : 0.0);
    }
    for (int h = 0; h < 32; ++h) {
        double a = to_float(b2[h]);
        for (int g = 0; g < 32; ++g) a += h1[g] * bf16_round(W2[g * 32 + h]);
        h2[h] = bf16_round(a > 0.0 ? a : 0.0);
    }
    for (int k = 0; k < 3; ++k) {
        double a = to_float(b3[k]);
        for (int h = 0; h < 32; ++h) a += h2[h] * bf16_round(W3[h * 3 + k]);
        z[k] = a;
    }
    /* prior: the classical fifth-order WENO weights d_k / (eps + beta_k)^2 of
     * the normalised stencil (taken as float, as the device holds it) */
    double xf[5];
    for (int j = 0; j < 5; ++j) xf[j] = to_float(x[j]);
    double beta[3];
    weno5_beta(xf, beta);
    const double d[3] = {1.0 / 16.0, 10.0 / 16.0, 5.0 / 16.0};
    double zc[3];
    for (int k = 0; k < 3; ++k) zc[k] = MLP_BOUND * tanh(z[k]);
    double m = fmax(zc[0], fmax(zc[1], zc[2]));
    double a[3], sum = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double eb = MLP_EPS + beta[k];
        a[k] = d[k] * exp(zc[k] - m) / (eb * eb);
        sum += a[k];
    }
    for (int k = 0; k < 3; ++k) omega[k] = a[k] / sum;
}

/* learned interpolation of u = (u_{i-2}..u_{i+2}); returns 0 (and leaves
 * *out alone) if a weight is not finite, so that the caller falls back */
static int mlp_interp(const double *P, const double *u, double *out, double *omega)
{
    double s = 0.0;
    for (int j = 0; j < 5; ++j) s = fmax(s, fabs(u[j] - u[2]));
    const double r = s > 0.0 ? 1.0 / s : 0.0;
    double x[5];
    for (int j = 0; j < 5; ++j) x[j] = (u[j] - u[2]) * r;
    mlp_weights(P, x, omega);
    for (int k = 0; k < 3; ++k)
        if (!isfinite(omega[k])) return 0;
    const double sl = (3.0 * u[0] - 10.0 * u[1] + 15.0 * u[2]) / 8.0;
    const double sc = (-u[1] + 6.0 * u[2] + 3.0 * u[3]) / 8.0;
    const double sr = (3.0 * u[2] + 6.0 * u[3] - u[4]) / 8.0;
    /* sum_k omega_k S_k with the weights summing to one, written so that a
     * constant stencil is reproduced exactly */
    *out = sc + omega[0] * (sl - sc) + omega[2] * (sr - sc);
    return 1;
}

/* ------------------------------------------------------------------------ */
/* App. C: left-biased incremental-stencil WENO interpolation at i+1/2 from   */
/* u = (u_{i-2}, u_{i-1}, u_i, u_{i+1}, u_{i+2}).                              */
/* ------------------------------------------------------------------------ */
static double weno_is(const double *u, double eps)
{
    const double um2 = u[0], um1 = u[1], u0 = u[2], up1 = u[3], up2 = u[4];
    /* sub-stencil interpolants S0..S3 */
    const double s0 = 0.5 * (u0 + up1);
    const double s1 = 0.5 * (-um1 + 3.0 * u0);
    const double s2 = (3.0 * u0 + 6.0 * up1 - up2) / 8.0;
    const double s3 = (3.0 * um2 - 10.0 * um1 + 15.0 * u0) / 8.0;
    /* linear weights */
    const double d0 = 15.0 / 32.0, d1 = 5.0 / 32.0, d2 = 5.0 / 16.0, d3 = 1.0 / 16.0;
    /* smoothness indicators */
    const double b0 = (u0 - up1) * (u0 - up1);
    const double b1 = (um1 - u0) * (um1 - u0);
    const double t01a = um1 - 2.0 * u0 + up1, t01b = um1 - up1;
    const double b01 = 13.0 / 12.0 * t01a * t01a + 0.25 * t01b * t01b;
    const double t2a = u0 - 2.0 * up1 + up2, t2b = 3.0 * u0 - 4.0 * up1 + up2;
    const double b2 = 13.0 / 12.0 * t2a * t2a + 0.25 * t2b * t2b;
    const double t3a = um2 - 2.0 * um1 + u0, t3b = um2 - 4.0 * um1 + 3.0 * u0;
    const double b3 = 13.0 / 12.0 * t3a * t3a + 0.25 * t3b * t3b;
    const double t5a = up2 - 4.0 * up1 + 6.0 * u0 - 4.0 * um1 + um2;
    const double t5b = up2 - 2.0 * up1 + 2.0 * um1 - um2;
    const double tau5 = 13.0 / 12.0 * t5a * t5a + 0.25 * t5b * t5b;
    /* unnormalised weights eta_k */
    const double e0 = d0 * (1.0 + tau5 / (b0 + eps) * (tau5 / (b01 + eps)));
    const double e1 = d1 * (1.0 + tau5 / (b1 + eps) * (tau5 / (b01 + eps)));
    const double e2 = d2 * (1.0 + tau5 / (b2 + eps));
    const double e3 = d3 * (1.0 + tau5 / (b3 + eps));
    const double esum = e0 + e1 + e2 + e3;
    const double w0 = e0 / esum, w1 = e1 / esum, w2 = e2 / esum, w3 = e3 / esum;
    return w0 * s0 + w1 * s1 + w2 * s2 + w3 * s3;
}

/* ------------------------------------------------------------------------ */
/* App. D: projection matrices R_A^{-1}, R_A at a midpoint for direction n,   */
/* from arithmetic means of alpha_k rho_k, rho and c of the two nodes.        */
/* Wave order: (u-c), alpha_k rho_k waves (k = 0..N-1), tangential            */
/* velocities in increasing direction index, alpha_k (k = 0..N-2), (u+c).     */
/* ------------------------------------------------------------------------ */
static void projection_matrices(const orc_setup *s, int n, const orc_state *A, const orc_state *B,
                                double Rinv[ORC_MAXM][ORC_MAXM], double Rm[ORC_MAXM][ORC_MAXM])
{
    const int N = s->N, D = s->D, M = NCOMP(s);
    double arb[ORC_MAXN];
    for (int k = 0; k < N; ++k) arb[k] = 0.5 * (A->W[k] + B->W[k]);
    const double rb = 0.5 * (A->rho + B->rho);
    const double cb = 0.5 * (A->c + B->c);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) Rinv[i][j] = Rm[i][j] = 0.0;
    const int up = IE(s), un = IMOM(s, n);
    /* R^{-1}: rows are waves, columns the primitive slots */
    Rinv[0][un] = 1.0;
    Rinv[0][up] = -1.0 / (rb * cb);
    for (int k = 0; k < N; ++k) {
        Rinv[1 + k][k] = 1.0;
        Rinv[1 + k][up] = -arb[k] / (rb * cb * cb);
    }
    int t = 0;
    for (int d = 0; d < D; ++d)
        if (d != n) {
            Rinv[1 + N + t][IMOM(s, d)] = 1.0;
            ++t;
        }
    for (int k = 0; k < N - 1; ++k) Rinv[N + D + k][IAL(s, k)] = 1.0;
    Rinv[M - 1][un] = 1.0;
    Rinv[M - 1][up] = 1.0 / (rb * cb);
    /* R: rows are the primitive slots, columns the waves */
    for (int k = 0; k < N; ++k) {
        Rm[k][0] = -arb[k] / (2.0 * cb);
        Rm[k][1 + k] = 1.0;
        Rm[k][M - 1] = arb[k] / (2.0 * cb);
    }
    Rm[un][0] = 0.5;
    Rm[un][M - 1] = 0.5;
    t = 0;
    for (int d = 0; d < D; ++d)
        if (d != n) {
            Rm[IMOM(s, d)][1 + N + t] = 1.0;
            ++t;
        }
    Rm[up][0] = -rb * cb / 2.0;
    Rm[up][M - 1] = rb * cb / 2.0;
    for (int k = 0; k < N - 1; ++k) Rm[IAL(s, k)][N + D + k] = 1.0;
}

static void matvec(int M, double A[ORC_MAXM][ORC_MAXM], const double *x, double *y)
{
    for (int i = 0; i < M; ++i) {
        double acc = 0.0;
        for (int j = 0; j < M; ++j) acc += A[i][j] * x[j];
        y[i] = acc;
    }
}

static int all_finite(int n, const double *x)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

/* theta solving (1-theta) a + theta b = min(eps, a), used only when
 * b < min(eps, a) (Alg. 1-4); otherwise theta = 1 */
static double limiter_theta(double a, double b, double eps)
{
    const double m = fmin(eps, a);
    if (b < m) return (a - m) / (a - b);
    return 1.0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.3.2: positivity-preserving interpolation limiter (Alg. 1, Alg. 2    */
/* and the hard switch) for one interpolated primitive state Vt against the   */
/* node state of its side.  Reading: the limiter acts on the interpolated     */
/* primitive vector, so velocity and pressure are held fixed while partial    */
/* densities and volume fractions are blended; the hard switch replaces the   */
/* whole state by the node state and also fires on non-finite values.         */
/* Returns 1 if the hard switch fired.                                        */
/* ------------------------------------------------------------------------ */
static int interp_limit(const orc_setup *s, double *Vt, const orc_state *node, long long *cnt)
{
    const int N = s->N, M = NCOMP(s);
    /* Alg. 1: each partial density on its own */
    for (int k = 0; k < N; ++k) {
        const double a = node->W[k], b = Vt[k];
        const double th = limiter_theta(a, b, s->eps_i_ar);
        if (th < 1.0) {
            Vt[k] = (1.0 - th) * a + th * b;
            cnt[ORC_C_ALG1]++;
        }
    }
    /* Alg. 2: one common theta for all N volume fractions */
    double at[ORC_MAXN], asum = 0.0;
    for (int k = 0; k < N - 1; ++k) {
        at[k] = Vt[IAL(s, k)];
        asum += at[k];
    }
    at[N - 1] = 1.0 - asum;
    double th = 1.0;
    for (int k = 0; k < N; ++k) th = fmin(th, limiter_theta(node->alpha[k], at[k], s->eps_i_a));
    if (th < 1.0) {
        for (int k = 0; k < N - 1; ++k) Vt[IAL(s, k)] = (1.0 - th) * node->alpha[k] + th * Vt[IAL(s, k)];
        cnt[ORC_C_ALG2]++;
    }
    /* hard switch */
    orc_state lim;
    state_from_prim(s, Vt, &lim);
    int hs = !all_finite(M, Vt) || !isfinite(lim.rhoc2);
    for (int k = 0; k < N; ++k) {
        if (Vt[k] < fmin(s->hs_i_ar, node->W[k])) hs = 1;
        if (lim.alpha[k] < fmin(s->hs_i_a, node->alpha[k])) hs = 1;
    }
    if (lim.rhoc2 < fmin(s->hs_i_rc2, node->rhoc2)) hs = 1;
    if (hs) {
        for (int c = 0; c < M; ++c) Vt[c] = node->V[c];
        cnt[ORC_C_IHS]++;
    }
    return hs;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.3.2: quasi-positivity-preserving flux limiter (Alg. 3, Alg. 4 and   */
/* the hard switch) at the face between nodes i (L) and i+1 (R).  The         */
/* half-cell states are                                                        */
/*   W_i^{+}     = W_i     - 2 lambda (G^{-}_{i+1/2} - F_i)                     */
/*   W_{i+1}^{-} = W_{i+1} + 2 lambda (G^{+}_{i+1/2} - F_{i+1})                 */
/* for the high-order pair (Gm_ho, Gp_ho) and the first-order HLLC pair.      */
/* ------------------------------------------------------------------------ */
static void half_cell_states(const orc_setup *s, const orc_state *L, const orc_state *R, const double *FL,
                             const double *FR, double lam, const double *Gm, const double *Gp, double *Wp,
                             double *Wm)
{
    for (int c = 0; c < NCOMP(s); ++c) {
        Wp[c] = L->W[c] - 2.0 * lam * (Gm[c] - FL[c]);
        Wm[c] = R->W[c] + 2.0 * lam * (Gp[c] - FR[c]);
    }
}

static void flux_limit(const orc_setup *s, int n, const orc_state *L, const orc_state *R, double lam,
                       const double *Gm_ho, const double *Gp_ho, const double *Gm_lo, const double *Gp_lo,
                       double *Gm, double *Gp, long long *cnt)
{
    const int N = s->N, M = NCOMP(s);
    double FL[ORC_MAXM], FR[ORC_MAXM];
    flux_vec(s, n, L, 0, FL);
    flux_vec(s, n, R, 0, FR);
    double Wp_ho[ORC_MAXM], Wm_ho[ORC_MAXM], Wp_lo[ORC_MAXM], Wm_lo[ORC_MAXM];
    half_cell_states(s, L, R, FL, FR, lam, Gm_ho, Gp_ho, Wp_ho, Wm_ho);
    half_cell_states(s, L, R, FL, FR, lam, Gm_lo, Gp_lo, Wp_lo, Wm_lo);

    /* Alg. 3: one theta from all partial densities and all volume fractions */
    double th = 1.0;
    for (int k = 0; k < N; ++k) {
        th = fmin(th, limiter_theta(Wp_lo[k], Wp_ho[k], s->eps_f_ar));
        th = fmin(th, limiter_theta(Wm_lo[k], Wm_ho[k], s->eps_f_ar));
    }
    double ap_ho[ORC_MAXN], am_ho[ORC_MAXN], ap_lo[ORC_MAXN], am_lo[ORC_MAXN];
    alphas_of(s, Wp_ho, ap_ho);
    alphas_of(s, Wm_ho, am_ho);
    alphas_of(s, Wp_lo, ap_lo);
    alphas_of(s, Wm_lo, am_lo);
    for (int k = 0; k < N; ++k) {
        th = fmin(th, limiter_theta(ap_lo[k], ap_ho[k], s->eps_f_a));
        th = fmin(th, limiter_theta(am_lo[k], am_ho[k], s->eps_f_a));
    }
    if (th < 1.0) cnt[ORC_C_ALG3]++;
    double Gsm[ORC_MAXM], Gsp[ORC_MAXM];
    for (int c = 0; c < M; ++c) {
        Gsm[c] = (1.0 - th) * Gm_lo[c] + th * Gm_ho[c];
        Gsp[c] = (1.0 - th) * Gp_lo[c] + th * Gp_ho[c];
    }

    /* Alg. 4: theta from rho e-tilde, linear in the values (reading: as printed) */
    double Wsp[ORC_MAXM], Wsm[ORC_MAXM];
    half_cell_states(s, L, R, FL, FR, lam, Gsm, Gsp, Wsp, Wsm);
    const double thp = limiter_theta(rhoe_tilde(s, Wp_lo), rhoe_tilde(s, Wsp), s->eps_f_re);
    const double thm = limiter_theta(rhoe_tilde(s, Wm_lo), rhoe_tilde(s, Wsm), s->eps_f_re);
    const double th2 = fmin(thp, thm);
    if (th2 < 1.0) cnt[ORC_C_ALG4]++;
    double Gssm[ORC_MAXM], Gssp[ORC_MAXM];
    for (int c = 0; c < M; ++c) {
        Gssm[c] = (1.0 - th2) * Gm_lo[c] + th2 * Gsm[c];
        Gssp[c] = (1.0 - th2) * Gp_lo[c] + th2 * Gsp[c];
    }

    /* hard switch on the final half-cell states */
    double Wssp[ORC_MAXM], Wssm[ORC_MAXM];
    half_cell_states(s, L, R, FL, FR, lam, Gssm, Gssp, Wssp, Wssm);
    int hs = !all_finite(M, Gssm) || !all_finite(M, Gssp);
    double assp[ORC_MAXN], assm[ORC_MAXN];
    alphas_of(s, Wssp, assp);
    alphas_of(s, Wssm, assm);
    for (int k = 0; k < N; ++k) {
        if (Wssp[k] < fmin(s->hs_f_ar, Wp_lo[k])) hs = 1;
        if (Wssm[k] < fmin(s->hs_f_ar, Wm_lo[k])) hs = 1;
        if (assp[k] < fmin(s->hs_f_a, ap_lo[k])) hs = 1;
        if (assm[k] < fmin(s->hs_f_a, am_lo[k])) hs = 1;
    }
    const double rep = rhoe_tilde(s, Wssp), rem = rhoe_tilde(s, Wssm);
    if (!isfinite(rep) || !isfinite(rem)) hs = 1;
    if (rep < fmin(s->hs_f_re, rhoe_tilde(s, Wp_lo))) hs = 1;
    if (rem < fmin(s->hs_f_re, rhoe_tilde(s, Wm_lo))) hs = 1;
    if (hs) cnt[ORC_C_FHS]++;
    for (int c = 0; c < M; ++c) {
        Gm[c] = hs ? Gm_lo[c] : Gssm[c];
        Gp[c] = hs ? Gp_lo[c] : Gssp[c];
    }
}

/* Sec. 4.3.1: normalised fourth-order second derivative of the shock sensor,
 * for five nodes v[0..4] centred on v[2] */
static double sensor_ratio(const double *v)
{
    const double num = fabs(-v[0] + 16.0 * v[1] - 30.0 * v[2] + 16.0 * v[3] - v[4]);
    const double den = fabs(v[0] + 16.0 * v[1] + 30.0 * v[2] + 16.0 * v[3] + v[4]);
    /* reading: a zero denominator (possible only for a liquid in tension)
     * counts as a discontinuity when the numerator is not zero */
    if (den > 0.0) return num / den;
    return num > 0.0 ? 1.0 : 0.0;
}

/* sigma_{i+1/2}(u) = (sigma^+ + sigma^-)/2 from nodes u[0..5] = u_{i-2..i+3} */
static double sensor_sigma(const double *u)
{
    return 0.5 * (sensor_ratio(u + 1) + sensor_ratio(u));
}

/* ------------------------------------------------------------------------ */
/* One face i+1/2 in direction n from the six nodes i-2..i+3 (nodes[0..5]).   */
/* Produces the limited quasi-conservative pair G^{**,-}, G^{**,+}.           */
/* ------------------------------------------------------------------------ */
static double hllc4(const orc_setup *s, int n, const double *WL, const double *WR, double *G);

static void face_flux(const orc_setup *s, int n, const orc_state *nodes, double lam, double *Gm, double *Gp,
                      long long *cnt)
{
    const int N = s->N, M = NCOMP(s);
    const orc_state *L = &nodes[2], *R = &nodes[3];

    if (s->flags & ORC_FOUR_EQ) {
        hllc4(s, n, L->W, R->W, Gm);
        for (int c = 0; c < M; ++c) Gp[c] = Gm[c];
        return;
    }

    /* first-order HLLC on the node pair and its quasi-conservative pair (eq:G_pm) */
    double Glo[ORC_MAXM], Gm_lo[ORC_MAXM], Gp_lo[ORC_MAXM];
    const double ss_lo = hllc(s, n, L, R, Glo);
    for (int c = 0; c < M; ++c) Gm_lo[c] = Gp_lo[c] = Glo[c];
    for (int k = 0; k < N - 1; ++k) {
        Gm_lo[IAL(s, k)] = Glo[IAL(s, k)] - ss_lo * L->alpha[k];
        Gp_lo[IAL(s, k)] = Glo[IAL(s, k)] - ss_lo * R->alpha[k];
    }
    if (s->flags & ORC_FIRST_ORDER) {
        for (int c = 0; c < M; ++c) {
            Gm[c] = Gm_lo[c];
            Gp[c] = Gp_lo[c];
        }
        return;
    }

    /* App. D: characteristic projection of the six stencil nodes */
    double Rinv[ORC_MAXM][ORC_MAXM], Rm[ORC_MAXM][ORC_MAXM];
    projection_matrices(s, n, L, R, Rinv, Rm);
    double U[6][ORC_MAXM];
    for (int j = 0; j < 6; ++j) matvec(M, Rinv, nodes[j].V, U[j]);

    /* App. C: left-biased from i-2..i+2, right-biased mirrored from i+3..i-1 */
    double UL[ORC_MAXM], UR[ORC_MAXM];
    for (int m = 0; m < M; ++m) {
        const double l5[5] = {U[0][m], U[1][m], U[2][m], U[3][m], U[4][m]};
        const double r5[5] = {U[5][m], U[4][m], U[3][m], U[2][m], U[1][m]};
        double om[3];
        /* learned weights, with App. C as the fallback for non-finite weights */
        if (s->weights != ORC_W_MLP || !mlp_interp(s->mlp, l5, &UL[m], om)) UL[m] = weno_is(l5, s->eps_weno);
        if (s->weights != ORC_W_MLP || !mlp_interp(s->mlp, r5, &UR[m], om)) UR[m] = weno_is(r5, s->eps_weno);
    }
    double VL[ORC_MAXM], VR[ORC_MAXM];
    matvec(M, Rm, UL, VL);
    matvec(M, Rm, UR, VR);

    /* Sec. 4.3.2: interpolation limiter, left state against node i, right against node i+1 */
    if (!(s->flags & ORC_NO_LIMITERS)) {
        interp_limit(s, VL, L, cnt);
        interp_limit(s, VR, R, cnt);
    }

    /* HLLC on the interpolated states: midpoint flux G-tilde and velocity u-tilde */
    orc_state SL, SR;
    state_from_prim(s, VL, &SL);
    state_from_prim(s, VR, &SR);
    double Gt[ORC_MAXM];
    const double ut = hllc(s, n, &SL, &SR, Gt);

    /* Sec. 4.3.1: HCS reconstructed flux and velocity (eq:reconstructed_G, eq:reconstructed_vel) */
    const double psi = s->psi;
    const double ca = 75.0 * psi / 128.0 - 37.0 / 60.0;
    const double cb = 25.0 * psi / 256.0 - 2.0 / 15.0;
    const double cc = 3.0 * psi / 256.0 - 1.0 / 60.0;
    double Gn[6][ORC_MAXM], un[6], rh[6], pr[6];
    for (int j = 0; j < 6; ++j) {
        flux_vec(s, n, &nodes[j], 1, Gn[j]);
        un[j] = nodes[j].V[IMOM(s, n)];
        rh[j] = nodes[j].rho;
        pr[j] = nodes[j].V[IE(s)];
    }
    double Ghcs[ORC_MAXM];
    for (int c = 0; c < M; ++c)
        Ghcs[c] = psi * Gt[c] - ca * (Gn[2][c] + Gn[3][c]) + cb * (Gn[1][c] + Gn[4][c]) - cc * (Gn[0][c] + Gn[5][c]);
    const double uhcs = psi * ut - ca * (un[2] + un[3]) + cb * (un[1] + un[4]) - cc * (un[0] + un[5]);

    /* shock sensor and blending (eq:flux_blending, eq:velocity_blending) */
    double sig = 0.0;
    if (!(s->flags & ORC_NO_BLEND)) {
        const double sr = sensor_sigma(rh), sp = sensor_sigma(pr);
        sig = tanh(s->Cs * pow(sr * sp, s->qexp));
    }
    double Gh[ORC_MAXM];
    for (int c = 0; c < M; ++c) Gh[c] = sig * Gt[c] + (1.0 - sig) * Ghcs[c];
    const double uh = sig * ut + (1.0 - sig) * uhcs;

    /* high-order quasi-conservative pair: alpha slots take alpha of node i (-) or i+1 (+) */
    double Gm_ho[ORC_MAXM], Gp_ho[ORC_MAXM];
    for (int c = 0; c < M; ++c) Gm_ho[c] = Gp_ho[c] = Gh[c];
    for (int k = 0; k < N - 1; ++k) {
        Gm_ho[IAL(s, k)] = Gh[IAL(s, k)] - uh * L->alpha[k];
        Gp_ho[IAL(s, k)] = Gh[IAL(s, k)] - uh * R->alpha[k];
    }
    if (s->flags & ORC_NO_LIMITERS) {
        for (int c = 0; c < M; ++c) {
            Gm[c] = Gm_ho[c];
            Gp[c] = Gp_ho[c];
        }
        return;
    }
    flux_limit(s, n, L, R, lam, Gm_ho, Gp_ho, Gm_lo, Gp_lo, Gm, Gp, cnt);
}

/* ghost index map: transmissive copies the edge cell, periodic wraps */
static int map_index(const orc_setup *s, int d, int i)
{
    const int n = s->n[d];
    if (i < 0) return s->bc_lo[d] == ORC_PERIODIC ? ((i % n) + n) % n : 0;
    if (i >= n) return s->bc_hi[d] == ORC_PERIODIC ? i % n : n - 1;
    return i;
}

static long cell_index(const orc_setup *s, const int *ijk)
{
    return ((long)ijk[2] * s->n[1] + ijk[1]) * s->n[0] + ijk[0];
}

static void load_state(const orc_setup *s, const double *W, long cell, orc_state *st)
{
    double w[ORC_MAXM];
    const long nc = NCELL(s);
    for (int c = 0; c < NCOMP(s); ++c) w[c] = W[(long)c * nc + cell];
    state_from_cons(s, w, st);
}

/* the two dimensions other than d, in increasing order */
static void other_dims(int d, int *a, int *b)
{
    *a = d == 0 ? 1 : 0;
    *b = d == 2 ? 1 : 2;
}

/* node i along dimension d of the line through ijk: a cell, or a ghost node
 * (index map for transmissive and periodic sides; for a Dirichlet side every
 * ghost node is the given state of the line) */
static void load_node(const orc_setup *s, const double *W, int d, int *ijk, int i, orc_state *st)
{
    const int side = i < 0 ? 0 : (i >= s->n[d] ? 1 : -1);
    if (side >= 0 && (side == 0 ? s->bc_lo[d] : s->bc_hi[d]) == ORC_DIRICHLET) {
        int a, b;
        other_dims(d, &a, &b);
        const long nf = (long)s->n[a] * s->n[b], t = ijk[a] + (long)s->n[a] * ijk[b];
        double w[ORC_MAXM];
        for (int c = 0; c < NCOMP(s); ++c) w[c] = s->bnd[d][side][(long)c * nf + t];
        state_from_cons(s, w, st);
        return;
    }
    ijk[d] = map_index(s, d, i);
    load_state(s, W, cell_index(s, ijk), st);
}

/* ------------------------------------------------------------------------ */
/* Semi-discrete right-hand side L(W) (eq:semi_W_G_pm_eqn):                   */
/*   L_i = - sum_d (G^{**,-}_{i+1/2} - G^{**,+}_{i-1/2}) / dx_d                */
/* lam[d] is the lambda_d of the flux limiter (Sec. 4.1.2).                    */
/* ------------------------------------------------------------------------ */
void orc_rhs(const orc_setup *s, const double *W, const double *lam, double *Lout, long long *cnt_out)
{
    const int M = NCOMP(s);
    const long nc = NCELL(s);
    for (long i = 0; i < (long)M * nc; ++i) Lout[i] = 0.0;
    long long cnt_total[ORC_NCOUNT] = {0};
    for (int d = 0; d < s->D; ++d) {
        const int nd = s->n[d];
        const int o1 = (d + 1) % 3, o2 = (d + 2) % 3;
        const long nlines = (long)s->n[o1] * s->n[o2];
#pragma omp parallel
        {
            long long cnt[ORC_NCOUNT] = {0};
            double *Gm = malloc(sizeof(double) * (size_t)(nd + 1) * M);
            double *Gp = malloc(sizeof(double) * (size_t)(nd + 1) * M);
            orc_state nodes[6];
#pragma omp for schedule(dynamic, 4)
            for (long line = 0; line < nlines; ++line) {
                int ijk[3];
                ijk[o1] = (int)(line % s->n[o1]);
                ijk[o2] = (int)(line / s->n[o1]);
                /* faces f = -1 .. nd-1 between nodes f and f+1, stored at f+1 */
                for (int f = -1; f < nd; ++f) {
                    for (int j = 0; j < 6; ++j) load_node(s, W, d, ijk, f - 2 + j, &nodes[j]);
                    face_flux(s, d, nodes, lam[d], Gm + (size_t)(f + 1) * M, Gp + (size_t)(f + 1) * M, cnt);
                }
                for (int i = 0; i < nd; ++i) {
                    ijk[d] = i;
                    const long cell = cell_index(s, ijk);
                    for (int c = 0; c < M; ++c)
                        Lout[(long)c * nc + cell] -= (Gm[(size_t)(i + 1) * M + c] - Gp[(size_t)i * M + c]) / s->dx[d];
                }
            }
            free(Gm);
            free(Gp);
#pragma omp critical
            for (int k = 0; k < ORC_NCOUNT; ++k) cnt_total[k] += cnt[k];
        }
    }
    if (cnt_out)
        for (int k = 0; k < ORC_NCOUNT; ++k) cnt_out[k] += cnt_total[k];
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.2: infinite-rate thermal relaxation of one cell.  Species 0 is the  */
/* only stiffened gas; the others are ideal gases.                             */
/*   A p^2 + B p + C = 0 (eq:Ap_Bp_Cp_1..3), p* the positive root (eq:p_relax)  */
/*   T* from the energy form (eq:T_relax_e)                                    */
/*   rho_k* = (p* + pinf_k)/((gamma_k - 1) cv_k T*) (eq:rho_k_thermally_relaxed) */
/*   alpha_k* = alpha_k rho_k / rho_k*                                         */
/* Readings: for B > 0 the positive root is taken in the algebraically equal   */
/* form 2C/(-B - sqrt(B^2 - 4AC)) to avoid cancellation; alpha_k* of the first */
/* N-1 species are stored as computed (alpha_N stays 1 minus their sum), with  */
/* no renormalisation: rescaling them would move the liquid fraction by the    */
/* round-off of the gas fractions, which p_inf amplifies in the pressure.      */
/* A cell with rho e-tilde <= 0 or no positive root is left unchanged and      */
/* returns 1.                                                                  */
/* ------------------------------------------------------------------------ */
/* p* and T* of the relaxed state (eq:p_relax, eq:T_relax_e); returns 1 for a
 * state with rho e-tilde <= 0 or without a positive root */
static int relaxed_pT(const orc_setup *s, const double *W, double *p_out, double *T_out)
{
    const int N = s->N;
    double rho = 0.0;
    for (int k = 0; k < N; ++k) rho += W[k];
    double Y[ORC_MAXN], cvb = 0.0, cpb = 0.0, qb = 0.0;
    for (int k = 0; k < N; ++k) {
        Y[k] = W[k] / rho;
        cvb += Y[k] * s->cv[k];
        cpb += Y[k] * s->gamma[k] * s->cv[k];
        qb += Y[k] * s->q[k];
    }
    double mom2 = 0.0;
    for (int d = 0; d < s->D; ++d) mom2 += W[IMOM(s, d)] * W[IMOM(s, d)];
    const double rhoe_t = W[IE(s)] - 0.5 * mom2 / rho - rho * qb; /* rho (e - qbar) */
    if (!(rhoe_t > 0.0) || !(rho > 0.0)) return 1;
    const double p1 = s->pinf[0];
    const double R1 = s->gamma[0] * s->cv[0] - s->cv[0]; /* c_p1 - c_v1 */
    const double A = cvb;
    const double B = -(rhoe_t * (cpb - cvb) - p1 * cvb - p1 * Y[0] * R1);
    const double C = -rhoe_t * p1 * ((cpb - cvb) - Y[0] * R1);
    const double disc = B * B - 4.0 * A * C;
    double p;
    if (B <= 0.0)
        p = (-B + sqrt(disc)) / (2.0 * A);
    else
        p = 2.0 * C / (-B - sqrt(disc));
    if (!(p > 0.0) || !isfinite(p)) return 1;
    const double e_t = rhoe_t / rho;
    const double T = e_t / (Y[0] * (p + s->gamma[0] * p1) * s->cv[0] / (p + p1) + cvb - Y[0] * s->cv[0]);
    if (!(T > 0.0) || !isfinite(T)) return 1;
    *p_out = p;
    *T_out = T;
    return 0;
}

int orc_relax_cell(const orc_setup *s, double *W, double *pT)
{
    double p, T;
    if (relaxed_pT(s, W, &p, &T)) return 1;
    for (int k = 0; k < s->N - 1; ++k) {
        const double rho_k = (p + s->pinf[k]) / ((s->gamma[k] - 1.0) * s->cv[k] * T);
        W[IAL(s, k)] = W[k] / rho_k;
    }
    if (pT) {
        pT[0] = p;
        pT[1] = T;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 3: equation of state and sound speed of the four-equation HRM.        */
/* p and T are the relaxed p*, T* of the conservative vector without the      */
/* volume fractions.  c^2 = sum_k Y_k Psi_k + Gamma p / rho (eq:4_eqn_sos),    */
/* with Psi_k = dp/d(alpha_k rho_k) at fixed e and Gamma = (1/rho) dp/de from  */
/* the implicit derivative of A_p p^2 + B_p p + C_p = 0 (Sec. 4.2):            */
/*   dp = -(dA_p p^2 + dB_p p + dC_p) / (2 A_p p + B_p),                       */
/* where, with rho = sum_k alpha_k rho_k, Y_k = alpha_k rho_k / rho and         */
/* rho (e - qbar) = sum_k alpha_k rho_k (e - q_k),                              */
/*   A_p = cvbar,  B_p = -[rho (e - qbar) G - pinf_1 cvbar - pinf_1 Y_1 R_1],    */
/*   C_p = -rho (e - qbar) pinf_1 (G - Y_1 R_1),  G = cpbar - cvbar,            */
/*   R_1 = c_p1 - c_v1, and                                                    */
/*   d cvbar / d(alpha_k rho_k) = (c_vk - cvbar)/rho,                          */
/*   d G / d(alpha_k rho_k) = (R_k - G)/rho,  d Y_1 / d(alpha_k rho_k) =        */
/*   (delta_k1 - Y_1)/rho,  d rho (e - qbar) / d(alpha_k rho_k) = e - q_k,      */
/*   d rho (e - qbar) / de = rho.                                              */
/* out = (p, T, c).  Returns 1 (out set to NaN) where relaxed_pT fails.        */
/* ------------------------------------------------------------------------ */
static int hrm_eos(const orc_setup *s, const double *W, double *out)
{
    const int N = s->N;
    double p, T;
    if (relaxed_pT(s, W, &p, &T)) {
        out[0] = out[1] = out[2] = NAN;
        return 1;
    }
    double rho = 0.0, mom2 = 0.0;
    for (int k = 0; k < N; ++k) rho += W[k];
    for (int d = 0; d < s->D; ++d) mom2 += W[IMOM(s, d)] * W[IMOM(s, d)];
    const double e = (W[IE(s)] - 0.5 * mom2 / rho) / rho; /* specific internal energy */
    double Y[ORC_MAXN] = {0}, Rk[ORC_MAXN] = {0}, cvb = 0.0, cpb = 0.0, re = 0.0;
    for (int k = 0; k < N; ++k) {
        Y[k] = W[k] / rho;
        Rk[k] = s->gamma[k] * s->cv[k] - s->cv[k];
        cvb += Y[k] * s->cv[k];
        cpb += Y[k] * s->gamma[k] * s->cv[k];
        re += W[k] * (e - s->q[k]);
    }
    const double p1 = s->pinf[0], R1 = Rk[0];
    const double A = cvb, G = cpb - cvb, H = G - Y[0] * R1;
    const double B = -(re * G - p1 * cvb - p1 * Y[0] * R1);
    const double den = 2.0 * A * p + B;
    double c2 = 0.0;
    for (int k = 0; k < N; ++k) {
        const double dA = (s->cv[k] - A) / rho;
        const double dG = (Rk[k] - G) / rho;
        const double dY1 = ((k == 0 ? 1.0 : 0.0) - Y[0]) / rho;
        const double dre = e - s->q[k];
        const double dB = -(dre * G + re * dG - p1 * dA - p1 * R1 * dY1);
        const double dC = -p1 * (dre * H + re * (dG - R1 * dY1));
        const double Psi = -(dA * p * p + dB * p + dC) / den;
        c2 += Y[k] * Psi;
    }
    const double dBde = -rho * G, dCde = -p1 * rho * H;
    const double Gamma = -(dBde * p + dCde) / den / rho;
    c2 += Gamma * p / rho;
    out[0] = p;
    out[1] = T;
    out[2] = c2 > 0.0 ? sqrt(c2) : NAN;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* First-order HLLC for the four-equation HRM solved directly (the reference */
/* scheme of the comparisons of Sec. 5.4 and App. A).  Reading: the solver of */
/* Sec. 4.1.1 applied to (alpha_k rho_k, rho u, E), with the HRM pressure and  */
/* sound speed of hrm_eos in place of the five-equation ones, the same wave-   */
/* speed estimates and sign(0) = 0.  The volume-fraction slots of G are zero.  */
/* Returns s_*.                                                                */
/* ------------------------------------------------------------------------ */
static double hllc4(const orc_setup *s, int n, const double *WL, const double *WR, double *G)
{
    const int N = s->N, D = s->D, M = NCOMP(s);
    double rho[2], u[2][3], p[2], c[2];
    const double *Wk[2] = {WL, WR};
    for (int side = 0; side < 2; ++side) {
        double pTc[3];
        hrm_eos(s, Wk[side], pTc);
        rho[side] = 0.0;
        for (int k = 0; k < N; ++k) rho[side] += Wk[side][k];
        for (int d = 0; d < D; ++d) u[side][d] = Wk[side][IMOM(s, d)] / rho[side];
        p[side] = pTc[0];
        c[side] = pTc[2];
    }
    const double uL = u[0][n], uR = u[1][n];
    const double ubar = 0.5 * (uL + uR), cbar = 0.5 * (c[0] + c[1]);
    const double sL = fmin(ubar - cbar, uL - c[0]);
    const double sR = fmax(ubar + cbar, uR + c[1]);
    const double sstar = (p[1] - p[0] + rho[0] * uL * (sL - uL) - rho[1] * uR * (sR - uR)) /
                         (rho[0] * (sL - uL) - rho[1] * (sR - uR));
    double Ws[2][ORC_MAXM], F[2][ORC_MAXM];
    for (int side = 0; side < 2; ++side) {
        const double *W = Wk[side];
        const double sK = side == 0 ? sL : sR, uK = u[side][n], pK = p[side];
        const double chi = (sK - uK) / (sK - sstar);
        for (int k = 0; k < N; ++k) {
            Ws[side][k] = chi * W[k];
            F[side][k] = W[k] * uK;
        }
        for (int d = 0; d < D; ++d) {
            Ws[side][IMOM(s, d)] = d == n ? chi * rho[side] * sstar : chi * rho[side] * u[side][d];
            F[side][IMOM(s, d)] = W[IMOM(s, d)] * uK + (d == n ? pK : 0.0);
        }
        Ws[side][IE(s)] = chi * (W[IE(s)] + (sstar - uK) * (rho[side] * sstar + pK / (sK - uK)));
        F[side][IE(s)] = (W[IE(s)] + pK) * uK;
    }
    const double sm = fmin(0.0, sL), sp = fmax(0.0, sR);
    const double sg = sstar > 0.0 ? 1.0 : (sstar < 0.0 ? -1.0 : 0.0);
    for (int c = 0; c <= IE(s); ++c)
        G[c] = 0.5 * (1.0 + sg) * (F[0][c] + sm * (Ws[0][c] - WL[c])) +
               0.5 * (1.0 - sg) * (F[1][c] + sp * (Ws[1][c] - WR[c]));
    for (int c = IE(s) + 1; c < M; ++c) G[c] = 0.0;
    return sstar;
}

/* relaxation of every cell of a state array (hot-path step a11) */
void orc_relax(const orc_setup *s, double *W, long long *cnt)
{
    const int M = NCOMP(s);
    const long nc = NCELL(s);
    long long bad = 0;
#pragma omp parallel for reduction(+ : bad)
    for (long cell = 0; cell < nc; ++cell) {
        double w[ORC_MAXM];
        for (int c = 0; c < M; ++c) w[c] = W[(long)c * nc + cell];
        if (orc_relax_cell(s, w, 0)) {
            bad++;
            continue;
        }
        for (int k = 0; k < s->N - 1; ++k) W[(long)IAL(s, k) * nc + cell] = w[IAL(s, k)];
    }
    if (cnt) cnt[ORC_C_RELAX_BAD] += bad;
}

/* Sec. 4.1.2: max over cells of |u_d| + c for each direction d (five-equation
 * c; the HRM c of hrm_eos when the four-equation model is solved directly) */
void orc_max_wavespeed(const orc_setup *s, const double *W, double *out)
{
    const long nc = NCELL(s);
    for (int d = 0; d < s->D; ++d) out[d] = 0.0;
    for (long cell = 0; cell < nc; ++cell) {
        orc_state st;
        load_state(s, W, cell, &st);
        double c = st.c;
        if (s->flags & ORC_FOUR_EQ) {
            double pTc[3];
            hrm_eos(s, st.W, pTc);
            c = pTc[2];
        }
        for (int d = 0; d < s->D; ++d) {
            const double v = fabs(st.V[IMOM(s, d)]) + c;
            if (v > out[d] || !(v == v)) out[d] = v;
        }
    }
    /* reading: the Dirichlet ghost states count for the direction normal to their face */
    for (int d = 0; d < s->D; ++d)
        for (int side = 0; side < 2; ++side) {
            if ((side == 0 ? s->bc_lo[d] : s->bc_hi[d]) != ORC_DIRICHLET) continue;
            int a, b;
            other_dims(d, &a, &b);
            const long nf = (long)s->n[a] * s->n[b];
            for (long t = 0; t < nf; ++t) {
                double w[ORC_MAXM], c;
                orc_state st;
                for (int k = 0; k < NCOMP(s); ++k) w[k] = s->bnd[d][side][(long)k * nf + t];
                state_from_cons(s, w, &st);
                c = st.c;
                if (s->flags & ORC_FOUR_EQ) {
                    double pTc[3];
                    hrm_eos(s, st.W, pTc);
                    c = pTc[2];
                }
                const double v = fabs(st.V[IMOM(s, d)]) + c;
                if (v > out[d] || !(v == v)) out[d] = v;
            }
        }
}

/* Sec. 4.1.2 multi-D time step: tau_d = max(|u_d|+c)/dx_d, dt = CFL/sum tau,
 * sigma_d = tau_d/sum tau, lambda_d = dt/(sigma_d dx_d).  With dt_fixed > 0
 * the step is fixed and only sigma_d comes from the state.
 * out = (dt, lambda_0, ..., lambda_{D-1}). */
void orc_dt(const orc_setup *s, const double *maxspeed, double cfl, double dt_fixed, double *out)
{
    double tau[3], tsum = 0.0;
    for (int d = 0; d < s->D; ++d) {
        tau[d] = maxspeed[d] / s->dx[d];
        tsum += tau[d];
    }
    const double dt = dt_fixed > 0.0 ? dt_fixed : cfl / tsum;
    out[0] = dt;
    for (int d = 0; d < s->D; ++d) {
        const double sigma = tau[d] / tsum;
        out[1 + d] = dt / (sigma * s->dx[d]);
    }
}

/* Shu-Osher combination of one explicit stage with a given right-hand side,
 * followed by the relaxation (Sec. 4.4: relaxation after every stage):
 *   W_out = a W^n + b (W^(s) + dt L)  then relax(W_out) if relax != 0 */
void orc_combine_ab(const orc_setup *s, double a, double b, const double *Wn, const double *Ws, const double *L,
                    double dt, double *Wout, int relax, long long *cnt)
{
    const long nv = (long)NCOMP(s) * NCELL(s);
    for (long i = 0; i < nv; ++i) Wout[i] = a * Wn[i] + b * (Ws[i] + dt * L[i]);
    if (relax) orc_relax(s, Wout, cnt);
}

/* SSP-RK3 of Shu and Osher (Sec. 4.4, Sec. 5), stage = 0, 1, 2:
 *   W1 = W^n + dt L(W^n)
 *   W2 = 3/4 W^n + 1/4 (W1 + dt L(W1))
 *   W^{n+1} = 1/3 W^n + 2/3 (W2 + dt L(W2)) */
static const double RK3_A[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
static const double RK3_B[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};

void orc_combine(const orc_setup *s, int stage, const double *Wn, const double *Ws, const double *L, double dt,
                 double *Wout, int relax, long long *cnt)
{
    orc_combine_ab(s, RK3_A[stage], RK3_B[stage], Wn, Ws, L, dt, Wout, relax, cnt);
}

/* one SSP-RK3 stage: L(W^(s)) from the spatial operator, then the combination */
void orc_stage(const orc_setup *s, int stage, const double *Wn, const double *Ws, double *Wout, double dt,
               const double *lam, int relax, long long *cnt)
{
    const long nv = (long)NCOMP(s) * NCELL(s);
    double *L = malloc(sizeof(double) * (size_t)nv);
    orc_rhs(s, Ws, lam, L, cnt);
    orc_combine(s, stage, Wn, Ws, L, dt, Wout, relax, cnt);
    free(L);
}

/* ---------------------------- unit entry points -------------------------- */

/* out = (rho, p, rho c^2, c, rho e-tilde, u_0..u_{D-1}) of one conservative vector */
void orc_prim(const orc_setup *s, const double *W, double *out)
{
    orc_state st;
    state_from_cons(s, W, &st);
    out[0] = st.rho;
    out[1] = st.V[IE(s)];
    out[2] = st.rhoc2;
    out[3] = st.c;
    out[4] = st.rhoe_t;
    for (int d = 0; d < s->D; ++d) out[5 + d] = st.V[IMOM(s, d)];
}

void orc_cons_from_prim(const orc_setup *s, const double *V, double *W)
{
    orc_state st;
    state_from_prim(s, V, &st);
    for (int c = 0; c < NCOMP(s); ++c) W[c] = st.W[c];
}

double orc_weno(const double *u5, double eps) { return weno_is(u5, eps); }

/* learned interpolation of one stencil; omega[3] receives the weights;
 * returns 0 if they are not finite (*out then untouched) */
int orc_mlp_interp(const double *params, const double *u5, double *out, double *omega)
{
    return mlp_interp(params, u5, out, omega);
}

double orc_bf16(double x) { return bf16_round(x); }

double orc_sensor(const double *u6) { return sensor_sigma(u6); }

/* out = (p, T, c) of the four-equation HRM; returns 1 for a state outside G */
int orc_hrm_eos(const orc_setup *s, const double *W, double *out) { return hrm_eos(s, W, out); }

double orc_hllc4(const orc_setup *s, int n, const double *WL, const double *WR, double *G)
{
    return hllc4(s, n, WL, WR, G);
}

double orc_hllc(const orc_setup *s, int n, const double *WL, const double *WR, double *G)
{
    orc_state L, R;
    state_from_cons(s, WL, &L);
    state_from_cons(s, WR, &R);
    return hllc(s, n, &L, &R, G);
}

/* characteristic projection of a primitive vector and back, for the pair of
 * nodes (WA, WB) that defines the midpoint averages */
void orc_project(const orc_setup *s, int n, const double *WA, const double *WB, const double *V, double *U,
                 double *Vback)
{
    orc_state A, B;
    state_from_cons(s, WA, &A);
    state_from_cons(s, WB, &B);
    double Rinv[ORC_MAXM][ORC_MAXM], Rm[ORC_MAXM][ORC_MAXM];
    projection_matrices(s, n, &A, &B, Rinv, Rm);
    matvec(NCOMP(s), Rinv, V, U);
    matvec(NCOMP(s), Rm, U, Vback);
}

/* face pair from six conservative node vectors W6[j*M + c], j = 0..5 */
void orc_face(const orc_setup *s, int n, const double *W6, double lam, double *Gm, double *Gp, long long *cnt)
{
    orc_state nodes[6];
    for (int j = 0; j < 6; ++j) state_from_cons(s, W6 + (size_t)j * NCOMP(s), &nodes[j]);
    face_flux(s, n, nodes, lam, Gm, Gp, cnt);
}

int orc_interp_limit(const orc_setup *s, double *Vt, const double *Wnode, long long *cnt)
{
    orc_state node;
    state_from_cons(s, Wnode, &node);
    return interp_limit(s, Vt, &node, cnt);
}

void orc_flux_limit(const orc_setup *s, int n, const double *WL, const double *WR, double lam,
                    const double *Gm_ho, const double *Gp_ho, const double *Gm_lo, const double *Gp_lo,
                    double *Gm, double *Gp, long long *cnt)
{
    orc_state L, R;
    state_from_cons(s, WL, &L);
    state_from_cons(s, WR, &R);
    flux_limit(s, n, &L, &R, lam, Gm_ho, Gp_ho, Gm_lo, Gp_lo, Gm, Gp, cnt);
}

void orc_hcs_coeffs(double psi, double *out)
{
    out[0] = 75.0 * psi / 128.0 - 37.0 / 60.0;
    out[1] = 25.0 * psi / 256.0 - 2.0 / 15.0;
    out[2] = 3.0 * psi / 256.0 - 1.0 / 60.0;
}

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
