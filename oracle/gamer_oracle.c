/*
 * gamer_oracle.c -- plain FP64 CPU oracle for one MUSCL-Hancock + Roe step
 * on batches of ghost-padded 16^3 patch groups.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path
 * (the HIP library and its Python binding) never links, loads or calls it,
 * and the two share no code: no headers, helpers, tables or constants.
 *
 * What it computes (paper, Sec. 2 "Extension I: hydrodynamic solver"): the
 * MUSCL-Hancock method in its four steps -- spatial data reconstruction,
 * half-step prediction, Riemann solver, full-step update -- applied unsplit
 * to the 3D Euler equations, with Roe's approximate Riemann solver and a
 * five-point stencil in each direction (hence two ghost cells per side).
 * The paper names the method and cites Toro (2009) and Roe (1981) for it;
 * the per-step formulas below follow those sources:
 *   - reconstruction and the conservative Hancock predictor: Toro 2009,
 *     Sec. 14.4 (1D), summed over the three directions for the unsplit step;
 *   - Roe's solver for the 3D Euler equations: Toro 2009, Sec. 11.2
 *     (eigenvalues, right eigenvectors, wave strengths);
 *   - entropy fix: Harten & Hyman (1983), as in Toro 2009, Sec. 11.4;
 *   - HLLE fallback with Einfeldt's signal speeds (Einfeldt 1988).
 * Where the paper is silent (primitive-variable generalised minmod with
 * parameter theta, the two positivity fallbacks, the CFL form, the flux
 * planes written out) the reading taken is stated at the function that
 * implements it.
 *
 * Everything is plain loops in IEEE double, one stage after another, in the
 * order the method states them.  Build with -O2 -ffp-contract=off and no
 * fast-math.  OpenMP (optional) only splits the independent groups.
 *
 * Pinning: every exported stage is checked by the CPU tests against values
 * fixed by the mathematics (uniform-state preservation, the limiter truth
 * table, exact linear reconstruction, the Roe property and eigen-structure,
 * consistency, stationary contact, conservation, flux-plane telescoping,
 * mirror symmetry, Sod against the exact Riemann solution, second-order
 * convergence, closed-form CFL, math.fsum for the sums).
 *
 * Layouts (x fastest everywhere):
 *   padded group   [5][20][20][20]   cell (i,j,k), i,j,k in -2..17
 *   interior group [5][16][16][16]   cell (i,j,k), i,j,k in 0..15
 *   flux planes    [3 dir][3 plane][5][16][16]; planes at face index 0, 8, 16;
 *                  transverse order (k,j) for x, (k,i) for y, (j,i) for z.
 *   variables      (rho, m_x, m_y, m_z, E) conserved, (rho, u, v, w, p) primitive.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NI 16          /* interior cells per axis */
#define NGH 2          /* ghost cells per side */
#define NP 20          /* padded cells per axis */
#define NF 18          /* face-state index range -1..16 */
#define NV 5

/* padded cell (v,i,j,k), i,j,k in -2..17 */
static size_t ip(int v, int i, int j, int k) {
    return (((size_t)v * NP + (size_t)(k + NGH)) * NP + (size_t)(j + NGH)) * NP + (size_t)(i + NGH);
}
/* interior cell (v,i,j,k), i,j,k in 0..15 */
static size_t ii(int v, int i, int j, int k) {
    return (((size_t)v * NI + (size_t)k) * NI + (size_t)j) * NI + (size_t)i;
}
/* face-state-set cell (v,i,j,k), i,j,k in -1..16 */
static size_t is(int v, int i, int j, int k) {
    return (((size_t)v * NF + (size_t)(k + 1)) * NF + (size_t)(j + 1)) * NF + (size_t)(i + 1);
}

static int oracle_threads = 1;

void gamer_oracle_set_threads(int n) { oracle_threads = n > 0 ? n : 1; }

int gamer_oracle_get_threads(void) { return oracle_threads; }

/* Test hook, outside the method's arithmetic: a count of the fallback
 * decisions that sit within a relative margin tau of their threshold, so a
 * test can bound how many decisions another implementation, rounding
 * differently, may legitimately take the other way.  A positivity decision on
 * a state U is counted when |2 rho E - |m|^2| <= tau (|2 rho E| + |m|^2), the
 * sign of p (the sign of rho is not counted: no state here has rho near 0);
 * the Roe solver's decision on a2 > 0 when |a2| <= tau (gamma - 1)(|H| +
 * |u|^2 / 2).  tau < 0 (the default)
 * turns counting off.  The counter is a plain global: use it with one thread
 * (gamer_oracle_set_threads(1)). */
static double margin_tau = -1.0;
static long long margin_hits = 0;

void gamer_oracle_margin_reset(double tau) {
    margin_tau = tau;
    margin_hits = 0;
}

long long gamer_oracle_margin_hits(void) { return margin_hits; }

void gamer_oracle_margin_note_state(const double *U) {
    if (margin_tau < 0.0) return;
    double q = 2.0 * U[0] * U[4], m2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
    if (fabs(q - m2) <= margin_tau * (fabs(q) + m2)) ++margin_hits;
}

static void margin_note_a2(double a2, double H, double q2, double g) {
    if (margin_tau < 0.0) return;
    if (fabs(a2) <= margin_tau * (g - 1.0) * (fabs(H) + 0.5 * q2)) ++margin_hits;
}

/* ---------------------------------------------------------------------- */
/* Ideal-gas state conversions (Toro 2009, Sec. 3.1).                      */

/* W = (rho, u, v, w, p) from U = (rho, m_x, m_y, m_z, E);
 * p = (gamma-1) (E - rho |u|^2 / 2). */
void gamer_oracle_prim_from_cons(const double *U, double g, double *W) {
    double rho = U[0];
    double u = U[1] / rho, v = U[2] / rho, w = U[3] / rho;
    W[0] = rho;
    W[1] = u;
    W[2] = v;
    W[3] = w;
    W[4] = (g - 1.0) * (U[4] - 0.5 * rho * (u * u + v * v + w * w));
}

/* U from W; E = p/(gamma-1) + rho |u|^2 / 2. */
void gamer_oracle_cons_from_prim(const double *W, double g, double *U) {
    double rho = W[0];
    U[0] = rho;
    U[1] = rho * W[1];
    U[2] = rho * W[2];
    U[3] = rho * W[3];
    U[4] = W[4] / (g - 1.0) + 0.5 * rho * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
}

/* Physical flux of U along direction d (0 = x, 1 = y, 2 = z):
 * F_d = (m_d, m u_d + p e_d, (E + p) u_d)  (Toro 2009, Sec. 3.2). */
void gamer_oracle_phys_flux(const double *U, int d, double g, double *F) {
    double W[NV];
    gamer_oracle_prim_from_cons(U, g, W);
    double un = W[1 + d];
    F[0] = U[1 + d];
    F[1] = U[1] * un;
    F[2] = U[2] * un;
    F[3] = U[3] * un;
    F[1 + d] += W[4];
    F[4] = (U[4] + W[4]) * un;
}

/* ---------------------------------------------------------------------- */
/* Step 1: spatial data reconstruction.                                    */

/* Generalised minmod slope of the two one-sided differences a = q_c - q_{c-1}
 * and b = q_{c+1} - q_c: zero at an extremum (a b <= 0), otherwise the
 * smallest of theta|a|, theta|b|, |a+b|/2 with the sign of a.  theta = 1
 * gives minmod, theta = 2 the monotonised-central limiter. */
double gamer_oracle_limiter(double a, double b, double theta) {
    if (a * b <= 0.0) return 0.0;
    double m = fmin(theta * fabs(a), fmin(theta * fabs(b), 0.5 * fabs(a + b)));
    return a > 0.0 ? m : -m;
}

/* A cell (i,j,k) with i,j,k in -1..16 belongs to the face-state set when at
 * most one coordinate lies outside the interior 0..15: the interior plus one
 * ghost layer across each face (5632 cells). */
static int in_face_state_set(int i, int j, int k) {
    int out = (i < 0 || i >= NI) + (j < 0 || j >= NI) + (k < 0 || k >= NI);
    return out <= 1;
}

static void neighbour(int d, int s, int *i, int *j, int *k) {
    if (d == 0) *i += s;
    if (d == 1) *j += s;
    if (d == 2) *k += s;
}

/* Primitive variables on every padded cell of one group.
 * U: [5][20][20][20]  ->  W: [5][20][20][20]. */
void gamer_oracle_group_prim(const double *U, double g, double *W) {
    for (int k = -NGH; k < NI + NGH; ++k)
        for (int j = -NGH; j < NI + NGH; ++j)
            for (int i = -NGH; i < NI + NGH; ++i) {
                double u[NV], w[NV];
                for (int v = 0; v < NV; ++v) u[v] = U[ip(v, i, j, k)];
                gamer_oracle_prim_from_cons(u, g, w);
                for (int v = 0; v < NV; ++v) W[ip(v, i, j, k)] = w[v];
            }
}

/* Limited slopes on the face-state set.
 * W: [5][20][20][20] primitives  ->  dW: [3 dir][5][18][18][18]
 * (entries outside the face-state set are set to zero). */
void gamer_oracle_group_slopes(const double *W, double theta, double *dW) {
    const size_t plane = (size_t)NV * NF * NF * NF;
    memset(dW, 0, 3 * plane * sizeof(double));
    for (int k = -1; k <= NI; ++k)
        for (int j = -1; j <= NI; ++j)
            for (int i = -1; i <= NI; ++i) {
                if (!in_face_state_set(i, j, k)) continue;
                for (int d = 0; d < 3; ++d) {
                    int im = i, jm = j, km = k, iq = i, jq = j, kq = k;
                    neighbour(d, -1, &im, &jm, &km);
                    neighbour(d, +1, &iq, &jq, &kq);
                    for (int v = 0; v < NV; ++v) {
                        double a = W[ip(v, i, j, k)] - W[ip(v, im, jm, km)];
                        double b = W[ip(v, iq, jq, kq)] - W[ip(v, i, j, k)];
                        dW[d * plane + is(v, i, j, k)] = gamer_oracle_limiter(a, b, theta);
                    }
                }
            }
}

/* Limited slope of one cell along direction d in characteristic variables
 * (limiting variant): the one-sided primitive differences a = W_c - W_{c-1}
 * and b = W_{c+1} - W_c are projected onto the left eigenvectors of the
 * primitive-variable system along d, evaluated at W_c; each wave's two
 * projections are limited with the generalised minmod; the limited wave
 * amplitudes are mapped back with the right eigenvectors (Toro 2009, Sec. 14
 * notes limiting in characteristic variables; the eigenvectors are those of
 * the quasi-linear primitive system, Toro 2009, Sec. 3.2).  With n the normal
 * velocity component, t1, t2 the transverse ones, c^2 = gamma p / rho:
 *   wave u - c:  l = (0, -rho/(2c), 0, 0, 1/(2c^2)),  r = (1, -c/rho, 0, 0, c^2)
 *   wave u (entropy):  l = (1, 0, 0, 0, -1/c^2),      r = (1, 0, 0, 0, 0)
 *   waves u (shear): l = r = unit vectors of t1, t2
 *   wave u + c:  l = (0, rho/(2c), 0, 0, 1/(2c^2)),   r = (1, c/rho, 0, 0, c^2)
 * (vector components in the order rho, n, t1, t2, p). */
void gamer_oracle_char_slope(const double *Wc, const double *a, const double *b, int d, double g,
                             double theta, double *dW) {
    const int n = 1 + d, t1 = d == 0 ? 2 : 1, t2 = d == 2 ? 2 : 3;
    const double rho = Wc[0];
    const double c2 = g * Wc[4] / rho;
    const double c = sqrt(c2);
    double la[5], lb[5], m[5];
    la[0] = -rho / (2.0 * c) * a[n] + a[4] / (2.0 * c2);
    lb[0] = -rho / (2.0 * c) * b[n] + b[4] / (2.0 * c2);
    la[1] = a[0] - a[4] / c2;
    lb[1] = b[0] - b[4] / c2;
    la[2] = a[t1];
    lb[2] = b[t1];
    la[3] = a[t2];
    lb[3] = b[t2];
    la[4] = rho / (2.0 * c) * a[n] + a[4] / (2.0 * c2);
    lb[4] = rho / (2.0 * c) * b[n] + b[4] / (2.0 * c2);
    for (int w = 0; w < 5; ++w) m[w] = gamer_oracle_limiter(la[w], lb[w], theta);
    dW[0] = m[0] + m[1] + m[4];
    dW[n] = c / rho * (m[4] - m[0]);
    dW[t1] = m[2];
    dW[t2] = m[3];
    dW[4] = c2 * (m[0] + m[4]);
}

/* Limited slopes in characteristic variables on the face-state set; layout
 * as gamer_oracle_group_slopes. */
void gamer_oracle_group_slopes_char(const double *W, double g, double theta, double *dW) {
    const size_t plane = (size_t)NV * NF * NF * NF;
    memset(dW, 0, 3 * plane * sizeof(double));
    for (int k = -1; k <= NI; ++k)
        for (int j = -1; j <= NI; ++j)
            for (int i = -1; i <= NI; ++i) {
                if (!in_face_state_set(i, j, k)) continue;
                double wc[NV];
                for (int v = 0; v < NV; ++v) wc[v] = W[ip(v, i, j, k)];
                for (int d = 0; d < 3; ++d) {
                    int im = i, jm = j, km = k, iq = i, jq = j, kq = k;
                    neighbour(d, -1, &im, &jm, &km);
                    neighbour(d, +1, &iq, &jq, &kq);
                    double a[NV], b[NV], out[NV];
                    for (int v = 0; v < NV; ++v) {
                        a[v] = wc[v] - W[ip(v, im, jm, km)];
                        b[v] = W[ip(v, iq, jq, kq)] - wc[v];
                    }
                    gamer_oracle_char_slope(wc, a, b, d, g, theta, out);
                    for (int v = 0; v < NV; ++v) dW[d * plane + is(v, i, j, k)] = out[v];
                }
            }
}

/* ---------------------------------------------------------------------- */
/* Step 2: half-step prediction (conservative Hancock step, unsplit).      */

/* For every face-state cell c: face values W^{d,-} = W_c - dW_d/2 and
 * W^{d,+} = W_c + dW_d/2, their conserved forms U^{d,+-}, and the common
 * half-step increment
 *   S_c = dt/(2 dh) * sum_d [ F_d(U^{d,-}) - F_d(U^{d,+}) ],
 * giving the predicted face states Ubar^{d,+-} = U^{d,+-} + S_c.
 * If any of the six predicted states has rho <= 0 or p <= 0, all six faces
 * of that cell take the cell average U_c instead (first-order fallback).
 *
 * U: padded conserved, W: padded primitives, dW: slopes from above.
 * Ub: [3 dir][2 side (0 = minus, 1 = plus)][5][18][18][18].
 * Returns the number of cells that took the fallback. */
long long gamer_oracle_group_predict(const double *U, const double *W, const double *dW,
                                     double dt, double dh, double g, double *Ub) {
    const size_t plane = (size_t)NV * NF * NF * NF;
    long long fallbacks = 0;
    memset(Ub, 0, 6 * plane * sizeof(double));
    for (int k = -1; k <= NI; ++k)
        for (int j = -1; j <= NI; ++j)
            for (int i = -1; i <= NI; ++i) {
                if (!in_face_state_set(i, j, k)) continue;
                double face[3][2][NV];   /* conserved face values U^{d,-}, U^{d,+} */
                double S[NV] = {0, 0, 0, 0, 0};
                for (int d = 0; d < 3; ++d) {
                    double wm[NV], wp[NV], fm[NV], fp[NV];
                    for (int v = 0; v < NV; ++v) {
                        double wc = W[ip(v, i, j, k)];
                        double dw = dW[d * plane + is(v, i, j, k)];
                        wm[v] = wc - 0.5 * dw;
                        wp[v] = wc + 0.5 * dw;
                    }
                    gamer_oracle_cons_from_prim(wm, g, face[d][0]);
                    gamer_oracle_cons_from_prim(wp, g, face[d][1]);
                    gamer_oracle_phys_flux(face[d][0], d, g, fm);
                    gamer_oracle_phys_flux(face[d][1], d, g, fp);
                    for (int v = 0; v < NV; ++v) S[v] += fm[v] - fp[v];
                }
                double coef = dt / (2.0 * dh);
                for (int v = 0; v < NV; ++v) S[v] *= coef;

                int bad = 0;
                double pred[3][2][NV];
                for (int d = 0; d < 3; ++d)
                    for (int s = 0; s < 2; ++s) {
                        for (int v = 0; v < NV; ++v) pred[d][s][v] = face[d][s][v] + S[v];
                        gamer_oracle_margin_note_state(pred[d][s]);
                        double w[NV];
                        gamer_oracle_prim_from_cons(pred[d][s], g, w);
                        if (!(w[0] > 0.0) || !(w[4] > 0.0)) bad = 1;
                    }
                if (bad) {
                    ++fallbacks;
                    for (int d = 0; d < 3; ++d)
                        for (int s = 0; s < 2; ++s)
                            for (int v = 0; v < NV; ++v) pred[d][s][v] = U[ip(v, i, j, k)];
                }
                for (int d = 0; d < 3; ++d)
                    for (int s = 0; s < 2; ++s)
                        for (int v = 0; v < NV; ++v)
                            Ub[(size_t)(2 * d + s) * plane + is(v, i, j, k)] = pred[d][s][v];
            }
    return fallbacks;
}

/* ---------------------------------------------------------------------- */
/* Step 3: Roe's approximate Riemann solver (Toro 2009, Sec. 11.2).       */
/* States are in a rotated frame whose component 1 is the normal momentum */
/* and components 2, 3 the two transverse momenta.                         */

typedef struct {
    double u, v, w, H, a2, a;  /* Roe averages; a = sqrt(a2) (NaN if a2 <= 0) */
    double alpha[NV];          /* wave strengths */
    double lambda[NV];         /* eigenvalues u-a, u, u, u, u+a */
    double K[NV][NV];          /* right eigenvectors K[wave][component] */
} roe_decomp;

static void roe_decompose(const double *L, const double *R, double g, roe_decomp *r) {
    double wl[NV], wr[NV];
    gamer_oracle_prim_from_cons(L, g, wl);
    gamer_oracle_prim_from_cons(R, g, wr);
    double HL = (L[4] + wl[4]) / wl[0];
    double HR = (R[4] + wr[4]) / wr[0];
    double sl = sqrt(wl[0]), sr = sqrt(wr[0]);
    double sum = sl + sr;
    /* Roe averages: square-root-density weighted means (Toro eq. 11.60). */
    r->u = (sl * wl[1] + sr * wr[1]) / sum;
    r->v = (sl * wl[2] + sr * wr[2]) / sum;
    r->w = (sl * wl[3] + sr * wr[3]) / sum;
    r->H = (sl * HL + sr * HR) / sum;
    double q2 = r->u * r->u + r->v * r->v + r->w * r->w;
    r->a2 = (g - 1.0) * (r->H - 0.5 * q2);
    r->a = r->a2 > 0.0 ? sqrt(r->a2) : NAN;
    double u = r->u, v = r->v, w = r->w, H = r->H, a = r->a;

    /* eigenvalues and right eigenvectors (Toro eqs. 11.58-11.59) */
    r->lambda[0] = u - a;
    r->lambda[1] = u;
    r->lambda[2] = u;
    r->lambda[3] = u;
    r->lambda[4] = u + a;
    double K[NV][NV] = {
        {1.0, u - a, v, w, H - u * a},
        {1.0, u, v, w, 0.5 * q2},
        {0.0, 0.0, 1.0, 0.0, v},
        {0.0, 0.0, 0.0, 1.0, w},
        {1.0, u + a, v, w, H + u * a},
    };
    memcpy(r->K, K, sizeof K);

    /* wave strengths (Toro eqs. 11.68-11.70) */
    double D[NV];
    for (int m = 0; m < NV; ++m) D[m] = R[m] - L[m];
    double a3 = D[2] - v * D[0];
    double a4 = D[3] - w * D[0];
    double d5 = D[4] - a3 * v - a4 * w;
    double a2w = (g - 1.0) / r->a2 * (D[0] * (H - u * u) + u * D[1] - d5);
    double a1 = (D[0] * (u + a) - D[1] - a * a2w) / (2.0 * a);
    double a5 = D[0] - (a1 + a2w);
    r->alpha[0] = a1;
    r->alpha[1] = a2w;
    r->alpha[2] = a3;
    r->alpha[3] = a4;
    r->alpha[4] = a5;
}

static double sound_speed(const double *U, double g, double *un) {
    double W[NV];
    gamer_oracle_prim_from_cons(U, g, W);
    *un = W[1];
    return sqrt(g * W[4] / W[0]);
}

static int physical(const double *U, double g) {
    double W[NV];
    gamer_oracle_margin_note_state(U);
    gamer_oracle_prim_from_cons(U, g, W);
    return W[0] > 0.0 && W[4] > 0.0;
}

/* Physical flux in the rotated frame (normal = component 1). */
static void rot_flux(const double *U, double g, double *F) { gamer_oracle_phys_flux(U, 0, g, F); }

/* HLLE flux (Einfeldt 1988) with signal speeds SL, SR. */
static void hlle(const double *L, const double *R, const double *FL, const double *FR, double SL,
                 double SR, double *F) {
    if (SL >= 0.0) {
        for (int m = 0; m < NV; ++m) F[m] = FL[m];
    } else if (SR <= 0.0) {
        for (int m = 0; m < NV; ++m) F[m] = FR[m];
    } else {
        for (int m = 0; m < NV; ++m)
            F[m] = (SR * FL[m] - SL * FR[m] + SL * SR * (R[m] - L[m])) / (SR - SL);
    }
}

/* Roe flux between rotated states L and R.
 *   F = (F(L) + F(R))/2 - (1/2) sum_k alpha_k |lambda_k| K_k,
 * with the Harten-Hyman entropy fix on the two acoustic waves: for wave k
 * with speeds lambda_left, lambda_right on its two sides,
 * delta = max(0, lambda_k - lambda_left, lambda_right - lambda_k), and if
 * |lambda_k| < delta then |lambda_k| is replaced by (lambda_k^2 + delta^2)/(2 delta).
 * The sides of wave 1 are L and L* = L + alpha_1 K_1; of wave 5,
 * R* = R - alpha_5 K_5 and R.
 * Guard: if a2 <= 0, or L* or R* has rho <= 0 or p <= 0, the HLLE flux is
 * used instead (signal speeds min(u_L - c_L, u~ - a~), max(u_R + c_R, u~ + a~),
 * or the outer ones alone when a2 <= 0).  Returns 1 when HLLE was used. */
static int roe_flux_rotated(const double *L, const double *R, double g, double *F) {
    double FL[NV], FR[NV];
    rot_flux(L, g, FL);
    rot_flux(R, g, FR);
    roe_decomp r;
    roe_decompose(L, R, g, &r);
    double uL, uR;
    double cL = sound_speed(L, g, &uL);
    double cR = sound_speed(R, g, &uR);

    margin_note_a2(r.a2, r.H, r.u * r.u + r.v * r.v + r.w * r.w, g);
    if (!(r.a2 > 0.0)) {
        hlle(L, R, FL, FR, uL - cL, uR + cR, F);
        return 1;
    }
    double Ls[NV], Rs[NV];
    for (int m = 0; m < NV; ++m) {
        Ls[m] = L[m] + r.alpha[0] * r.K[0][m];
        Rs[m] = R[m] - r.alpha[4] * r.K[4][m];
    }
    if (!physical(Ls, g) || !physical(Rs, g)) {
        hlle(L, R, FL, FR, fmin(uL - cL, r.u - r.a), fmax(uR + cR, r.u + r.a), F);
        return 1;
    }

    double absl[NV];
    for (int k = 0; k < NV; ++k) absl[k] = fabs(r.lambda[k]);
    {
        double us, cs = sound_speed(Ls, g, &us);
        double lleft = uL - cL, lright = us - cs, lam = r.lambda[0];
        double delta = fmax(0.0, fmax(lam - lleft, lright - lam));
        if (fabs(lam) < delta) absl[0] = (lam * lam + delta * delta) / (2.0 * delta);
    }
    {
        double us, cs = sound_speed(Rs, g, &us);
        double lleft = us + cs, lright = uR + cR, lam = r.lambda[4];
        double delta = fmax(0.0, fmax(lam - lleft, lright - lam));
        if (fabs(lam) < delta) absl[4] = (lam * lam + delta * delta) / (2.0 * delta);
    }
    for (int m = 0; m < NV; ++m) {
        double diss = 0.0;
        for (int k = 0; k < NV; ++k) diss += r.alpha[k] * absl[k] * r.K[k][m];
        F[m] = 0.5 * (FL[m] + FR[m]) - 0.5 * diss;
    }
    return 0;
}

/* Rotation for direction d: (rho, m_d, m_{d+1}, m_{d+2}, E), indices cyclic. */
static void rotate(const double *U, int d, double *Ur) {
    Ur[0] = U[0];
    Ur[1] = U[1 + d];
    Ur[2] = U[1 + (d + 1) % 3];
    Ur[3] = U[1 + (d + 2) % 3];
    Ur[4] = U[4];
}
static void unrotate(const double *Fr, int d, double *F) {
    F[0] = Fr[0];
    F[1 + d] = Fr[1];
    F[1 + (d + 1) % 3] = Fr[2];
    F[1 + (d + 2) % 3] = Fr[3];
    F[4] = Fr[4];
}

/* Roe flux along direction d between unrotated conserved states UL, UR.
 * Returns 1 if the HLLE fallback was taken. */
int gamer_oracle_roe_flux(const double *UL, const double *UR, int d, double g, double *F) {
    double L[NV], R[NV], Fr[NV];
    rotate(UL, d, L);
    rotate(UR, d, R);
    int fb = roe_flux_rotated(L, R, g, Fr);
    unrotate(Fr, d, F);
    return fb;
}

/* Test hook: the Roe decomposition of rotated states L, R (normal = x).
 * avg: [u, v, w, H, a2, a]; alpha, lambda: [5]; K: [5 wave][5 component]. */
void gamer_oracle_roe_decompose(const double *L, const double *R, double g, double *avg,
                                double *alpha, double *lambda, double *K) {
    roe_decomp r;
    roe_decompose(L, R, g, &r);
    avg[0] = r.u;
    avg[1] = r.v;
    avg[2] = r.w;
    avg[3] = r.H;
    avg[4] = r.a2;
    avg[5] = r.a;
    for (int k = 0; k < NV; ++k) {
        alpha[k] = r.alpha[k];
        lambda[k] = r.lambda[k];
        for (int m = 0; m < NV; ++m) K[k * NV + m] = r.K[k][m];
    }
}

/* Fluxes at every face of one group.  Face f = 0..16 along d lies between
 * cells f-1 and f; left state Ubar^{d,+} of cell f-1, right state
 * Ubar^{d,-} of cell f.  Fl: [3 dir][5][17 face][16 t2][16 t1], with
 * (t1, t2) = (j, k) for x, (i, k) for y, (i, j) for z.
 * Returns the number of faces that took the HLLE fallback. */
long long gamer_oracle_group_fluxes(const double *Ub, double g, double *Fl) {
    const size_t plane = (size_t)NV * NF * NF * NF;
    const size_t fplane = (size_t)NV * 17 * NI * NI;
    long long fallbacks = 0;
    for (int d = 0; d < 3; ++d)
        for (int t2 = 0; t2 < NI; ++t2)
            for (int t1 = 0; t1 < NI; ++t1)
                for (int f = 0; f <= NI; ++f) {
                    int i, j, k;
                    if (d == 0) { i = f; j = t1; k = t2; }
                    else if (d == 1) { i = t1; j = f; k = t2; }
                    else { i = t1; j = t2; k = f; }
                    int il = i, jl = j, kl = k;
                    neighbour(d, -1, &il, &jl, &kl);
                    double UL[NV], UR[NV], F[NV];
                    for (int v = 0; v < NV; ++v) {
                        UL[v] = Ub[(size_t)(2 * d + 1) * plane + is(v, il, jl, kl)];
                        UR[v] = Ub[(size_t)(2 * d + 0) * plane + is(v, i, j, k)];
                    }
                    fallbacks += gamer_oracle_roe_flux(UL, UR, d, g, F);
                    for (int v = 0; v < NV; ++v)
                        Fl[d * fplane + (((size_t)v * 17 + f) * NI + t2) * NI + t1] = F[v];
                }
    return fallbacks;
}

/* ---------------------------------------------------------------------- */
/* Step 4: full-step conservative update.                                  */

/* U^{n+1}_c = U^n_c - (dt/dh) ((dF_x + dF_y) + dF_z), dF_d = F_{c+e_d/2} - F_{c-e_d/2}.
 * Also copies the face-index 0, 8, 16 planes to flux_planes when non-NULL. */
void gamer_oracle_group_update(const double *U, const double *Fl, double dt, double dh,
                               double *Uout, double *flux_planes) {
    const size_t fplane = (size_t)NV * 17 * NI * NI;
#define FL(d, v, f, t2, t1) Fl[(d) * fplane + ((((size_t)(v) * 17 + (f)) * NI + (t2)) * NI + (t1))]
    double r = dt / dh;
    for (int v = 0; v < NV; ++v)
        for (int k = 0; k < NI; ++k)
            for (int j = 0; j < NI; ++j)
                for (int i = 0; i < NI; ++i) {
                    double dfx = FL(0, v, i + 1, k, j) - FL(0, v, i, k, j);
                    double dfy = FL(1, v, j + 1, k, i) - FL(1, v, j, k, i);
                    double dfz = FL(2, v, k + 1, j, i) - FL(2, v, k, j, i);
                    Uout[ii(v, i, j, k)] = U[ip(v, i, j, k)] - r * ((dfx + dfy) + dfz);
                }
    if (flux_planes) {
        for (int d = 0; d < 3; ++d)
            for (int p = 0; p < 3; ++p)
                for (int v = 0; v < NV; ++v)
                    for (int t2 = 0; t2 < NI; ++t2)
                        for (int t1 = 0; t1 < NI; ++t1)
                            flux_planes[((((size_t)d * 3 + p) * NV + v) * NI + t2) * NI + t1] =
                                FL(d, v, 8 * p, t2, t1);
    }
#undef FL
}

/* ---------------------------------------------------------------------- */
/* One full step on a batch of groups.                                     */

/* groups_in: [n][5][20][20][20]; groups_out: [n][5][16][16][16];
 * fluxes_out: [n][3][3][5][16][16] or NULL; counts: [2] or NULL receives
 * (predictor fallbacks, HLLE fallbacks) summed over the batch.
 * Returns 0, or -1 on invalid arguments / allocation failure. */
int gamer_oracle_hydro_solve_lim(const double *groups_in, int64_t n_groups, double dt, double dh,
                                 double gamma, double theta, int char_limiting, double *fluxes_out,
                                 double *groups_out, long long *counts);

int gamer_oracle_hydro_solve(const double *groups_in, int64_t n_groups, double dt, double dh,
                             double gamma, double theta, double *fluxes_out, double *groups_out,
                             long long *counts) {
    return gamer_oracle_hydro_solve_lim(groups_in, n_groups, dt, dh, gamma, theta, 0, fluxes_out,
                                        groups_out, counts);
}

/* As gamer_oracle_hydro_solve; char_limiting != 0 takes the slopes in
 * characteristic variables (gamer_oracle_group_slopes_char). */
int gamer_oracle_hydro_solve_lim(const double *groups_in, int64_t n_groups, double dt, double dh,
                                 double gamma, double theta, int char_limiting, double *fluxes_out,
                                 double *groups_out, long long *counts) {
    if (n_groups < 0 || (n_groups > 0 && (!groups_in || !groups_out))) return -1;
    if (!(dt > 0.0) || !(dh > 0.0) || !(gamma > 1.0)) return -1;
    const size_t in_sz = (size_t)NV * NP * NP * NP;
    const size_t out_sz = (size_t)NV * NI * NI * NI;
    const size_t fl_sz = (size_t)3 * 3 * NV * NI * NI;
    const size_t s_sz = (size_t)NV * NF * NF * NF;
    const size_t face_sz = (size_t)3 * NV * 17 * NI * NI;
    long long bad_pred = 0, bad_roe = 0;
    int err = 0;
#pragma omp parallel num_threads(oracle_threads) reduction(+ : bad_pred, bad_roe)
    {
        double *W = malloc(in_sz * sizeof(double));
        double *dW = malloc(3 * s_sz * sizeof(double));
        double *Ub = malloc(6 * s_sz * sizeof(double));
        double *Fl = malloc(face_sz * sizeof(double));
        int ok = W && dW && Ub && Fl;
        if (!ok) {
#pragma omp atomic write
            err = 1;
        }
        /* every thread reaches the worksharing loop, even one whose
         * allocation failed (it then skips its share) */
#pragma omp for schedule(static)
        for (int64_t gi = 0; gi < n_groups; ++gi) {
            if (!ok) continue;
            const double *U = groups_in + (size_t)gi * in_sz;
            gamer_oracle_group_prim(U, gamma, W);
            if (char_limiting)
                gamer_oracle_group_slopes_char(W, gamma, theta, dW);
            else
                gamer_oracle_group_slopes(W, theta, dW);
            bad_pred += gamer_oracle_group_predict(U, W, dW, dt, dh, gamma, Ub);
            bad_roe += gamer_oracle_group_fluxes(Ub, gamma, Fl);
            gamer_oracle_group_update(U, Fl, dt, dh, groups_out + (size_t)gi * out_sz,
                                      fluxes_out ? fluxes_out + (size_t)gi * fl_sz : NULL);
        }
        free(W);
        free(dW);
        free(Ub);
        free(Fl);
    }
    if (counts) {
        counts[0] = bad_pred;
        counts[1] = bad_roe;
    }
    return err ? -1 : 0;
}

/* ---------------------------------------------------------------------- */
/* CFL time step and conserved sums.  The paper gives no formula for      */
/* either; the reading is the usual unsplit one: the time step is limited */
/* by the sum over the three directions of |u_d| + c_s (the 3D donor-cell */
/* stability bound), and the sums are plain dh^3-weighted totals.          */

/* Largest signal-speed sum max_c (|u|+|v|+|w| + 3 c_s), c_s = sqrt(gamma p / rho),
 * over all interior cells of groups [n][5][16][16][16].  A cell with rho <= 0,
 * p <= 0 or a speed that is not finite has no sound speed: the maximum, and so
 * the time step, is then NaN (undefined) rather than the maximum over the
 * remaining cells. */
double gamer_oracle_max_speed(const double *groups, int64_t n_groups, double gamma) {
    const size_t out_sz = (size_t)NV * NI * NI * NI;
    double smax = 0.0;
    for (int64_t gi = 0; gi < n_groups; ++gi) {
        const double *U = groups + (size_t)gi * out_sz;
        for (int k = 0; k < NI; ++k)
            for (int j = 0; j < NI; ++j)
                for (int i = 0; i < NI; ++i) {
                    double u[NV], w[NV];
                    for (int v = 0; v < NV; ++v) u[v] = U[ii(v, i, j, k)];
                    gamer_oracle_prim_from_cons(u, gamma, w);
                    if (!(w[0] > 0.0) || !(w[4] > 0.0)) return NAN;
                    double cs = sqrt(gamma * w[4] / w[0]);
                    double s = fabs(w[1]) + fabs(w[2]) + fabs(w[3]) + 3.0 * cs;
                    if (!isfinite(s)) return NAN;
                    if (s > smax) smax = s;
                }
    }
    return smax;
}

/* dt = cfl * dh / max_c sum_d (|u_d| + c_s). */
double gamer_oracle_cfl_dt(const double *groups, int64_t n_groups, double dh, double gamma,
                           double cfl) {
    return cfl * dh / gamer_oracle_max_speed(groups, n_groups, gamma);
}

/* sums5 = dh^3 * (sum rho, sum m_x, sum m_y, sum m_z, sum E) over the interior,
 * each accumulated with Neumaier's compensated summation. */
void gamer_oracle_conserved_sums(const double *groups, int64_t n_groups, double dh, double *sums5) {
    const size_t cells = (size_t)NI * NI * NI;
    for (int v = 0; v < NV; ++v) {
        double s = 0.0, c = 0.0;
        for (int64_t gi = 0; gi < n_groups; ++gi) {
            const double *q = groups + ((size_t)gi * NV + v) * cells;
            for (size_t m = 0; m < cells; ++m) {
                double x = q[m], t = s + x;
                if (fabs(s) >= fabs(x))
                    c += (s - t) + x;
                else
                    c += (x - t) + s;
                s = t;
            }
        }
        sums5[v] = dh * dh * dh * (s + c);
    }
}

/* ---------------------------------------------------------------------- */
/* Same-level periodic ghost fill (test utility for uniform grids).        */

/* state: groups [gz][gy][gx][5][16][16][16] (group index g = gx + Gx (gy + Gy gz))
 * padded: [G][5][20][20][20]; every padded cell takes the value of the cell at
 * the same global position wrapped periodically. */
void gamer_oracle_pack_periodic(const double *state, int gx, int gy, int gz, double *padded) {
    const int NX = gx * NI, NY = gy * NI, NZ = gz * NI;
    const size_t cells = (size_t)NI * NI * NI;
    for (int bz = 0; bz < gz; ++bz)
        for (int by = 0; by < gy; ++by)
            for (int bx = 0; bx < gx; ++bx) {
                size_t g = (size_t)bx + (size_t)gx * ((size_t)by + (size_t)gy * bz);
                double *P = padded + g * (size_t)NV * NP * NP * NP;
                for (int v = 0; v < NV; ++v)
                    for (int k = -NGH; k < NI + NGH; ++k)
                        for (int j = -NGH; j < NI + NGH; ++j)
                            for (int i = -NGH; i < NI + NGH; ++i) {
                                int X = ((bx * NI + i) % NX + NX) % NX;
                                int Y = ((by * NI + j) % NY + NY) % NY;
                                int Z = ((bz * NI + k) % NZ + NZ) % NZ;
                                size_t sg = (size_t)(X / NI) + (size_t)gx * ((size_t)(Y / NI) + (size_t)gy * (Z / NI));
                                P[ip(v, i, j, k)] = state[(sg * NV + v) * cells +
                                                          ((size_t)(Z % NI) * NI + (Y % NI)) * NI + (X % NI)];
                            }
            }
}
