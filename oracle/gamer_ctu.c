/*
 * gamer_ctu.c -- plain FP64 CPU oracle for the corner-transport-upwind (CTU)
 * variant of the MUSCL-Hancock step on ghost-padded 16^3 patch groups.  TEST
 * INFRASTRUCTURE ONLY (same rules as gamer_oracle.c).
 *
 * The paper applies MUSCL-Hancock unsplit (Sec. 2) without saying how the
 * directions are coupled; the default path couples them through the
 * conservative Hancock predictor (the face states of a cell see the flux
 * differences of all three directions of that cell).  This variant couples
 * them instead with upwind transverse fluxes, as in Colella's (1990)
 * corner-transport-upwind method (the six-Riemann-solve form without the
 * 3D corner terms):
 *
 *  1. slopes as in the default path, on the cells of [-1,16]^3 with at most
 *     two coordinates outside the interior 0..15 (set E1);
 *  2. normal predictor per direction d: U^{d,+-} = cons(W +- dW_d/2)
 *       + dt/(2dh) [F_d(U^{d,-}) - F_d(U^{d,+})]  (direction d alone); if
 *     either state is unphysical both take the cell average (counted);
 *  3. transverse fluxes: Roe fluxes at every face between two E1 cells;
 *  4. correction of the states the group's faces use: the states of
 *     direction d of every cell whose coordinates other than d lie in the
 *     interior, the minus state for c_d = 0..16 and the plus state for
 *     c_d = -1..15 (the faces 0..16 along d lie between c_d - 1 and c_d):
 *       U^{d,+-} -= dt/(2dh) sum_{d' != d} [Ft_{d'}(c + e_{d'}/2) - Ft_{d'}(c - e_{d'}/2)];
 *     a corrected state that is unphysical keeps its step-2 value (counted
 *     with the predictor fallbacks);
 *  5. Roe fluxes at the group's 3 x 17 x 16^2 faces from the corrected
 *     states, and the same full-step update as the default path.
 * Two ghost cells per side suffice: step 1 at an E1 cell reads its
 * neighbours in -2..17.  HLLE fallbacks of steps 3 and 5 are both counted.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CI 16 /* interior cells per axis */
#define CP 20 /* padded cells per axis */
#define CE 18 /* cells -1..16 */
#define CV 5

int gamer_oracle_get_threads(void);
void gamer_oracle_prim_from_cons(const double *U, double g, double *W);
void gamer_oracle_cons_from_prim(const double *W, double g, double *U);
void gamer_oracle_phys_flux(const double *U, int d, double g, double *F);
double gamer_oracle_limiter(double a, double b, double theta);
int gamer_oracle_roe_flux(const double *UL, const double *UR, int d, double g, double *F);
void gamer_oracle_group_update(const double *U, const double *Fl, double dt, double dh, double *out,
                               double *flux_planes);

static size_t pidx(int v, int i, int j, int k) { /* padded, -2..17 */
    return (((size_t)v * CP + (size_t)(k + 2)) * CP + (size_t)(j + 2)) * CP + (size_t)(i + 2);
}
static size_t eidx(int v, int i, int j, int k) { /* -1..16 */
    return (((size_t)v * CE + (size_t)(k + 1)) * CE + (size_t)(j + 1)) * CE + (size_t)(i + 1);
}
static int n_out(int i, int j, int k) {
    return (i < 0 || i >= CI) + (j < 0 || j >= CI) + (k < 0 || k >= CI);
}
static int in_e1(int i, int j, int k) {
    return i >= -1 && i <= CI && j >= -1 && j <= CI && k >= -1 && k <= CI && n_out(i, j, k) <= 2;
}
/* rho > 0 and p > 0, with p > 0 written as 2 rho E > |m|^2 (p = (gamma-1)
 * (2 rho E - |m|^2) / (2 rho)): the kernels decide with this expression, so a
 * state with p within rounding of zero falls on the same side in both. */
void gamer_oracle_margin_note_state(const double *U);
static int physical(const double *U) {
    gamer_oracle_margin_note_state(U);
    return U[0] > 0.0 && 2.0 * U[0] * U[4] > U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
}
static void step(int d, int s, int *i, int *j, int *k) {
    if (d == 0) *i += s;
    if (d == 1) *j += s;
    if (d == 2) *k += s;
}

/* One group: U padded [5][20][20][20] -> out [5][16][16][16] (+ flux planes
 * [3][3][5][16][16] when non-NULL).  counts[0]: predictor fallbacks (step 2
 * cell-directions plus step 4 faces), counts[1]: HLLE fallbacks (steps 3 and
 * 5).  Returns 0 or -1 (allocation). */
int gamer_oracle_ctu_group(const double *U, double dt, double dh, double g, double theta,
                           double *out, double *planes, long long counts[2]) {
    const size_t pe = (size_t)CV * CE * CE * CE;
    double *W = malloc(sizeof(double) * CV * CP * CP * CP);
    double *Ub = malloc(sizeof(double) * 6 * pe);  /* [d][side][5][18^3] */
    double *Ft = malloc(sizeof(double) * 3 * pe);  /* [d][5][18^3], face c + e_d/2 */
    double *Fl = malloc(sizeof(double) * 3 * CV * 17 * CI * CI);
    if (!W || !Ub || !Ft || !Fl) {
        free(W), free(Ub), free(Ft), free(Fl);
        return -1;
    }
    const double hdt = 0.5 * dt / dh;
    for (int k = -2; k < CI + 2; ++k)
        for (int j = -2; j < CI + 2; ++j)
            for (int i = -2; i < CI + 2; ++i) {
                double u[CV], w[CV];
                for (int v = 0; v < CV; ++v) u[v] = U[pidx(v, i, j, k)];
                gamer_oracle_prim_from_cons(u, g, w);
                for (int v = 0; v < CV; ++v) W[pidx(v, i, j, k)] = w[v];
            }
    /* steps 1 and 2 */
    for (int k = -1; k <= CI; ++k)
        for (int j = -1; j <= CI; ++j)
            for (int i = -1; i <= CI; ++i) {
                if (!in_e1(i, j, k)) continue;
                for (int d = 0; d < 3; ++d) {
                    int im = i, jm = j, km = k, iq = i, jq = j, kq = k;
                    step(d, -1, &im, &jm, &km);
                    step(d, +1, &iq, &jq, &kq);
                    double wm[CV], wp[CV], um[CV], up[CV], fm[CV], fp[CV];
                    for (int v = 0; v < CV; ++v) {
                        const double w0 = W[pidx(v, i, j, k)];
                        const double dw = gamer_oracle_limiter(w0 - W[pidx(v, im, jm, km)],
                                                               W[pidx(v, iq, jq, kq)] - w0, theta);
                        wm[v] = w0 - 0.5 * dw;
                        wp[v] = w0 + 0.5 * dw;
                    }
                    gamer_oracle_cons_from_prim(wm, g, um);
                    gamer_oracle_cons_from_prim(wp, g, up);
                    gamer_oracle_phys_flux(um, d, g, fm);
                    gamer_oracle_phys_flux(up, d, g, fp);
                    for (int v = 0; v < CV; ++v) {
                        const double s = hdt * (fm[v] - fp[v]);
                        um[v] += s;
                        up[v] += s;
                    }
                    if (!physical(um) || !physical(up)) {
                        ++counts[0];
                        for (int v = 0; v < CV; ++v) um[v] = up[v] = U[pidx(v, i, j, k)];
                    }
                    for (int v = 0; v < CV; ++v) {
                        Ub[(size_t)(2 * d + 0) * pe + eidx(v, i, j, k)] = um[v];
                        Ub[(size_t)(2 * d + 1) * pe + eidx(v, i, j, k)] = up[v];
                    }
                }
            }
    /* step 3: transverse fluxes between E1 cells */
    for (int d = 0; d < 3; ++d)
        for (int k = -1; k <= CI; ++k)
            for (int j = -1; j <= CI; ++j)
                for (int i = -1; i <= CI; ++i) {
                    int iq = i, jq = j, kq = k;
                    step(d, +1, &iq, &jq, &kq);
                    if (!in_e1(i, j, k) || !in_e1(iq, jq, kq)) continue;
                    double L[CV], R[CV], F[CV];
                    for (int v = 0; v < CV; ++v) {
                        L[v] = Ub[(size_t)(2 * d + 1) * pe + eidx(v, i, j, k)];
                        R[v] = Ub[(size_t)(2 * d + 0) * pe + eidx(v, iq, jq, kq)];
                    }
                    counts[1] += gamer_oracle_roe_flux(L, R, d, g, F);
                    for (int v = 0; v < CV; ++v) Ft[(size_t)d * pe + eidx(v, i, j, k)] = F[v];
                }
    /* step 4: transverse corrections of the states the final faces use */
    for (int d = 0; d < 3; ++d)
        for (int k = -1; k <= CI; ++k)
            for (int j = -1; j <= CI; ++j)
                for (int i = -1; i <= CI; ++i) {
                    const int c[3] = {i, j, k};
                    int ok = 1;
                    for (int e = 0; e < 3; ++e)
                        if (e != d && (c[e] < 0 || c[e] >= CI)) ok = 0;
                    if (!ok) continue;
                    double corr[CV] = {0, 0, 0, 0, 0};
                    for (int e = 0; e < 3; ++e) {
                        if (e == d) continue;
                        int im = i, jm = j, km = k;
                        step(e, -1, &im, &jm, &km);
                        for (int v = 0; v < CV; ++v)
                            corr[v] += Ft[(size_t)e * pe + eidx(v, i, j, k)] -
                                       Ft[(size_t)e * pe + eidx(v, im, jm, km)];
                    }
                    for (int s = 0; s < 2; ++s) {
                        /* no face of the group uses the minus state of cell -1
                         * or the plus state of cell 16 along d */
                        if ((s == 0 && c[d] < 0) || (s == 1 && c[d] >= CI)) continue;
                        double u[CV];
                        double *dst = Ub + (size_t)(2 * d + s) * pe;
                        for (int v = 0; v < CV; ++v) u[v] = dst[eidx(v, i, j, k)] - hdt * corr[v];
                        if (!physical(u)) {
                            ++counts[0];
                            continue;
                        }
                        for (int v = 0; v < CV; ++v) dst[eidx(v, i, j, k)] = u[v];
                    }
                }
    /* step 5: final fluxes, layout of the default path's face array
     * [3 dir][5][17 face][16 t2][16 t1] */
    const size_t fplane = (size_t)CV * 17 * CI * CI;
    for (int d = 0; d < 3; ++d)
        for (int t2 = 0; t2 < CI; ++t2)
            for (int t1 = 0; t1 < CI; ++t1)
                for (int f = 0; f <= CI; ++f) {
                    int i, j, k;
                    if (d == 0) { i = f; j = t1; k = t2; }
                    else if (d == 1) { i = t1; j = f; k = t2; }
                    else { i = t1; j = t2; k = f; }
                    int il = i, jl = j, kl = k;
                    step(d, -1, &il, &jl, &kl);
                    double L[CV], R[CV], F[CV];
                    for (int v = 0; v < CV; ++v) {
                        L[v] = Ub[(size_t)(2 * d + 1) * pe + eidx(v, il, jl, kl)];
                        R[v] = Ub[(size_t)(2 * d + 0) * pe + eidx(v, i, j, k)];
                    }
                    counts[1] += gamer_oracle_roe_flux(L, R, d, g, F);
                    for (int v = 0; v < CV; ++v) Fl[d * fplane + (((size_t)v * 17 + f) * CI + t2) * CI + t1] = F[v];
                }
    gamer_oracle_group_update(U, Fl, dt, dh, out, planes);
    free(W), free(Ub), free(Ft), free(Fl);
    return 0;
}

/* Batch as gamer_oracle_hydro_solve. */
int gamer_oracle_ctu_solve(const double *groups_in, int64_t n_groups, double dt, double dh, double gamma,
                           double theta, double *fluxes_out, double *groups_out, long long *counts) {
    if (n_groups < 0 || (n_groups > 0 && (!groups_in || !groups_out))) return -1;
    if (!(dt > 0.0) || !(dh > 0.0) || !(gamma > 1.0)) return -1;
    const size_t in_sz = (size_t)CV * CP * CP * CP, out_sz = (size_t)CV * CI * CI * CI;
    const size_t fl_sz = (size_t)3 * 3 * CV * CI * CI;
    long long c0 = 0, c1 = 0;
    int err = 0;
#pragma omp parallel for schedule(static) num_threads(gamer_oracle_get_threads()) reduction(+ : c0, c1)
    for (int64_t gi = 0; gi < n_groups; ++gi) {
        long long c[2] = {0, 0};
        if (gamer_oracle_ctu_group(groups_in + (size_t)gi * in_sz, dt, dh, gamma, theta,
                                   groups_out + (size_t)gi * out_sz,
                                   fluxes_out ? fluxes_out + (size_t)gi * fl_sz : NULL, c) != 0) {
#pragma omp atomic write
            err = 1;
        }
        c0 += c[0];
        c1 += c[1];
    }
    if (counts) {
        counts[0] = c0;
        counts[1] = c1;
    }
    return err ? -1 : 0;
}
