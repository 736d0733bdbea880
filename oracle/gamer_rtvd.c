/*
 * gamer_rtvd.c -- plain FP64 CPU oracle for one step of the relaxing TVD
 * scheme on ghost-padded 16^3 patch groups.  TEST INFRASTRUCTURE ONLY (same
 * rules as gamer_oracle.c: only tests, the smoke check and the benchmark's CPU
 * leg may load it; it shares no code with the HIP library).
 *
 * What it computes: the paper's Sec. 2 names the solver GAMER used before the
 * MUSCL-Hancock one -- the second-order relaxing total-variation-diminishing
 * scheme of Trac & Pen (2003), three-dimensional through dimensional
 * splitting -- and notes that it needs a seven-point stencil per direction
 * (three ghost cells per side).  The per-sweep formulas follow Trac & Pen:
 *
 *   freezing speed c = |v_d| + sqrt(gamma p / rho) per cell, w = F_d(u) / c;
 *   right- and left-moving fluxes  fr = c (u + w),  fl = c (u - w);
 *   half step (first order):   F_{i+1/2} = (fr_i - fl_{i+1}) / 2,
 *                              u*_i = u_i - dt/(2 dx) (F_{i+1/2} - F_{i-1/2});
 *   full step (second order): fr, fl from u*, each made second order by the
 *     van Leer limiter on its upwind side,
 *       R = fr_i     + VL((fr_i - fr_{i-1})/2, (fr_{i+1} - fr_i)/2),
 *       L = fl_{i+1} + VL((fl_i - fl_{i+1})/2, (fl_{i+1} - fl_{i+2})/2),
 *     F_{i+1/2} = (R - L) / 2,  u^{n+1}_i = u_i - dt/dx (F_{i+1/2} - F_{i-1/2});
 *   VL(a, b) = 2ab/(a+b) when ab > 0, else 0.
 *
 * A step sweeps x, y, z in turn (order 0) or z, y, x (order 1); alternating
 * the two from step to step is the usual symmetric splitting.  Each sweep
 * updates the cells whose seven-point stencil along its direction lies in the
 * current block, so the block shrinks by three cells per side along that
 * direction only: 22^3 -> 16 x 22 x 22 -> 16 x 16 x 22 -> 16^3 for order 0.
 *
 * Layouts (x fastest): padded group [5][22][22][22], cells -3..18 per axis;
 * interior group [5][16][16][16].  Variables (rho, m_x, m_y, m_z, E).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RI 16 /* interior cells per axis */
#define RG 3  /* ghost cells per side */
#define RP 22 /* padded cells per axis */
#define RV 5

int gamer_oracle_get_threads(void);
void gamer_oracle_phys_flux(const double *U, int d, double g, double *F);

/* van Leer's harmonic limiter */
double gamer_oracle_vanleer(double a, double b) {
    const double ab = a * b;
    return ab > 0.0 ? 2.0 * ab / (a + b) : 0.0;
}

/* c and w = F_d(u) / c of one cell; returns 0 if rho <= 0 or p <= 0 */
static int freeze(const double *u, int d, double g, double *c, double *w) {
    const double rho = u[0];
    const double vd = u[1 + d] / rho;
    const double ke = 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / rho;
    const double p = (g - 1.0) * (u[4] - ke);
    *c = fabs(vd) + sqrt(g * p / rho);
    double F[RV];
    gamer_oracle_phys_flux(u, d, g, F);
    for (int v = 0; v < RV; ++v) w[v] = F[v] / *c;
    return rho > 0.0 && p > 0.0;
}

/* One relaxing-TVD update of a pencil of n >= 7 cells along direction d.
 * u: [n][5]; out: [n - 6][5] for cells 3 .. n-4.  Returns the number of cells
 * met with rho <= 0 or p <= 0 (their results are not meaningful). */
long long gamer_oracle_rtvd_pencil(const double *u, int n, int d, double dtdx, double g, double *out) {
    double *fr = malloc(sizeof(double) * (size_t)n * RV);
    double *fl = malloc(sizeof(double) * (size_t)n * RV);
    double *h = malloc(sizeof(double) * (size_t)n * RV);
    double *F = malloc(sizeof(double) * (size_t)n * RV);
    long long bad = 0;
    if (!fr || !fl || !h || !F) {
        free(fr), free(fl), free(h), free(F);
        return -1;
    }
    /* half step, first-order fluxes */
    for (int i = 0; i < n; ++i) {
        double c, w[RV];
        bad += !freeze(u + (size_t)i * RV, d, g, &c, w);
        for (int v = 0; v < RV; ++v) {
            fr[i * RV + v] = c * (u[i * RV + v] + w[v]);
            fl[i * RV + v] = c * (u[i * RV + v] - w[v]);
        }
    }
    for (int i = 0; i + 1 < n; ++i) /* face i+1/2 */
        for (int v = 0; v < RV; ++v) F[i * RV + v] = 0.5 * (fr[i * RV + v] - fl[(i + 1) * RV + v]);
    for (int i = 1; i + 1 < n; ++i)
        for (int v = 0; v < RV; ++v)
            h[i * RV + v] = u[i * RV + v] - 0.5 * dtdx * (F[i * RV + v] - F[(i - 1) * RV + v]);
    /* full step, second-order fluxes from the half-step state */
    for (int i = 1; i + 1 < n; ++i) {
        double c, w[RV];
        bad += !freeze(h + (size_t)i * RV, d, g, &c, w);
        for (int v = 0; v < RV; ++v) {
            fr[i * RV + v] = c * (h[i * RV + v] + w[v]);
            fl[i * RV + v] = c * (h[i * RV + v] - w[v]);
        }
    }
    for (int i = 2; i + 4 <= n; ++i) /* face i+1/2 */
        for (int v = 0; v < RV; ++v) {
            const double r0 = fr[(i - 1) * RV + v], r1 = fr[i * RV + v], r2 = fr[(i + 1) * RV + v];
            const double l1 = fl[i * RV + v], l2 = fl[(i + 1) * RV + v], l3 = fl[(i + 2) * RV + v];
            const double R = r1 + gamer_oracle_vanleer(0.5 * (r1 - r0), 0.5 * (r2 - r1));
            const double L = l2 + gamer_oracle_vanleer(0.5 * (l1 - l2), 0.5 * (l2 - l3));
            F[i * RV + v] = 0.5 * (R - L);
        }
    for (int i = 3; i + 3 < n; ++i)
        for (int v = 0; v < RV; ++v)
            out[(i - 3) * RV + v] = u[i * RV + v] - dtdx * (F[i * RV + v] - F[(i - 1) * RV + v]);
    free(fr), free(fl), free(h), free(F);
    return bad;
}

/* One sweep along d over a block of extents e[3] (x, y, z), [5][e2][e1][e0];
 * out has extent e[d] - 6 along d. */
static long long sweep(const double *in, const int e[3], int d, double dtdx, double g, double *out) {
    int eo[3] = {e[0], e[1], e[2]};
    eo[d] -= 2 * RG;
    const int n = e[d];
    const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2; /* transverse axes */
    const size_t plane_in = (size_t)e[0] * e[1] * e[2];
    const size_t plane_out = (size_t)eo[0] * eo[1] * eo[2];
    double *pu = malloc(sizeof(double) * (size_t)n * RV);
    double *po = malloc(sizeof(double) * (size_t)n * RV);
    long long bad = 0;
    if (!pu || !po) {
        free(pu), free(po);
        return -1;
    }
    for (int tb = 0; tb < e[b]; ++tb)
        for (int ta = 0; ta < e[a]; ++ta) {
            int idx[3];
            idx[a] = ta;
            idx[b] = tb;
            for (int s = 0; s < n; ++s) {
                idx[d] = s;
                const size_t off = ((size_t)idx[2] * e[1] + idx[1]) * e[0] + idx[0];
                for (int v = 0; v < RV; ++v) pu[s * RV + v] = in[v * plane_in + off];
            }
            const long long r = gamer_oracle_rtvd_pencil(pu, n, d, dtdx, g, po);
            if (r < 0) bad = -1;
            if (bad >= 0) bad += r;
            for (int s = 0; s < n - 2 * RG; ++s) {
                idx[d] = s;
                const size_t off = ((size_t)idx[2] * eo[1] + idx[1]) * eo[0] + idx[0];
                for (int v = 0; v < RV; ++v) out[v * plane_out + off] = po[s * RV + v];
            }
        }
    free(pu), free(po);
    return bad;
}

/* One step of one padded group [5][22][22][22] -> [5][16][16][16]; order 0
 * sweeps x, y, z; order 1 sweeps z, y, x.  Returns the bad-cell count or -1. */
long long gamer_oracle_rtvd_group(const double *in, double dt, double dh, double g, int order,
                                  double *out) {
    const double dtdx = dt / dh;
    const int dirs[2][3] = {{0, 1, 2}, {2, 1, 0}};
    double *b1 = malloc(sizeof(double) * RV * RP * RP * RI);
    double *b2 = malloc(sizeof(double) * RV * RP * RI * RI);
    if (!b1 || !b2) {
        free(b1), free(b2);
        return -1;
    }
    int e[3] = {RP, RP, RP};
    long long bad = 0, r;
    const int d0 = dirs[order][0], d1 = dirs[order][1], d2 = dirs[order][2];
    r = sweep(in, e, d0, dtdx, g, b1);
    bad = r < 0 ? -1 : bad + r;
    e[d0] -= 2 * RG;
    r = sweep(b1, e, d1, dtdx, g, b2);
    bad = (r < 0 || bad < 0) ? -1 : bad + r;
    e[d1] -= 2 * RG;
    r = sweep(b2, e, d2, dtdx, g, out);
    bad = (r < 0 || bad < 0) ? -1 : bad + r;
    free(b1), free(b2);
    return bad;
}

/* Batch: groups_in [n][5][22][22][22] -> groups_out [n][5][16][16][16].
 * Returns 0 (and the bad-cell count in *bad when non-NULL) or -1. */
int gamer_oracle_rtvd_solve(const double *groups_in, int64_t n_groups, double dt, double dh,
                            double gamma, int order, double *groups_out, long long *bad) {
    if (n_groups < 0 || (n_groups > 0 && (!groups_in || !groups_out))) return -1;
    if (!(dt > 0.0) || !(dh > 0.0) || !(gamma > 1.0) || (order != 0 && order != 1)) return -1;
    const size_t in_sz = (size_t)RV * RP * RP * RP, out_sz = (size_t)RV * RI * RI * RI;
    long long total = 0;
    int err = 0;
#pragma omp parallel for schedule(static) num_threads(gamer_oracle_get_threads()) reduction(+ : total)
    for (int64_t gi = 0; gi < n_groups; ++gi) {
        const long long r = gamer_oracle_rtvd_group(groups_in + (size_t)gi * in_sz, dt, dh, gamma, order,
                                                    groups_out + (size_t)gi * out_sz);
        if (r < 0) {
#pragma omp atomic write
            err = 1;
        } else {
            total += r;
        }
    }
    if (bad) *bad = total;
    return err ? -1 : 0;
}
