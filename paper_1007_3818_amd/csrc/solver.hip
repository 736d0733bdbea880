// solver.hip -- fused MUSCL-Hancock + Roe step for 16^3 patch groups (gfx950).
//
// Method (paper Sec. 2): reconstruction, half-step prediction, Roe Riemann
// solver, full-step update, unsplit in 3D with a five-point stencil.  Formula
// details follow Toro (2009) Sec. 14.4 and Sec. 11.2, the sources the paper
// cites; see include/gamer_hydro.h for the interface.
//
// Kernel design (one work-group of 320 threads = 5 wave64s per group):
//  - The group is swept in z.  At sweep position k the work-group holds the
//    primitive variables of planes k-1, k, k+1 (20 x 20 each) in a three-slot
//    LDS ring, and each thread owns one cell of the face-state plane: threads
//    0..255 the 16 x 16 interior columns, threads 256..319 the 64 ghost cells
//    just outside the four side faces (the face states of those cells are
//    needed by the group's boundary faces).
//  - A thread computes its cell's limited slopes in x, y, z from the LDS ring,
//    the half-step increment, and its predicted face states.  States that a
//    neighbour needs (the +x and +y faces) go to LDS; the -x, -y, -z and +z
//    states stay in registers.  The z face between planes k-1 and k is solved
//    in registers (the +z state of plane k-1 was kept from the last step of the
//    sweep), the x and y faces after one barrier, with the flux written over
//    the consumed LDS state.
//  - The update of plane k-1 completes at step k, once the z flux above it is
//    known: U - dt/dh ((dF_x + dF_y) + dF_z), in double for both precisions.
//  - The next padded plane is prefetched into registers one step ahead.
//  - Per-group stats of the updated cells (sums, max signal speed, fallback
//    counts) are reduced in a fixed order in the epilogue.
#include "device_math.h"
#include "internal.h"

namespace gamer {
namespace {

constexpr int NTHR = 320;
constexpr int NINNER = NI * NI;  // 256 interior columns

template <typename T>
struct alignas(16) Lds {
    T w[3][NV][NPL];       // primitive planes, ring indexed by (plane + 3) % 3
    T sx[NV][NI][NI + 1];  // [v][j][f]: +x state of cell f-1, then x flux at face f
    T sy[NV][NI + 1][NI];  // [v][f][i]: +y state of cell f-1, then y flux at face f
    double dxy[NV][NINNER];  // (dF_x + dF_y) of each interior cell of the previous plane
};

template <typename T>
__device__ __forceinline__ T limiter(T a, T b, T theta) {
    // generalised minmod: 0 at extrema, else sign(a) min(theta|a|, theta|b|, |a+b|/2)
    if (a * b <= T(0)) return T(0);
    T m = fmin(theta * fabs(a), fmin(theta * fabs(b), T(0.5) * fabs(a + b)));
    return a > T(0) ? m : -m;
}

// Physical flux along direction D of primitive state (rho, u_x, u_y, u_z, p);
// writes F.
template <int D, typename T>
__device__ __forceinline__ void flux_prim(const T w[NV], const Consts<T> &c, T f[NV]) {
    const T un = w[1 + D];
    const T e = w[4] * c.igm1 + c.half * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
    const T mn = w[0] * un;
    f[0] = mn;
    f[1] = mn * w[1];
    f[2] = mn * w[2];
    f[3] = mn * w[3];
    f[1 + D] += w[4];
    f[4] = (e + w[4]) * un;
}

template <typename T>
__device__ __forceinline__ void cons_prim(const T w[NV], const Consts<T> &c, T u[NV]) {
    u[0] = w[0];
    u[1] = w[0] * w[1];
    u[2] = w[0] * w[2];
    u[3] = w[0] * w[3];
    u[4] = w[4] * c.igm1 + c.half * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
}

template <typename T>
__device__ __forceinline__ bool physical(const T u[NV]) {
    // rho > 0 and p > 0  <=>  rho > 0 and 2 rho E > |m|^2
    return u[0] > T(0) && T(2) * u[0] * u[4] > u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
}

// Physical flux of a rotated conserved state (normal = component 1), given
// its normal velocity and pressure.
template <typename T>
__device__ __forceinline__ void rot_flux(const T U[NV], T un, T p, T F[NV]) {
    F[0] = U[1];
    F[1] = U[1] * un + p;
    F[2] = U[2] * un;
    F[3] = U[3] * un;
    F[4] = (U[4] + p) * un;
}

// HLLE flux (Einfeldt) with signal speeds SL, SR.
template <typename T>
__device__ __forceinline__ void hlle(const T L[NV], const T R[NV], T uL, T pL, T uR, T pR, T SL, T SR,
                                  T F[NV]) {
    T FL[NV], FR[NV];
    rot_flux(L, uL, pL, FL);
    rot_flux(R, uR, pR, FR);
    if (SL >= T(0)) {
#pragma unroll
        for (int m = 0; m < NV; ++m) F[m] = FL[m];
    } else if (SR <= T(0)) {
#pragma unroll
        for (int m = 0; m < NV; ++m) F[m] = FR[m];
    } else {
        const T id = rcp(SR - SL);
#pragma unroll
        for (int m = 0; m < NV; ++m) F[m] = (SR * FL[m] - SL * FR[m] + SL * SR * (R[m] - L[m])) * id;
    }
}

// Roe flux between rotated conserved states (component 1 = normal momentum).
// Harten-Hyman entropy fix on the acoustic waves, HLLE when a2 <= 0 or an
// intermediate state is unphysical.  Returns true when HLLE was used.
// Arithmetic layout: one reciprocal square root per side gives sqrt(rho) and
// 1/rho; one of a2 gives a and 1/a; the intermediate states' positivity and
// rho c come from Q = 2 rho E - |m|^2 (p > 0 <=> Q > 0, (rho c)^2 = gq Q), so
// they need no reciprocal unless the entropy fix is active on that lane.
template <typename T>
__device__ __forceinline__ bool roe(const T L[NV], const T R[NV], const Consts<T> &c, T F[NV]) {
    const T h = c.half;
    const T qL = rsq(L[0]), qR = rsq(R[0]);
    const T irL = qL * qL, irR = qR * qR;
    const T uL = L[1] * irL, vL = L[2] * irL, wL = L[3] * irL;
    const T uR = R[1] * irR, vR = R[2] * irR, wR = R[3] * irR;
    const T pL = c.gm1 * (L[4] - h * (L[1] * uL + L[2] * vL + L[3] * wL));
    const T pR = c.gm1 * (R[4] - h * (R[1] * uR + R[2] * vR + R[3] * wR));
    const T cL = sqrt_(c.g * pL * irL), cR = sqrt_(c.g * pR * irR);

    // Roe averages with weights sqrt(rho): sqrt(rho) u = m / sqrt(rho)
    const T is = rcp(L[0] * qL + R[0] * qR);
    const T u = (L[1] * qL + R[1] * qR) * is;
    const T v = (L[2] * qL + R[2] * qR) * is;
    const T w = (L[3] * qL + R[3] * qR) * is;
    const T H = ((L[4] + pL) * qL + (R[4] + pR) * qR) * is;
    const T q2 = u * u + v * v + w * w;
    const T a2 = c.gm1 * (H - h * q2);
    if (!(a2 > T(0))) {
        hlle(L, R, uL, pL, uR, pR, uL - cL, uR + cR, F);
        return true;
    }
    const T ia = rsq(a2);
    const T a = a2 * ia;
    const T D0 = R[0] - L[0], D1 = R[1] - L[1], D2 = R[2] - L[2], D3 = R[3] - L[3],
            D4 = R[4] - L[4];
    const T al3 = D2 - v * D0;
    const T al4 = D3 - w * D0;
    const T d5 = D4 - al3 * v - al4 * w;
    const T al2 = c.gm1 * (ia * ia) * (D0 * (H - u * u) + u * D1 - d5);
    const T al1 = (D0 * (u + a) - D1 - a * al2) * (h * ia);
    const T al5 = D0 - (al1 + al2);
    const T ua = u * a;

    // states on the inner sides of the two acoustic waves
    const T Ls[NV] = {L[0] + al1, L[1] + al1 * (u - a), L[2] + al1 * v, L[3] + al1 * w,
                      L[4] + al1 * (H - ua)};
    const T Rs[NV] = {R[0] - al5, R[1] - al5 * (u + a), R[2] - al5 * v, R[3] - al5 * w,
                      R[4] - al5 * (H + ua)};
    const T QL = T(2) * Ls[0] * Ls[4] - (Ls[1] * Ls[1] + Ls[2] * Ls[2] + Ls[3] * Ls[3]);
    const T QR = T(2) * Rs[0] * Rs[4] - (Rs[1] * Rs[1] + Rs[2] * Rs[2] + Rs[3] * Rs[3]);
    if (!(Ls[0] > T(0) && QL > T(0) && Rs[0] > T(0) && QR > T(0))) {
        hlle(L, R, uL, pL, uR, pR, fmin(uL - cL, u - a), fmax(uR + cR, u + a), F);
        return true;
    }
    const T rcLs = sqrt_(c.gq * QL), rcRs = sqrt_(c.gq * QR);  // rho* c*

    // Harten-Hyman: wave 1 between L (speed uL - cL) and L* (speed (m* - rho* c*)/rho*),
    // wave 5 between R* (speed (m* + rho* c*)/rho*) and R (speed uR + cR).  The fix is
    // active when |lambda| < lambda - lambda_left or |lambda| < lambda_right - lambda.
    const T lam1 = u - a, lam5 = u + a;
    const T t1a = lam1 - (uL - cL);
    const T t1b_r = (Ls[1] - rcLs) - lam1 * Ls[0];  // (lambda_right - lambda) rho*
    const T t5b = (uR + cR) - lam5;
    const T t5a_r = lam5 * Rs[0] - (Rs[1] + rcRs);  // (lambda - lambda_left) rho*
    T ab1 = fabs(lam1), ab5 = fabs(lam5);
    if (ab1 < t1a || ab1 * Ls[0] < t1b_r) {
        const T e = fmax(t1a, t1b_r * rcp(Ls[0]));
        ab1 = (lam1 * lam1 + e * e) * (h * rcp(e));
    }
    if (ab5 < t5b || ab5 * Rs[0] < t5a_r) {
        const T e = fmax(t5b, t5a_r * rcp(Rs[0]));
        ab5 = (lam5 * lam5 + e * e) * (h * rcp(e));
    }
    const T ab2 = fabs(u);

    const T c1 = al1 * ab1, c2 = al2 * ab2, c3 = al3 * ab2, c4 = al4 * ab2, c5 = al5 * ab5;
    F[0] = h * ((L[1] + R[1]) - ((c1 + c2) + c5));
    F[1] = h * ((L[1] * uL + pL + R[1] * uR + pR) - ((c1 * (u - a) + c2 * u) + c5 * (u + a)));
    F[2] = h * ((L[2] * uL + R[2] * uR) - (((c1 * v + c2 * v) + c3) + c5 * v));
    F[3] = h * ((L[3] * uL + R[3] * uR) - (((c1 * w + c2 * w) + c4) + c5 * w));
    F[4] = h * (((L[4] + pL) * uL + (R[4] + pR) * uR) -
                ((((c1 * (H - ua) + c2 * (h * q2)) + c3 * v) + c4 * w) + c5 * (H + ua)));
    return false;
}

// Roe flux along direction D for unrotated conserved states.
template <int D, typename T>
__device__ __forceinline__ bool roe_dir(const T UL[NV], const T UR[NV], const Consts<T> &c,
                                        T F[NV]) {
    constexpr int n = 1 + D, t1 = 1 + (D + 1) % 3, t2 = 1 + (D + 2) % 3;
    const T L[NV] = {UL[0], UL[n], UL[t1], UL[t2], UL[4]};
    const T R[NV] = {UR[0], UR[n], UR[t1], UR[t2], UR[4]};
    T Fr[NV];
    const bool fb = roe(L, R, c, Fr);
    F[0] = Fr[0];
    F[n] = Fr[1];
    F[t1] = Fr[2];
    F[t2] = Fr[3];
    F[4] = Fr[4];
    return fb;
}

// Fixed-order reduction of NSTAT doubles per thread over NTHREADS threads:
// stats 0..4 and 6..7 are summed, stat 5 is a maximum.  Lane 0 of wave 0
// writes the result.  `red` must hold NTHREADS * NSTAT doubles of LDS.
template <int NTHREADS>
__device__ __forceinline__ void block_reduce_stats(double st[NSTAT], double *red, double *dst) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < NSTAT; ++q) red[q * NTHREADS + t] = st[q];
    __syncthreads();
    if (t < 64) {
        double acc[NSTAT];
#pragma unroll
        for (int q = 0; q < NSTAT; ++q) {
            double a = red[q * NTHREADS + t];
            for (int s = t + 64; s < NTHREADS; s += 64) {
                const double b = red[q * NTHREADS + s];
                a = (q == 5) ? fmax(a, b) : a + b;
            }
            acc[q] = a;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
            for (int q = 0; q < NSTAT; ++q) {
                const double b = __shfl_down(acc[q], off, 64);
                acc[q] = (q == 5) ? fmax(acc[q], b) : acc[q] + b;
            }
        }
        if (t == 0) {
#pragma unroll
            for (int q = 0; q < NSTAT; ++q) dst[q] = acc[q];
        }
    }
    __syncthreads();
}

// Variants: the waves per SIMD that the register allocation must allow.  LDS
// allows three 5-wave float work-groups per CU (45 KB each) and two double
// ones (80 KB each); more waves trade registers for spills.  The first entry
// of each list is the default; the tuner may pick another at run time.
template <typename T>
struct Variants;
template <>
struct Variants<float> {
    static constexpr int count = 2;
    static constexpr int waves[count] = {4, 3};
};
template <>
struct Variants<double> {
    static constexpr int count = 2;
    static constexpr int waves[count] = {2, 3};
};

template <typename T, int WAVES>
__global__ __launch_bounds__(NTHR, WAVES) void solve_kernel(SolveParams<T> P) {
    __shared__ Lds<T> S;
    const int t = threadIdx.x;

    // ---- this thread's cell in the face-state plane ----
    const bool inner = t < NINNER;
    int ci, cj;
    if (inner) {
        ci = t & 15;
        cj = t >> 4;
    } else {
        const int r = t - NINNER, q = r & 15;
        switch (r >> 4) {
            case 0: ci = -1; cj = q; break;   // -x ghost layer: gives +x state of face 0
            case 1: ci = NI; cj = q; break;   // +x ghost layer: solves x face 16
            case 2: ci = q; cj = -1; break;   // -y ghost layer
            default: ci = q; cj = NI; break;  // +y ghost layer
        }
    }
    const int pos = (cj + NG) * NP + (ci + NG);
    // roles within the plane (k = 0..15)
    const bool put_xp = ci <= NI - 1 && cj >= 0 && cj < NI;  // +x state feeds face ci+1
    const bool put_yp = cj <= NI - 1 && ci >= 0 && ci < NI;  // +y state feeds face cj+1
    const bool do_x = ci >= 0 && cj >= 0 && cj < NI;          // solves x face ci
    const bool do_y = cj >= 0 && ci >= 0 && ci < NI;          // solves y face cj

    const Consts<T> c = make_consts<T>(P.gamma, P.theta);

    for (int64_t g = blockIdx.x; g < P.n_groups; g += gridDim.x) {
        double dt = P.dt, dh = P.dh;
        if (P.dt_dev) {
            const int lev = P.level ? int(P.level[g]) : 0;
            dt = P.dt_dev[lev];
            dh = P.dh_dev[lev];
        }
        const double dtdh = dt / dh;
        const T hdt = T(0.5 * dtdh);
        const T *__restrict__ in = P.in + g * GIN;

        // ---- load helpers: positions t and t + NTHR of a padded plane ----
        const int p0 = t, p1 = t + NTHR;
        const bool has1 = p1 < NPL;
        T pre0[NV], pre1[NV];
        auto fetch = [&](int plane) {  // plane in -2..17
            const T *src = in + (plane + NG) * NPL;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                pre0[v] = src[v * NP * NPL + p0];
                pre1[v] = has1 ? src[v * NP * NPL + p1] : T(1);
            }
        };
        auto store = [&](int plane) {  // prefetched conserved -> primitive LDS plane
            const int slot = (plane + 3) % 3;
            {
                const T ir = rcp(pre0[0]);
                const T u = pre0[1] * ir, v = pre0[2] * ir, w = pre0[3] * ir;
                S.w[slot][0][p0] = pre0[0];
                S.w[slot][1][p0] = u;
                S.w[slot][2][p0] = v;
                S.w[slot][3][p0] = w;
                S.w[slot][4][p0] = c.gm1 * (pre0[4] - c.half * pre0[0] * (u * u + v * v + w * w));
            }
            if (has1) {
                const T ir = rcp(pre1[0]);
                const T u = pre1[1] * ir, v = pre1[2] * ir, w = pre1[3] * ir;
                S.w[slot][0][p1] = pre1[0];
                S.w[slot][1][p1] = u;
                S.w[slot][2][p1] = v;
                S.w[slot][3][p1] = w;
                S.w[slot][4][p1] = c.gm1 * (pre1[4] - c.half * pre1[0] * (u * u + v * v + w * w));
            }
        };

        fetch(-2);
        store(-2);
        fetch(-1);
        store(-1);
        fetch(0);

        // carried across sweep steps
        T zp[NV];            // +z state of this column at the previous plane
        T fz[NV];            // z flux below the current plane
        double st[6];        // sums of the 5 conserved variables, max signal speed
        int n_pred = 0, n_roe = 0;  // fallback counts
#pragma unroll
        for (int q = 0; q < 6; ++q) st[q] = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            zp[v] = T(0);
            fz[v] = T(0);
        }

        for (int k = -1; k <= NI; ++k) {
            store(k + 1);
            if (k + 2 <= NI + 1) fetch(k + 2);
            __syncthreads();  // B1: plane k+1 visible; planes k-1, k, k+1 in the ring

            const bool edge = (k < 0 || k >= NI);
            const bool active = inner || !edge;
            T xm[NV], ym[NV], zm[NV], zpn[NV];
            if (active) {
                const T(*wm)[NPL] = S.w[(k + 2) % 3];
                const T(*w0)[NPL] = S.w[(k + 3) % 3];
                const T(*wq)[NPL] = S.w[(k + 4) % 3];
                T W0[NV], dW[3][NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const T q0 = w0[v][pos];
                    W0[v] = q0;
                    dW[0][v] = limiter(q0 - w0[v][pos - 1], w0[v][pos + 1] - q0, c.theta);
                    dW[1][v] = limiter(q0 - w0[v][pos - NP], w0[v][pos + NP] - q0, c.theta);
                    dW[2][v] = limiter(q0 - wm[v][pos], wq[v][pos] - q0, c.theta);
                }
                // half-step increment S = dt/(2dh) sum_d [F_d(W^{d,-}) - F_d(W^{d,+})]
                T Sv[NV] = {T(0), T(0), T(0), T(0), T(0)};
                {
                    T wmf[NV], wpf[NV], fm[NV], fp[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        wmf[v] = W0[v] - c.half * dW[0][v];
                        wpf[v] = W0[v] + c.half * dW[0][v];
                    }
                    flux_prim<0>(wmf, c, fm);
                    flux_prim<0>(wpf, c, fp);
#pragma unroll
                    for (int v = 0; v < NV; ++v) Sv[v] += fm[v] - fp[v];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        wmf[v] = W0[v] - c.half * dW[1][v];
                        wpf[v] = W0[v] + c.half * dW[1][v];
                    }
                    flux_prim<1>(wmf, c, fm);
                    flux_prim<1>(wpf, c, fp);
#pragma unroll
                    for (int v = 0; v < NV; ++v) Sv[v] += fm[v] - fp[v];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        wmf[v] = W0[v] - c.half * dW[2][v];
                        wpf[v] = W0[v] + c.half * dW[2][v];
                    }
                    flux_prim<2>(wmf, c, fm);
                    flux_prim<2>(wpf, c, fp);
#pragma unroll
                    for (int v = 0; v < NV; ++v) Sv[v] += fm[v] - fp[v];
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) Sv[v] *= hdt;

                // predicted face states Ubar^{d,+-} = cons(W0 +- dW_d/2) + S
                bool ok = true;
                T xp[NV], yp[NV];
                auto face = [&](const T dw[NV], T sgn, T out[NV]) {
                    T wf[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) wf[v] = W0[v] + sgn * (c.half * dw[v]);
                    cons_prim(wf, c, out);
#pragma unroll
                    for (int v = 0; v < NV; ++v) out[v] += Sv[v];
                    ok = ok && physical(out);
                };
                face(dW[0], T(-1), xm);
                face(dW[0], T(1), xp);
                face(dW[1], T(-1), ym);
                face(dW[1], T(1), yp);
                face(dW[2], T(-1), zm);
                face(dW[2], T(1), zpn);
                if (!ok) {
                    // first-order fallback: every face of the cell takes the cell average
                    ++n_pred;
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const T u0 = in[v * NP * NPL + (k + NG) * NPL + pos];
                        xm[v] = xp[v] = ym[v] = yp[v] = zm[v] = zpn[v] = u0;
                    }
                }
                if (!edge) {
                    if (put_xp) {
#pragma unroll
                        for (int v = 0; v < NV; ++v) S.sx[v][cj][ci + 1] = xp[v];
                    }
                    if (put_yp) {
#pragma unroll
                        for (int v = 0; v < NV; ++v) S.sy[v][cj + 1][ci] = yp[v];
                    }
                }
            }

            // z face between planes k-1 and k (registers only)
            T fzn[NV];
            if (inner && k >= 0) {
                n_roe += roe_dir<2>(zp, zm, c, fzn);
                if (P.flux && (k & 7) == 0) {
                    T *dst = P.flux + g * GFLX + ((2 * 3 + (k >> 3)) * NV) * NINNER + cj * NI + ci;
#pragma unroll
                    for (int v = 0; v < NV; ++v) dst[v * NINNER] = fzn[v];
                }
            }
            __syncthreads();  // B2: +x / +y states visible

            if (!edge) {
                if (do_x) {
                    T UL[NV], F[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) UL[v] = S.sx[v][cj][ci];
                    n_roe += roe_dir<0>(UL, xm, c, F);
#pragma unroll
                    for (int v = 0; v < NV; ++v) S.sx[v][cj][ci] = F[v];
                    if (P.flux && (ci & 7) == 0) {
                        T *dst = P.flux + g * GFLX + ((0 * 3 + (ci >> 3)) * NV) * NINNER + k * NI + cj;
#pragma unroll
                        for (int v = 0; v < NV; ++v) dst[v * NINNER] = F[v];
                    }
                }
                if (do_y) {
                    T UL[NV], F[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) UL[v] = S.sy[v][cj][ci];
                    n_roe += roe_dir<1>(UL, ym, c, F);
#pragma unroll
                    for (int v = 0; v < NV; ++v) S.sy[v][cj][ci] = F[v];
                    if (P.flux && (cj & 7) == 0) {
                        T *dst = P.flux + g * GFLX + ((1 * 3 + (cj >> 3)) * NV) * NINNER + k * NI + ci;
#pragma unroll
                        for (int v = 0; v < NV; ++v) dst[v * NINNER] = F[v];
                    }
                }
            }
            __syncthreads();  // B3: x / y fluxes visible

            if (inner) {
                if (k >= 1) {
                    // plane k-1 is complete: U - dt/dh ((dF_x + dF_y) + dF_z)
                    const int kk = k - 1;
                    T *dst = P.out + g * GOUT + kk * NINNER + cj * NI + ci;
                    const T *src = in + (kk + NG) * NPL + pos;
                    T un[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const double dfz = double(fzn[v]) - double(fz[v]);
                        const double r = double(src[v * NP * NPL]) - dtdh * (S.dxy[v][t] + dfz);
                        const T o = T(r);
                        dst[v * NI * NINNER] = o;
                        un[v] = o;
                        st[v] += double(o);
                    }
                    st[5] = fmax(st[5], double(signal_speed(un[0], un[1], un[2], un[3], un[4], c)));
                }
                if (!edge) {
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        S.dxy[v][t] = (double(S.sx[v][cj][ci + 1]) - double(S.sx[v][cj][ci])) +
                                      (double(S.sy[v][cj + 1][ci]) - double(S.sy[v][cj][ci]));
                }
                if (k >= 0) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) fz[v] = fzn[v];
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) zp[v] = zpn[v];
            }
        }

        if (P.stats) {
            double all[NSTAT] = {st[0], st[1], st[2], st[3], st[4], st[5], double(n_pred),
                                 double(n_roe)};
            // S.w is free now (B3 of the last step passed); reuse it for the reduction
            block_reduce_stats<NTHR>(all, reinterpret_cast<double *>(&S.w[0][0][0]),
                                     P.stats + g * NSTAT);
        } else {
            __syncthreads();
        }
    }
}

static_assert(sizeof(Lds<float>::w) >= NTHR * NSTAT * sizeof(double),
              "stats reduction must fit in the primitive ring");

}  // namespace

template <typename T>
int solve_variant_count() {
    return Variants<T>::count;
}

template <typename T>
int solve_variant_waves(int v) {
    return (v >= 0 && v < Variants<T>::count) ? Variants<T>::waves[v] : 0;
}

// variant < 0 selects the default; grid <= 0 launches one work-group per group,
// grid > 0 a persistent grid that strides over the groups.
template <typename T>
hipError_t launch_solve(const SolveParams<T> &p, int variant, int64_t grid, hipStream_t s) {
    if (p.n_groups <= 0) return hipSuccess;
    const int64_t max_grid = int64_t(1) << 30;
    int64_t g = grid > 0 ? (grid < p.n_groups ? grid : p.n_groups) : p.n_groups;
    if (g > max_grid) g = max_grid;
    const dim3 blocks = dim3(unsigned(g)), threads = dim3(NTHR);
    switch (variant < 0 ? 0 : variant) {
        case 0:
            hipLaunchKernelGGL((solve_kernel<T, Variants<T>::waves[0]>), blocks, threads, 0, s, p);
            break;
        case 1:
            hipLaunchKernelGGL((solve_kernel<T, Variants<T>::waves[1]>), blocks, threads, 0, s, p);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template int solve_variant_count<float>();
template int solve_variant_count<double>();
template int solve_variant_waves<float>(int);
template int solve_variant_waves<double>(int);
template hipError_t launch_solve<float>(const SolveParams<float> &, int, int64_t, hipStream_t);
template hipError_t launch_solve<double>(const SolveParams<double> &, int, int64_t, hipStream_t);

}  // namespace gamer
