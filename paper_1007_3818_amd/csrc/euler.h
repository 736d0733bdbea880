// euler.h -- per-cell and per-face arithmetic of the Euler equations shared by
// the fused MUSCL-Hancock solver and its CTU variant: positivity test,
// limiters, physical fluxes, the Hancock predictor, Roe's flux with the
// Harten-Hyman entropy fix and the HLLE fallback, and the fixed-order
// per-group stats reduction.
#pragma once

#include "device_math.h"
#include "internal.h"

namespace gamer {
namespace {

template <typename T>
__device__ __forceinline__ bool physical(const T u[NV]) {
    // rho > 0 and p > 0  <=>  rho > 0 and 2 rho E > |m|^2
    return u[0] > T(0) && T(2) * u[0] * u[4] > u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
}

// Generalised minmod: 0 at extrema (a b <= 0), else sign(a) min(theta|a|,
// theta|b|, |a+b|/2).  In float it is evaluated as med3(theta a,
// med3(theta b, (a+b)/2, 0), 0): the median with 0 is the two-argument minmod,
// and nesting it gives the same value bitwise whenever a and b share a sign
// (and 0 otherwise); only an a b that underflows to 0 would differ.
__device__ __forceinline__ float limiter(float a, float b, float theta) {
    const float inner = __builtin_amdgcn_fmed3f(theta * b, 0.5f * (a + b), 0.0f);
    return __builtin_amdgcn_fmed3f(theta * a, inner, 0.0f);
}
// In double, without a branch: bs = b with the sign of a is positive exactly
// when a and b share a sign, and then |a| + bs = |a + b|; otherwise theta bs <= 0
// and the clamp at 0 gives a zero slope (of either sign).  The min is taken
// over the same three values as in the definition, so a nonzero slope is the
// same bitwise.
__device__ __forceinline__ double limiter(double a, double b, double theta) {
    const double aa = fabs(a);
    const double bs = __builtin_copysign(1.0, a) * b;
    const double m = fmin(theta * aa, fmin(theta * bs, 0.5 * (aa + bs)));
    return __builtin_copysign(fmax(m, 0.0), a);
}

// Limited slope along direction D in characteristic variables: the one-sided
// primitive differences a, b are projected on the left eigenvectors of the
// primitive system along D at the cell state, each wave's pair is limited,
// and the limited amplitudes are mapped back with the right eigenvectors.
// Component order (rho, normal velocity, two transverse velocities, p):
//   u - c: l = (0, -rho/2c, 0, 0, 1/2c^2), r = (1, -c/rho, 0, 0, c^2)
//   u (entropy): l = (1, 0, 0, 0, -1/c^2), r = (1, 0, 0, 0, 0)
//   u (shear, two): unit vectors of the transverse velocities
//   u + c: l = (0, rho/2c, 0, 0, 1/2c^2), r = (1, c/rho, 0, 0, c^2)
// h = rho/(2c), q = 1/(2c^2), cr = c/rho, c2 = c^2 of the cell.
template <int D, typename T>
__device__ __forceinline__ void char_slope(const T a[NV], const T b[NV], T h, T q, T cr, T c2,
                                           T theta, T dw[NV]) {
    constexpr int N = 1 + D, T1 = D == 0 ? 2 : 1, T2 = D == 2 ? 2 : 3;
    const T m0 = limiter(q * a[4] - h * a[N], q * b[4] - h * b[N], theta);
    const T m1 = limiter(a[0] - T(2) * q * a[4], b[0] - T(2) * q * b[4], theta);
    const T m4 = limiter(q * a[4] + h * a[N], q * b[4] + h * b[N], theta);
    dw[0] = m0 + m1 + m4;
    dw[N] = cr * (m4 - m0);
    dw[T1] = limiter(a[T1], b[T1], theta);
    dw[T2] = limiter(a[T2], b[T2], theta);
    dw[4] = c2 * (m0 + m4);
}

// Physical flux along direction D of a primitive state (rho, u_x, u_y, u_z, p).
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

// Conserved variables of a primitive state.
template <typename T>
__device__ __forceinline__ void cons_prim(const T w[NV], const Consts<T> &c, T u[NV]) {
    u[0] = w[0];
    u[1] = w[0] * w[1];
    u[2] = w[0] * w[2];
    u[3] = w[0] * w[3];
    u[4] = w[4] * c.igm1 + c.half * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
}

// S += F_D(W0 - dW/2) - F_D(W0 + dW/2)
template <int D, typename T>
__device__ __forceinline__ void flux_difference(const T W0[NV], const T dw[NV], const Consts<T> &c,
                                                T Sv[NV]) {
    T wm[NV], wp[NV], fm[NV], fp[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        wm[v] = W0[v] - c.half * dw[v];
        wp[v] = W0[v] + c.half * dw[v];
    }
    flux_prim<D>(wm, c, fm);
    flux_prim<D>(wp, c, fp);
#pragma unroll
    for (int v = 0; v < NV; ++v) Sv[v] += fm[v] - fp[v];
}

// Half-step prediction of one cell (conservative Hancock step, all three
// directions): face values W0 -+ dW_d/2, the common increment
//   S = dt/(2dh) sum_d [F_d(W0 - dW_d/2) - F_d(W0 + dW_d/2)],
// and Ub[d][0] (minus face), Ub[d][1] (plus face) = cons(W0 -+ dW_d/2) + S.
// Returns false if any of the six has rho <= 0 or p <= 0.
template <typename T>
__device__ __forceinline__ bool predict(const T W0[NV], const T dW[3][NV], T hdt,
                                        const Consts<T> &c, T Ub[3][2][NV]) {
    T Sv[NV] = {T(0), T(0), T(0), T(0), T(0)};
    flux_difference<0>(W0, dW[0], c, Sv);
    flux_difference<1>(W0, dW[1], c, Sv);
    flux_difference<2>(W0, dW[2], c, Sv);
#pragma unroll
    for (int v = 0; v < NV; ++v) Sv[v] *= hdt;
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            T wf[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) wf[v] = W0[v] + T(side ? 1 : -1) * (c.half * dW[d][v]);
            cons_prim(wf, c, Ub[d][side]);
#pragma unroll
            for (int v = 0; v < NV; ++v) Ub[d][side][v] += Sv[v];
            ok = ok && physical(Ub[d][side]);
        }
    }
    return ok;
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
// they need no reciprocal unless the entropy fix is active on that lane.  In
// double, where a square root is a refined estimate of about fifteen
// instructions, the entropy fix is tested on squared speeds (c^2 = gamma p /
// rho, (rho* c*)^2 = gq Q*), and the square roots are taken only on lanes where
// the fix is active or HLLE is used; in float the square root is one hardware
// instruction and the speeds are formed directly.
//
// TWICE: return 2F instead of F.  Every component of F is half of a sum, and
// halving is exact, so a caller that scales its use of the flux by 1/2 (the
// update's dt/dh, the flux planes it stores) gets the same values bitwise
// without the five multiplications.
template <typename T, bool TWICE = false>
__device__ __forceinline__ bool roe(const T L[NV], const T R[NV], const Consts<T> &c, T F[NV]) {
    const T h = c.half;
    const T hf = TWICE ? T(1) : h;  // the flux sums' factor
    const T qL = rsq(L[0]), qR = rsq(R[0]);
    const T irL = qL * qL, irR = qR * qR;
    const T uL = L[1] * irL, vL = L[2] * irL, wL = L[3] * irL;
    const T uR = R[1] * irR, vR = R[2] * irR, wR = R[3] * irR;
    const T pL = c.gm1 * (L[4] - h * (L[1] * uL + L[2] * vL + L[3] * wL));
    const T pR = c.gm1 * (R[4] - h * (R[1] * uR + R[2] * vR + R[3] * wR));
    const T c2L = c.g * pL * irL, c2R = c.g * pR * irR;  // squared sound speeds

    // Roe averages with weights sqrt(rho): sqrt(rho) u = m / sqrt(rho)
    const T is = rcp(L[0] * qL + R[0] * qR);
    const T u = (L[1] * qL + R[1] * qR) * is;
    const T v = (L[2] * qL + R[2] * qR) * is;
    const T w = (L[3] * qL + R[3] * qR) * is;
    const T H = ((L[4] + pL) * qL + (R[4] + pR) * qR) * is;
    const T q2 = u * u + v * v + w * w;
    const T a2 = c.gm1 * (H - h * q2);
    if (!(a2 > T(0))) {
        hlle(L, R, uL, pL, uR, pR, uL - sqrt_(c2L), uR + sqrt_(c2R), F);
        if (TWICE) {
#pragma unroll
            for (int m = 0; m < NV; ++m) F[m] *= T(2);
        }
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
        hlle(L, R, uL, pL, uR, pR, fmin(uL - sqrt_(c2L), u - a), fmax(uR + sqrt_(c2R), u + a), F);
        if (TWICE) {
#pragma unroll
            for (int m = 0; m < NV; ++m) F[m] *= T(2);
        }
        return true;
    }
    // Harten-Hyman: wave 1 between L (speed uL - cL) and L* (speed (m* - rho* c*)/rho*),
    // wave 5 between R* (speed (m* + rho* c*)/rho*) and R (speed uR + cR).  The fix is
    // active when |lambda| < lambda - lambda_left or |lambda| < lambda_right - lambda.
    const T lam1 = u - a, lam5 = u + a;
    T ab1 = fabs(lam1), ab5 = fabs(lam5);
    if constexpr (sizeof(T) == 4) {
        const T cL = sqrt_(c2L), cR = sqrt_(c2R);
        const T rcLs = sqrt_(c.gq * QL), rcRs = sqrt_(c.gq * QR);  // rho* c*
        const T t1a = lam1 - (uL - cL);
        const T t1b_r = (Ls[1] - rcLs) - lam1 * Ls[0];  // (lambda_right - lambda) rho*
        const T t5b = (uR + cR) - lam5;
        const T t5a_r = lam5 * Rs[0] - (Rs[1] + rcRs);  // (lambda - lambda_left) rho*
        if (ab1 < t1a || ab1 * Ls[0] < t1b_r) {
            const T e = fmax(t1a, t1b_r * rcp(Ls[0]));
            ab1 = (lam1 * lam1 + e * e) * (h * rcp(e));
        }
        if (ab5 < t5b || ab5 * Rs[0] < t5a_r) {
            const T e = fmax(t5b, t5a_r * rcp(Rs[0]));
            ab5 = (lam5 * lam5 + e * e) * (h * rcp(e));
        }
    } else {
        // with the speeds' square roots isolated the tests read, for wave 1,
        //   cL > |lam1| - (lam1 - uL)     and   rho* c* < m* - (lam1 + |lam1|) rho*,
        // and for wave 5
        //   cR > |lam5| + (lam5 - uR)     and   rho* c* < (lam5 - |lam5|) rho* - m*,
        // each compared through the squares when its right-hand side is positive
        const T A1 = ab1 - (lam1 - uL), B1 = Ls[1] - (lam1 + ab1) * Ls[0];
        const T A5 = ab5 + (lam5 - uR), B5 = (lam5 - ab5) * Rs[0] - Rs[1];
        if (A1 < T(0) || c2L > A1 * A1 || (B1 > T(0) && c.gq * QL < B1 * B1)) {
            const T t1a = lam1 - (uL - sqrt_(c2L));
            const T t1b_r = (Ls[1] - sqrt_(c.gq * QL)) - lam1 * Ls[0];
            const T e = fmax(t1a, t1b_r * rcp(Ls[0]));
            ab1 = (lam1 * lam1 + e * e) * (h * rcp(e));
        }
        if (A5 < T(0) || c2R > A5 * A5 || (B5 > T(0) && c.gq * QR < B5 * B5)) {
            const T t5b = (uR + sqrt_(c2R)) - lam5;
            const T t5a_r = lam5 * Rs[0] - (Rs[1] + sqrt_(c.gq * QR));
            const T e = fmax(t5b, t5a_r * rcp(Rs[0]));
            ab5 = (lam5 * lam5 + e * e) * (h * rcp(e));
        }
    }
    const T ab2 = fabs(u);

    // dissipation sum_k |lambda_k| alpha_k K_k: waves 1, 2 and 5 share the
    // transverse components v and w of their eigenvectors, so those rows take
    // the sum of the three amplitudes once
    const T c1 = al1 * ab1, c2 = al2 * ab2, c3 = al3 * ab2, c4 = al4 * ab2, c5 = al5 * ab5;
    const T s125 = (c1 + c2) + c5;
    F[0] = hf * ((L[1] + R[1]) - s125);
    F[1] = hf * ((L[1] * uL + pL + R[1] * uR + pR) - ((c1 * (u - a) + c2 * u) + c5 * (u + a)));
    F[2] = hf * ((L[2] * uL + R[2] * uR) - (s125 * v + c3));
    F[3] = hf * ((L[3] * uL + R[3] * uR) - (s125 * w + c4));
    F[4] = hf * (((L[4] + pL) * uL + (R[4] + pR) * uR) -
                 ((((c1 * (H - ua) + c2 * (h * q2)) + c3 * v) + c4 * w) + c5 * (H + ua)));
    return false;
}

// Roe flux along direction D for unrotated conserved states (2F with TWICE).
template <int D, bool TWICE = false, typename T>
__device__ __forceinline__ bool roe_dir(const T UL[NV], const T UR[NV], const Consts<T> &c,
                                        T F[NV]) {
    constexpr int n = 1 + D, t1 = 1 + (D + 1) % 3, t2 = 1 + (D + 2) % 3;
    const T L[NV] = {UL[0], UL[n], UL[t1], UL[t2], UL[4]};
    const T R[NV] = {UR[0], UR[n], UR[t1], UR[t2], UR[4]};
    T Fr[NV];
    const bool fb = roe<T, TWICE>(L, R, c, Fr);
    F[0] = Fr[0];
    F[n] = Fr[1];
    F[t1] = Fr[2];
    F[t2] = Fr[3];
    F[4] = Fr[4];
    return fb;
}

// Fixed-order reduction of NSTAT doubles per thread over NTHREADS threads
// (thread index t, 0 .. NTHREADS - 1, NTHREADS a multiple of 64 when the
// work-group holds several such sets): stats 0..4 and 6..7 are summed, stat 5
// is a maximum that keeps NaN.  Thread 0 writes the result to dst (if not
// null).  The values go through LDS PART at a time; `red` must hold
// NTHREADS * PART doubles.  Each value is folded in the same order whatever
// PART is: thread t takes the values of threads t, t + 64, ..., then the 64
// partial results are folded by halving.
template <int NTHREADS, int PART = NSTAT>
__device__ __forceinline__ void block_reduce_stats(double st[NSTAT], double *red, double *dst,
                                                   int t = threadIdx.x) {
    static_assert(NSTAT % PART == 0, "whole passes");
#pragma unroll
    for (int q0 = 0; q0 < NSTAT; q0 += PART) {
#pragma unroll
        for (int q = 0; q < PART; ++q) red[q * NTHREADS + t] = st[q0 + q];
        __syncthreads();
        if (t < 64) {
            double acc[PART];
#pragma unroll
            for (int q = 0; q < PART; ++q) {
                double a = red[q * NTHREADS + t];
                for (int s = t + 64; s < NTHREADS; s += 64) {
                    const double b = red[q * NTHREADS + s];
                    a = (q0 + q == 5) ? max_nan(a, b) : a + b;
                }
                acc[q] = a;
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
                for (int q = 0; q < PART; ++q) {
                    const double b = __shfl_down(acc[q], off, 64);
                    acc[q] = (q0 + q == 5) ? max_nan(acc[q], b) : acc[q] + b;
                }
            }
            if (t == 0 && dst) {
#pragma unroll
                for (int q = 0; q < PART; ++q) dst[q0 + q] = acc[q];
            }
        }
        __syncthreads();
    }
}

}  // namespace
}  // namespace gamer
