// solver.hip -- fused MUSCL-Hancock + Roe step for 16^3 patch groups (gfx950).
//
// Method (paper Sec. 2): reconstruction, half-step prediction, Roe Riemann
// solver, full-step update, unsplit in 3D with a five-point stencil.  Formula
// details follow Toro (2009) Sec. 14.4 and Sec. 11.2, the sources the paper
// cites; see include/gamer_hydro.h for the interface.
//
// Kernel design (one work-group per group at a time):
//  - The group is swept in z.  At sweep position k the work-group holds the
//    primitive variables of planes k-1, k, k+1 (20 x 20 each) in a three-slot
//    LDS ring.  Threads 0..255 own the 16 x 16 interior columns.  The 64 ghost
//    cells just outside the four side faces (whose face states the group's
//    boundary faces need) are computed either by 64 extra threads (320-thread
//    shape, 5 waves) or, in the 256-thread shape (one wave per SIMD), by one
//    wave in a second round, rotating over the waves plane by plane.
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

constexpr int NINNER = NI * NI;  // 256 interior columns

template <typename T>
struct alignas(16) Lds {
    T w[3][NV][NPL];       // primitive planes, ring indexed by (plane + 3) % 3
    T sx[NV][NI][NI + 1];  // [v][j][f]: +x state of cell f-1, then x flux at face f
    T sy[NV][NI + 1][NI];  // [v][f][i]: +y state of cell f-1, then y flux at face f
    double dxy[NV][NINNER];  // (dF_x + dF_y) of each interior cell of the previous plane
};

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
__device__ __forceinline__ double limiter(double a, double b, double theta) {
    if (a * b <= 0.0) return 0.0;
    const double m = fmin(theta * fabs(a), fmin(theta * fabs(b), 0.5 * fabs(a + b)));
    return a > 0.0 ? m : -m;
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

// Compiled variants: work-group size (320: ghost-layer cells on their own wave;
// 256: one wave per SIMD, ghost-layer cells as a second round) and the waves
// per SIMD the register allocation must allow.  LDS allows three float
// work-groups per CU (45 KB each) and two double ones (80 KB each).  The first
// entry of each list is the default; the tuner may pick another at run time.
struct Shape {
    int threads, waves;
};
template <typename T>
struct Variants;
template <>
struct Variants<float> {
    static constexpr int count = 3;
    static constexpr Shape shape[count] = {{256, 3}, {320, 4}, {320, 3}};
};
template <>
struct Variants<double> {
    static constexpr int count = 2;
    static constexpr Shape shape[count] = {{256, 2}, {320, 2}};
};

// The 64 cells of the ghost layer just outside the four side faces of a plane,
// numbered r = 0..63: -x layer (gives the +x state of face 0), +x layer (solves
// x face 16), -y layer, +y layer.
__device__ __forceinline__ void ring_cell(int r, int &ci, int &cj) {
    const int q = r & 15;
    switch (r >> 4) {
        case 0: ci = -1; cj = q; break;
        case 1: ci = NI; cj = q; break;
        case 2: ci = q; cj = -1; break;
        default: ci = q; cj = NI; break;
    }
}

// One work-group of NT threads advances one group at a time (grid-stride).
//  NT = 320: threads 0..255 own the interior columns, 256..319 the ghost-layer
//            cells of every plane (5 waves).
//  NT = 256: threads own the interior columns; in plane k the wave k mod 4 also
//            computes the 64 ghost-layer cells in a second round (4 waves, one
//            per SIMD).
template <typename S_, typename T, int NT, int WAVES, bool PERIODIC, bool CHAR>
__global__ __attribute__((amdgpu_flat_work_group_size(NT, NT), amdgpu_waves_per_eu(WAVES, 8)))
void solve_kernel(SolveParams<S_> P) {
    static_assert(NT == 320 || NT == 256, "work-group shape");
    constexpr bool SPLIT = NT == 320;
    __shared__ Lds<T> S;
    const int t = threadIdx.x;
    const int wave = t >> 6;

    const bool inner = t < NINNER;
    const int ii = t & 15, jj = t >> 4;  // interior column of threads 0..255
    const int my_ring = SPLIT ? t - NINNER : (t & 63);

    const Consts<T> c = make_consts<T>(P.gamma, P.theta);

    for (int64_t g = blockIdx.x; g < P.n_groups; g += gridDim.x) {
        double dt = P.dt, dh = P.dh;
        if (P.dt_dev) {
            const int lev = P.level ? int(P.level[g]) : 0;
            dt = P.dt_dev[lev];
            dh = P.dh_dev[lev];
        }
        const double dtdh = dt / dh;

        // ---- where padded cell (ip, jp, kp) of this group lives in the input ----
        // Padded input: the group's own padded block.  Periodic input: the cell at
        // the wrapped global position, in whichever group holds it; an offset is
        // (group index) * 20480 + (cell within the group), the group index split
        // into an x/y part and a z part.
        constexpr int VSTRIDE = PERIODIC ? NI * NI * NI : NP * NP * NP;
        int bx = 0, by = 0, bz = 0;
        if (PERIODIC) {
            bx = int(g % P.gx);
            by = int((g / P.gx) % P.gy);
            bz = int(g / (int64_t(P.gx) * P.gy));
        }
        // x/y part: (group index part, cell part)
        auto xy_part = [&](int ip, int jp, int &gpart) -> int {
            if (!PERIODIC) {
                gpart = 0;
                return jp * NP + ip;
            }
            int X = bx * NI + ip - NG, Y = by * NI + jp - NG;
            const int NX = P.gx * NI, NY = P.gy * NI;
            X = X < 0 ? X + NX : (X >= NX ? X - NX : X);
            Y = Y < 0 ? Y + NY : (Y >= NY ? Y - NY : Y);
            gpart = X / NI + P.gx * (Y / NI);
            return (Y % NI) * NI + (X % NI);
        };
        // z part, and the base pointer of a plane for the x/y group part 0
        auto plane_base = [&](int kp) -> const S_ * {
            if (!PERIODIC) return P.in + g * GIN + kp * NPL;
            int Z = bz * NI + kp - NG;
            const int NZ = P.gz * NI;
            Z = Z < 0 ? Z + NZ : (Z >= NZ ? Z - NZ : Z);
            return P.in + int64_t(P.gx) * P.gy * (Z / NI) * GOUT + (Z % NI) * (NI * NI);
        };
        auto cell_ptr = [&](int ip, int jp, int kp) -> const S_ * {
            int gp;
            const int cp = xy_part(ip, jp, gp);
            return plane_base(kp) + int64_t(gp) * GOUT + cp;
        };

        // ---- load helpers: positions t and t + NT of a padded plane ----
        const int p0 = t, p1 = t + NT;
        const bool has1 = p1 < NPL;
        int gp0, gp1 = 0;
        const int cp0 = xy_part(p0 % NP, p0 / NP, gp0);
        const int cp1 = has1 ? xy_part(p1 % NP, p1 / NP, gp1) : cp0;
        T pre0[NV], pre1[NV];
        auto fetch = [&](int plane) {  // plane in -2..17
            const S_ *src = plane_base(plane + NG);
            const S_ *s0 = src + int64_t(gp0) * GOUT + cp0;
            const S_ *s1 = src + int64_t(gp1) * GOUT + cp1;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                pre0[v] = T(s0[v * VSTRIDE]);
                pre1[v] = has1 ? T(s1[v * VSTRIDE]) : T(1);
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
            // ghost-layer cell of this thread in this plane (-1: none)
            const int ring = edge ? -1 : (SPLIT ? my_ring : (wave == (k & 3) ? my_ring : -1));

            // ---- face states: the interior cell, then the ghost-layer cell ----
            // (one code path for both, so a face state is computed identically
            // wherever its cell sits)
            T xm[NV], ym[NV], zm[NV], zpn[NV], rs[NV];  // rs: kept state of a ghost-layer cell
            const T(*wm)[NPL] = S.w[(k + 2) % 3];
            const T(*w0)[NPL] = S.w[(k + 3) % 3];
            const T(*wq)[NPL] = S.w[(k + 4) % 3];
#pragma unroll 1
            for (int round = 0; round < 2; ++round) {
                int ci, cj;
                if (round == 0) {
                    if (!inner) continue;
                    ci = ii;
                    cj = jj;
                } else {
                    if (ring < 0) continue;
                    ring_cell(ring, ci, cj);
                }
                const int pos = (cj + NG) * NP + (ci + NG);
                T W0[NV], dW[3][NV];
                if constexpr (!CHAR) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const T q0 = w0[v][pos];
                        W0[v] = q0;
                        dW[0][v] = limiter(q0 - w0[v][pos - 1], w0[v][pos + 1] - q0, c.theta);
                        dW[1][v] = limiter(q0 - w0[v][pos - NP], w0[v][pos + NP] - q0, c.theta);
                        dW[2][v] = limiter(q0 - wm[v][pos], wq[v][pos] - q0, c.theta);
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < NV; ++v) W0[v] = w0[v][pos];
                    const T c2 = c.g * W0[4] * rcp(W0[0]);
                    const T ic = rsq(c2);                    // 1/c
                    const T h = c.half * W0[0] * ic;         // rho/(2c)
                    const T q = c.half * ic * ic;            // 1/(2c^2)
                    const T cr = c2 * ic * rcp(W0[0]);       // c/rho
                    T a[NV], b[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        a[v] = W0[v] - w0[v][pos - 1];
                        b[v] = w0[v][pos + 1] - W0[v];
                    }
                    char_slope<0>(a, b, h, q, cr, c2, c.theta, dW[0]);
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        a[v] = W0[v] - w0[v][pos - NP];
                        b[v] = w0[v][pos + NP] - W0[v];
                    }
                    char_slope<1>(a, b, h, q, cr, c2, c.theta, dW[1]);
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        a[v] = W0[v] - wm[v][pos];
                        b[v] = wq[v][pos] - W0[v];
                    }
                    char_slope<2>(a, b, h, q, cr, c2, c.theta, dW[2]);
                }
                // predicted face states Ubar^{d,+-} = cons(W0 +- dW_d/2) + S
                T Ub[3][2][NV];
                if (!predict(W0, dW, T(0.5 * dtdh), c, Ub)) {
                    // first-order fallback: every face of the cell takes the cell average
                    ++n_pred;
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const T u0 = T(cell_ptr(ci + NG, cj + NG, k + NG)[v * VSTRIDE]);
#pragma unroll
                        for (int d = 0; d < 3; ++d) Ub[d][0][v] = Ub[d][1][v] = u0;
                    }
                }
                if (round == 0) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        xm[v] = Ub[0][0][v];
                        ym[v] = Ub[1][0][v];
                        zm[v] = Ub[2][0][v];
                        zpn[v] = Ub[2][1][v];
                    }
                    if (!edge) {
#pragma unroll
                        for (int v = 0; v < NV; ++v) {
                            S.sx[v][cj][ci + 1] = Ub[0][1][v];
                            S.sy[v][cj + 1][ci] = Ub[1][1][v];
                        }
                    }
                } else {
                    switch (ring >> 4) {
                        case 0:  // +x state of face 0
#pragma unroll
                            for (int v = 0; v < NV; ++v) S.sx[v][cj][0] = Ub[0][1][v];
                            break;
                        case 1:  // -x state of face 16, kept
#pragma unroll
                            for (int v = 0; v < NV; ++v) rs[v] = Ub[0][0][v];
                            break;
                        case 2:  // +y state of face 0
#pragma unroll
                            for (int v = 0; v < NV; ++v) S.sy[v][0][ci] = Ub[1][1][v];
                            break;
                        default:  // -y state of face 16, kept
#pragma unroll
                            for (int v = 0; v < NV; ++v) rs[v] = Ub[1][0][v];
                            break;
                    }
                }
            }

            // z face between planes k-1 and k (registers only)
            T fzn[NV];
            if (inner && k >= 0) {
                n_roe += roe_dir<2>(zp, zm, c, fzn);
                if (P.flux && (k & 7) == 0) {
                    S_ *dst = P.flux + g * GFLX + ((2 * 3 + (k >> 3)) * NV) * NINNER + jj * NI + ii;
#pragma unroll
                    for (int v = 0; v < NV; ++v) dst[v * NINNER] = S_(fzn[v]);
                }
            }
            __syncthreads();  // B2: +x / +y states visible

            if (!edge) {
                // x faces: face ci of each interior cell, then face 16 of each row
#pragma unroll 1
                for (int round = 0; round < 2; ++round) {
                    int row, f;
                    const T *R;
                    if (round == 0) {
                        if (!inner) continue;
                        row = jj;
                        f = ii;
                        R = xm;
                    } else {
                        if (ring < 0 || (ring >> 4) != 1) continue;
                        row = ring & 15;
                        f = NI;
                        R = rs;
                    }
                    T UL[NV], UR[NV], F[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        UL[v] = S.sx[v][row][f];
                        UR[v] = R[v];
                    }
                    n_roe += roe_dir<0>(UL, UR, c, F);
#pragma unroll
                    for (int v = 0; v < NV; ++v) S.sx[v][row][f] = F[v];
                    if (P.flux && (f & 7) == 0) {
                        S_ *dst = P.flux + g * GFLX + ((0 * 3 + (f >> 3)) * NV) * NINNER + k * NI + row;
#pragma unroll
                        for (int v = 0; v < NV; ++v) dst[v * NINNER] = S_(F[v]);
                    }
                }
                // y faces: face cj of each interior cell, then face 16 of each column
#pragma unroll 1
                for (int round = 0; round < 2; ++round) {
                    int col, f;
                    const T *R;
                    if (round == 0) {
                        if (!inner) continue;
                        col = ii;
                        f = jj;
                        R = ym;
                    } else {
                        if (ring < 0 || (ring >> 4) != 3) continue;
                        col = ring & 15;
                        f = NI;
                        R = rs;
                    }
                    T UL[NV], UR[NV], F[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        UL[v] = S.sy[v][f][col];
                        UR[v] = R[v];
                    }
                    n_roe += roe_dir<1>(UL, UR, c, F);
#pragma unroll
                    for (int v = 0; v < NV; ++v) S.sy[v][f][col] = F[v];
                    if (P.flux && (f & 7) == 0) {
                        S_ *dst = P.flux + g * GFLX + ((1 * 3 + (f >> 3)) * NV) * NINNER + k * NI + col;
#pragma unroll
                        for (int v = 0; v < NV; ++v) dst[v * NINNER] = S_(F[v]);
                    }
                }
            }
            __syncthreads();  // B3: x / y fluxes visible

            if (inner) {
                if (k >= 1) {
                    // plane k-1 is complete: U - dt/dh ((dF_x + dF_y) + dF_z)
                    const int kk = k - 1;
                    S_ *dst = P.out + g * GOUT + kk * NINNER + t;
                    const S_ *src = cell_ptr(ii + NG, jj + NG, kk + NG);
                    T un[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const double dfz = double(fzn[v]) - double(fz[v]);
                        const double r = double(src[v * VSTRIDE]) - dtdh * (S.dxy[v][t] + dfz);
                        const S_ o = S_(r);
                        dst[v * NI * NINNER] = o;
                        un[v] = T(o);
                        st[v] += double(o);
                    }
                    st[5] = fmax(st[5], double(signal_speed(un[0], un[1], un[2], un[3], un[4], c)));
                }
                if (!edge) {
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        S.dxy[v][t] = (double(S.sx[v][jj][ii + 1]) - double(S.sx[v][jj][ii])) +
                                      (double(S.sy[v][jj + 1][ii]) - double(S.sy[v][jj][ii]));
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
            block_reduce_stats<NT>(all, reinterpret_cast<double *>(&S.w[0][0][0]),
                                   P.stats + g * NSTAT);
        } else {
            __syncthreads();
        }
    }
}

static_assert(sizeof(Lds<float>::w) >= 320 * NSTAT * sizeof(double),
              "stats reduction must fit in the primitive ring");

}  // namespace

template <typename T>
int solve_variant_count() {
    return Variants<T>::count;
}

template <typename T>
int solve_variant_shape(int v, int *threads, int *waves) {
    if (v < 0 || v >= Variants<T>::count) return 0;
    *threads = Variants<T>::shape[v].threads;
    *waves = Variants<T>::shape[v].waves;
    return 1;
}

namespace {
template <typename S_, typename T, int V, bool CHAR>
void launch_shape(const SolveParams<S_> &p, dim3 blocks, hipStream_t s) {
    constexpr Shape sh = Variants<T>::shape[V];
    if (p.gx > 0)
        hipLaunchKernelGGL((solve_kernel<S_, T, sh.threads, sh.waves, true, CHAR>), blocks,
                           dim3(sh.threads), 0, s, p);
    else
        hipLaunchKernelGGL((solve_kernel<S_, T, sh.threads, sh.waves, false, CHAR>), blocks,
                           dim3(sh.threads), 0, s, p);
}
template <typename S_, typename T, int V>
void launch_variant(const SolveParams<S_> &p, dim3 blocks, hipStream_t s) {
    if (p.char_limiting)
        launch_shape<S_, T, V, true>(p, blocks, s);
    else
        launch_shape<S_, T, V, false>(p, blocks, s);
}
}  // namespace

// Storage type S_, arithmetic type T (float or S_).  variant < 0 selects the
// default; grid <= 0 launches one work-group per group, grid > 0 a persistent
// grid that strides over the groups.
template <typename S_, typename T>
hipError_t launch_solve(const SolveParams<S_> &p, int variant, int64_t grid, hipStream_t s) {
    if (p.n_groups <= 0) return hipSuccess;
    const int64_t max_grid = int64_t(1) << 30;
    int64_t g = grid > 0 ? (grid < p.n_groups ? grid : p.n_groups) : p.n_groups;
    if (g > max_grid) g = max_grid;
    const dim3 blocks = dim3(unsigned(g));
    switch (variant < 0 ? 0 : variant) {
        case 0: launch_variant<S_, T, 0>(p, blocks, s); break;
        case 1: launch_variant<S_, T, 1>(p, blocks, s); break;
        case 2:
            if constexpr (Variants<T>::count > 2) {
                launch_variant<S_, T, 2>(p, blocks, s);
                break;
            }
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template int solve_variant_count<float>();
template int solve_variant_count<double>();
template int solve_variant_shape<float>(int, int *, int *);
template int solve_variant_shape<double>(int, int *, int *);
template hipError_t launch_solve<float, float>(const SolveParams<float> &, int, int64_t, hipStream_t);
template hipError_t launch_solve<double, double>(const SolveParams<double> &, int, int64_t, hipStream_t);
template hipError_t launch_solve<double, float>(const SolveParams<double> &, int, int64_t, hipStream_t);

}  // namespace gamer
