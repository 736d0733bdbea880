// ctu.hip -- the corner-transport-upwind (CTU) coupling of the MUSCL-Hancock
// step: face states predicted along their own direction, corrected by upwind
// transverse Roe fluxes, then the final Roe fluxes and the same full-step
// update as the default path.  Two implementations:
//
// ctu_fused (variant 0, the default): 384 threads per group sweeping z with
// every intermediate on chip (two groups side by side per work-group in
// float, so that the work-group's 12 waves sit three to a SIMD).  Thread
// t < 324 of a group owns the column (i, j) of the 18 x 18 square of cells
// -1..16; step s (planes s = -1..16):
//   A  the z predictor of plane s, the transverse z flux between planes s - 1
//      and s (registers: this thread holds the plus-z state below), the
//      corrections of plane s - 1's x and y states (they need that flux and the
//      one below it, both in registers, and plane s - 1's transverse x and y
//      fluxes from LDS), then the x and y predictor of plane s;
//   C  (after a barrier) the transverse x and y fluxes of plane s and the final
//      x and y fluxes of plane s - 1, into LDS;
//   E  (after a barrier) the corrected z states of plane s, the final z flux
//      between planes s - 1 and s, the update of plane s - 1 and the primitive
//      states of padded plane s + 2 into the ring.
// Nothing is written to memory but the result, the flux planes and the stats.
//
// The pipeline (variant 1) keeps its intermediate arrays in a caller-provided
// workspace and runs as a short sequence of launches, one stage each:
//   ctu_zero      clear the per-group fallback counters
//   ctu_predict   one work-group per group sweeping z: slopes and the
//                 one-direction Hancock predictor on the cells of [-1,16]^3
//                 with at most two coordinates outside the interior (set E1),
//                 primitive planes in an LDS ring            -> Ub [6][5][18^3]
//                 and the Roe fluxes between neighbouring E1 cells
//                                                            -> Ft [3][5][18^3]
//   ctu_final     one work-group per group sweeping z: corrected states and the
//                 final Roe fluxes of each plane (x and y faces through LDS, z
//                 faces in registers), then U - dt/dh ((dF_x + dF_y) + dF_z) of
//                 the plane below and the per-group stats
#include "device_math.h"
#include "euler.h"
#include "internal.h"

namespace gamer {
namespace {

constexpr int CE = 18;                        // cells -1..16 per axis
constexpr int NINNER = NI * NI;
constexpr int64_t E3 = int64_t(CE) * CE * CE;  // 5832
constexpr int64_t UB_VALUES = 6 * NV * E3;
constexpr int64_t FT_VALUES = 3 * NV * E3;
constexpr int64_t WORK_VALUES = UB_VALUES + FT_VALUES;  // per group

__device__ __forceinline__ int eidx(int i, int j, int k) { return ((k + 1) * CE + (j + 1)) * CE + (i + 1); }
__device__ __forceinline__ int n_out(int i, int j, int k) {
    return (i < 0 || i >= NI) + (j < 0 || j >= NI) + (k < 0 || k >= NI);
}
__device__ __forceinline__ bool in_e1(int i, int j, int k) {
    return i >= -1 && i <= NI && j >= -1 && j <= NI && k >= -1 && k <= NI && n_out(i, j, k) <= 2;
}

template <typename T>
struct CtuArgs {
    const T *in;          // [n][5][20][20][20]
    T *out;               // [n][5][16][16][16]
    T *flux;              // [n][3][3][5][16][16] or nullptr
    double *stats;        // [n][8] or nullptr
    const int8_t *level;
    const double *dt_dev, *dh_dev;
    int n_levels;
    double gamma, theta;
    int64_t n_groups;
    T *work;              // [n][WORK_VALUES]
    int *counts;          // [n][2]
    unsigned long long *bad;  // as in the default solver, or nullptr
};

// dt and dh of group g (NaN for a level byte out of range, see level_dt)
template <typename T>
__device__ __forceinline__ bool group_dt(const CtuArgs<T> &P, int64_t g, double &dt, double &dh) {
    return level_dt(P.level, g, P.n_levels, P.dt_dev, P.dh_dev, dt, dh);
}

template <typename T>
__global__ __launch_bounds__(256) void ctu_zero(CtuArgs<T> P) {
    const int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (q < 2 * P.n_groups) P.counts[q] = 0;
}

template <int D>
__device__ __forceinline__ void nb(int s, int &i, int &j, int &k) {
    if (D == 0) i += s;
    if (D == 1) j += s;
    if (D == 2) k += s;
}

// primitive state of padded cell (i, j, k)
template <typename T>
__device__ __forceinline__ void prim_at(const T *U, int i, int j, int k, const Consts<T> &c, T w[NV]) {
    const int o = ((k + NG) * NP + (j + NG)) * NP + (i + NG);
    const T r = U[o];
    const T ir = rcp(r);
    const T u = U[o + 1 * NP * NP * NP] * ir, v = U[o + 2 * NP * NP * NP] * ir,
            wz = U[o + 3 * NP * NP * NP] * ir;
    w[0] = r;
    w[1] = u;
    w[2] = v;
    w[3] = wz;
    w[4] = c.gm1 * (U[o + 4 * NP * NP * NP] - c.half * r * (u * u + v * v + wz * wz));
}

// One-direction Hancock predictor of a cell along D, from its primitive state
// W0 and those of its two neighbours along D: the limited slope, the face
// values W0 -+ dW/2, and their conserved states advanced by dt/(2dh) times the
// flux difference along D.  False if either state is unphysical.
template <int D, typename T>
__device__ __forceinline__ bool predict_from(const T W0[NV], const T wl[NV], const T wr[NV], T hdt,
                                             const Consts<T> &c, T um[NV], T up[NV]) {
    T wm[NV], wp[NV], fm[NV], fp[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const T dw = limiter(W0[v] - wl[v], wr[v] - W0[v], c.theta);
        wm[v] = W0[v] - c.half * dw;
        wp[v] = W0[v] + c.half * dw;
    }
    cons_prim(wm, c, um);
    cons_prim(wp, c, up);
    flux_prim<D>(wm, c, fm);
    flux_prim<D>(wp, c, fp);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const T s = hdt * (fm[v] - fp[v]);
        um[v] += s;
        up[v] += s;
    }
    return physical(um) && physical(up);
}

template <typename T>
struct PredLds {
    T w[3][NV][NP][NP];  // primitive states of padded planes: plane m in slot (m + 3) % 3
    T xm[NV][CE][CE];    // minus-x predicted state of the plane's E1 cells, at [v][j + 1][i + 1]
    T ym[NV][CE][CE];    // minus-y, likewise
};

// Work-group size of the predictor, one E1 cell of a plane per thread (the
// 324 positions of the 18 x 18 square), so that every phase is one pass: in
// double (156 VGPRs, two waves per SIMD) one work-group fills the CU; in float
// (86 VGPRs) two fit.
constexpr int PRED_THREADS = 512;

// One work-group per group, sweeping k = -1..16; thread t < 324 owns the cell
// at position t of the 18 x 18 plane.  At step k: the primitive states of
// padded plane k + 1 into the LDS ring (planes k - 1 and k are there from the
// previous steps); after a barrier, the predicted states of the plane's E1
// cells (the one-direction Hancock predictor, per direction) -> Ub, their
// minus-x and minus-y states also to LDS, and the transverse z flux between the
// cell below, whose plus-z state this thread kept from the previous step, and
// the cell -> Ft; after a second barrier, the transverse x and y fluxes of the
// plane from each cell's plus states and its neighbours' minus states -> Ft.
template <typename T>
__global__ __launch_bounds__(PRED_THREADS) void ctu_predict(CtuArgs<T> P) {
    constexpr int NT = PRED_THREADS;
    static_assert(NT >= CE * CE, "one thread per cell of a plane");
    __shared__ PredLds<T> S;
    const int64_t g = blockIdx.x;
    if (g >= P.n_groups) return;
    const Consts<T> c = make_consts<T>(P.gamma, P.theta);
    double dt, dh;
    group_dt(P, g, dt, dh);
    const T hdt = T(0.5 * dt / dh);
    const T *U = P.in + g * GIN;
    T *Ub = P.work + g * WORK_VALUES;
    T *Ft = Ub + UB_VALUES;
    const int t = threadIdx.x;
    const int i = t % CE - 1, j = t / CE - 1;  // meaningful for t < 324 only
    const int ii = i + NG, jj = j + NG;
    int bad = 0, bad_roe = 0;
    T zp[NV];  // plus-z predicted state of this thread's cell in the plane below

    // primitive states of padded plane m (-2..17) into its slot of the ring
    auto fill = [&](int m) {
        const int slot = (m + 3) % 3;
        for (int q = t; q < NPL; q += NT) {
            const int qi = q % NP, qj = q / NP;
            T w[NV];
            prim_at(U, qi - NG, qj - NG, m, c, w);
#pragma unroll
            for (int v = 0; v < NV; ++v) S.w[slot][v][qj][qi] = w[v];
        }
    };
    fill(-2);
    fill(-1);
    for (int k = -1; k <= NI; ++k) {
        fill(k + 1);
        __syncthreads();  // planes k - 1, k and k + 1 in LDS
        const int sm = (k + 2) % 3, s0 = (k + 3) % 3, sp = (k + 4) % 3;
        const bool mine = t < CE * CE && in_e1(i, j, k);
        T xp[NV], yp[NV];
        if (mine) {
            const int e = eidx(i, j, k);
            const int o = ((k + NG) * NP + jj) * NP + ii;
            T W0[NV], wl[NV], wr[NV], um[NV], up[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) W0[v] = S.w[s0][v][jj][ii];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    wl[v] = d == 0 ? S.w[s0][v][jj][ii - 1] : d == 1 ? S.w[s0][v][jj - 1][ii] : S.w[sm][v][jj][ii];
                    wr[v] = d == 0 ? S.w[s0][v][jj][ii + 1] : d == 1 ? S.w[s0][v][jj + 1][ii] : S.w[sp][v][jj][ii];
                }
                const bool ok = d == 0   ? predict_from<0>(W0, wl, wr, hdt, c, um, up)
                                : d == 1 ? predict_from<1>(W0, wl, wr, hdt, c, um, up)
                                         : predict_from<2>(W0, wl, wr, hdt, c, um, up);
                if (!ok) {
                    ++bad;
#pragma unroll
                    for (int v = 0; v < NV; ++v) um[v] = up[v] = U[o + v * NP * NP * NP];
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    Ub[((2 * d + 0) * NV + v) * E3 + e] = um[v];
                    Ub[((2 * d + 1) * NV + v) * E3 + e] = up[v];
                }
                if (d == 0) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        S.xm[v][j + 1][i + 1] = um[v];
                        xp[v] = up[v];
                    }
                } else if (d == 1) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        S.ym[v][j + 1][i + 1] = um[v];
                        yp[v] = up[v];
                    }
                } else {
                    // transverse z flux at the face between the cell below and this one
                    if (k >= 0 && in_e1(i, j, k - 1)) {
                        T F[NV];
                        bad_roe += roe_dir<2>(zp, um, c, F);
                        const int eb = eidx(i, j, k - 1);
#pragma unroll
                        for (int v = 0; v < NV; ++v) Ft[(2 * NV + v) * E3 + eb] = F[v];
                    }
#pragma unroll
                    for (int v = 0; v < NV; ++v) zp[v] = up[v];
                }
            }
        }
        __syncthreads();  // the plane's minus-x and minus-y states visible
        if (mine) {
            const int e = eidx(i, j, k);
            T R[NV], F[NV];
            if (in_e1(i + 1, j, k)) {
#pragma unroll
                for (int v = 0; v < NV; ++v) R[v] = S.xm[v][j + 1][i + 2];
                bad_roe += roe_dir<0>(xp, R, c, F);
#pragma unroll
                for (int v = 0; v < NV; ++v) Ft[(0 * NV + v) * E3 + e] = F[v];
            }
            if (in_e1(i, j + 1, k)) {
#pragma unroll
                for (int v = 0; v < NV; ++v) R[v] = S.ym[v][j + 2][i + 1];
                bad_roe += roe_dir<1>(yp, R, c, F);
#pragma unroll
                for (int v = 0; v < NV; ++v) Ft[(1 * NV + v) * E3 + e] = F[v];
            }
        }
    }
    if (bad) atomicAdd(P.counts + 2 * g, bad);
    if (bad_roe) atomicAdd(P.counts + 2 * g + 1, bad_roe);
}

// corrected state of direction D, side s, at cell (i, j, k); false when the
// correction would make it unphysical (the predicted state is kept)
template <int D, typename T>
__device__ __forceinline__ bool corrected(const T *Ub, const T *Ft, int s, int i, int j, int k, T hdt,
                                          T u[NV]) {
    const int e = eidx(i, j, k);
    T corr[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) corr[v] = T(0);
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) {
        if (dd == D) continue;
        const int em = dd == 0 ? eidx(i - 1, j, k) : dd == 1 ? eidx(i, j - 1, k) : eidx(i, j, k - 1);
#pragma unroll
        for (int v = 0; v < NV; ++v) corr[v] += Ft[(dd * NV + v) * E3 + e] - Ft[(dd * NV + v) * E3 + em];
    }
    T p[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        p[v] = Ub[((2 * D + s) * NV + v) * E3 + e];
        u[v] = p[v] - hdt * corr[v];
    }
    if (physical(u)) return true;
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = p[v];
    return false;
}

// Final flux along D at the face between cell (i, j, k) - e_D and cell (i, j, k):
// Roe between the two corrected states; the flux planes at face index 0, 8, 16
// are written out when requested.
template <int D, typename T>
__device__ __forceinline__ void final_flux(const CtuArgs<T> &P, int64_t g, int i, int j, int k, T hdt,
                                           const Consts<T> &c, int &n_pred, int &n_roe, T F[NV]) {
    const T *Ub = P.work + g * WORK_VALUES;
    const T *Ft = Ub + UB_VALUES;
    int il = i, jl = j, kl = k;
    nb<D>(-1, il, jl, kl);
    T L[NV], R[NV];
    n_pred += !corrected<D>(Ub, Ft, 1, il, jl, kl, hdt, L);
    n_pred += !corrected<D>(Ub, Ft, 0, i, j, k, hdt, R);
    n_roe += roe_dir<D>(L, R, c, F);
    const int f = D == 0 ? i : (D == 1 ? j : k);
    if (P.flux && (f & 7) == 0) {
        // transverse order (t1, t2): (j, k) for x, (i, k) for y, (i, j) for z
        const int t1 = D == 0 ? j : i, t2 = D == 2 ? j : k;
        T *dst = P.flux + g * GFLX + ((D * 3 + (f >> 3)) * NV) * NINNER + t2 * NI + t1;
#pragma unroll
        for (int v = 0; v < NV; ++v) dst[v * NINNER] = F[v];
    }
}

template <typename T>
struct FinalLds {
    union {
        struct {
            T fx[NV][NI][NI + 1];  // [v][j][f]: x flux at face f of row j
            T fy[NV][NI + 1][NI];  // [v][f][i]: y flux at face f of column i
        } f;
        double red[256 * NSTAT];  // the stats reduction, after the sweep
    };
};

// One work-group of 256 threads per group; thread (i, j) owns column (i, j)
// and sweeps k = 0..16.  At step k: the z face k (below plane k) in registers;
// the update of plane k - 1, whose x and y flux differences were kept from the
// previous step; the x and y faces of plane k into LDS (faces 16 by one wave
// each, rotating); after a barrier, this column's x and y flux differences of
// plane k.
template <typename T>
__global__ __launch_bounds__(256) void ctu_final(CtuArgs<T> P) {
    __shared__ FinalLds<T> S;
    const int64_t g = blockIdx.x;
    if (g >= P.n_groups) return;
    const Consts<T> c = make_consts<T>(P.gamma, P.theta);
    double dt, dh;
    const bool lev_ok = group_dt(P, g, dt, dh);
    const T hdt = T(0.5 * dt / dh);
    const double dtdh = dt / dh;
    const int t = threadIdx.x;
    const int i = t & 15, j = t >> 4;
    if (!lev_ok && P.bad && t == 0) atomicAdd(P.bad + 1, 1ull);
    unsigned n_bad = 0;  // output cells that are not physical or not finite
    const T *U = P.in + g * GIN;
    T *out = P.out + g * GOUT;
    int n_pred = 0, n_roe = 0;
    double st[NSTAT];
#pragma unroll
    for (int q = 0; q < NSTAT; ++q) st[q] = 0.0;
    T fz[NV];         // z flux below the current plane
    double dxy[NV];   // (dF_x + dF_y) of this column in the previous plane
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        fz[v] = T(0);
        dxy[v] = 0.0;
    }
    for (int k = 0; k <= NI; ++k) {
        // the old state of this column's cell in plane k - 1, loaded before the z
        // face's solve so that its latency overlaps it
        T uold[NV];
        if (k >= 1) {
#pragma unroll
            for (int v = 0; v < NV; ++v) uold[v] = U[v * (NP * NP * NP) + ((k - 1 + NG) * NP + (j + NG)) * NP + (i + NG)];
        }
        T fzn[NV];
        final_flux<2>(P, g, i, j, k, hdt, c, n_pred, n_roe, fzn);
        if (k >= 1) {
            // plane k - 1 is complete: U - dt/dh ((dF_x + dF_y) + dF_z)
            const int kk = k - 1;
            T un[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double dfz = double(fzn[v]) - double(fz[v]);
                const double u0 = double(uold[v]);
                const T o = T(u0 - dtdh * (dxy[v] + dfz));
                out[v * (NI * NI * NI) + (kk * NI + j) * NI + i] = o;
                un[v] = o;
                st[v] += double(o);
            }
            const double sp = double(signal_speed(un[0], un[1], un[2], un[3], un[4], c));
            n_bad += sp != sp;
            st[5] = max_nan(st[5], sp);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) fz[v] = fzn[v];
        if (k == NI) break;
        // x and y faces of plane k: face i of row j and face j of column i; then
        // the faces 16 of the rows (lanes 0..15 of wave k mod 4) and of the
        // columns (lanes 0..15 of wave k + 1 mod 4), so that no wave takes both
        {
            T F[NV];
            final_flux<0>(P, g, i, j, k, hdt, c, n_pred, n_roe, F);
#pragma unroll
            for (int v = 0; v < NV; ++v) S.f.fx[v][j][i] = F[v];
            final_flux<1>(P, g, i, j, k, hdt, c, n_pred, n_roe, F);
#pragma unroll
            for (int v = 0; v < NV; ++v) S.f.fy[v][j][i] = F[v];
            const int wave = t >> 6, lane = t & 63;
            if (lane < NI && wave == (k & 3)) {
                final_flux<0>(P, g, NI, lane, k, hdt, c, n_pred, n_roe, F);
#pragma unroll
                for (int v = 0; v < NV; ++v) S.f.fx[v][lane][NI] = F[v];
            }
            if (lane < NI && wave == ((k + 1) & 3)) {
                final_flux<1>(P, g, lane, NI, k, hdt, c, n_pred, n_roe, F);
#pragma unroll
                for (int v = 0; v < NV; ++v) S.f.fy[v][NI][lane] = F[v];
            }
        }
        __syncthreads();  // the plane's x and y fluxes visible
#pragma unroll
        for (int v = 0; v < NV; ++v)
            dxy[v] = (double(S.f.fx[v][j][i + 1]) - double(S.f.fx[v][j][i])) +
                     (double(S.f.fy[v][j + 1][i]) - double(S.f.fy[v][j][i]));
        __syncthreads();  // read before the next plane's fluxes overwrite them
    }
    // fallback counts: this stage's, plus those of the predictor and the
    // transverse fluxes, added once by thread 0
    st[6] = double(n_pred) + (t == 0 ? double(P.counts[2 * g]) : 0.0);
    st[7] = double(n_roe) + (t == 0 ? double(P.counts[2 * g + 1]) : 0.0);
    if (P.bad && n_bad) atomicAdd(P.bad, (unsigned long long)n_bad);
    if (P.stats) block_reduce_stats<256>(st, S.red, P.stats + g * NSTAT);
}


// ---- the fused z-sweep (variant 0) -------------------------------------------

template <typename T>
struct FusedLds {
    union {
        struct {
            T w[3][NV][NP][NP];    // primitive states of padded planes: plane m in slot (m + 3) % 3
            T xm[NV][CE][CE];      // predicted minus-x state of plane s at [v][j + 1][i + 1]
            T ym[NV][CE][CE];      // predicted minus-y state, likewise
            T ftx[NV][CE][CE];     // transverse x flux of plane s at face (i + 1/2, j): [v][j + 1][i + 1]
            T fty[NV][CE][CE];     // transverse y flux at face (i, j + 1/2): [v][j + 1][i + 1]
            T cxp[NV][NI][NI + 1];  // corrected plus-x state of plane s - 1, cell (f - 1, j) at [v][j][f]
            T cyp[NV][NI + 1][NI];  // corrected plus-y state, cell (i, f - 1) at [v][f][i]
            T fx[NV][NI][NI + 1];   // final x flux of plane s - 1 at face f of row j: [v][j][f]
            T fy[NV][NI + 1][NI];   // final y flux at face f of column i: [v][f][i]
        } a;
        double red[384 * NSTAT];  // the stats reduction, after the sweep
    };
};

// Threads per group: one per cell of an 18 x 18 plane (324 of 384 busy).
// LDS per group: 70 KB in float, 140 KB in double.  A work-group sweeps
// FusedShape::groups groups side by side, so that its waves spread evenly over
// the CU's four SIMDs (a lone 6-wave work-group puts two waves on two SIMDs
// and one on the others): float two groups (12 waves, 140 KB, three waves per
// SIMD), double one.
constexpr int FUSED_THREADS = 384;

template <typename T>
struct FusedShape;
template <>
struct FusedShape<float> {
    static constexpr int waves = 3, groups = 2;
};
template <>
struct FusedShape<double> {
    static constexpr int waves = 2, groups = 1;
};

// u = p - hdt (a + b), or p itself (and false) when that leaves the physical
// set; a, b are the two transverse flux differences in the order of the
// pipeline's `corrected` (the lower direction first)
template <typename T>
__device__ __forceinline__ bool correct_state(const T p[NV], const T a[NV], const T b[NV], T hdt, T u[NV]) {
    T q[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const T corr = a[v] + b[v];
        q[v] = p[v] - hdt * corr;
    }
    if (!physical(q)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = p[v];
        return false;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = q[v];
    return true;
}

template <typename T>
__global__ __attribute__((amdgpu_flat_work_group_size(FUSED_THREADS * FusedShape<T>::groups,
                                                      FUSED_THREADS * FusedShape<T>::groups),
                          amdgpu_waves_per_eu(FusedShape<T>::waves, 8)))
void ctu_fused(CtuArgs<T> P) {
    constexpr int NT = FUSED_THREADS;
    static_assert(NT >= CE * CE && NT % 64 == 0, "one thread per cell of a plane, whole waves");
    constexpr int G = FusedShape<T>::groups;
    __shared__ FusedLds<T> SS[G];
    const int half = G > 1 ? int(threadIdx.x) / NT : 0;
    FusedLds<T> &S = SS[half];
    const int64_t g_raw = int64_t(blockIdx.x) * G + half;
    if (G == 1 && g_raw >= P.n_groups) return;
    // with several groups per work-group the last slot may lie past the batch:
    // its threads then take no cell (they read group 0's input and write
    // nothing) but still meet every barrier
    const bool live = G == 1 || g_raw < P.n_groups;
    const int64_t g = live ? g_raw : 0;
    const Consts<T> c = make_consts<T>(P.gamma, P.theta);
    double dt, dh;
    const bool lev_ok = group_dt(P, g, dt, dh);
    const T hdt = T(0.5 * dt / dh);
    const double dtdh = dt / dh;
    // The Roe fluxes of this sweep are kept doubled (roe_dir<..., true>: 2F, the
    // flux sums without their exact factor 1/2); the corrections, the update and
    // the stored flux planes take that 1/2 instead, with the same values bitwise.
    const T hdt2 = c.half * hdt;
    const double hdtdh = 0.5 * dtdh;
    const T *U = P.in + g * GIN;
    T *out = P.out + g * GOUT;
    const int t = threadIdx.x - half * NT;
    if (live && !lev_ok && P.bad && t == 0) atomicAdd(P.bad + 1, 1ull);
    const bool mine = live && t < CE * CE;
    const int i = t % CE - 1, j = t / CE - 1;  // this thread's column, meaningful when mine
    const int ii = i + NG, jj = j + NG;        // its padded position
    const bool in_i = i >= 0 && i < NI, in_j = j >= 0 && j < NI;
    int n_pred = 0, n_roe = 0;
    unsigned n_bad = 0;
    double st[NSTAT];
#pragma unroll
    for (int q = 0; q < NSTAT; ++q) st[q] = 0.0;

    // carried from step s - 1 to step s
    T zpp[NV];   // predicted plus-z state of plane s - 1 (transverse z flux)
    T czp[NV];   // corrected plus-z state of plane s - 1 (final z flux)
    T ftzb[NV];  // transverse z flux below plane s - 1
    T fzb[NV];   // final z flux below plane s - 1
    T xp[NV], yp[NV];  // predicted plus-x and plus-y states of plane s - 1
#pragma unroll
    for (int v = 0; v < NV; ++v) zpp[v] = czp[v] = ftzb[v] = fzb[v] = xp[v] = yp[v] = T(0);

    auto fill = [&](int m) {  // padded plane m (-2..17) into its ring slot
        const int slot = (m + 3) % 3;
        for (int q = t; q < NPL; q += NT) {
            const int qi = q % NP, qj = q / NP;
            T w[NV];
            prim_at(U, qi - NG, qj - NG, m, c, w);
#pragma unroll
            for (int v = 0; v < NV; ++v) S.a.w[slot][v][qj][qi] = w[v];
        }
    };
    // The sweep's next plane: in float its conserved values are loaded into
    // registers at the top of a step (positions t and t + NT of the 20 x 20
    // plane) and converted into the ring at the step's end, so the loads overlap
    // the step (2.17 -> 2.04 ms at 256^3).  In double those registers spill
    // (3.39 -> 4.39 ms), and the plane is loaded and converted at the step's end.
    constexpr bool PREFETCH = sizeof(T) == 4;
    constexpr int NPOS = (NPL + NT - 1) / NT;
    T pre[NPOS][NV];
    auto fetch = [&](int m) {
#pragma unroll
        for (int r = 0; r < NPOS; ++r) {
            const int q = t + r * NT;
            if (q < NPL) {
                const T *src = U + (m + NG) * NPL + q;
#pragma unroll
                for (int v = 0; v < NV; ++v) pre[r][v] = src[v * NP * NP * NP];
            }
        }
    };
    auto store = [&](int m) {
        const int slot = (m + 3) % 3;
#pragma unroll
        for (int r = 0; r < NPOS; ++r) {
            const int q = t + r * NT;
            if (q < NPL) {
                const T ir = rcp(pre[r][0]);
                const T u = pre[r][1] * ir, v = pre[r][2] * ir, wz = pre[r][3] * ir;
                T *dst = &S.a.w[slot][0][0][0] + q;
                dst[0 * NPL] = pre[r][0];
                dst[1 * NPL] = u;
                dst[2 * NPL] = v;
                dst[3 * NPL] = wz;
                dst[4 * NPL] = c.gm1 * (pre[r][4] - c.half * pre[r][0] * (u * u + v * v + wz * wz));
            }
        }
    };
    // cell average of padded cell (i, j, k): the predictor's first-order fallback
    auto average = [&](int k, T u[NV]) {
        const int o = ((k + NG) * NP + jj) * NP + ii;
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = U[o + v * NP * NP * NP];
    };
    fill(-2);
    fill(-1);
    fill(0);

    for (int s = -1; s <= NI; ++s) {
        const bool ahead = s + 2 <= NI + 1;
        if (PREFETCH && ahead) fetch(s + 2);
        __syncthreads();  // B0: padded planes s - 1, s, s + 1 in the ring
        const int sm = (s + 2) % 3, s0 = (s + 3) % 3, sp = (s + 4) % 3;
        const bool e1 = mine && in_e1(i, j, s);
        const int kb = s - 1;  // the plane whose x / y states are corrected and fluxes finished

        // ---- A: z predictor, transverse z flux, corrections of plane s - 1, x / y predictor
        T W0[NV], zm[NV], zpn[NV], ftz[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) W0[v] = zm[v] = zpn[v] = ftz[v] = T(0);
        if (e1) {
            T wl[NV], wr[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                W0[v] = S.a.w[s0][v][jj][ii];
                wl[v] = S.a.w[sm][v][jj][ii];
                wr[v] = S.a.w[sp][v][jj][ii];
            }
            if (!predict_from<2>(W0, wl, wr, hdt, c, zm, zpn)) {
                ++n_pred;
                average(s, zm);
#pragma unroll
                for (int v = 0; v < NV; ++v) zpn[v] = zm[v];
            }
            if (s >= 0 && in_e1(i, j, s - 1)) n_roe += roe_dir<2, true>(zpp, zm, c, ftz);
        }
        // corrected x and y states of plane kb (whose other two coordinates lie in
        // the interior); the plus states go to LDS for the neighbour's face
        T cxm[NV], cym[NV];
        if (mine && kb >= 0 && kb < NI) {
            T a[NV], b[NV], u[NV], p[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) b[v] = ftz[v] - ftzb[v];
            if (in_j) {  // x states: y and z differences
#pragma unroll
                for (int v = 0; v < NV; ++v) a[v] = S.a.fty[v][j + 1][i + 1] - S.a.fty[v][j][i + 1];
                if (i >= 0) {  // minus-x state: face i
#pragma unroll
                    for (int v = 0; v < NV; ++v) p[v] = S.a.xm[v][j + 1][i + 1];
                    n_pred += !correct_state(p, a, b, hdt2, cxm);
                }
                if (i < NI) {  // plus-x state: face i + 1
                    n_pred += !correct_state(xp, a, b, hdt2, u);
#pragma unroll
                    for (int v = 0; v < NV; ++v) S.a.cxp[v][j][i + 1] = u[v];
                }
            }
            if (in_i) {  // y states: x and z differences
#pragma unroll
                for (int v = 0; v < NV; ++v) a[v] = S.a.ftx[v][j + 1][i + 1] - S.a.ftx[v][j + 1][i];
                if (j >= 0) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) p[v] = S.a.ym[v][j + 1][i + 1];
                    n_pred += !correct_state(p, a, b, hdt2, cym);
                }
                if (j < NI) {
                    n_pred += !correct_state(yp, a, b, hdt2, u);
#pragma unroll
                    for (int v = 0; v < NV; ++v) S.a.cyp[v][j + 1][i] = u[v];
                }
            }
        }
        if (e1) {
            T wl[NV], wr[NV], um[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                wl[v] = S.a.w[s0][v][jj][ii - 1];
                wr[v] = S.a.w[s0][v][jj][ii + 1];
            }
            if (!predict_from<0>(W0, wl, wr, hdt, c, um, xp)) {
                ++n_pred;
                average(s, um);
#pragma unroll
                for (int v = 0; v < NV; ++v) xp[v] = um[v];
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                S.a.xm[v][j + 1][i + 1] = um[v];
                wl[v] = S.a.w[s0][v][jj - 1][ii];
                wr[v] = S.a.w[s0][v][jj + 1][ii];
            }
            if (!predict_from<1>(W0, wl, wr, hdt, c, um, yp)) {
                ++n_pred;
                average(s, um);
#pragma unroll
                for (int v = 0; v < NV; ++v) yp[v] = um[v];
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) S.a.ym[v][j + 1][i + 1] = um[v];
        }
        __syncthreads();  // B1: minus states of plane s and corrected plus states of plane kb
        // the old state of the cell of plane kb that E updates, loaded before C so
        // that the load overlaps the C phase instead of waiting in E (256^3 step:
        // 1.357 -> 1.317 ms FP32, 3.347 -> 3.230 ms FP64)
        T uold[NV];
        if (mine && in_i && in_j && kb >= 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v) uold[v] = U[v * (NP * NP * NP) + ((kb + NG) * NP + jj) * NP + ii];
        }

        // ---- C: transverse x / y fluxes of plane s, final x / y fluxes of plane kb
        if (e1) {
            T R[NV], F[NV];
            if (in_e1(i + 1, j, s)) {
#pragma unroll
                for (int v = 0; v < NV; ++v) R[v] = S.a.xm[v][j + 1][i + 2];
                n_roe += roe_dir<0, true>(xp, R, c, F);
#pragma unroll
                for (int v = 0; v < NV; ++v) S.a.ftx[v][j + 1][i + 1] = F[v];
            }
            if (in_e1(i, j + 1, s)) {
#pragma unroll
                for (int v = 0; v < NV; ++v) R[v] = S.a.ym[v][j + 2][i + 1];
                n_roe += roe_dir<1, true>(yp, R, c, F);
#pragma unroll
                for (int v = 0; v < NV; ++v) S.a.fty[v][j + 1][i + 1] = F[v];
            }
        }
        if (mine && kb >= 0 && kb < NI) {
            T L[NV], F[NV];
            if (in_j && i >= 0) {  // x face i of row j: plus-x of cell i - 1, minus-x of cell i
#pragma unroll
                for (int v = 0; v < NV; ++v) L[v] = S.a.cxp[v][j][i];
                n_roe += roe_dir<0, true>(L, cxm, c, F);
#pragma unroll
                for (int v = 0; v < NV; ++v) S.a.fx[v][j][i] = F[v];
                if (P.flux && (i & 7) == 0) {
                    T *dst = P.flux + g * GFLX + ((0 * 3 + (i >> 3)) * NV) * NINNER + kb * NI + j;
#pragma unroll
                    for (int v = 0; v < NV; ++v) dst[v * NINNER] = c.half * F[v];
                }
            }
            if (in_i && j >= 0) {  // y face j of column i
#pragma unroll
                for (int v = 0; v < NV; ++v) L[v] = S.a.cyp[v][j][i];
                n_roe += roe_dir<1, true>(L, cym, c, F);
#pragma unroll
                for (int v = 0; v < NV; ++v) S.a.fy[v][j][i] = F[v];
                if (P.flux && (j & 7) == 0) {
                    T *dst = P.flux + g * GFLX + ((1 * 3 + (j >> 3)) * NV) * NINNER + kb * NI + i;
#pragma unroll
                    for (int v = 0; v < NV; ++v) dst[v * NINNER] = c.half * F[v];
                }
            }
        }
        __syncthreads();  // B2: transverse fluxes of plane s, final x / y fluxes of plane kb

        // ---- E: corrected z states of plane s, final z flux below it, update of plane kb
        if (mine && in_i && in_j) {
            T a[NV], b[NV], czm[NV], fz[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                fz[v] = T(0);
                a[v] = S.a.ftx[v][j + 1][i + 1] - S.a.ftx[v][j + 1][i];
                b[v] = S.a.fty[v][j + 1][i + 1] - S.a.fty[v][j][i + 1];
            }
            if (s >= 0) n_pred += !correct_state(zm, a, b, hdt2, czm);
            if (s >= 0) {  // final z flux at face s: plus-z of plane s - 1, minus-z of plane s
                n_roe += roe_dir<2, true>(czp, czm, c, fz);
                if (P.flux && (s & 7) == 0) {
                    T *dst = P.flux + g * GFLX + ((2 * 3 + (s >> 3)) * NV) * NINNER + j * NI + i;
#pragma unroll
                    for (int v = 0; v < NV; ++v) dst[v * NINNER] = c.half * fz[v];
                }
            }
            if (kb >= 0) {
                // plane kb is complete: U - dt/dh ((dF_x + dF_y) + dF_z)
                T un[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const double dxy = (double(S.a.fx[v][j][i + 1]) - double(S.a.fx[v][j][i])) +
                                       (double(S.a.fy[v][j + 1][i]) - double(S.a.fy[v][j][i]));
                    const double dfz = double(fz[v]) - double(fzb[v]);
                    const double u0 = double(uold[v]);
                    const T o = T(u0 - hdtdh * (dxy + dfz));
                    out[v * (NI * NI * NI) + (kb * NI + j) * NI + i] = o;
                    un[v] = o;
                    st[v] += double(o);
                }
                const double sp_ = double(signal_speed(un[0], un[1], un[2], un[3], un[4], c));
                n_bad += sp_ != sp_;
                st[5] = max_nan(st[5], sp_);
            }
            if (s < NI) n_pred += !correct_state(zpn, a, b, hdt2, czp);
#pragma unroll
            for (int v = 0; v < NV; ++v) fzb[v] = fz[v];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            zpp[v] = zpn[v];
            ftzb[v] = ftz[v];
        }
        if (ahead) {  // into the slot of plane s - 1, no longer read
            if constexpr (PREFETCH)
                store(s + 2);
            else
                fill(s + 2);
        }
    }
    if (P.bad && n_bad) atomicAdd(P.bad, (unsigned long long)n_bad);
    if (P.stats) {
        st[6] = double(n_pred);
        st[7] = double(n_roe);
        __syncthreads();  // the ring and the plane arrays are no longer read
        block_reduce_stats<NT>(st, S.red, live ? P.stats + g * NSTAT : nullptr, t);
    }
}

}  // namespace

size_t ctu_workspace_bytes(int64_t n, int elem) {
    // per group: the intermediate arrays, then two int32 counters per group
    return size_t(n) * size_t(WORK_VALUES) * size_t(elem) + size_t(n) * 2 * sizeof(int) + 256;
}

template <typename T>
hipError_t launch_ctu(const T *in, int64_t n, const int8_t *level, int n_levels, const double *dt_dev,
                      const double *dh_dev, double gamma, double theta, T *fluxes, T *out, double *stats,
                      unsigned long long *bad, int variant, void *work, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    CtuArgs<T> P;
    P.in = in;
    P.out = out;
    P.flux = fluxes;
    P.stats = stats;
    P.level = level;
    P.dt_dev = dt_dev;
    P.dh_dev = dh_dev;
    P.n_levels = n_levels;
    P.bad = bad;
    P.gamma = gamma;
    P.theta = theta;
    P.n_groups = n;
    P.work = nullptr;
    P.counts = nullptr;
    if (variant == 0) {
        constexpr int G = FusedShape<T>::groups;
        hipLaunchKernelGGL(ctu_fused<T>, dim3(unsigned((n + G - 1) / G)), dim3(FUSED_THREADS * G), 0, s, P);
        return hipGetLastError();
    }
    P.work = static_cast<T *>(work);
    // counters after the arrays, 256-byte aligned
    const size_t off = (size_t(n) * size_t(WORK_VALUES) * sizeof(T) + 255) & ~size_t(255);
    P.counts = reinterpret_cast<int *>(static_cast<char *>(work) + off);
    hipLaunchKernelGGL(ctu_zero<T>, dim3(unsigned((2 * n + 255) / 256)), dim3(256), 0, s, P);
    hipLaunchKernelGGL(ctu_predict<T>, dim3(unsigned(n)), dim3(PRED_THREADS), 0, s, P);
    hipLaunchKernelGGL(ctu_final<T>, dim3(unsigned(n)), dim3(256), 0, s, P);
    return hipGetLastError();
}

template hipError_t launch_ctu<float>(const float *, int64_t, const int8_t *, int, const double *,
                                      const double *, double, double, float *, float *, double *,
                                      unsigned long long *, int, void *, hipStream_t);
template hipError_t launch_ctu<double>(const double *, int64_t, const int8_t *, int, const double *,
                                       const double *, double, double, double *, double *, double *,
                                       unsigned long long *, int, void *, hipStream_t);

}  // namespace gamer
