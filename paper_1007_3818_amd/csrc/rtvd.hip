// rtvd.hip -- the relaxing TVD scheme (the solver the paper compares
// MUSCL-Hancock with): three dimensionally split sweeps per step, one launch
// per sweep, each advancing every pencil along the sweep direction by the
// relaxing scheme's half step and full step.  The block shrinks by three cells
// per side along the sweep direction only, so the three sweeps go 22^3 ->
// 16 x 22 x 22 -> 16 x 16 x 22 -> 16^3 (x, y, z order) through two workspace
// arrays.  x sweeps: a work-group stages 11 pencils in LDS, one lane per
// position, so that the loads along x coalesce.  y and z sweeps: one thread per pencil, streaming along it
// in registers, with consecutive threads on consecutive x.
#include "device_math.h"
#include "internal.h"

namespace gamer {
namespace {

constexpr int RP = 22;      // padded cells per axis (three ghost cells per side)
constexpr int RG = 3;
constexpr int XPEN = 11;    // x pencils per work-group, 22 lanes each
// LDS stride per pencil: unpadded, so that the 64 lanes of a wave, which hold
// consecutive positions of consecutive pencils, take consecutive words (a
// one-word pad put some of them on the same bank; 23 -> 22 took the FP32 step
// from 1.018 to 0.977 ms at 256^3)
constexpr int XSTR = RP;

template <typename T>
struct SweepArgs {
    const T *in;      // block [n][5][ez][ey][ex], or the periodic state (gx > 0)
    int gx, gy, gz;   // > 0: the first sweep reads a periodic grid of groups
    int ex, ey, ez;   // input block extents
    int d;            // sweep axis
    T *out;           // [n][5][..] with extent e[d] - 6 along d
    const int8_t *level;
    const double *dt_dev, *dh_dev;
    int n_levels;     // a level byte outside [0, n_levels) gives the group NaN dt and dh
    double gamma;
    int64_t n_groups;
};

template <typename T>
struct RtvdLds {
    T u[NV][XPEN][XSTR];   // the pencils' input
    T fr[NV][XPEN][XSTR];  // c (u + w), then from the half-step state
    T fl[NV][XPEN][XSTR];  // c (u - w), likewise
    T fc[NV][XPEN][XSTR];  // second-order flux of face c0 + 1/2 at index c0
};

// freezing speed c = |v_d| + c_s and the right/left-moving fluxes
// fr = c (u + w), fl = c (u - w) with w = F_d(u) / c, evaluated as c u + F and
// c u - F (the same values up to rounding, without the division by c)
template <typename T>
__device__ __forceinline__ void relax(const T u[NV], int d, T g, T gm1, T fr[NV], T fl[NV]) {
    const T ir = rcp(u[0]);
    const T vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
    const T vd = d == 0 ? vx : (d == 1 ? vy : vz);
    const T p = gm1 * (u[4] - T(0.5) * (u[1] * vx + u[2] * vy + u[3] * vz));
    const T c = fabs(vd) + sqrt_(g * p * ir);
    T F[NV];
    F[0] = u[1 + d];
    F[1] = u[1] * vd;
    F[2] = u[2] * vd;
    F[3] = u[3] * vd;
    F[1 + d] += p;
    F[4] = (u[4] + p) * vd;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const T cu = c * u[v];
        fr[v] = cu + F[v];
        fl[v] = cu - F[v];
    }
}

// Van Leer's limiter of the half differences, VL(x/2, y/2) = 2 (x/2)(y/2) /
// (x/2 + y/2) if their product is positive, else 0, written as x y / (x + y):
// halving is exact and the reciprocal scales exactly, so the value is the
// same bitwise (subnormal products aside) with three fewer multiplications.
template <typename T>
__device__ __forceinline__ T vanleer_half(T x, T y) {
    const T xy = x * y;
    return xy > T(0) ? xy * rcp(x + y) : T(0);
}

// x sweeps: 11 pencils per work-group, one lane per position (22 lanes per
// pencil, lanes 242..255 idle), positions fastest in LDS.  Each phase is one
// pass: load, relaxed fluxes of the 22 input cells, half-step state and its
// relaxed fluxes at positions 1..20, the second-order flux of each of the 17
// faces once, and the update of the 16 output cells.  Consecutive lanes read
// consecutive x, so the loads of a wave are contiguous along each pencil.
// E is the block's extent along y and z (22 for the first sweep of a step, 16
// for the last), so every index below divides by a constant.  Work-groups: the
// padded input runs a grid of TILES * XCHUNK by ceil(n / XCHUNK), group-major
// within a row; the periodic input a grid of TILES * gx by gy by gz, one row
// of tiles per group.
template <int E>
constexpr int x_tiles() { return (E * E + XPEN - 1) / XPEN; }
constexpr int XCHUNK = 8192;  // groups per grid row of the padded-input x sweep

template <typename T, int E, bool PERIODIC>
__global__ __launch_bounds__(256) void rtvd_sweep_kernel(SweepArgs<T> P) {
    constexpr int TILES = x_tiles<E>();
    constexpr int VIN = RP * E * E, VOUT = NI * E * E;  // cells per variable, input and output
    __shared__ RtvdLds<T> S;
    const int t = threadIdx.x;
    int gi, tile, bx = 0, by = 0, bz = 0;
    if constexpr (PERIODIC) {
        bx = int(blockIdx.x / unsigned(TILES));
        tile = int(blockIdx.x) - bx * TILES;
        by = int(blockIdx.y);
        bz = int(blockIdx.z);
        gi = bx + P.gx * (by + P.gy * bz);
    } else {
        const int gl = int(blockIdx.x / unsigned(TILES));
        tile = int(blockIdx.x) - gl * TILES;
        gi = int(blockIdx.y) * XCHUNK + gl;  // < 2^31: the host caps n_groups
        if (gi >= P.n_groups) return;
    }
    const int64_t g = gi;
    const int q = t / RP, l = t - q * RP;  // pencil within the tile, position
    const int p = tile * XPEN + q;        // pencil index within the group: (y, z), y fastest
    const bool live = q < XPEN && p < E * E;
    const int iy = live ? p % E : 0, iz = live ? p / E : 0;

    double dt, dh;
    level_dt(P.level, g, P.n_levels, P.dt_dev, P.dh_dev, dt, dh);
    const double dtdx = dt / dh;
    const T g_ = T(P.gamma), gm1 = T(P.gamma - 1.0);
    const T hdt2 = T(0.25 * dtdx);     // half of dt/(2 dx): the fluxes below are kept doubled
    const double hdtdx = 0.5 * dtdx;

    // ---- load position l of pencil q ----
    if (live) {
        const T *src;
        int64_t vs;
        if constexpr (PERIODIC) {
            const int NX = P.gx * NI, NY = P.gy * NI, NZ = P.gz * NI;
            int X = bx * NI + l - RG, Y = by * NI + iy - RG, Z = bz * NI + iz - RG;
            X = X < 0 ? X + NX : (X >= NX ? X - NX : X);
            Y = Y < 0 ? Y + NY : (Y >= NY ? Y - NY : Y);
            Z = Z < 0 ? Z + NZ : (Z >= NZ ? Z - NZ : Z);
            const int64_t grp = X / NI + int64_t(P.gx) * (Y / NI + int64_t(P.gy) * (Z / NI));
            src = P.in + grp * GOUT + ((Z % NI) * NI + (Y % NI)) * NI + (X % NI);
            vs = NI * NI * NI;
        } else {
            src = P.in + g * (NV * VIN) + (iz * E + iy) * RP + l;
            vs = VIN;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) S.u[v][q][l] = src[v * vs];
    }
    __syncthreads();

    // ---- half step: first-order relaxed fluxes of the input ----
    if (live) {
        T u[NV], fr[NV], fl[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = S.u[v][q][l];
        relax(u, 0, g_, gm1, fr, fl);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            S.fr[v][q][l] = fr[v];
            S.fl[v][q][l] = fl[v];
        }
    }
    __syncthreads();
    // half-step state of positions 1..20
    const bool hs = live && l >= 1 && l <= RP - 2;
    T h[NV];
    if (hs) {
        // first-order fluxes (fr_i - fl_{i+1}) / 2, their 1/2 taken into hdt2
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const T Fp = S.fr[v][q][l] - S.fl[v][q][l + 1];
            const T Fm = S.fr[v][q][l - 1] - S.fl[v][q][l];
            h[v] = S.u[v][q][l] - hdt2 * (Fp - Fm);
        }
    }
    __syncthreads();  // every first-order flux read before it is overwritten
    if (hs) {
        T fr[NV], fl[NV];
        relax(h, 0, g_, gm1, fr, fl);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            S.fr[v][q][l] = fr[v];
            S.fl[v][q][l] = fl[v];
        }
    }
    __syncthreads();

    // ---- full step: the second-order flux of face c0 + 1/2, c0 = l + 2 ----
    if (live && l <= NI) {
        const int c0 = l + 2;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const T r0 = S.fr[v][q][c0 - 1], r1 = S.fr[v][q][c0], r2 = S.fr[v][q][c0 + 1];
            const T l1 = S.fl[v][q][c0], l2 = S.fl[v][q][c0 + 1], l3 = S.fl[v][q][c0 + 2];
            const T R = r1 + vanleer_half(r1 - r0, r2 - r1);
            const T L = l2 + vanleer_half(l1 - l2, l2 - l3);
            S.fc[v][q][c0] = R - L;  // twice the face flux (R - L) / 2
        }
    }
    __syncthreads();
    // update of cell i = l + 3 (output position l)
    if (live && l < NI) {
        const int i = l + RG;
        T *dst = P.out + g * (NV * VOUT) + (iz * E + iy) * NI + l;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double o = double(S.u[v][q][i]) - hdtdx * (double(S.fc[v][q][i]) - double(S.fc[v][q][i - 1]));
            dst[v * VOUT] = T(o);
        }
    }
}

// The same sweep with one thread per pencil, streaming along it: the relaxed
// fluxes of each cell, its half-step state and each face flux are computed once,
// in registers, with no LDS and no barrier.  Consecutive threads take
// consecutive pencils along the fastest transverse axis, so for y and z sweeps
// the loads and stores of one position are contiguous across the wave.  D is
// the sweep axis; PERIODIC reads the periodic grid of unpadded groups (first
// sweep of a step) with the ghost cells taken from the neighbouring groups.
template <typename T, int D, bool PERIODIC>
__global__ __launch_bounds__(256) void rtvd_stream_kernel(SweepArgs<T> P) {
    constexpr int A = D == 0 ? 1 : 0, B = D == 2 ? 1 : 2;  // transverse axes, A fastest
    const int e[3] = {P.ex, P.ey, P.ez};
    int eo[3] = {P.ex, P.ey, P.ez};
    eo[D] -= 2 * RG;
    const int ea = e[A], npen = e[A] * e[B];
    // 32-bit index arithmetic: the host caps n_groups * pencils below 2^31.
    // Work-groups go to the 8 XCDs round-robin (work-group b to XCD b mod 8),
    // each with its own L2; the periodic first sweep numbers them so that each
    // XCD takes a contiguous run of pencils, and so mostly whole groups with
    // their x and y neighbours, whose cells it reads again as ghost cells.
    int b = int(blockIdx.x);
    if constexpr (PERIODIC) {
        const int nb = int(gridDim.x), x = b % 8, j = b / 8, q = nb / 8, r = nb % 8;
        b = x * q + (x < r ? x : r) + j;
    }
    const int tid = b * 256 + int(threadIdx.x);
    if (int64_t(tid) >= P.n_groups * npen) return;
    const int gi = tid / npen;
    const int p = tid - gi * npen;
    const int64_t g = gi;
    const int ia = p % ea, ib = p / ea;
    const int64_t vin = int64_t(e[0]) * e[1] * e[2], vout = int64_t(eo[0]) * eo[1] * eo[2];
    const int si[3] = {1, e[0], e[0] * e[1]}, so[3] = {1, eo[0], eo[0] * eo[1]};

    // cell s of the pencil (s = 0..21 along D) is src(s)[v * vstride]
    const T *base[3];  // padded input: one base; periodic: the groups below, at, above along D
    int64_t vstride;
    if constexpr (PERIODIC) {
        const int gx = P.gx, gy = P.gy, gz = P.gz;
        const int bc[3] = {gi % gx, (gi / gx) % gy, gi / (gx * gy)};
        const int nb[3] = {gx, gy, gz};
        // transverse global coordinates, wrapped
        int gc[3], lc[3];
        const int tr[2] = {A, B}, ti[2] = {ia, ib};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int ax = tr[q], N = nb[ax] * NI;
            int X = bc[ax] * NI + ti[q] - RG;
            X = X < 0 ? X + N : (X >= N ? X - N : X);
            gc[ax] = X / NI;
            lc[ax] = X % NI;
        }
        lc[D] = 0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {  // the group along D: below, own, above
            int G = bc[D] + q - 1;
            G = G < 0 ? G + nb[D] : (G >= nb[D] ? G - nb[D] : G);
            gc[D] = G;
            const int64_t grp = gc[0] + int64_t(gx) * (gc[1] + int64_t(gy) * gc[2]);
            base[q] = P.in + grp * GOUT + (lc[2] * NI + lc[1]) * NI + lc[0];
        }
        vstride = NI * NI * NI;
    } else {
        base[0] = base[1] = base[2] = P.in + g * NV * vin + int64_t(ia) * si[A] + int64_t(ib) * si[B];
        vstride = vin;
    }
    T *dst = P.out + g * NV * vout + int64_t(ia) * so[A] + int64_t(ib) * so[B];

    double dt, dh;
    level_dt(P.level, g, P.n_levels, P.dt_dev, P.dh_dev, dt, dh);
    const double dtdx = dt / dh;
    const T hdt2 = T(0.25 * dtdx);     // half of dt/(2 dx): the fluxes below are kept doubled
    const double hdtdx = 0.5 * dtdx;
    const T g_ = T(P.gamma), gm1 = T(P.gamma - 1.0);
    constexpr int LSTR[3] = {1, NI, NI * NI};  // strides inside an unpadded group

    T u[RP][NV], fr[RP][NV], fl[RP][NV], fr2[RP][NV], fl2[RP][NV], Fc[RP][NV];
    // cell s of the pencil into u[s]; issued PREFETCH cells ahead of its use,
    // so that a wave's loads are in flight while it computes the cells before
    auto load = [&](int s) {
        const T *src;
        if constexpr (PERIODIC) {
            const int q = s < RG ? 0 : (s < RG + NI ? 1 : 2);
            const int l = s < RG ? s + NI - RG : (s < RG + NI ? s - RG : s - RG - NI);
            src = base[q] + l * LSTR[D];
        } else {
            src = base[0] + s * si[D];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) u[s][v] = src[v * vstride];
    };
    constexpr int PREFETCH = 2;  // 256^3 step: 0.976 -> 0.951 ms FP32, 1.757 -> 1.717 ms FP64
#pragma unroll
    for (int s = 0; s < PREFETCH; ++s) load(s);
#pragma unroll
    for (int s = 0; s < RP; ++s) {
        if (s + PREFETCH < RP) load(s + PREFETCH);
        relax(u[s], D, g_, gm1, fr[s], fl[s]);
        if (s < 2) continue;
        // half-step state of cell m = s - 1 and its relaxed fluxes
        const int m = s - 1;
        T h[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const T Fp = fr[m][v] - fl[m + 1][v];  // twice the first-order fluxes
            const T Fm = fr[m - 1][v] - fl[m][v];
            h[v] = u[m][v] - hdt2 * (Fp - Fm);
        }
        relax(h, D, g_, gm1, fr2[m], fl2[m]);
        // second-order flux at face c0 + 1/2, c0 = m - 2 (faces 2..18)
        const int c0 = m - 2;
        if (c0 < 2) continue;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const T r0 = fr2[c0 - 1][v], r1 = fr2[c0][v], r2 = fr2[c0 + 1][v];
            const T l1 = fl2[c0][v], l2 = fl2[c0 + 1][v], l3 = fl2[c0 + 2][v];
            const T R = r1 + vanleer_half(r1 - r0, r2 - r1);
            const T L = l2 + vanleer_half(l1 - l2, l2 - l3);
            Fc[c0][v] = R - L;  // twice the face flux
        }
        if (c0 < RG) continue;
        // update of cell i = c0 (output position i - 3)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double o = double(u[c0][v]) - hdtdx * (double(Fc[c0][v]) - double(Fc[c0 - 1][v]));
            dst[v * vout + int64_t(c0 - RG) * so[D]] = T(o);
        }
    }
}

}  // namespace

template <typename T>
size_t rtvd_workspace_elems(int64_t n_groups) {
    // two intermediate blocks: 16 x 22 x 22 and 16 x 16 x 22 cells per group
    return size_t(n_groups) * NV * (NI * RP * RP + NI * NI * RP);
}

template <typename T>
hipError_t launch_rtvd(const T *in, int gx, int gy, int gz, int64_t n, const int8_t *level,
                       int n_levels, const double *dt_dev, const double *dh_dev, double gamma,
                       int order, T *work, T *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int dirs[2][3] = {{0, 1, 2}, {2, 1, 0}};
    T *b1 = work;
    T *b2 = work + size_t(n) * NV * NI * RP * RP;
    int e[3] = {RP, RP, RP};
    const T *src = in;
    for (int k = 0; k < 3; ++k) {
        const int d = dirs[order][k];
        SweepArgs<T> P;
        P.in = src;
        P.gx = k == 0 ? gx : 0;
        P.gy = gy;
        P.gz = gz;
        P.ex = e[0];
        P.ey = e[1];
        P.ez = e[2];
        P.d = d;
        P.out = k == 0 ? b1 : (k == 1 ? b2 : out);
        P.level = level;
        P.dt_dev = dt_dev;
        P.dh_dev = dh_dev;
        P.n_levels = n_levels;
        P.gamma = gamma;
        P.n_groups = n;
        const int ta = d == 0 ? 1 : 0, tb = d == 2 ? 1 : 2;
        if (d != 0) {
            // y and z pencils: one thread each, streaming (contiguous across the wave)
            if (n * e[ta] * e[tb] >= int64_t(1) << 31) return hipErrorInvalidValue;
            const int64_t blocks = (n * e[ta] * e[tb] + 255) / 256;
            const dim3 gr(static_cast<unsigned>(blocks)), bl(256);
            if (d == 1) {
                if (P.gx > 0) hipLaunchKernelGGL((rtvd_stream_kernel<T, 1, true>), gr, bl, 0, s, P);
                else hipLaunchKernelGGL((rtvd_stream_kernel<T, 1, false>), gr, bl, 0, s, P);
            } else {
                if (P.gx > 0) hipLaunchKernelGGL((rtvd_stream_kernel<T, 2, true>), gr, bl, 0, s, P);
                else hipLaunchKernelGGL((rtvd_stream_kernel<T, 2, false>), gr, bl, 0, s, P);
            }
        } else {
            // x pencils: 11 per work-group through LDS, so that loads along x coalesce;
            // the block is 22 x E x E with E = 22 (first sweep) or 16 (last)
            const int E = e[1];
            const int64_t tiles = E == RP ? x_tiles<RP>() : x_tiles<NI>();
            if (P.gx > 0) {
                // periodic input: first sweep, E = 22; one row of tiles per group
                if (int64_t(gx) * tiles * 256 >= int64_t(1) << 32 || gy > 65535 || gz > 65535)
                    return hipErrorInvalidValue;
                const dim3 gr(unsigned(gx * tiles), unsigned(gy), unsigned(gz));
                hipLaunchKernelGGL((rtvd_sweep_kernel<T, RP, true>), gr, dim3(256), 0, s, P);
            } else {
                const int64_t rows = (n + XCHUNK - 1) / XCHUNK;
                if (rows > 65535) return hipErrorInvalidValue;
                const dim3 gr(unsigned(tiles * (n < XCHUNK ? n : XCHUNK)), unsigned(rows));
                if (E == RP)
                    hipLaunchKernelGGL((rtvd_sweep_kernel<T, RP, false>), gr, dim3(256), 0, s, P);
                else
                    hipLaunchKernelGGL((rtvd_sweep_kernel<T, NI, false>), gr, dim3(256), 0, s, P);
            }
        }
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
        src = P.out;
        e[d] -= 2 * RG;
    }
    return hipSuccess;
}

template size_t rtvd_workspace_elems<float>(int64_t);
template size_t rtvd_workspace_elems<double>(int64_t);
template hipError_t launch_rtvd<float>(const float *, int, int, int, int64_t, const int8_t *, int,
                                       const double *, const double *, double, int, float *, float *,
                                       hipStream_t);
template hipError_t launch_rtvd<double>(const double *, int, int, int, int64_t, const int8_t *, int,
                                        const double *, const double *, double, int, double *,
                                        double *, hipStream_t);

}  // namespace gamer
