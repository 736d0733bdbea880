// aux_kernels.hip -- periodic ghost fill, per-group stats and the fixed-order
// reduction of group stats to per-level time steps and conserved totals.
#include "device_math.h"
#include "internal.h"

namespace gamer {
namespace {

// ---- same-level periodic ghost fill --------------------------------------
// One work-group per (group, variable, padded z-plane): 400 values, written by
// consecutive threads along x; 32-bit index arithmetic only.
template <typename T>
__global__ __launch_bounds__(256) void pack_periodic_kernel(const T *__restrict__ state, int gx,
                                                            int gy, int gz, T *__restrict__ padded,
                                                            int n_planes) {
    const int NX = gx * NI, NY = gy * NI, NZ = gz * NI;
    for (int b = blockIdx.x; b < n_planes; b += gridDim.x) {
        const int kp = b % NP;
        const int v = (b / NP) % NV;
        const int g = b / (NP * NV);
        const int bx = g % gx, by = (g / gx) % gy, bz = g / (gx * gy);
        int Z = bz * NI + kp - NG;
        Z = Z < 0 ? Z + NZ : (Z >= NZ ? Z - NZ : Z);
        const T *src_z = state + int64_t(gx) * gy * (Z / NI) * GOUT + v * (NI * NI * NI) +
                         (Z % NI) * (NI * NI);
        T *dst = padded + int64_t(b) * NPL;
        for (int p = threadIdx.x; p < NPL; p += blockDim.x) {
            const int ip = p % NP, jp = p / NP;
            int X = bx * NI + ip - NG, Y = by * NI + jp - NG;
            X = X < 0 ? X + NX : (X >= NX ? X - NX : X);
            Y = Y < 0 ? Y + NY : (Y >= NY ? Y - NY : Y);
            const int sg = X / NI + gx * (Y / NI);
            dst[p] = src_z[int64_t(sg) * GOUT + (Y % NI) * NI + (X % NI)];
        }
    }
}

// ---- per-group stats of interior groups -----------------------------------
// 256 threads per group, thread (i, j) walks its z column in order; the block
// reduction matches the solver epilogue's order, so stats of the same cells
// agree bitwise with the ones the solver writes.
template <typename T>
__global__ __launch_bounds__(256) void group_stats_kernel(const T *__restrict__ groups, int64_t n,
                                                          double gamma, double *__restrict__ stats) {
    __shared__ double red[320 * NSTAT];
    const int t = threadIdx.x;
    const Consts<T> c = make_consts<T>(gamma, 1.5);
    for (int64_t g = blockIdx.x; g < n; g += gridDim.x) {
        const T *src = groups + g * GOUT + t;
        double st[NSTAT] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int k = 0; k < NI; ++k) {
            T u[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                u[v] = src[v * NI * NI * NI + k * NI * NI];
                st[v] += double(u[v]);
            }
            st[5] = fmax(st[5], double(signal_speed(u[0], u[1], u[2], u[3], u[4], c)));
        }
        // same layout and order as the solver's 320-thread reduction, with
        // the 64 entries of its ghost-cell threads equal to zero
#pragma unroll
        for (int q = 0; q < NSTAT; ++q) {
            red[q * 320 + t] = st[q];
            if (t < 64) red[q * 320 + 256 + t] = 0.0;
        }
        __syncthreads();
        if (t < 64) {
            double acc[NSTAT];
#pragma unroll
            for (int q = 0; q < NSTAT; ++q) {
                double a = red[q * 320 + t];
                for (int s = t + 64; s < 320; s += 64) {
                    const double b = red[q * 320 + s];
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
                for (int q = 0; q < NSTAT; ++q) stats[g * NSTAT + q] = acc[q];
            }
        }
        __syncthreads();
    }
}

// ---- fixed-order reduction of group stats ----------------------------------
// One work-group of RT threads.  Thread t folds groups t, t+RT, ... in order,
// then a fixed tree combines the threads; the result does not depend on timing.
constexpr int RT = 1024;

__device__ double block_tree(double x, bool is_max, double *red) {
    const int t = threadIdx.x;
    red[t] = x;
    __syncthreads();
    for (int s = RT / 2; s >= 1; s >>= 1) {
        if (t < s) red[t] = is_max ? fmax(red[t], red[t + s]) : red[t] + red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(RT) void reduce_kernel(const double *__restrict__ stats, int64_t n,
                                                    const int8_t *__restrict__ level,
                                                    const double *__restrict__ dh_dev, double dh,
                                                    int n_levels, double cfl,
                                                    double *__restrict__ dt_out,
                                                    double *__restrict__ totals_out) {
    __shared__ double red[RT];
    const int t = threadIdx.x;
    if (dt_out) {
        for (int L = 0; L < n_levels; ++L) {
            double m = 0.0;
            for (int64_t g = t; g < n; g += RT) {
                const int lg = level ? int(level[g]) : 0;
                if (lg == L) m = fmax(m, stats[g * NSTAT + 5]);
            }
            m = block_tree(m, true, red);
            if (t == 0) {
                const double h = dh_dev ? dh_dev[L] : dh;
                dt_out[L] = m > 0.0 ? cfl * h / m : INFINITY;
            }
        }
    }
    if (totals_out) {
        for (int q = 0; q < 7; ++q) {
            const int src = q < 5 ? q : q + 1;  // stats 0..4, then 6, 7
            double s = 0.0;
            for (int64_t g = t; g < n; g += RT) {
                double w = 1.0;
                if (q < 5) {
                    const double h = dh_dev ? dh_dev[level ? int(level[g]) : 0] : dh;
                    w = h * h * h;
                }
                s += w * stats[g * NSTAT + src];
            }
            s = block_tree(s, false, red);
            if (t == 0) totals_out[q] = s;
        }
    }
}

}  // namespace

template <typename T>
hipError_t launch_pack_periodic(const T *state, int gx, int gy, int gz, T *padded, hipStream_t s) {
    // n_planes = groups * 5 * 20 must fit in int (the ABI caps the group count)
    const int64_t n_planes = int64_t(gx) * gy * gz * NV * NP;
    if (n_planes == 0) return hipSuccess;
    const int64_t cap = int64_t(256) * 1024;
    const unsigned grid = unsigned(n_planes < cap ? n_planes : cap);
    hipLaunchKernelGGL(pack_periodic_kernel<T>, dim3(grid), dim3(256), 0, s, state, gx, gy, gz,
                       padded, int(n_planes));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_group_stats(const T *groups, int64_t n, double gamma, double *stats,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t cap = int64_t(1) << 30;
    hipLaunchKernelGGL(group_stats_kernel<T>, dim3(unsigned(n < cap ? n : cap)), dim3(256), 0, s,
                       groups, n, gamma, stats);
    return hipGetLastError();
}

hipError_t launch_reduce(const double *stats, int64_t n, const int8_t *level, const double *dh_dev,
                         double dh, int n_levels, double cfl, double *dt_out, double *totals_out,
                         hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(RT), 0, s, stats, n, level, dh_dev, dh,
                       n_levels, cfl, dt_out, totals_out);
    return hipGetLastError();
}

template hipError_t launch_pack_periodic<float>(const float *, int, int, int, float *, hipStream_t);
template hipError_t launch_pack_periodic<double>(const double *, int, int, int, double *,
                                                 hipStream_t);
template hipError_t launch_group_stats<float>(const float *, int64_t, double, double *,
                                              hipStream_t);
template hipError_t launch_group_stats<double>(const double *, int64_t, double, double *,
                                               hipStream_t);

}  // namespace gamer
