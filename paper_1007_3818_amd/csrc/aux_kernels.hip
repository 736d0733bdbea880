// aux_kernels.hip -- periodic ghost fill, per-group stats and the fixed-order
// reduction of group stats to per-level time steps and conserved totals.
#include "device_math.h"
#include "internal.h"

namespace gamer {
namespace {

// ---- same-level periodic ghost fill --------------------------------------
// One work-group per (group, variable) pair: the pair's padded block of 20^3
// values is one contiguous run of the output, written as 2,000 pieces of four
// values (padded x = 4k - 2 .. 4k + 1 of one padded row), consecutive threads
// on consecutive pieces.  A piece takes two pairs of source values: from the
// left x neighbour (x = 14, 15) and the group's own row for k = 0, from the own
// row and the right x neighbour (x = 0, 1) for k = 4, and from the own row
// otherwise.  The group's position and its periodic neighbours are worked out
// once per work-group; per piece, the padded y and z indices pick the source
// group (own, or the neighbour below or above) and the row within it with
// compares, shifts and masks.  Each thread loads all its pieces before it
// stores any, so that eight pieces' loads are in flight at once.
//
// Work-groups go to the 8 XCDs round-robin by flat index; they are numbered so
// that each XCD takes a contiguous run of (group, variable) pairs, which puts a
// group and its x neighbours (5 pairs apart) under one L2.  The other order
// sent them to different L2s, and the x ghost cells were fetched again from
// memory: reads of 3.8 (256^3) and 4.7 (1024^3) times the field, against 1.5
// and 1.7 with this numbering.
template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
    using type = float4;
};
template <>
struct Vec4<double> {
    using type = double4;
};
template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
    using type = float2;
};
template <>
struct Vec2<double> {
    using type = double2;
};

constexpr int PIECES = NP * NP * 5;  // 4-value pieces in one padded block of one variable

template <typename T>
__global__ __launch_bounds__(256) void pack_block_kernel(const T *__restrict__ state, int gx, int gy,
                                                         int gz, T *__restrict__ padded, int64_t n_blocks) {
    using V = typename Vec4<T>::type;
    using V2 = typename Vec2<T>::type;
    static_assert(NI == 16 && NG == 2, "the masks below assume 16 interior cells and 2 ghost cells");
    unsigned xb = blockIdx.x;
    if ((gridDim.x & 7) == 0) xb = (xb & 7) * (gridDim.x >> 3) + (xb >> 3);
    for (int64_t gv = xb; gv < n_blocks; gv += gridDim.x) {
        const int64_t g = gv / NV;
        const int v = int(gv - g * NV);
        const int bx = int(g % gx);
        const int64_t g1 = g / gx;
        const int by = int(g1 % gy), bz = int(g1 / gy);
        const int ym = by == 0 ? gy - 1 : by - 1, yp = by == gy - 1 ? 0 : by + 1;
        const int zm = bz == 0 ? gz - 1 : bz - 1, zp = bz == gz - 1 ? 0 : bz + 1;
        const int xm = bx == 0 ? gx - 1 : bx - 1, xp = bx == gx - 1 ? 0 : bx + 1;
        const T *src = state + int64_t(v) * (NI * NI * NI);
        V *dst = reinterpret_cast<V *>(padded + gv * (NP * NP * NP));
        constexpr int PER = (PIECES + 255) / 256;
        V2 a[PER], b[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int o = int(threadIdx.x) + 256 * q;
            if (o < PIECES) {
                const int row = o / 5, k = o - row * 5;  // row = kp * 20 + jp
                const int kp = row / NP, jp = row - kp * NP;
                const int yb = jp < NG ? ym : (jp >= NG + NI ? yp : by);
                const int zb = kp < NG ? zm : (kp >= NG + NI ? zp : bz);
                const int yo = (jp - NG) & (NI - 1), zo = (kp - NG) & (NI - 1);
                const int64_t grow = int64_t(gx) * (yb + int64_t(gy) * zb);  // group of x block 0
                const int off = zo * (NI * NI) + yo * NI;
                const int xa = k == 0 ? xm : bx, xc = k == 4 ? xp : bx;  // groups of the two pairs
                const int x0 = k == 0 ? NI - 2 : 4 * k - 2, x1 = k == 4 ? 0 : 4 * k;
                a[q] = *reinterpret_cast<const V2 *>(src + (grow + xa) * GOUT + off + x0);
                b[q] = *reinterpret_cast<const V2 *>(src + (grow + xc) * GOUT + off + x1);
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int o = int(threadIdx.x) + 256 * q;
            if (o < PIECES) dst[o] = V{a[q].x, a[q].y, b[q].x, b[q].y};
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
            st[5] = max_nan(st[5], double(signal_speed(u[0], u[1], u[2], u[3], u[4], c)));
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
                    a = (q == 5) ? max_nan(a, b) : a + b;
                }
                acc[q] = a;
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
                for (int q = 0; q < NSTAT; ++q) {
                    const double b = __shfl_down(acc[q], off, 64);
                    acc[q] = (q == 5) ? max_nan(acc[q], b) : acc[q] + b;
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
// One work-group of RT threads.  Thread t folds groups t, t+RT, ... in order;
// each wave combines its lanes by a fixed shuffle tree and wave 0 combines the
// waves in order.  The result does not depend on timing.  Maxima keep NaN, so
// a level holding a non-physical cell gets a NaN time step.
constexpr int RT = 1024;
constexpr int RW = RT / 64;
constexpr int RU = 4;  // groups per thread whose loads are in flight together
constexpr int RL = 4;  // levels whose maxima are taken in the totals' pass

template <int N>
__device__ void block_fold(double (&x)[N], const bool (&is_max)[N], double (*red)[RW]) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const double y = __shfl_down(x[q], off, 64);
            x[q] = is_max[q] ? max_nan(x[q], y) : x[q] + y;
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < N; ++q) red[q][wave] = x[q];
    }
    __syncthreads();
    if (t == 0) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            double a = red[q][0];
            for (int w = 1; w < RW; ++w) a = is_max[q] ? max_nan(a, red[q][w]) : a + red[q][w];
            x[q] = a;
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(RT) void reduce_kernel(const double *__restrict__ stats, int64_t n,
                                                    const int8_t *__restrict__ level,
                                                    const double *__restrict__ dh_dev, double dh,
                                                    int n_levels, double cfl,
                                                    double *__restrict__ dt_out,
                                                    double *__restrict__ totals_out) {
    // values folded: [0..4] dh^3-weighted sums of stats 0..4, [5..6] sums of
    // stats 6..7, [7..7+RL) the signal-speed maxima of levels 0..RL-1
    __shared__ double red[7 + RL][RW];
    const int t = threadIdx.x;
    // one pass over the stats for the totals and, up to RL levels, the maxima;
    // more levels take one further pass per level for their maxima
    const bool tot = totals_out != nullptr;
    const int lv_one = dt_out ? (n_levels <= RL ? n_levels : 0) : 0;
    double x[7 + RL];
    bool is_max[7 + RL];
#pragma unroll
    for (int q = 0; q < 7 + RL; ++q) {
        x[q] = 0.0;
        is_max[q] = q >= 7;
    }
    // RU groups' loads are issued before any is folded (a pass over 10^5
    // groups is otherwise one memory latency per group per thread); each
    // thread folds its groups in the order t, t + RT, t + 2 RT, ...
    if (tot || lv_one > 0) {
        for (int64_t g0 = t; g0 < n; g0 += int64_t(RT) * RU) {
            double s[RU][NSTAT], w[RU];
            int lv[RU];
            bool ok[RU];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int64_t g1 = g0 + int64_t(u) * RT;
                ok[u] = g1 < n;
                const int64_t g = ok[u] ? g1 : g0;  // a valid group to read; its values are not used
                lv[u] = level ? int(level[g]) : 0;
                double h = dh;
                if (dh_dev) {
                    // a level out of range is never used as an index; it makes the totals NaN
                    h = (lv[u] >= 0 && lv[u] < n_levels) ? dh_dev[lv[u]] : __builtin_nan("");
                }
                w[u] = h * h * h;
                const double *st = stats + g * NSTAT;
#pragma unroll
                for (int q = 0; q < NSTAT; ++q) s[u][q] = st[q];
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                if (!ok[u]) continue;
                if (tot) {
#pragma unroll
                    for (int q = 0; q < 5; ++q) x[q] += w[u] * s[u][q];
                    x[5] += s[u][6];
                    x[6] += s[u][7];
                }
#pragma unroll
                for (int L = 0; L < RL; ++L)
                    if (L < lv_one && lv[u] == L) x[7 + L] = max_nan(x[7 + L], s[u][5]);
            }
        }
        block_fold(x, is_max, red);
        if (t == 0) {
            if (tot) {
#pragma unroll
                for (int q = 0; q < 7; ++q) totals_out[q] = x[q];
            }
        }
    }
    if (dt_out) {
        const bool max1[1] = {true};
        for (int L = 0; L < n_levels; ++L) {
            double m[1] = {0.0};
            if (L < lv_one) {
                m[0] = x[7 + (L < RL ? L : 0)];  // thread 0 holds the folded value
            } else {
                for (int64_t g0 = t; g0 < n; g0 += int64_t(RT) * RU) {
                    double sp[RU];
                    bool take[RU];
#pragma unroll
                    for (int u = 0; u < RU; ++u) {
                        const int64_t g1 = g0 + int64_t(u) * RT;
                        const int64_t g = g1 < n ? g1 : g0;
                        take[u] = g1 < n && (level ? int(level[g]) : 0) == L;
                        sp[u] = stats[g * NSTAT + 5];
                    }
#pragma unroll
                    for (int u = 0; u < RU; ++u)
                        if (take[u]) m[0] = max_nan(m[0], sp[u]);
                }
                block_fold(m, max1, red);
            }
            if (t == 0) {
                const double hL = dh_dev ? dh_dev[L] : dh;
                // NaN when a group of the level has a non-physical cell
                dt_out[L] = m[0] > 0.0 ? cfl * hL / m[0] : (m[0] != m[0] ? m[0] : INFINITY);
            }
        }
    }
}

}  // namespace

template <typename T>
hipError_t launch_pack_periodic(const T *state, int gx, int gy, int gz, T *padded, hipStream_t s) {
    const int64_t n_blocks = int64_t(gx) * gy * gz * NV;  // (group, variable) pairs
    if (n_blocks == 0) return hipSuccess;
    const int64_t cap = int64_t(256) * 2048;  // a multiple of 8, as the XCD numbering wants
    hipLaunchKernelGGL(pack_block_kernel<T>, dim3(unsigned(n_blocks < cap ? n_blocks : cap)), dim3(256), 0, s,
                       state, gx, gy, gz, padded, n_blocks);
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
