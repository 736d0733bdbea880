// amr.hip -- the steps that follow the solver when two refinement levels are
// advanced together: time-weighted accumulation of the fine levels' face
// fluxes, conservative correction of the coarse cells next to coarse/fine
// faces, and restriction of fine groups onto the coarse cells they cover.
// All three are memory-bound gathers with a few flops per value; results are
// formed in double and stored in the level's precision.
#include "internal.h"

namespace gamer {
namespace {

constexpr int64_t FLUX_VALUES = int64_t(3) * 3 * NV * NI * NI;  // per group

// acc = (reset ? 0 : acc) + dt * F over whole flux-plane arrays, 2 values per thread.
template <typename T>
__global__ __launch_bounds__(256) void flux_accumulate_kernel(const T *__restrict__ F, int64_t n_pairs,
                                                              const double *__restrict__ dt_dev, int reset,
                                                              double *__restrict__ acc) {
    const double dt = dt_dev[0];
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n_pairs;
         p += int64_t(gridDim.x) * blockDim.x) {
        const double f0 = double(F[2 * p]), f1 = double(F[2 * p + 1]);
        double2 a = reset ? double2{0.0, 0.0} : reinterpret_cast<const double2 *>(acc)[p];
        a.x += dt * f0;
        a.y += dt * f1;
        reinterpret_cast<double2 *>(acc)[p] = a;
    }
}

// One wave per face record, one lane per coarse cell of its 8 x 8 patch face,
// all five variables per lane.  Only records of direction `dir` are applied,
// so that a cell on a concave corner of the fine region takes its x, y and z
// corrections in that order, from three launches.
template <typename T>
__global__ __launch_bounds__(256) void flux_correct_kernel(
    T *__restrict__ U, int64_t n_coarse, const T *__restrict__ Fc, const double *__restrict__ acc,
    int64_t n_fine, const gamer_cf_face *__restrict__ faces, int64_t n_faces,
    const double *__restrict__ dt_dev, const double *__restrict__ dh_dev, int dir,
    int32_t *__restrict__ n_bad) {
    const int lane = threadIdx.x & 63;
    const int64_t r = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (r >= n_faces) return;
    const gamer_cf_face rec = faces[r];
    const bool dir_ok = rec.dir >= 0 && rec.dir <= 2;
    if (!dir_ok) {  // counted once, in the x pass
        if (dir == 0 && lane == 0 && n_bad) atomicAdd(n_bad, 1);
        return;
    }
    if (rec.dir != dir) return;
    const int cf = rec.coarse_face, side = rec.side;
    const int n = 8 * cf - 1 + side;  // the coarse cells' index along dir
    const bool ok = rec.coarse_group >= 0 && rec.coarse_group < n_coarse && rec.fine_group >= 0 &&
                    rec.fine_group < n_fine && cf >= 0 && cf <= 2 && (side == 0 || side == 1) &&
                    n >= 0 && n < NI && (rec.qs == 0 || rec.qs == 1) && (rec.qf == 0 || rec.qf == 1);
    if (!ok) {
        if (lane == 0 && n_bad) atomicAdd(n_bad, 1);
        return;
    }
    const int s = 8 * rec.qs + (lane >> 3), f = 8 * rec.qf + (lane & 7);  // coarse plane position
    const int sf = 2 * (lane >> 3), ff = 2 * (lane & 7);                  // fine plane position
    int i, j, k;
    if (dir == 0) { i = n; j = f; k = s; }
    else if (dir == 1) { i = f; j = n; k = s; }
    else { i = f; j = s; k = n; }
    const double dt = dt_dev[0], dh = dh_dev[0];
    const T *fc = Fc + rec.coarse_group * FLUX_VALUES + (dir * 3 + cf) * (NV * NI * NI) + s * NI + f;
    const double *fa =
        acc + rec.fine_group * FLUX_VALUES + (dir * 3 + 2 * side) * (NV * NI * NI) + sf * NI + ff;
    T *u = U + rec.coarse_group * GOUT + (k * NI + j) * NI + i;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double *a = fa + v * (NI * NI);
        const double phi = (((a[0] + a[1]) + a[NI]) + a[NI + 1]) * 0.25;
        double delta = (dt * double(fc[v * (NI * NI)]) - phi) / dh;
        if (side) delta = -delta;
        T *uv = u + v * (NI * NI * NI);
        *uv = T(double(*uv) + delta);
    }
}

// One thread per coarse cell of one variable: grid (n_fine * 5 * 2), 256
// threads = 4 coarse planes of 8 x 8 cells.
template <typename T>
__global__ __launch_bounds__(256) void restrict_kernel(const T *__restrict__ fine,
                                                       const int64_t *__restrict__ parent, int64_t n_fine,
                                                       T *__restrict__ coarse, int64_t n_coarse,
                                                       int32_t *__restrict__ n_bad) {
    const int64_t b = blockIdx.x;
    const int64_t fg = b / (NV * 2);
    const int v = int((b / 2) % NV);
    const int K = int(b % 2) * 4 + (threadIdx.x >> 6);
    const int J = (threadIdx.x >> 3) & 7, I = threadIdx.x & 7;
    if (fg >= n_fine) return;
    const int64_t code = parent[fg];
    if (code < 0) return;  // no parent: nothing to restrict
    if (code >= 8 * n_coarse) {
        if (threadIdx.x == 0 && v == 0 && (b % 2) == 0 && n_bad) atomicAdd(n_bad, 1);
        return;
    }
    const int64_t g = code >> 3;
    const int o = int(code & 7);
    const T *src = fine + fg * GOUT + v * (NI * NI * NI) + ((2 * K) * NI + 2 * J) * NI + 2 * I;
    const double s00 = double(src[0]) + double(src[1]);
    const double s01 = double(src[NI]) + double(src[NI + 1]);
    const double s10 = double(src[NI * NI]) + double(src[NI * NI + 1]);
    const double s11 = double(src[NI * NI + NI]) + double(src[NI * NI + NI + 1]);
    const double mean = ((s00 + s01) + (s10 + s11)) * 0.125;
    const int ci = 8 * (o & 1) + I, cj = 8 * ((o >> 1) & 1) + J, ck = 8 * ((o >> 2) & 1) + K;
    coarse[g * GOUT + v * (NI * NI * NI) + (ck * NI + cj) * NI + ci] = T(mean);
}

int grid_for(int64_t items, int per_block) {
    const int64_t b = (items + per_block - 1) / per_block;
    return int(b < 65536 * 4 ? b : 65536 * 4);
}

}  // namespace

template <typename T>
hipError_t launch_flux_accumulate(const T *fluxes, int64_t n_groups, const double *dt_dev, int reset,
                                  double *acc, hipStream_t s) {
    const int64_t pairs = n_groups * FLUX_VALUES / 2;
    if (pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(flux_accumulate_kernel<T>, dim3(grid_for(pairs, 256)), dim3(256), 0, s, fluxes,
                       pairs, dt_dev, reset, acc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_flux_correct(T *coarse, int64_t n_coarse, const T *coarse_fluxes, const double *acc,
                               int64_t n_fine, const gamer_cf_face *faces, int64_t n_faces,
                               const double *dt_dev, const double *dh_dev, int32_t *n_bad,
                               hipStream_t s) {
    if (n_faces == 0) return hipSuccess;
    const dim3 blocks(unsigned((n_faces + 3) / 4));
    for (int d = 0; d < 3; ++d) {
        hipLaunchKernelGGL(flux_correct_kernel<T>, blocks, dim3(256), 0, s, coarse, n_coarse, coarse_fluxes,
                           acc, n_fine, faces, n_faces, dt_dev, dh_dev, d, n_bad);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_restrict(const T *fine, const int64_t *parent, int64_t n_fine, T *coarse,
                           int64_t n_coarse, int32_t *n_bad, hipStream_t s) {
    if (n_fine == 0) return hipSuccess;
    hipLaunchKernelGGL(restrict_kernel<T>, dim3(unsigned(n_fine * NV * 2)), dim3(256), 0, s, fine, parent,
                       n_fine, coarse, n_coarse, n_bad);
    return hipGetLastError();
}

template hipError_t launch_flux_accumulate<float>(const float *, int64_t, const double *, int, double *,
                                                  hipStream_t);
template hipError_t launch_flux_accumulate<double>(const double *, int64_t, const double *, int, double *,
                                                   hipStream_t);
template hipError_t launch_flux_correct<float>(float *, int64_t, const float *, const double *, int64_t,
                                               const gamer_cf_face *, int64_t, const double *,
                                               const double *, int32_t *, hipStream_t);
template hipError_t launch_flux_correct<double>(double *, int64_t, const double *, const double *, int64_t,
                                                const gamer_cf_face *, int64_t, const double *,
                                                const double *, int32_t *, hipStream_t);
template hipError_t launch_restrict<float>(const float *, const int64_t *, int64_t, float *, int64_t,
                                           int32_t *, hipStream_t);
template hipError_t launch_restrict<double>(const double *, const int64_t *, int64_t, double *, int64_t,
                                            int32_t *, hipStream_t);

}  // namespace gamer
