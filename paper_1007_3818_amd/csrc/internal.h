// internal.h -- declarations shared by the translation units of libgamer_hydro.so.
// Not installed; the public interface is include/gamer_hydro.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gamer_hydro.h"

namespace gamer {

// Patch-group geometry: 16^3 interior cells, two ghost cells per side (the
// five-point stencil of MUSCL-Hancock), five conserved variables.
constexpr int NI = 16;
constexpr int NG = 2;
constexpr int NP = NI + 2 * NG;               // 20
constexpr int NPL = NP * NP;                  // cells in one padded z-plane
constexpr int NV = 5;
constexpr int64_t GIN = int64_t(NV) * NP * NP * NP;    // values per padded group
constexpr int64_t GOUT = int64_t(NV) * NI * NI * NI;   // values per interior group
constexpr int64_t GFLX = int64_t(3) * 3 * NV * NI * NI;  // values per flux-plane set
constexpr int NSTAT = 8;                      // doubles of group stats
constexpr int MAX_LEVELS = 32;

template <typename T>
struct SolveParams {
    // Input: padded groups [n][5][20][20][20] (gx == 0), or the interior state of
    // a periodic grid of gx x gy x gz groups [n][5][16][16][16] whose ghost cells
    // are read from the neighbouring groups (gx > 0).
    const T *in;
    int gx, gy, gz;
    T *out;               // [n][5][16][16][16]
    T *flux;              // [n][3][3][5][16][16] or nullptr
    double *stats;        // [n][8] or nullptr
    const int8_t *level;  // [n] or nullptr
    const double *dt_dev; // [n_levels] or nullptr (then dt, dh below)
    const double *dh_dev;
    double dt, dh;
    double gamma, theta;
    int64_t n_groups;
    int n_levels;       // entries of dt_dev and dh_dev
    int char_limiting;  // 0: limit primitive variables, 1: characteristic variables
    int zseg;           // periodic input: groups per z segment of a column that one
                        // work-group sweeps in one pass (>= 1)
    // device counters or nullptr: [0] output cells that are not physical or not
    // finite, [1] groups whose level byte lies outside [0, n_levels)
    unsigned long long *bad;
};

// dt and dh of group g read on the device from its level.  A level byte outside
// [0, n_levels) is never used as an index: the group gets NaN for both (so its
// whole output and stats come out NaN) and lev_ok is false.
__device__ __forceinline__ bool level_dt(const int8_t *level, int64_t g, int n_levels,
                                         const double *dt_dev, const double *dh_dev, double &dt,
                                         double &dh) {
    const int lev = level ? int(level[g]) : 0;
    if (lev < 0 || lev >= n_levels) {
        dt = dh = __builtin_nan("");
        return false;
    }
    dt = dt_dev[lev];
    dh = dh_dev[lev];
    return true;
}

// Compiled solver variants (work-group size, occupancy target) and the launcher.
template <typename T>
int solve_variant_count();
template <typename T>
int solve_variant_shape(int variant, int *threads, int *waves_per_simd);
// Storage type S (the arrays of P), arithmetic type T: <float, float>,
// <double, double>, or <double, float> (FP64 state, FP32 arithmetic).
template <typename S, typename T>
hipError_t launch_solve(const SolveParams<S> &p, int variant, int64_t grid, hipStream_t s);

template <typename T>
hipError_t launch_pack_periodic(const T *state, int gx, int gy, int gz, T *padded, hipStream_t s);

template <typename T>
hipError_t launch_group_stats(const T *groups, int64_t n, double gamma, double *stats,
                              hipStream_t s);

// dt_out[L] and totals_out[7] from group stats; dh_dev may be nullptr (then the
// scalar dh applies to every group, and level must be nullptr too).  A group
// whose level lies outside [0, n_levels) counts towards no level's dt and
// makes the totals NaN.
hipError_t launch_reduce(const double *stats, int64_t n, const int8_t *level, const double *dh_dev,
                         double dh, int n_levels, double cfl, double *dt_out, double *totals_out,
                         hipStream_t s);

// relaxing TVD (rtvd.hip): elements of workspace for n groups; one step of
// padded groups [n][5][22][22][22] (gx == 0) or of a periodic grid of groups
template <typename T>
size_t rtvd_workspace_elems(int64_t n_groups);
template <typename T>
hipError_t launch_rtvd(const T *in, int gx, int gy, int gz, int64_t n, const int8_t *level,
                       int n_levels, const double *dt_dev, const double *dh_dev, double gamma,
                       int order, T *work, T *out, hipStream_t s);

// CTU coupling (ctu.hip): workspace bytes for n groups of elem-byte values (the
// pipeline, variant 1), and one step of padded groups (variant 0: the fused
// sweep, which takes no workspace)
size_t ctu_workspace_bytes(int64_t n, int elem);
template <typename T>
hipError_t launch_ctu(const T *in, int64_t n, const int8_t *level, int n_levels, const double *dt_dev,
                      const double *dh_dev, double gamma, double theta, T *fluxes, T *out, double *stats,
                      unsigned long long *bad, int variant, void *work, hipStream_t s);

// two refinement levels (amr.hip)
template <typename T>
hipError_t launch_flux_accumulate(const T *fluxes, int64_t n_groups, const double *dt_dev, int reset,
                                  double *acc, hipStream_t s);
template <typename T>
hipError_t launch_flux_correct(T *coarse, int64_t n_coarse, const T *coarse_fluxes, const double *acc,
                               int64_t n_fine, const gamer_cf_face *faces, int64_t n_faces,
                               const double *dt_dev, const double *dh_dev, int32_t *n_bad,
                               hipStream_t s);
template <typename T>
hipError_t launch_restrict(const T *fine, const int64_t *parent, int64_t n_fine, T *coarse,
                           int64_t n_coarse, int32_t *n_bad, hipStream_t s);

}  // namespace gamer
