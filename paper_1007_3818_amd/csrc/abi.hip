// abi.hip -- the extern "C" entry points of include/gamer_hydro.h: argument
// checks, per-thread stream and error state, library scratch, dispatch.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <mutex>

#include "../../include/gamer_hydro.h"
#include "internal.h"

using namespace gamer;

// Fixed scratch of gamer_cfl_dt_noalloc: the per-group stats of up to
// GAMER_NOALLOC_MAX_GROUPS groups, then a 256-byte tail.  Every device the
// library runs on holds its own copy until the process ends.  In host code this
// name is not a device address: host code uses only the address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch below).
constexpr size_t kNoAllocBytes = size_t(GAMER_NOALLOC_MAX_GROUPS) * NSTAT * sizeof(double) + 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

thread_local char g_err[512] = "";
thread_local hipStream_t g_stream = nullptr;

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return GAMER_OK;
    return fail(GAMER_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

// Library scratch: one growing device buffer per device, guarded by a mutex.
// Calls that use it and overlap on different streams of one device race.
struct Scratch {
    std::mutex mu;
    void *ptr[64] = {};
    size_t size[64] = {};
};
Scratch g_scratch;

int grow_scratch(size_t bytes, void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return fail(GAMER_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lock(g_scratch.mu);
    if (g_scratch.size[dev] < bytes) {
        if (g_scratch.ptr[dev]) {
            // the old buffer may still be in use by queued work on any stream
            if (hipDeviceSynchronize() != hipSuccess) return fail(GAMER_EHIP, "hipDeviceSynchronize");
            (void)hipFree(g_scratch.ptr[dev]);
            g_scratch.ptr[dev] = nullptr;
            g_scratch.size[dev] = 0;
        }
        size_t want = bytes < 4096 ? 4096 : bytes;
        if (hipMalloc(&g_scratch.ptr[dev], want) != hipSuccess) {
            g_scratch.ptr[dev] = nullptr;
            return fail(GAMER_ENOMEM, "could not allocate %zu bytes of scratch", want);
        }
        g_scratch.size[dev] = want;
    }
    *out = g_scratch.ptr[dev];
    return GAMER_OK;
}

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
struct NoAllocScratch {
    std::mutex mu;
    void *ptr[64] = {};
};
NoAllocScratch g_noalloc;

int noalloc_scratch(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return fail(GAMER_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lock(g_noalloc.mu);
    if (!g_noalloc.ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GAMER_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_noalloc.ptr[dev] = p;
    }
    *out = g_noalloc.ptr[dev];
    return GAMER_OK;
}

// Groups per z segment of a periodic grid when the caller leaves it to the
// library: the largest divisor of gz that still leaves at least 12,288
// segments (sixteen per slot of a full chip: 256 CUs x 3 work-groups), so that
// the last round of work-groups is a small part of the launch; 1 on grids too
// small for that.
int auto_zseg(int gx, int gy, int gz) {
    const int64_t cols = int64_t(gx) * gy;
    int best = 1;
    for (int d = 2; d <= gz; ++d)
        if (gz % d == 0 && cols * (gz / d) >= 12288) best = d;
    return best;
}

// Tunables shared by the solver entry points; returns GAMER_OK or an error.
template <typename T>
int parse_opts(const gamer_opts *opts, double *theta, int *variant, int64_t *grid, int *limiting,
               unsigned long long **bad, int *zseg = nullptr) {
    *theta = (opts && opts->theta != 0.0) ? opts->theta : 1.5;
    if (!(*theta >= 1.0 && *theta <= 2.0)) return fail(GAMER_EINVAL, "theta must lie in [1, 2]");
    *variant = opts ? opts->variant : 0;
    *grid = opts ? opts->grid : 0;
    *limiting = opts ? opts->limiting : 0;
    if (*variant < 0 || *variant >= solve_variant_count<T>())
        return fail(GAMER_EINVAL, "variant must lie in [0, %d)", solve_variant_count<T>());
    if (*grid < 0) return fail(GAMER_EINVAL, "grid must be >= 0");
    if (*limiting != GAMER_LIMIT_PRIMITIVE && *limiting != GAMER_LIMIT_CHARACTERISTIC)
        return fail(GAMER_EINVAL, "limiting must be GAMER_LIMIT_PRIMITIVE or GAMER_LIMIT_CHARACTERISTIC");
    const int zs = opts ? opts->zseg : 0;
    if (zseg) {
        if (zs < 0) return fail(GAMER_EINVAL, "gamer_opts.zseg must be >= 0");
        *zseg = zs;
    } else if (zs != 0) {
        return fail(GAMER_EINVAL, "gamer_opts.zseg applies to the periodic entry points only (must be 0)");
    }
    *bad = opts ? reinterpret_cast<unsigned long long *>(opts->bad_count_dev) : nullptr;
    if (reinterpret_cast<uintptr_t>(*bad) % 8)
        return fail(GAMER_EINVAL, "gamer_opts.bad_count_dev must be 8-byte aligned");
    return GAMER_OK;
}

// Storage type S (the arrays), arithmetic type T.
template <typename S, typename T>
int solve_common(const S *in, int64_t n, const int8_t *level, const double *dt_dev,
                 const double *dh_dev, int n_levels, double dt, double dh, double gamma,
                 S *fluxes, S *out, double *stats, const gamer_opts *opts, hipStream_t stream) {
    g_err[0] = 0;
    if (n < 0) return fail(GAMER_EINVAL, "n_groups < 0");
    if (!(isfinite(gamma) && gamma > 1.0)) return fail(GAMER_EINVAL, "gamma must be > 1");
    double theta;
    int variant, limiting;
    int64_t grid;
    unsigned long long *bad;
    if (const int e = parse_opts<T>(opts, &theta, &variant, &grid, &limiting, &bad)) return e;
    if (!dt_dev && (!finite_pos(dt) || !finite_pos(dh)))
        return fail(GAMER_EINVAL, "dt and dh must be finite and positive");
    if (n == 0) return GAMER_OK;
    if (!in || !out) return fail(GAMER_EINVAL, "NULL groups_in or groups_out");
    if (dt_dev && !dh_dev) return fail(GAMER_EINVAL, "NULL dh_dev");
    if (dt_dev && (n_levels < 1 || n_levels > GAMER_MAX_LEVELS))
        return fail(GAMER_EINVAL, "n_levels must lie in [1, %d]", GAMER_MAX_LEVELS);
    SolveParams<S> p;
    p.in = in;
    p.gx = p.gy = p.gz = 0;
    p.out = out;
    p.flux = fluxes;
    p.stats = stats;
    p.level = level;
    p.dt_dev = dt_dev;
    p.dh_dev = dh_dev;
    p.dt = dt;
    p.dh = dh;
    p.gamma = gamma;
    p.theta = theta;
    p.n_groups = n;
    p.n_levels = dt_dev ? n_levels : 1;
    p.char_limiting = limiting;
    p.zseg = 1;
    p.bad = bad;
    return check_hip(launch_solve<S, T>(p, variant, grid, stream), "solver launch");
}

template <typename S, typename T>
int periodic_common(const S *state, int gx, int gy, int gz, const double *dt_dev,
                    const double *dh_dev, double gamma, S *fluxes, S *out, double *stats,
                    const gamer_opts *opts) {
    g_err[0] = 0;
    if (gx < 1 || gy < 1 || gz < 1) return fail(GAMER_EINVAL, "gx, gy, gz must be >= 1");
    const int64_t n = int64_t(gx) * gy * gz;
    if (int64_t(gx) * NI > (1 << 28) || int64_t(gy) * NI > (1 << 28) || int64_t(gz) * NI > (1 << 28) ||
        n > INT32_MAX)
        return fail(GAMER_EINVAL, "grid too large: gx, gy, gz <= 2^24 and gx*gy*gz < 2^31 required");
    if (!state || !out || !dt_dev || !dh_dev) return fail(GAMER_EINVAL, "NULL array argument");
    if (static_cast<const void *>(state) == static_cast<const void *>(out))
        return fail(GAMER_EINVAL, "state and state_out must be different arrays");
    if (!(isfinite(gamma) && gamma > 1.0)) return fail(GAMER_EINVAL, "gamma must be > 1");
    double theta;
    int variant, limiting, zseg;
    int64_t grid;
    unsigned long long *bad;
    if (const int e = parse_opts<T>(opts, &theta, &variant, &grid, &limiting, &bad, &zseg)) return e;
    SolveParams<S> p;
    p.in = state;
    p.gx = gx;
    p.gy = gy;
    p.gz = gz;
    p.out = out;
    p.flux = fluxes;
    p.stats = stats;
    p.level = nullptr;
    p.dt_dev = dt_dev;
    p.dh_dev = dh_dev;
    p.dt = p.dh = 0.0;
    p.gamma = gamma;
    p.theta = theta;
    p.n_groups = n;
    p.n_levels = 1;
    p.char_limiting = limiting;
    p.zseg = zseg == 0 ? auto_zseg(gx, gy, gz) : (zseg < gz ? zseg : gz);
    p.bad = bad;
    return check_hip(launch_solve<S, T>(p, variant, grid, g_stream), "solver launch");
}

template <typename T>
int cfl_common(const T *groups, int64_t n, double dh, double gamma, double cfl, double *dt_out,
               int dt_dev) {
    g_err[0] = 0;
    if (n < 0) return fail(GAMER_EINVAL, "n_groups < 0");
    if (!finite_pos(dh) || !finite_pos(cfl) || !(isfinite(gamma) && gamma > 1.0))
        return fail(GAMER_EINVAL, "dh and cfl must be finite and positive, gamma > 1");
    if (n == 0) return GAMER_OK;
    if (!dt_out) return fail(GAMER_EINVAL, "NULL dt_out");
    if (!groups) return fail(GAMER_EINVAL, "NULL groups");
    void *buf = nullptr;
    int rc = grow_scratch(size_t(n) * NSTAT * sizeof(double) + 64, &buf);
    if (rc) return rc;
    double *stats = static_cast<double *>(buf);
    double *dt_tmp = stats + size_t(n) * NSTAT;
    if ((rc = check_hip(launch_group_stats<T>(groups, n, gamma, stats, g_stream), "stats launch")))
        return rc;
    double *dst = dt_dev ? dt_out : dt_tmp;
    if ((rc = check_hip(launch_reduce(stats, n, nullptr, nullptr, dh, 1, cfl, dst, nullptr, g_stream),
                        "reduce launch")))
        return rc;
    if (!dt_dev) {
        if ((rc = check_hip(hipMemcpyAsync(dt_out, dt_tmp, sizeof(double), hipMemcpyDeviceToHost,
                                           g_stream), "copy dt")))
            return rc;
        return check_hip(hipStreamSynchronize(g_stream), "stream sync");
    }
    return GAMER_OK;
}

template <typename T>
int sums_common(const T *groups, int64_t n, double dh, double *sums5, int is_dev) {
    g_err[0] = 0;
    if (n < 0) return fail(GAMER_EINVAL, "n_groups < 0");
    if (!finite_pos(dh)) return fail(GAMER_EINVAL, "dh must be finite and positive");
    if (n == 0) return GAMER_OK;
    if (!sums5) return fail(GAMER_EINVAL, "NULL sums5_out");
    if (!groups) return fail(GAMER_EINVAL, "NULL groups");
    void *buf = nullptr;
    int rc = grow_scratch(size_t(n) * NSTAT * sizeof(double) + 64, &buf);
    if (rc) return rc;
    double *stats = static_cast<double *>(buf);
    double *tot = stats + size_t(n) * NSTAT;  // 7 doubles (56 B) fit in the 64 B tail
    // gamma only enters stat 5, which the totals ignore
    if ((rc = check_hip(launch_group_stats<T>(groups, n, 2.0, stats, g_stream), "stats launch")))
        return rc;
    if ((rc = check_hip(launch_reduce(stats, n, nullptr, nullptr, dh, 1, 1.0, nullptr, tot, g_stream),
                        "reduce launch")))
        return rc;
    if (is_dev)
        return check_hip(hipMemcpyAsync(sums5, tot, 5 * sizeof(double), hipMemcpyDeviceToDevice,
                                        g_stream), "copy sums");
    if ((rc = check_hip(hipMemcpyAsync(sums5, tot, 5 * sizeof(double), hipMemcpyDeviceToHost,
                                       g_stream), "copy sums")))
        return rc;
    return check_hip(hipStreamSynchronize(g_stream), "stream sync");
}

template <typename T>
int pack_common(const T *state, int gx, int gy, int gz, T *padded) {
    g_err[0] = 0;
    if (gx < 1 || gy < 1 || gz < 1) return fail(GAMER_EINVAL, "gx, gy, gz must be >= 1");
    if (int64_t(gx) * gy * gz * NV * NP > INT32_MAX)
        return fail(GAMER_EINVAL, "grid too large (gx*gy*gz*100 must fit in int32)");
    if (!state || !padded) return fail(GAMER_EINVAL, "NULL state or padded");
    // rows are moved with 4-element vector loads and stores
    if (reinterpret_cast<uintptr_t>(state) % (4 * sizeof(T)) ||
        reinterpret_cast<uintptr_t>(padded) % (4 * sizeof(T)))
        return fail(GAMER_EINVAL, "state and padded must be aligned to 4 elements");
    return check_hip(launch_pack_periodic<T>(state, gx, gy, gz, padded, g_stream), "pack launch");
}

template <typename T>
int stats_common(const T *groups, int64_t n, double gamma, double *stats) {
    g_err[0] = 0;
    if (n < 0) return fail(GAMER_EINVAL, "n_groups < 0");
    if (!(isfinite(gamma) && gamma > 1.0)) return fail(GAMER_EINVAL, "gamma must be > 1");
    if (n == 0) return GAMER_OK;
    if (!groups || !stats) return fail(GAMER_EINVAL, "NULL groups or group_stats");
    return check_hip(launch_group_stats<T>(groups, n, gamma, stats, g_stream), "stats launch");
}

template <typename T>
int accumulate_common(const T *fluxes, int64_t n, const double *dt_dev, int reset, double *acc) {
    g_err[0] = 0;
    if (n < 0) return fail(GAMER_EINVAL, "n_groups < 0");
    if (n == 0) return GAMER_OK;
    if (!fluxes || !dt_dev || !acc) return fail(GAMER_EINVAL, "NULL array argument");
    if (reinterpret_cast<uintptr_t>(acc) % 16) return fail(GAMER_EINVAL, "acc must be 16-byte aligned");
    return check_hip(launch_flux_accumulate<T>(fluxes, n, dt_dev, reset, acc, g_stream),
                     "flux accumulate launch");
}

template <typename T>
int correct_common(T *coarse, int64_t n_coarse, const T *coarse_fluxes, const double *fine_acc,
                   int64_t n_fine, const gamer_cf_face *faces, int64_t n_faces, const double *dt_dev,
                   const double *dh_dev, int32_t *n_bad) {
    g_err[0] = 0;
    if (n_coarse < 0 || n_fine < 0 || n_faces < 0) return fail(GAMER_EINVAL, "negative count");
    if (n_faces > (int64_t(1) << 32)) return fail(GAMER_EINVAL, "n_faces above 2^32");
    if (n_faces == 0) return GAMER_OK;
    if (!coarse || !coarse_fluxes || !fine_acc || !faces || !dt_dev || !dh_dev)
        return fail(GAMER_EINVAL, "NULL array argument");
    if (reinterpret_cast<uintptr_t>(faces) % 8) return fail(GAMER_EINVAL, "faces must be 8-byte aligned");
    return check_hip(launch_flux_correct<T>(coarse, n_coarse, coarse_fluxes, fine_acc, n_fine, faces,
                                            n_faces, dt_dev, dh_dev, n_bad, g_stream),
                     "flux correct launch");
}

template <typename T>
int restrict_common(const T *fine, const int64_t *parent, int64_t n_fine, T *coarse, int64_t n_coarse,
                    int32_t *n_bad) {
    g_err[0] = 0;
    if (n_fine < 0 || n_coarse < 0) return fail(GAMER_EINVAL, "negative count");
    if (n_fine > (int64_t(1) << 27)) return fail(GAMER_EINVAL, "n_fine above 2^27");
    if (n_fine == 0) return GAMER_OK;
    if (!fine || !parent || !coarse) return fail(GAMER_EINVAL, "NULL array argument");
    return check_hip(launch_restrict<T>(fine, parent, n_fine, coarse, n_coarse, n_bad, g_stream),
                     "restrict launch");
}

template <typename T>
int ctu_common(const T *in, int64_t n, const int8_t *level, const double *dt_dev, const double *dh_dev,
               int n_levels, double gamma, T *fluxes, T *out, double *stats, const gamer_opts *opts,
               void *work, size_t work_bytes) {
    g_err[0] = 0;
    if (n < 0) return fail(GAMER_EINVAL, "n_groups < 0");
    if (!(isfinite(gamma) && gamma > 1.0)) return fail(GAMER_EINVAL, "gamma must be > 1");
    double theta;
    int variant, limiting;
    int64_t grid;
    unsigned long long *bad;
    if (const int e = parse_opts<T>(opts, &theta, &variant, &grid, &limiting, &bad)) return e;
    if (variant > 1 || grid != 0 || limiting != GAMER_LIMIT_PRIMITIVE)
        return fail(GAMER_EINVAL,
                    "the CTU step takes theta, bad_count_dev and variant 0 (fused) or 1 (pipeline) only "
                    "(grid 0; primitive limiting)");
    if (n == 0) return GAMER_OK;
    if (!in || !out || !dt_dev || !dh_dev) return fail(GAMER_EINVAL, "NULL array argument");
    if (n_levels < 1 || n_levels > GAMER_MAX_LEVELS)
        return fail(GAMER_EINVAL, "n_levels must lie in [1, %d]", GAMER_MAX_LEVELS);
    if (n > INT32_MAX / 51) return fail(GAMER_EINVAL, "too many groups for one launch");
    if (variant == 1) {
        const size_t need = ctu_workspace_bytes(n, int(sizeof(T)));
        if (!work || work_bytes < need) return fail(GAMER_EINVAL, "workspace of %zu bytes required", need);
        if (reinterpret_cast<uintptr_t>(work) % 256)
            return fail(GAMER_EINVAL, "workspace must be 256-byte aligned");
    }
    return check_hip(launch_ctu<T>(in, n, level, n_levels, dt_dev, dh_dev, gamma, theta, fluxes, out, stats,
                                   bad, variant, work, g_stream),
                     "CTU launch");
}

template <typename T>
int rtvd_common(const T *in, int gx, int gy, int gz, int64_t n, const int8_t *level,
                const double *dt_dev, const double *dh_dev, int n_levels, double gamma, int order,
                void *work, size_t work_bytes, T *out) {
    g_err[0] = 0;
    if (n < 0) return fail(GAMER_EINVAL, "n_groups < 0");
    if (!(isfinite(gamma) && gamma > 1.0)) return fail(GAMER_EINVAL, "gamma must be > 1");
    if (order != 0 && order != 1) return fail(GAMER_EINVAL, "order must be 0 (x, y, z) or 1 (z, y, x)");
    if (n == 0) return GAMER_OK;
    if (!in || !out || !dt_dev || !dh_dev) return fail(GAMER_EINVAL, "NULL array argument");
    if (n_levels < 1 || n_levels > GAMER_MAX_LEVELS)
        return fail(GAMER_EINVAL, "n_levels must lie in [1, %d]", GAMER_MAX_LEVELS);
    if (static_cast<const void *>(in) == static_cast<const void *>(out))
        return fail(GAMER_EINVAL, "input and output must be different arrays");
    const size_t need = rtvd_workspace_elems<T>(n) * sizeof(T);
    if (!work || work_bytes < need)
        return fail(GAMER_EINVAL, "workspace of %zu bytes required", need);
    if (reinterpret_cast<uintptr_t>(work) % 16) return fail(GAMER_EINVAL, "workspace must be 16-byte aligned");
    if (n * 31 > INT32_MAX) return fail(GAMER_EINVAL, "too many groups for one launch");
    return check_hip(launch_rtvd<T>(in, gx, gy, gz, n, level, n_levels, dt_dev, dh_dev, gamma, order,
                                    static_cast<T *>(work), out, g_stream),
                     "relaxing TVD launch");
}

template <typename T>
int rtvd_periodic_common(const T *state, int gx, int gy, int gz, const double *dt_dev,
                         const double *dh_dev, double gamma, int order, void *work, size_t work_bytes,
                         T *out) {
    g_err[0] = 0;
    if (gx < 1 || gy < 1 || gz < 1) return fail(GAMER_EINVAL, "gx, gy, gz must be >= 1");
    const int64_t n = int64_t(gx) * gy * gz;
    if (int64_t(gx) * NI > (1 << 28) || int64_t(gy) * NI > (1 << 28) || int64_t(gz) * NI > (1 << 28) ||
        n > INT32_MAX)
        return fail(GAMER_EINVAL, "grid too large: gx, gy, gz <= 2^24 and gx*gy*gz < 2^31 required");
    // the first x sweep runs one grid row of 44 work-groups per group along x
    if (gx > 381300 || gy > 65535 || gz > 65535)
        return fail(GAMER_EINVAL, "grid too large for the relaxing TVD step: gx <= 381300, gy, gz <= 65535");
    return rtvd_common<T>(state, gx, gy, gz, n, nullptr, dt_dev, dh_dev, 1, gamma, order, work,
                          work_bytes, out);
}

}  // namespace

extern "C" {

int gamer_version(void) { return 200; }

int gamer_set_stream(void *hip_stream) {
    g_stream = static_cast<hipStream_t>(hip_stream);
    return GAMER_OK;
}

void *gamer_get_stream(void) { return g_stream; }

const char *gamer_last_error(void) { return g_err; }

int gamer_solver_variants(int f32) {
    return f32 ? solve_variant_count<float>() : solve_variant_count<double>();
}

int gamer_solver_variant_shape(int f32, int variant, int *threads, int *waves_per_simd) {
    g_err[0] = 0;
    if (!threads || !waves_per_simd) return fail(GAMER_EINVAL, "NULL output");
    const int ok = f32 ? solve_variant_shape<float>(variant, threads, waves_per_simd)
                       : solve_variant_shape<double>(variant, threads, waves_per_simd);
    return ok ? GAMER_OK : fail(GAMER_EINVAL, "no variant %d", variant);
}

int gamer_hydro_solve(const double *groups_in, int64_t n_groups, double dt, double dh,
                      double gamma, double *fluxes_out, double *groups_out) {
    return solve_common<double, double>(groups_in, n_groups, nullptr, nullptr, nullptr, 1, dt, dh, gamma,
                                        fluxes_out, groups_out, nullptr, nullptr, g_stream);
}

int gamer_hydro_solve_f32(const float *groups_in, int64_t n_groups, double dt, double dh,
                          double gamma, float *fluxes_out, float *groups_out) {
    return solve_common<float, float>(groups_in, n_groups, nullptr, nullptr, nullptr, 1, dt, dh, gamma,
                                      fluxes_out, groups_out, nullptr, nullptr, g_stream);
}

// the stream argument of the batched entry points: NULL keeps the thread's stream
static hipStream_t pick_stream(void *s) { return s ? static_cast<hipStream_t>(s) : g_stream; }

int gamer_hydro_solve_batched(const double *groups_in, int64_t n_groups, const int8_t *level,
                              const double *dt_dev, const double *dh_dev, int n_levels,
                              double gamma, double *fluxes_out, double *groups_out,
                              double *group_stats, const gamer_opts *opts, void *hip_stream) {
    g_err[0] = 0;
    if (!dt_dev && n_groups > 0) return fail(GAMER_EINVAL, "NULL dt_dev");
    return solve_common<double, double>(groups_in, n_groups, level, dt_dev, dh_dev, n_levels, 0.0,
                                        0.0, gamma, fluxes_out, groups_out, group_stats, opts,
                                        pick_stream(hip_stream));
}

int gamer_hydro_solve_batched_f32(const float *groups_in, int64_t n_groups, const int8_t *level,
                                  const double *dt_dev, const double *dh_dev, int n_levels,
                                  double gamma, float *fluxes_out, float *groups_out,
                                  double *group_stats, const gamer_opts *opts, void *hip_stream) {
    g_err[0] = 0;
    if (!dt_dev && n_groups > 0) return fail(GAMER_EINVAL, "NULL dt_dev");
    return solve_common<float, float>(groups_in, n_groups, level, dt_dev, dh_dev, n_levels, 0.0, 0.0,
                                      gamma, fluxes_out, groups_out, group_stats, opts,
                                      pick_stream(hip_stream));
}

int gamer_hydro_solve_periodic(const double *state, int gx, int gy, int gz, const double *dt_dev,
                               const double *dh_dev, double gamma, double *fluxes_out,
                               double *state_out, double *group_stats, const gamer_opts *opts) {
    return periodic_common<double, double>(state, gx, gy, gz, dt_dev, dh_dev, gamma, fluxes_out, state_out,
                                   group_stats, opts);
}

int gamer_hydro_solve_periodic_f32(const float *state, int gx, int gy, int gz, const double *dt_dev,
                                   const double *dh_dev, double gamma, float *fluxes_out,
                                   float *state_out, double *group_stats, const gamer_opts *opts) {
    return periodic_common<float, float>(state, gx, gy, gz, dt_dev, dh_dev, gamma, fluxes_out, state_out,
                                  group_stats, opts);
}

int gamer_hydro_solve_batched_mixed(const double *groups_in, int64_t n_groups, const int8_t *level,
                                    const double *dt_dev, const double *dh_dev, int n_levels,
                                    double gamma, double *fluxes_out, double *groups_out,
                                    double *group_stats, const gamer_opts *opts, void *hip_stream) {
    g_err[0] = 0;
    if (!dt_dev && n_groups > 0) return fail(GAMER_EINVAL, "NULL dt_dev");
    return solve_common<double, float>(groups_in, n_groups, level, dt_dev, dh_dev, n_levels, 0.0, 0.0,
                                       gamma, fluxes_out, groups_out, group_stats, opts,
                                       pick_stream(hip_stream));
}

int gamer_hydro_solve_periodic_mixed(const double *state, int gx, int gy, int gz,
                                     const double *dt_dev, const double *dh_dev, double gamma,
                                     double *fluxes_out, double *state_out, double *group_stats,
                                     const gamer_opts *opts) {
    return periodic_common<double, float>(state, gx, gy, gz, dt_dev, dh_dev, gamma, fluxes_out,
                                          state_out, group_stats, opts);
}

int gamer_step_reduce(const double *group_stats, int64_t n_groups, const int8_t *level,
                      const double *dh_dev, int n_levels, double cfl, double *dt_dev_out,
                      double *totals_dev_out) {
    g_err[0] = 0;
    if (n_groups < 0) return fail(GAMER_EINVAL, "n_groups < 0");
    if (!finite_pos(cfl)) return fail(GAMER_EINVAL, "cfl must be finite and positive");
    if (n_levels < 1 || n_levels > GAMER_MAX_LEVELS)
        return fail(GAMER_EINVAL, "n_levels must lie in [1, %d]", GAMER_MAX_LEVELS);
    if (!dh_dev) return fail(GAMER_EINVAL, "NULL dh_dev");
    if (n_groups > 0 && !group_stats) return fail(GAMER_EINVAL, "NULL group_stats");
    if (!dt_dev_out && !totals_dev_out) return GAMER_OK;
    return check_hip(launch_reduce(group_stats, n_groups, level, dh_dev, 0.0, n_levels, cfl,
                                   dt_dev_out, totals_dev_out, g_stream),
                     "reduce launch");
}

int gamer_group_stats(const double *groups, int64_t n_groups, double gamma, double *group_stats) {
    return stats_common<double>(groups, n_groups, gamma, group_stats);
}

int gamer_group_stats_f32(const float *groups, int64_t n_groups, double gamma,
                          double *group_stats) {
    return stats_common<float>(groups, n_groups, gamma, group_stats);
}

int gamer_cfl_dt(const double *groups, int64_t n_groups, double dh, double gamma, double cfl,
                 double *dt_out, int dt_out_is_device) {
    return cfl_common<double>(groups, n_groups, dh, gamma, cfl, dt_out, dt_out_is_device);
}

int gamer_cfl_dt_f32(const float *groups, int64_t n_groups, double dh, double gamma, double cfl,
                     double *dt_out, int dt_out_is_device) {
    return cfl_common<float>(groups, n_groups, dh, gamma, cfl, dt_out, dt_out_is_device);
}

int gamer_cfl_dt_noalloc(const double *groups, int64_t n_groups, double dh, double gamma, double cfl,
                         double *dt_out_dev) {
    g_err[0] = 0;
    if (n_groups < 0) return fail(GAMER_EINVAL, "n_groups < 0");
    if (n_groups > GAMER_NOALLOC_MAX_GROUPS)
        return fail(GAMER_EINVAL, "n_groups %lld above the fixed scratch's %d groups",
                    (long long)n_groups, GAMER_NOALLOC_MAX_GROUPS);
    if (!finite_pos(dh) || !finite_pos(cfl) || !(isfinite(gamma) && gamma > 1.0))
        return fail(GAMER_EINVAL, "dh and cfl must be finite and positive, gamma > 1");
    if (n_groups == 0) return GAMER_OK;
    if (!dt_out_dev) return fail(GAMER_EINVAL, "NULL dt_out_dev");
    if (!groups) return fail(GAMER_EINVAL, "NULL groups");
    void *buf = nullptr;
    int rc = noalloc_scratch(&buf);
    if (rc) return rc;
    // every group's 8 stats are written before the reduction reads them, so
    // nothing left by an earlier call is read
    double *stats = static_cast<double *>(buf);
    if ((rc = check_hip(launch_group_stats<double>(groups, n_groups, gamma, stats, g_stream), "stats launch")))
        return rc;
    return check_hip(launch_reduce(stats, n_groups, nullptr, nullptr, dh, 1, cfl, dt_out_dev, nullptr, g_stream),
                     "reduce launch");
}

int gamer_conserved_sums(const double *groups, int64_t n_groups, double dh, double *sums5_out,
                         int is_device) {
    return sums_common<double>(groups, n_groups, dh, sums5_out, is_device);
}

int gamer_conserved_sums_f32(const float *groups, int64_t n_groups, double dh,
                             double *sums5_out, int is_device) {
    return sums_common<float>(groups, n_groups, dh, sums5_out, is_device);
}

int gamer_pack_periodic(const double *state, int gx, int gy, int gz, double *padded) {
    return pack_common<double>(state, gx, gy, gz, padded);
}

int gamer_pack_periodic_f32(const float *state, int gx, int gy, int gz, float *padded) {
    return pack_common<float>(state, gx, gy, gz, padded);
}

size_t gamer_ctu_workspace_bytes(int64_t n_groups, int f32) {
    if (n_groups <= 0) return 0;
    return ctu_workspace_bytes(n_groups, f32 ? 4 : 8);
}

int gamer_ctu_solve_batched(const double *groups_in, int64_t n_groups, const int8_t *level,
                            const double *dt_dev, const double *dh_dev, int n_levels, double gamma,
                            double *fluxes_out, double *groups_out, double *group_stats,
                            const gamer_opts *opts, void *work, size_t work_bytes) {
    return ctu_common<double>(groups_in, n_groups, level, dt_dev, dh_dev, n_levels, gamma, fluxes_out,
                              groups_out, group_stats, opts, work, work_bytes);
}

int gamer_ctu_solve_batched_f32(const float *groups_in, int64_t n_groups, const int8_t *level,
                                const double *dt_dev, const double *dh_dev, int n_levels, double gamma,
                                float *fluxes_out, float *groups_out, double *group_stats,
                                const gamer_opts *opts, void *work, size_t work_bytes) {
    return ctu_common<float>(groups_in, n_groups, level, dt_dev, dh_dev, n_levels, gamma, fluxes_out,
                             groups_out, group_stats, opts, work, work_bytes);
}

size_t gamer_rtvd_workspace_bytes(int64_t n_groups, int f32) {
    if (n_groups <= 0) return 0;
    return f32 ? rtvd_workspace_elems<float>(n_groups) * sizeof(float)
               : rtvd_workspace_elems<double>(n_groups) * sizeof(double);
}

int gamer_rtvd_solve_batched(const double *groups_in, int64_t n_groups, const int8_t *level,
                             const double *dt_dev, const double *dh_dev, int n_levels, double gamma,
                             int order, void *work, size_t work_bytes, double *groups_out) {
    return rtvd_common<double>(groups_in, 0, 0, 0, n_groups, level, dt_dev, dh_dev, n_levels, gamma,
                               order, work, work_bytes, groups_out);
}

int gamer_rtvd_solve_batched_f32(const float *groups_in, int64_t n_groups, const int8_t *level,
                                 const double *dt_dev, const double *dh_dev, int n_levels,
                                 double gamma, int order, void *work, size_t work_bytes,
                                 float *groups_out) {
    return rtvd_common<float>(groups_in, 0, 0, 0, n_groups, level, dt_dev, dh_dev, n_levels, gamma,
                              order, work, work_bytes, groups_out);
}

int gamer_rtvd_solve_periodic(const double *state, int gx, int gy, int gz, const double *dt_dev,
                              const double *dh_dev, double gamma, int order, void *work,
                              size_t work_bytes, double *state_out) {
    return rtvd_periodic_common<double>(state, gx, gy, gz, dt_dev, dh_dev, gamma, order, work,
                                        work_bytes, state_out);
}

int gamer_rtvd_solve_periodic_f32(const float *state, int gx, int gy, int gz, const double *dt_dev,
                                  const double *dh_dev, double gamma, int order, void *work,
                                  size_t work_bytes, float *state_out) {
    return rtvd_periodic_common<float>(state, gx, gy, gz, dt_dev, dh_dev, gamma, order, work,
                                       work_bytes, state_out);
}

int gamer_flux_accumulate(const double *fluxes, int64_t n_groups, const double *dt_dev, int reset,
                          double *acc) {
    return accumulate_common<double>(fluxes, n_groups, dt_dev, reset, acc);
}

int gamer_flux_accumulate_f32(const float *fluxes, int64_t n_groups, const double *dt_dev,
                              int reset, double *acc) {
    return accumulate_common<float>(fluxes, n_groups, dt_dev, reset, acc);
}

int gamer_flux_correct(double *coarse, int64_t n_coarse, const double *coarse_fluxes,
                       const double *fine_acc, int64_t n_fine, const gamer_cf_face *faces,
                       int64_t n_faces, const double *dt_dev, const double *dh_dev,
                       int32_t *n_bad_dev) {
    return correct_common<double>(coarse, n_coarse, coarse_fluxes, fine_acc, n_fine, faces, n_faces,
                                  dt_dev, dh_dev, n_bad_dev);
}

int gamer_flux_correct_f32(float *coarse, int64_t n_coarse, const float *coarse_fluxes,
                           const double *fine_acc, int64_t n_fine, const gamer_cf_face *faces,
                           int64_t n_faces, const double *dt_dev, const double *dh_dev,
                           int32_t *n_bad_dev) {
    return correct_common<float>(coarse, n_coarse, coarse_fluxes, fine_acc, n_fine, faces, n_faces,
                                 dt_dev, dh_dev, n_bad_dev);
}

int gamer_restrict(const double *fine, const int64_t *parent, int64_t n_fine, double *coarse,
                   int64_t n_coarse, int32_t *n_bad_dev) {
    return restrict_common<double>(fine, parent, n_fine, coarse, n_coarse, n_bad_dev);
}

int gamer_restrict_f32(const float *fine, const int64_t *parent, int64_t n_fine, float *coarse,
                       int64_t n_coarse, int32_t *n_bad_dev) {
    return restrict_common<float>(fine, parent, n_fine, coarse, n_coarse, n_bad_dev);
}

}  // extern "C"
