/*
 * gamer_hydro.h -- C ABI of the MI355X (gfx950) MUSCL-Hancock + Roe hydro solver
 * for batches of ghost-padded 16^3 patch groups.
 *
 * The method is the GPU hydrodynamic solver of "GAMER with out-of-core
 * computation" (Schive, Tsai & Chiueh), Sec. 2: the MUSCL-Hancock scheme in
 * four steps (spatial data reconstruction, half-step prediction, Riemann
 * solver, full-step update), applied unsplit in 3D, with Roe's Riemann
 * solver and a five-point stencil per direction, i.e. two ghost cells per
 * side of every patch group.  The paper's Sec. 2 also states the division
 * of labour kept here: the host prepares ghost-padded groups, the GPU
 * advances them.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers owned by the caller, unless an
 *    argument says otherwise.  The library never frees or retains them.
 *  - Layouts are C-contiguous with x fastest:
 *      padded group    [n][5][20][20][20]  conserved (rho, m_x, m_y, m_z, E),
 *                                          cell (i,j,k) at i,j,k = -2..17
 *      interior group  [n][5][16][16][16]  cells 0..15
 *      flux planes     [n][3 dir][3 plane][5][16][16]: the flux density F_d
 *                      (not multiplied by dt or area) on the faces with index
 *                      0, 8 and 16 along d (face f lies between cells f-1 and
 *                      f: the two outer faces and the mid-plane between the
 *                      2x2x2 sibling 8^3 patches); transverse order (k,j)
 *                      for x, (k,i) for y, (j,i) for z.
 *      group stats     [n][8] doubles: sum rho, sum m_x, sum m_y, sum m_z,
 *                      sum E over the 16^3 output cells (not multiplied by
 *                      dh^3), max over output cells of |u|+|v|+|w|+3 c_s
 *                      (evaluated in the working precision; NaN if any
 *                      output cell has rho <= 0, p <= 0 or a non-finite
 *                      value, since such a state has no sound speed),
 *                      number of cells whose half-step prediction fell back
 *                      to first order, number of faces whose Roe flux fell
 *                      back to HLLE.
 *  - Ideal gas, p = (gamma - 1)(E - rho |u|^2 / 2), c_s = sqrt(gamma p / rho).
 *  - Every call is asynchronous and ordered on the calling host thread's
 *    current stream (gamer_set_stream; default: the null stream).  Errors a
 *    kernel meets later surface at the next synchronising call.
 *  - Return value: GAMER_OK (0) or a negative code; gamer_last_error() then
 *    holds a message (per host thread).  n_groups == 0 is a successful no-op
 *    (gamer_step_reduce then writes the reduction over no groups: dt = +inf
 *    for every level, totals 0).
 *  - Inputs and outputs must not overlap.
 *  - Non-physical intermediate states are not errors: the solver falls back
 *    (first-order prediction for the cell, HLLE for the face) and counts them
 *    in the group stats.
 *  - FP32 entry points (suffix _f32) store and compute in float, but form
 *    the full-step update U - dt/dh * sum(dF) and all sums in double,
 *    rounding once on store.
 */
#ifndef GAMER_HYDRO_H
#define GAMER_HYDRO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GAMER_OK 0
#define GAMER_EINVAL (-1) /* invalid argument: nothing was launched */
#define GAMER_EHIP (-2)   /* a HIP runtime call failed; see gamer_last_error() */
#define GAMER_ENOMEM (-3) /* the library could not allocate its scratch space */

#define GAMER_MAX_LEVELS 32 /* largest n_levels of the batched entry points */

/* Tunables.  NULL, or a zero-initialised struct, selects the defaults. */
typedef struct gamer_opts {
    /* Generalised-minmod parameter of the slope limiter, 1 <= theta <= 2
     * (1: minmod, 2: monotonised central); 0 selects the default 1.5. */
    double theta;
    /* Compiled solver variant, 0 .. gamer_solver_variants(f32)-1 (0 is the
     * default).  Variants differ in work-group size and in the register budget
     * they were built for (waves per SIMD).  Each is deterministic, and its
     * launch grids give bitwise equal results; across variants FP64 results
     * agree to about 1e-13 and FP32 results to about 1e-6 relative (the
     * compiler may contract multiply-adds differently). */
    int32_t variant;
    /* Work-groups launched: 0 launches one per group (periodic entry points:
     * one per z segment, see zseg); g > 0 launches at most g persistent
     * work-groups that stride over the groups (segments). */
    int32_t grid;
    /* Variables the slopes are limited in: GAMER_LIMIT_PRIMITIVE (0, the
     * default) limits each primitive variable; GAMER_LIMIT_CHARACTERISTIC (1)
     * limits the wave amplitudes of the primitive system's eigen-decomposition
     * along each direction (the paper does not say which; both are common
     * choices of the MUSCL-Hancock reconstruction step, Toro 2009, Sec. 14). */
    int32_t limiting;
    /* Periodic entry points (gamer_hydro_solve_periodic*): the groups of one
     * (x, y) column of the grid are taken zseg at a time along z, and one
     * work-group sweeps such a segment as one run of planes, so the planes and z
     * faces that neighbouring groups of the segment share are computed once and
     * read once.  Results, flux planes and stats (fallback counts included) are
     * the same for every zseg.  0 lets the library choose (the largest divisor
     * of gz that leaves at least 12,288 segments, else 1); values above gz act
     * as gz.  Must be 0 for the other entry points. */
    int32_t zseg;
    /* Two device counters the step adds to, or NULL (8-byte aligned device
     * memory, zeroed by the caller; accumulated with atomics, so their order of
     * arrival is free but the totals are exact):
     *   bad_count_dev[0] += updated cells that are not physical (rho <= 0 or
     *                       p <= 0) or not finite;
     *   bad_count_dev[1] += groups whose level byte lies outside [0, n_levels).
     * Such cells are not errors of the call (see the conventions above).  The
     * positivity reading: the method keeps states physical through its two
     * fallbacks; a cell that still leaves the physical set is reported, never
     * clipped, so the stored state stays conservative. */
    uint64_t *bad_count_dev;
} gamer_opts;

#define GAMER_LIMIT_PRIMITIVE 0
#define GAMER_LIMIT_CHARACTERISTIC 1

/* Number of compiled solver variants for the float (f32 != 0) or double path,
 * and the shape of variant v: work-group size in threads and the waves per
 * SIMD its register allocation allows (GAMER_EINVAL for an unknown v).  Used
 * by the tuner that picks a variant and a grid for a given batch. */
int gamer_solver_variants(int f32);
int gamer_solver_variant_shape(int f32, int variant, int *threads, int *waves_per_simd);

/* Library version, major * 10000 + minor * 100 + patch. */
int gamer_version(void);

/* Make `hip_stream` (a hipStream_t, may be NULL for the null stream) the
 * stream of every later call from this host thread. */
int gamer_set_stream(void *hip_stream);
void *gamer_get_stream(void);

/* Message of the last failing call on this host thread ("" if none). */
const char *gamer_last_error(void);

/* ---- one MUSCL-Hancock + Roe step (paper Sec. 2, all four steps) --------
 * Advances every padded group in `groups_in` by dt with cell size dh and
 * writes the 16^3 interior to `groups_out`.  Per group:
 *   1. reconstruction: primitive variables, generalised-minmod limited
 *      slopes along x, y, z on the interior plus one ghost layer per face;
 *   2. half-step prediction: the conservative Hancock step with the flux
 *      differences of all three directions added to all six face states;
 *   3. Roe fluxes (Harten-Hyman entropy fix; HLLE when an intermediate
 *      state is unphysical) at the 3 x 17 x 16 x 16 faces;
 *   4. full-step update U^{n+1} = U^n - dt/dh sum_d (F_{d,+} - F_{d,-}).
 * `fluxes_out` may be NULL.  Errors: GAMER_EINVAL for n_groups < 0, a NULL
 * array with n_groups > 0, dt or dh not finite and positive, gamma <= 1. */
int gamer_hydro_solve(const double *groups_in, int64_t n_groups, double dt, double dh,
                      double gamma, double *fluxes_out, double *groups_out);
int gamer_hydro_solve_f32(const float *groups_in, int64_t n_groups, double dt, double dh,
                          double gamma, float *fluxes_out, float *groups_out);

/* ---- batched step over groups of uneven refinement level ---------------
 * Same step as gamer_hydro_solve in ONE launch, with each group's dt and dh
 * read ON THE DEVICE: group g uses dt_dev[level[g]] and dh_dev[level[g]]
 * (level == NULL: every group uses level 0), so a captured HIP graph can be
 * replayed while dt changes.  level: device int8 [n_groups], values in
 * 0..n_levels-1.  The device checks every level byte: a group whose level
 * lies outside [0, n_levels) never indexes dt_dev or dh_dev; it is advanced
 * with NaN dt and dh, so its output block and stats row come out NaN, and it
 * is counted in opts->bad_count_dev[1].  dt_dev, dh_dev: device double
 * [n_levels], 1 <= n_levels <= GAMER_MAX_LEVELS.  group_stats: device double
 * [n_groups][8] (see conventions) or NULL.  opts may be NULL.  hip_stream: the
 * hipStream_t to launch on, or NULL for the calling thread's current stream
 * (gamer_set_stream).  The null stream's handle is NULL too, so a caller that
 * means the null stream makes it the thread's stream first
 * (gamer_set_stream(NULL)). */
int gamer_hydro_solve_batched(const double *groups_in, int64_t n_groups, const int8_t *level,
                              const double *dt_dev, const double *dh_dev, int n_levels,
                              double gamma, double *fluxes_out, double *groups_out,
                              double *group_stats, const gamer_opts *opts, void *hip_stream);
int gamer_hydro_solve_batched_f32(const float *groups_in, int64_t n_groups, const int8_t *level,
                                  const double *dt_dev, const double *dh_dev, int n_levels,
                                  double gamma, float *fluxes_out, float *groups_out,
                                  double *group_stats, const gamer_opts *opts, void *hip_stream);

/* ---- one step of a uniform periodic grid, ghost cells fetched in place ---
 * The same step as gamer_hydro_solve_batched, for the interior state of a
 * uniform periodic grid of gx x gy x gz groups ([gx*gy*gz][5][16][16][16],
 * group index x + gx (y + gy z)): each group's two ghost layers are read from
 * its periodic neighbours while it is advanced, so no padded copy is built.
 * (The paper's Sec. 2 notes that preparing ghost zones costs more than the GPU
 * solver itself; for this uniform case the preparation disappears.)  Results
 * equal those of gamer_pack_periodic followed by the batched step with the
 * same variant: bitwise in FP64 with primitive limiting, to rounding otherwise
 * (the two are separate compilations, whose multiply-adds may contract
 * differently); fallback counts are equal.  dt_dev, dh_dev: device double
 * [1].  state_out must not be state.  group_stats, fluxes_out, opts as in the
 * batched step; opts->zseg as described with gamer_opts.
 * Errors: GAMER_EINVAL for gx, gy, gz outside [1, 2^24] or gx*gy*gz >= 2^31,
 * NULL state / state_out / dt_dev / dh_dev, state_out == state, gamma or opts
 * as in the batched step. */
int gamer_hydro_solve_periodic(const double *state, int gx, int gy, int gz, const double *dt_dev,
                               const double *dh_dev, double gamma, double *fluxes_out,
                               double *state_out, double *group_stats, const gamer_opts *opts);
int gamer_hydro_solve_periodic_f32(const float *state, int gx, int gy, int gz, const double *dt_dev,
                                   const double *dh_dev, double gamma, float *fluxes_out,
                                   float *state_out, double *group_stats, const gamer_opts *opts);

/* ---- FP64 state, FP32 arithmetic ----------------------------------------
 * The batched and periodic steps on double arrays with the reconstruction,
 * prediction and Riemann solver evaluated in float, and the full-step update
 * U - dt/dh * sum(dF) formed and stored in double: the state keeps FP64
 * resolution (no float rounding of the state accumulates over steps) at about
 * the FP32 arithmetic cost.  Arguments, layouts and errors as in
 * gamer_hydro_solve_batched / gamer_hydro_solve_periodic with double arrays;
 * fluxes_out holds the float fluxes widened to double; opts->variant indexes
 * the float variants (gamer_solver_variants(1)). */
int gamer_hydro_solve_batched_mixed(const double *groups_in, int64_t n_groups, const int8_t *level,
                                    const double *dt_dev, const double *dh_dev, int n_levels,
                                    double gamma, double *fluxes_out, double *groups_out,
                                    double *group_stats, const gamer_opts *opts, void *hip_stream);
int gamer_hydro_solve_periodic_mixed(const double *state, int gx, int gy, int gz,
                                     const double *dt_dev, const double *dh_dev, double gamma,
                                     double *fluxes_out, double *state_out, double *group_stats,
                                     const gamer_opts *opts);

/* ---- reduction of group stats to time steps and totals -----------------
 * From group_stats [n_groups][8] (as written by the batched step or by
 * gamer_group_stats), computes on the device, in a fixed order (results are
 * bitwise reproducible):
 *   dt_dev_out[L] = cfl * dh_dev[L] / max over groups of level L of stat 5
 *                   (+inf when level L has no group or a zero maximum; NaN
 *                   when a group of level L has a NaN stat 5, i.e. holds a
 *                   cell that is not physical);
 *   totals_dev_out[0..4] = sum over groups of dh_dev[level]^3 * stats 0..4,
 *   totals_dev_out[5..6] = sum over groups of stats 6..7.
 * A group whose level lies outside [0, n_levels) is read with no index into
 * dh_dev: it belongs to no level's dt and makes totals 0..4 NaN.
 * Either output may be NULL.  level, dh_dev, n_levels as in the batched step.
 * Errors: GAMER_EINVAL for cfl not finite and positive, bad sizes. */
int gamer_step_reduce(const double *group_stats, int64_t n_groups, const int8_t *level,
                      const double *dh_dev, int n_levels, double cfl, double *dt_dev_out,
                      double *totals_dev_out);

/* ---- per-group stats of interior groups --------------------------------
 * group_stats [n][8] for interior groups [n][5][16][16][16] (stats 6, 7 set to 0). */
int gamer_group_stats(const double *groups, int64_t n_groups, double gamma, double *group_stats);
int gamer_group_stats_f32(const float *groups, int64_t n_groups, double gamma,
                          double *group_stats);

/* ---- CFL time step ------------------------------------------------------
 * dt = cfl * dh / max over all interior cells of (|u| + |v| + |w| + 3 c_s), the
 * 3D unsplit stability bound (the paper does not state its CFL form),
 * evaluated in the working precision (the _f32 variant in float).  NaN when
 * a cell is not physical (rho <= 0 or p <= 0) or not finite.
 * groups: interior [n][5][16][16][16].  dt_out is a device pointer when
 * dt_out_is_device != 0 (asynchronous), else a host pointer (the call then
 * synchronises the stream).  Uses library scratch of 64 B per group. */
int gamer_cfl_dt(const double *groups, int64_t n_groups, double dh, double gamma, double cfl,
                 double *dt_out, int dt_out_is_device);
int gamer_cfl_dt_f32(const float *groups, int64_t n_groups, double dh, double gamma, double cfl,
                     double *dt_out, int dt_out_is_device);

/* ---- CFL time step without allocation -----------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * time step as gamer_cfl_dt (same kernels, bitwise the same value) for FP64
 * interior groups [n][5][16][16][16], written to the device pointer
 * dt_out_dev, asynchronously on the thread's stream.  The per-group stats go
 * to a fixed scratch array inside the library, 64 B per group for at most
 * GAMER_NOALLOC_MAX_GROUPS groups (16 MiB + 256 B per device, held until the
 * process ends); the call allocates and frees nothing.  The first call on a
 * device looks up that array's address (hipGetSymbolAddress): make it before
 * any graph capture.  Calls that overlap on one device (two streams, two
 * threads) share the array and race.
 * Errors: GAMER_EINVAL for n_groups < 0 or above GAMER_NOALLOC_MAX_GROUPS,
 * dh or cfl not finite and positive, gamma <= 1, NULL pointers (n_groups == 0
 * is a no-op success); GAMER_EHIP for a failed launch. */
#define GAMER_NOALLOC_MAX_GROUPS 262144
int gamer_cfl_dt_noalloc(const double *groups, int64_t n_groups, double dh, double gamma, double cfl,
                         double *dt_out_dev);

/* ---- conserved totals ---------------------------------------------------
 * sums5_out = dh^3 (sum rho, sum m_x, sum m_y, sum m_z, sum E) over interior
 * groups [n][5][16][16][16], accumulated in double in a fixed order.
 * Device pointer when is_device != 0, else host (synchronising). */
int gamer_conserved_sums(const double *groups, int64_t n_groups, double dh, double *sums5_out,
                         int is_device);
int gamer_conserved_sums_f32(const float *groups, int64_t n_groups, double dh,
                             double *sums5_out, int is_device);

/* ---- same-level periodic ghost fill (harness utility) -------------------
 * state: interior groups of a uniform periodic grid of gx x gy x gz groups,
 * [gx*gy*gz][5][16][16][16] with group index g = x + gx (y + gy z).
 * padded: [gx*gy*gz][5][20][20][20]; each padded cell takes the value of
 * the cell at its periodically wrapped global position.  The paper prepares
 * ghost zones on the host from the AMR hierarchy; this covers the uniform
 * periodic case on the device.  Both arrays must be aligned to 4 elements
 * (16 B float, 32 B double).  Errors: GAMER_EINVAL for gx, gy, gz < 1,
 * gx*gy*gz*100 > INT32_MAX (about 21 million groups), NULL or misaligned arrays. */
int gamer_pack_periodic(const double *state, int gx, int gy, int gz, double *padded);
int gamer_pack_periodic_f32(const float *state, int gx, int gy, int gz, float *padded);

/* ---- corner-transport-upwind coupling (a variant of the unsplit step) -----
 * The paper applies MUSCL-Hancock unsplit (Sec. 2) without saying how the
 * three directions are coupled.  The default entry points couple them through
 * the conservative Hancock predictor; this variant couples them as Colella's
 * (1990) corner transport upwind method does (its six-Riemann-solve form):
 *  1. slopes as in the default path (primitive, generalised minmod) on the
 *     cells of [-1,16]^3 with at most two coordinates outside 0..15;
 *  2. per direction d, face states cons(W -+ dW_d/2) advanced by
 *     dt/(2dh) [F_d(U^{d,-}) - F_d(U^{d,+})] (direction d alone); if either is
 *     unphysical both take the cell average (counted in stat 6);
 *  3. Roe fluxes Ft between every two neighbouring cells of that set;
 *  4. the states the group's faces use are corrected by
 *     -dt/(2dh) sum_{d' != d} [Ft_{d'}(c + e_{d'}/2) - Ft_{d'}(c - e_{d'}/2)]; a
 *     corrected state that is unphysical keeps its step-2 value (stat 6);
 *  5. Roe fluxes at the 3 x 17 x 16^2 faces and the default full-step update.
 * HLLE fallbacks of steps 3 and 5 are counted in stat 7.  Arguments, layouts
 * and outputs as in gamer_hydro_solve_batched (padded input); opts may set
 * theta, bad_count_dev and variant: 0 (default) runs one z-sweeping launch
 * with every intermediate on chip and ignores work (which may be NULL); 1 runs
 * the three-launch pipeline, whose intermediates go through work: a device
 * workspace of gamer_ctu_workspace_bytes(n, f32) bytes, 256-byte aligned,
 * owned by the caller.  The two agree to rounding (FP64: about 1e-16 of each
 * cell's update terms), with equal fallback counts.  Neither allocates.
 * Errors as the batched step, plus opts fields other than theta, variant and
 * bad_count_dev, a variant other than 0 or 1, and for variant 1 a missing,
 * short or misaligned workspace. */
size_t gamer_ctu_workspace_bytes(int64_t n_groups, int f32);
int gamer_ctu_solve_batched(const double *groups_in, int64_t n_groups, const int8_t *level,
                            const double *dt_dev, const double *dh_dev, int n_levels, double gamma,
                            double *fluxes_out, double *groups_out, double *group_stats,
                            const gamer_opts *opts, void *work, size_t work_bytes);
int gamer_ctu_solve_batched_f32(const float *groups_in, int64_t n_groups, const int8_t *level,
                                const double *dt_dev, const double *dh_dev, int n_levels, double gamma,
                                float *fluxes_out, float *groups_out, double *group_stats,
                                const gamer_opts *opts, void *work, size_t work_bytes);

/* ---- the relaxing TVD scheme (the solver the paper compares with) --------
 * The paper's Sec. 2 compares MUSCL-Hancock with the scheme GAMER used
 * before: the second-order relaxing total-variation-diminishing scheme of
 * Trac & Pen (2003), made three-dimensional by dimensional splitting, whose
 * seven-point stencil needs three ghost cells per side.  One step sweeps x,
 * y, z (order 0) or z, y, x (order 1; alternate the two between steps).  Per
 * sweep along d, with the freezing speed c = |v_d| + c_s and w = F_d(u)/c of
 * each cell, the right- and left-moving fluxes fr = c (u + w), fl = c (u - w)
 * give first-order face fluxes (fr_i - fl_{i+1})/2 for a half step of dt/2,
 * then, from the half-step state, second-order face fluxes with van Leer's
 * limiter on each moving part for the full step of dt:
 *   R = fr_i + VL((fr_i - fr_{i-1})/2, (fr_{i+1} - fr_i)/2),
 *   L = fl_{i+1} + VL((fl_i - fl_{i+1})/2, (fl_{i+1} - fl_{i+2})/2),
 *   F = (R - L)/2,   VL(a, b) = 2ab/(a+b) if ab > 0 else 0.
 * Input: padded groups [n][5][22][22][22] (cells -3..18 per axis) or, for the
 * periodic entry points, the state of a periodic grid of groups as in
 * gamer_hydro_solve_periodic.  Output: [n][5][16][16][16]; it must not alias
 * the input.  dt and dh are read on the device per level as in the batched
 * MUSCL-Hancock step (level may be NULL; the periodic entry points use
 * dt_dev[0], dh_dev[0]).  The FP32 variants compute in float and form each
 * sweep's update u - dt/dx (F_{i+1/2} - F_{i-1/2}) in double, rounding once.
 * work: device workspace of gamer_rtvd_workspace_bytes(n, f32) bytes, 16-byte
 * aligned, owned by the caller (nothing is allocated inside).  States with
 * rho <= 0 or p <= 0 are not caught (the scheme has no fallback).
 * Errors: GAMER_EINVAL for bad sizes or order (periodic grids: gx <= 381300,
 * gy, gz <= 65535), NULL or aliased arrays, a missing or short workspace. */
size_t gamer_rtvd_workspace_bytes(int64_t n_groups, int f32);
int gamer_rtvd_solve_batched(const double *groups_in, int64_t n_groups, const int8_t *level,
                             const double *dt_dev, const double *dh_dev, int n_levels, double gamma,
                             int order, void *work, size_t work_bytes, double *groups_out);
int gamer_rtvd_solve_batched_f32(const float *groups_in, int64_t n_groups, const int8_t *level,
                                 const double *dt_dev, const double *dh_dev, int n_levels,
                                 double gamma, int order, void *work, size_t work_bytes,
                                 float *groups_out);
int gamer_rtvd_solve_periodic(const double *state, int gx, int gy, int gz, const double *dt_dev,
                              const double *dh_dev, double gamma, int order, void *work,
                              size_t work_bytes, double *state_out);
int gamer_rtvd_solve_periodic_f32(const float *state, int gx, int gy, int gz, const double *dt_dev,
                                  const double *dh_dev, double gamma, int order, void *work,
                                  size_t work_bytes, float *state_out);

/* ---- two refinement levels: flux correction and restriction -------------
 * The steps that follow the solver when a coarse level and a fine level at
 * half the spacing are advanced together, as in GAMER's patch-based AMR
 * (Schive et al. 2010, the code the paper extends, Sec. 1): a coarse group is
 * 2x2x2 patches of 8^3 cells; refining a patch gives one fine group of 16^3
 * cells.  After one coarse step and the fine level's sub-steps:
 *   - flux correction (conservative refluxing, Berger & Colella 1989): an
 *     unrefined coarse cell next to a coarse/fine face was updated with the
 *     coarse flux F_C through that face; it is corrected to use instead the
 *     fine fluxes through the same face, summed over the fine sub-steps s with
 *     their dt_s and averaged over the 2x2 fine faces that tile the coarse face:
 *       Phi = sum_s dt_s (1/4) sum_faces F_f,s,   delta = (dt_C F_C - Phi) / dh_C,
 *     the cell below the face (lower index along d) gains delta, the cell
 *     above it loses delta;
 *   - restriction: each coarse cell covered by a fine group takes the mean of
 *     its 2x2x2 fine children.
 * Together they keep the composite (coarse + fine) totals conserved. */

/* One coarse/fine face: an 8x8 patch face of coarse cells next to a fine group.
 * 24 bytes, 8-byte aligned. */
typedef struct gamer_cf_face {
    int64_t coarse_group; /* group holding the unrefined coarse cells */
    int64_t fine_group;   /* fine group on the other side of the face */
    int8_t dir;           /* face normal: 0 x, 1 y, 2 z */
    int8_t coarse_face;   /* 0, 1, 2: the face at index 0, 8 or 16 of the coarse
                             group along dir (the coarse flux-plane index) */
    int8_t side;          /* 0: the coarse cells lie below the face (index
                             8*coarse_face - 1) and the fine group's face 0 is
                             the face; 1: above (index 8*coarse_face), the fine
                             group's face 16 */
    int8_t qs, qf;        /* 0/1: which 8x8 quarter of the 16x16 coarse plane,
                             along the plane's slow and fast transverse axes */
    int8_t reserved[3];
} gamer_cf_face;

/* acc (double, the flux-plane layout [n_groups][3][3][5][16][16]) =
 * (reset ? 0 : acc) + dt_dev[0] * fluxes, element by element.  Summing a fine
 * level's fluxes_out over its sub-steps gives the Phi above (before the 1/4
 * area average).  acc must be 16-byte aligned.
 * Errors: GAMER_EINVAL for n_groups < 0, NULL or misaligned arrays. */
int gamer_flux_accumulate(const double *fluxes, int64_t n_groups, const double *dt_dev, int reset,
                          double *acc);
int gamer_flux_accumulate_f32(const float *fluxes, int64_t n_groups, const double *dt_dev,
                              int reset, double *acc);

/* Applies every face record's correction to the coarse interior groups
 * coarse [n_coarse][5][16][16][16] in place, with coarse_fluxes the coarse
 * step's fluxes_out, fine_acc [n_fine][3][3][5][16][16] the fine level's
 * accumulated fluxes (gamer_flux_accumulate), dt_dev / dh_dev the coarse
 * level's dt and dh (device double [1]), faces [n_faces] in device memory.
 * The x records are applied first, then y, then z (three launches); records
 * of one direction must name distinct coarse cells.  A record with an index
 * or field out of range is skipped and, when n_bad_dev (device int32) is not
 * NULL, counted there (the caller zeroes it).  The FP32 variant forms each
 * corrected value in double and rounds once per record.
 * Errors: GAMER_EINVAL for negative counts, NULL arrays, misaligned faces. */
int gamer_flux_correct(double *coarse, int64_t n_coarse, const double *coarse_fluxes,
                       const double *fine_acc, int64_t n_fine, const gamer_cf_face *faces,
                       int64_t n_faces, const double *dt_dev, const double *dh_dev,
                       int32_t *n_bad_dev);
int gamer_flux_correct_f32(float *coarse, int64_t n_coarse, const float *coarse_fluxes,
                           const double *fine_acc, int64_t n_fine, const gamer_cf_face *faces,
                           int64_t n_faces, const double *dt_dev, const double *dh_dev,
                           int32_t *n_bad_dev);

/* Restriction: for each fine group f [n_fine][5][16][16][16] with
 * parent[f] = coarse_group * 8 + octant (octant = ox + 2 oy + 4 oz: the
 * coarse group's patch it covers), the 8^3 coarse cells of that patch take the
 * mean of their 2x2x2 children, summed in double and rounded once.  parent[f]
 * < 0 skips the group; a parent beyond the coarse array is skipped and counted
 * in n_bad_dev as above.  parent is device memory.
 * Errors: GAMER_EINVAL for negative counts, n_fine above 2^27, NULL arrays. */
int gamer_restrict(const double *fine, const int64_t *parent, int64_t n_fine, double *coarse,
                   int64_t n_coarse, int32_t *n_bad_dev);
int gamer_restrict_f32(const float *fine, const int64_t *parent, int64_t n_fine, float *coarse,
                       int64_t n_coarse, int32_t *n_bad_dev);

#ifdef __cplusplus
}
#endif

#endif /* GAMER_HYDRO_H */
