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
//  - Work between two barriers is spread so that no wave carries more than the
//    heaviest share: in the 256-thread shape the wave that computed the ghost
//    layer solves its z faces after the x and y faces, while the x faces 16 (on
//    wave k+1 mod 4) and the y faces 16 (on wave k+2 mod 4) are solved by
//    other waves, from right states the ghost-layer wave left in LDS.
//  - The update of plane k-1 completes at step k, once the z flux above it is
//    known: U - dt/dh ((dF_x + dF_y) + dF_z), in double for both precisions.
//  - Plane k+2 is loaded into registers at the top of step k and written to
//    the ring after the step's last barrier.  The old state of plane k-1 is
//    loaded in one batch before the update's stores.  Both orderings keep the
//    waits for loads from also waiting out earlier output stores (vector memory
//    operations complete in issue order).
//  - Template parameters select the storage and arithmetic types (float,
//    double, or double state with float arithmetic), the input (padded groups
//    or a periodic grid of unpadded groups read in place) and the limited
//    variables (primitive or characteristic).
//  - Per-group stats of the updated cells (sums, max signal speed, fallback
//    counts) are reduced in a fixed order in the epilogue.  An updated cell
//    that is not physical (rho <= 0, p <= 0) or not finite makes the group's
//    signal speed NaN and is counted in an optional device counter.
#include "device_math.h"
#include "euler.h"
#include "internal.h"

namespace gamer {
namespace {

constexpr int NINNER = NI * NI;  // 256 interior columns

// Element `off` of a wave-uniform base pointer, for a lane offset known to be
// non-negative and below 2^32: the access can then take the base in scalar
// registers and a 32-bit lane offset, with no 64-bit address arithmetic per lane.
template <typename P>
__device__ __forceinline__ P &at(P *base, unsigned off) {
    return base[off];
}

template <typename T>
struct alignas(16) Lds {
    T w[3][NV][NPL];       // primitive planes, ring indexed by (plane + 3) % 3
    T sx[NV][NI][NI + 1];  // [v][j][f]: +x state of cell f-1, then x flux at face f
    T sy[NV][NI + 1][NI];  // [v][f][i]: +y state of cell f-1, then y flux at face f
    T rf[2][NV][NI];       // -x state of ghost cell (16, j), -y state of ghost cell (i, 16)
    double dxy[NV][NINNER];  // (dF_x + dF_y) of each interior cell of the previous plane
};

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

// Work-groups are dispatched to the 8 XCDs round-robin (work-group b to XCD
// b mod 8), and each XCD has its own L2.  Launch slot i (work-group b at its
// k-th pass of the grid-stride loop, i = b + k * gridDim.x, with gridDim.x a
// multiple of 8 or the whole batch) is mapped to a group so that each XCD
// takes a contiguous run of groups: neighbouring groups, which read each
// other's cells as ghost cells, then mostly share an L2.  A bijection on
// [0, n) for any n.
constexpr int NXCD = 8;
__device__ __forceinline__ int64_t xcd_group(int64_t i, int64_t n) {
    const int64_t x = i % NXCD, j = i / NXCD, q = n / NXCD, r = n % NXCD;
    return x * q + (x < r ? x : r) + j;
}

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

// Stats values reduced per pass when a group's stats go out in the middle of a
// unit: the pass's values for every thread must fit in the flux arrays and the
// face-16 states (sx, sy, rf), the LDS free at that point.
template <typename T>
constexpr int FLUSH_PART = sizeof(T) == 4 ? 4 : 8;
template <typename T>
constexpr size_t FLUX_LDS = sizeof(Lds<T>::sx) + sizeof(Lds<T>::sy) + sizeof(Lds<T>::rf);
static_assert(320 * FLUSH_PART<float> * sizeof(double) <= FLUX_LDS<float> &&
                  320 * FLUSH_PART<double> * sizeof(double) <= FLUX_LDS<double> &&
                  NSTAT % FLUSH_PART<float> == 0 && NSTAT % FLUSH_PART<double> == 0,
              "a stats pass must fit in the flux arrays");

// Position (j * 20 + i) of the q-th of the 400 cells of a padded plane in the
// periodic load order: the 16 x 16 interior row by row, then the two ghost rows
// below and above it (20 cells each), then the ghost cells beside it, row by row.
__device__ __forceinline__ int plane_pos(int q) {
    if (q < NINNER) return ((q >> 4) + NG) * NP + (q & 15) + NG;
    int r = q - NINNER;
    if (r < 4 * NP) {
        const int row = r / NP;
        return (row < NG ? row : row + NI) * NP + r % NP;
    }
    r -= 4 * NP;
    const int col = r & 3;
    return ((r >> 2) + NG) * NP + (col < NG ? col : col + NI);
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

    // A unit is one group of padded input, or, for periodic input, a run of
    // nseg groups along z of one (x, y) column, swept as one sequence of planes
    // (units numbered column fastest, then z segment).
    const int64_t cols = PERIODIC ? int64_t(P.gx) * P.gy : 1;
    const int64_t n_units = PERIODIC ? cols * ((P.gz + P.zseg - 1) / P.zseg) : P.n_groups;
    for (int64_t slot = blockIdx.x; slot < n_units; slot += gridDim.x) {
        const int64_t unit = xcd_group(slot, n_units);
        int bx = 0, by = 0, bz = 0, nseg = 1;
        int64_t g = unit;  // the unit's first group; group q of the unit is g + q * cols
        if (PERIODIC) {
            const int64_t col = unit % cols;
            bx = int(col % P.gx);
            by = int(col / P.gx);
            bz = int(unit / cols) * P.zseg;
            nseg = P.gz - bz < P.zseg ? P.gz - bz : P.zseg;
            g = col + cols * bz;
        }
        const int nplanes = NI * nseg;  // interior planes 0 .. nplanes-1 of the unit
        double dt = P.dt, dh = P.dh;
        if (P.dt_dev && !level_dt(P.level, g, P.n_levels, P.dt_dev, P.dh_dev, dt, dh)) {
            // a level byte out of range: the group runs on NaN dt and dh (its
            // output and stats come out NaN) and is counted once
            if (P.bad && t == 0) atomicAdd(P.bad + 1, 1ull);
        }
        const double dtdh = dt / dh;
        const double hdtdh = 0.5 * dtdh;  // the Roe fluxes below are kept doubled (2F)

        // ---- where padded cell (ip, jp, kp) of this unit lives in the input ----
        // Padded input: the group's own padded block.  Periodic input: the cell at
        // the wrapped global position, in whichever group holds it; an offset is
        // (group index) * 20480 + (cell within the group), the group index split
        // into an x/y part and a z part.  kp counts planes from the unit's first
        // group, so it runs past 19 when the unit holds several groups.
        constexpr int VSTRIDE = PERIODIC ? NI * NI * NI : NP * NP * NP;
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
        // Padded input: position q of the plane, row by row (the plane is one
        // contiguous block).  Periodic float input: the 256 interior positions
        // first, then the 144 ghost positions, so that a wave's load of the
        // interior reads contiguous rows of the group itself (1024^3: 35.5 ->
        // 35.0 ms).  With double storage the extra registers of that order spill
        // (15 -> 22) and cost more than it saves; it keeps the row order.
        constexpr bool INTERIOR_FIRST = PERIODIC && sizeof(S_) == 4;
        const bool has1 = t + NT < NPL;
        const int p0 = INTERIOR_FIRST ? plane_pos(t) : t;
        const int p1 = INTERIOR_FIRST ? (has1 ? plane_pos(t + NT) : p0) : t + NT;
        int gp0;
        const int cp0 = xy_part(p0 % NP, p0 / NP, gp0);
        int gp1 = gp0;  // threads without a second position reload their first
        const int cp1 = has1 ? xy_part(p1 % NP, p1 / NP, gp1) : cp0;
        T pre0[NV], pre1[NV];
        auto fetch = [&](int plane) {  // plane in -2..17
            const S_ *src = plane_base(plane + NG);
            S_ r0[NV], r1[NV];
            if constexpr (!PERIODIC) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    r0[v] = at(src + v * VSTRIDE, unsigned(cp0));
                    r1[v] = at(src + v * VSTRIDE, unsigned(cp1));
                }
            } else {
                const S_ *s0 = src + int64_t(gp0) * GOUT + cp0;
                const S_ *s1 = src + int64_t(gp1) * GOUT + cp1;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    r0[v] = s0[v * VSTRIDE];
                    r1[v] = s1[v * VSTRIDE];
                }
            }
            // With double storage and float arithmetic the values are narrowed
            // here.  Every load is issued before the first conversion, so their
            // latencies overlap; left to itself the scheduler may pair each load
            // with its conversion, one memory wait per value.
            if constexpr (sizeof(S_) != sizeof(T)) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                pre0[v] = T(r0[v]);
                pre1[v] = T(r1[v]);
            }
        };
        // conserved -> primitive, into the LDS slot of a plane
        auto to_lds = [&](int slot, int pos, const T q[NV]) {
            const T ir = rcp(q[0]);
            const T u = q[1] * ir, v = q[2] * ir, w = q[3] * ir;
            S.w[slot][0][pos] = q[0];
            S.w[slot][1][pos] = u;
            S.w[slot][2][pos] = v;
            S.w[slot][3][pos] = w;
            S.w[slot][4][pos] = c.gm1 * (q[4] - c.half * q[0] * (u * u + v * v + w * w));
        };
        auto store = [&](int plane) {  // the prefetched plane -> its LDS slot
            const int slot = (plane + 3) % 3;
            to_lds(slot, p0, pre0);
            if (has1) to_lds(slot, p1, pre1);
        };

        // planes -2, -1, 0: every load issued before the first is consumed, so the
        // group start waits for memory once.  (Threads without a second position
        // loaded their first one again and write it again: same value, same place.)
        {
            T q0[3][NV], q1[3][NV];
#pragma unroll
            for (int pl = 0; pl < 3; ++pl) {
                fetch(pl - 2);
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    q0[pl][v] = pre0[v];
                    q1[pl][v] = pre1[v];
                }
            }
#pragma unroll
            for (int pl = 0; pl < 3; ++pl) {
                const int slot = (pl + 1) % 3;  // (plane + 3) % 3 of plane pl - 2
                to_lds(slot, p0, q0[pl]);
                to_lds(slot, has1 ? p1 : p0, q1[pl]);
            }
        }

        // carried across sweep steps
        T zp[NV];            // +z state of this column at the previous plane
        T fz[NV];            // z flux below the current plane
        double st[6];        // sums of the 5 conserved variables, max signal speed
        int n_pred = 0, n_roe = 0;  // fallback counts of the group being finished
        unsigned n_bad = 0;  // output cells that are not physical or not finite
        // With several groups per unit, a plane next to a group boundary serves
        // two groups: plane 16q is group q's plane 0 and group q-1's ghost plane
        // 16, plane 16q-1 also group q's ghost plane -1, and the z face between
        // them is face 16 of one and face 0 of the other.  Each group's counts
        // take such a plane's interior predictions and z face as its own padded
        // step would, so they equal a one-group sweep's.  `step` holds this
        // step's fallbacks (bit 0 interior cell, bit 1 ghost-layer cell, bit 2 z
        // face, bits 3.. number of x and y faces), `carry` the next group's
        // counts so far (predictions + 65536 * faces).
        int step = 0, carry = 0;
#pragma unroll
        for (int q = 0; q < 6; ++q) st[q] = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            zp[v] = T(0);
            fz[v] = T(0);
        }

        // Plane k+2 is fetched into registers at the top of step k and written
        // to the ring after B3, into the slot of plane k-1, which step k no
        // longer reads by then.  Consuming it there, before the update's stores
        // are issued, keeps the wait for the loads from also waiting out those
        // stores (memory operations complete in issue order).
        for (int k = -1; k <= nplanes; ++k) {
            // plane k of the unit is plane kl of its group gk (k in 0 .. nplanes-1;
            // with padded input, the group itself and k)
            const int kq = PERIODIC ? k >> 4 : 0, kl = PERIODIC ? k & 15 : k;
            const int64_t gk = PERIODIC ? g + int64_t(kq) * cols : g;
            const bool ahead = k + 2 <= nplanes + 1;
            if (ahead) fetch(k + 2);
            __syncthreads();  // B1: plane k+1 visible; planes k-1, k, k+1 in the ring

            const bool edge = (k < 0 || k >= nplanes);
            if constexpr (PERIODIC) step = 0;
            // ghost-layer cell of this thread in this plane (-1: none)
            const int ring = edge ? -1 : (SPLIT ? my_ring : (wave == (k & 3) ? my_ring : -1));

            // ---- face states: the interior cell, then the ghost-layer cell ----
            // (one code path for both, so a face state is computed identically
            // wherever its cell sits)
            T xm[NV], ym[NV], zm[NV], zpn[NV];
            const T(*wm)[NPL] = S.w[(k + 2) % 3];
            const T(*w0)[NPL] = S.w[(k + 3) % 3];
            const T(*wq)[NPL] = S.w[(k + 4) % 3];
#pragma unroll
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
                    if constexpr (PERIODIC)
                        step |= round == 0 ? 1 : 2;
                    else
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
                        case 1:  // -x state of face 16
#pragma unroll
                            for (int v = 0; v < NV; ++v) S.rf[0][v][cj] = Ub[0][0][v];
                            break;
                        case 2:  // +y state of face 0
#pragma unroll
                            for (int v = 0; v < NV; ++v) S.sy[v][0][ci] = Ub[1][1][v];
                            break;
                        default:  // -y state of face 16
#pragma unroll
                            for (int v = 0; v < NV; ++v) S.rf[1][v][ci] = Ub[1][0][v];
                            break;
                    }
                }
            }

            // z face between planes k-1 and k (registers only).  A wave that
            // computed ghost-layer cells in this plane solves it after the x and
            // y faces instead, while the two waves that take the faces 16 are
            // busy with them, so that no wave does more than one cell and three
            // Roe solves between two barriers.
            T fzn[NV];
            auto solve_z = [&]() {
                if (inner && k >= 0) {
                    const bool fb = roe_dir<2, true>(zp, zm, c, fzn);
                    if constexpr (PERIODIC)
                        step |= int(fb) << 2;
                    else
                        n_roe += fb;
                    if (P.flux) {
                        const int off = jj * NI + ii;
                        if constexpr (PERIODIC) {
                            // face kl of group gk (below the unit's last plane), and face 16
                            // of the group below when the face lies on a group boundary
                            if (k < nplanes && (kl & 7) == 0) {
                                S_ *dst = P.flux + gk * GFLX + ((2 * 3 + (kl >> 3)) * NV) * NINNER + off;
#pragma unroll
                                for (int v = 0; v < NV; ++v) dst[v * NINNER] = S_(c.half * fzn[v]);
                            }
                            if (kl == 0 && k > 0) {
                                S_ *dst = P.flux + (gk - cols) * GFLX + ((2 * 3 + 2) * NV) * NINNER + off;
#pragma unroll
                                for (int v = 0; v < NV; ++v) dst[v * NINNER] = S_(c.half * fzn[v]);
                            }
                        } else if ((k & 7) == 0) {
                            S_ *dst = P.flux + g * GFLX + ((2 * 3 + (k >> 3)) * NV) * NINNER + off;
#pragma unroll
                            for (int v = 0; v < NV; ++v) dst[v * NINNER] = S_(c.half * fzn[v]);
                        }
                    }
                }
            };
            const bool late_z = !SPLIT && ring >= 0;
            if (!late_z) solve_z();
            __syncthreads();  // B2: +x / +y states and the right states of faces 16 visible

            // faces 16: x by wave k+1 mod 4 and y by wave k+2 mod 4 (320 threads:
            // both by the ghost-layer wave), lanes 0..15
            const int lane = t & 63;
            const bool x16 = lane < NI && (SPLIT ? wave == 4 : wave == ((k + 1) & 3));
            const bool y16 = lane < NI && (SPLIT ? wave == 4 : wave == ((k + 2) & 3));

            if (!edge) {
                // x faces: face ci of each interior cell, then face 16 of each row
#pragma unroll
                for (int round = 0; round < 2; ++round) {
                    int row, f;
                    if (round == 0) {
                        if (!inner) continue;
                        row = jj;
                        f = ii;
                    } else {
                        if (!x16) continue;
                        row = lane;
                        f = NI;
                    }
                    T UL[NV], UR[NV], F[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        UL[v] = S.sx[v][row][f];
                        UR[v] = round == 0 ? xm[v] : S.rf[0][v][row];
                    }
                    const bool fb = roe_dir<0, true>(UL, UR, c, F);
                    if constexpr (PERIODIC)
                        step += int(fb) << 3;
                    else
                        n_roe += fb;
#pragma unroll
                    for (int v = 0; v < NV; ++v) S.sx[v][row][f] = F[v];
                    if (P.flux && (f & 7) == 0) {
                        S_ *dst = P.flux + gk * GFLX + ((0 * 3 + (f >> 3)) * NV) * NINNER + kl * NI + row;
#pragma unroll
                        for (int v = 0; v < NV; ++v) dst[v * NINNER] = S_(c.half * F[v]);
                    }
                }
                // y faces: face cj of each interior cell, then face 16 of each column
#pragma unroll
                for (int round = 0; round < 2; ++round) {
                    int col, f;
                    if (round == 0) {
                        if (!inner) continue;
                        col = ii;
                        f = jj;
                    } else {
                        if (!y16) continue;
                        col = lane;
                        f = NI;
                    }
                    T UL[NV], UR[NV], F[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        UL[v] = S.sy[v][f][col];
                        UR[v] = round == 0 ? ym[v] : S.rf[1][v][col];
                    }
                    const bool fb = roe_dir<1, true>(UL, UR, c, F);
                    if constexpr (PERIODIC)
                        step += int(fb) << 3;
                    else
                        n_roe += fb;
#pragma unroll
                    for (int v = 0; v < NV; ++v) S.sy[v][f][col] = F[v];
                    if (P.flux && (f & 7) == 0) {
                        S_ *dst = P.flux + gk * GFLX + ((1 * 3 + (f >> 3)) * NV) * NINNER + kl * NI + col;
#pragma unroll
                        for (int v = 0; v < NV; ++v) dst[v * NINNER] = S_(c.half * F[v]);
                    }
                }
            }
            if (late_z) solve_z();
            // The old state of plane k-1 for its update below, all five values
            // loaded before any of the update's stores (the compiler cannot prove
            // the arrays distinct, and would otherwise wait out a store before
            // each load).  With float arithmetic, where registers allow, the loads
            // are issued before the barrier, so their latency overlaps the wait.
            constexpr bool EARLY = sizeof(T) == 4;
            S_ uold[NV];
            // plane k-1 of the unit: plane ul of group gu
            const int ul = PERIODIC ? (k - 1) & 15 : k - 1;
            const int64_t gu = PERIODIC ? g + int64_t((k - 1) >> 4) * cols : g;
            auto load_old = [&]() {
                // an interior cell: in the group's own block in both input kinds
                const S_ *src = PERIODIC ? P.in + gu * GOUT + ul * NINNER
                                         : P.in + g * GIN + (k - 1 + NG) * NPL + NG * NP + NG;
                const unsigned off = PERIODIC ? unsigned(t) : unsigned(jj * NP + ii);
#pragma unroll
                for (int v = 0; v < NV; ++v) uold[v] = at(src + v * VSTRIDE, off);
            };
            if (EARLY && inner && k >= 1) load_old();
            __syncthreads();  // B3: x / y fluxes visible; plane k-1 no longer read
            if (ahead) store(k + 2);

            if (inner) {
                if (k >= 1) {
                    // plane k-1 is complete: U - dt/dh ((dF_x + dF_y) + dF_z)
                    S_ *dst = P.out + gu * GOUT + ul * NINNER;
                    if (!EARLY) load_old();
                    T un[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const double dfz = double(fzn[v]) - double(fz[v]);
                        const double r = double(uold[v]) - hdtdh * (S.dxy[v][t] + dfz);
                        const S_ o = S_(r);
                        at(dst + v * NI * NINNER, unsigned(t)) = o;
                        un[v] = T(o);
                        st[v] += double(o);
                    }
                    const double sp = double(signal_speed(un[0], un[1], un[2], un[3], un[4], c));
                    n_bad += sp != sp;
                    st[5] = max_nan(st[5], sp);
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

            if constexpr (PERIODIC) {
                // this step's fallbacks to the groups they belong to (see `step`)
                const int pi = step & 1, pr = (step >> 1) & 1, rz = (step >> 2) & 1, rxy = step >> 3;
                if (k < 0) {
                    n_pred += pi;  // the first group's ghost plane -1
                } else if (k == nplanes) {
                    n_pred += pi;  // the last group's ghost plane 16 and face 16
                    n_roe += rz;
                } else if (kl == 0 && k > 0) {
                    n_pred += pi;  // group kq - 1: ghost plane 16, face 16
                    n_roe += rz;
                    carry += (pi + pr) + ((rz + rxy) << 16);  // group kq: plane 0, face 0
                } else {
                    n_pred += pi + pr;
                    n_roe += rz + rxy;
                    if (kl == 15 && k < nplanes - 1) carry += pi;  // group kq + 1's ghost plane -1
                }
                // Group kq - 1 is complete at a boundary inside the unit: its stats
                // go out now (the unit's last group after the sweep).  The flux
                // arrays are free until the next step's predictions; they hold the
                // reduction's values once every thread has read this step's fluxes.
                if (kl == 0 && k > 0 && k < nplanes) {
                    if (P.stats) {
                        __syncthreads();
                        double all[NSTAT] = {st[0], st[1], st[2], st[3], st[4], st[5], double(n_pred),
                                             double(n_roe)};
                        block_reduce_stats<NT, FLUSH_PART<T>>(all, reinterpret_cast<double *>(&S.sx[0][0][0]),
                                                              P.stats + (gk - cols) * NSTAT);
                    }
                    n_pred = carry & 0xffff;
                    n_roe = carry >> 16;
                    carry = 0;
#pragma unroll
                    for (int q = 0; q < 6; ++q) st[q] = 0.0;
                }
            }
        }

        if (P.bad && n_bad) atomicAdd(P.bad, (unsigned long long)n_bad);
        if (P.stats) {
            double all[NSTAT] = {st[0], st[1], st[2], st[3], st[4], st[5], double(n_pred),
                                 double(n_roe)};
            // S.w is free now (B3 of the last step passed); reuse it for the reduction
            block_reduce_stats<NT>(all, reinterpret_cast<double *>(&S.w[0][0][0]),
                                   P.stats + (g + int64_t(nseg - 1) * cols) * NSTAT);
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
    // work units: groups, or z segments of the columns of a periodic grid
    int64_t units = p.n_groups;
    if (p.gx > 0) {
        if (p.zseg < 1 || p.zseg > p.gz) return hipErrorInvalidValue;
        units = int64_t(p.gx) * p.gy * ((p.gz + p.zseg - 1) / p.zseg);
    }
    const int64_t max_grid = int64_t(1) << 30;
    int64_t g = grid > 0 ? (grid < units ? grid : units) : units;
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
