"""Multi-step drivers around the CPU oracle (test helper).

Periodic uniform grids held as groups: ghost fill with the oracle's own pack,
one oracle step, time step from the oracle's CFL function.
"""
import numpy as np

import oracle


def run_periodic(state, gx, gy, gz, dh, gamma, cfl=0.5, steps=None, t_end=None, theta=oracle.THETA):
    """Advance ``state`` (G,5,16,16,16) float64.  Returns (state, t, n_steps, counts)."""
    s = np.ascontiguousarray(state, dtype=np.float64)
    t, n = 0.0, 0
    counts = [0, 0]
    while True:
        if steps is not None and n >= steps:
            break
        if t_end is not None and t >= t_end * (1 - 1e-14):
            break
        dt = oracle.cfl_dt(s, dh, gamma, cfl)
        if t_end is not None:
            dt = min(dt, t_end - t)
        s, c = oracle.step_periodic(s, gx, gy, gz, dt, dh, gamma, theta)
        counts[0] += c[0]
        counts[1] += c[1]
        t += dt
        n += 1
    return s, t, n, tuple(counts)


def to_global(groups, gx, gy, gz):
    """(G,5,16,16,16) -> (5, NZ, NY, NX) numpy."""
    g = np.asarray(groups).reshape(gz, gy, gx, 5, 16, 16, 16)
    return g.transpose(3, 0, 4, 1, 5, 2, 6).reshape(5, gz * 16, gy * 16, gx * 16)


def from_global(field, gx, gy, gz):
    f = np.asarray(field).reshape(5, gz, 16, gy, 16, gx, 16)
    return np.ascontiguousarray(f.transpose(1, 3, 5, 0, 2, 4, 6).reshape(gx * gy * gz, 5, 16, 16, 16))


# ------------------------------------------------------------------ two levels

def fine_global(coarse, gx, gy, gz, fine, parent):
    """The fine-resolution field (5, 32 gz, 32 gy, 32 gx): every coarse cell
    injected into its 2 x 2 x 2 children, then the fine groups laid over it."""
    c = to_global(coarse, gx, gy, gz)
    f = c.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)
    for n, code in enumerate(np.asarray(parent)):
        g, o = divmod(int(code), 8)
        bx, by, bz = g % gx, (g // gx) % gy, g // (gx * gy)
        x0, y0, z0 = 32 * bx + 16 * (o & 1), 32 * by + 16 * ((o >> 1) & 1), 32 * bz + 16 * ((o >> 2) & 1)
        f[:, z0:z0 + 16, y0:y0 + 16, x0:x0 + 16] = fine[n]
    return f


def fine_padded(coarse, gx, gy, gz, fine, parent):
    """Padded fine groups (n, 5, 20, 20, 20): ghost cells from neighbouring fine
    groups where they exist, else from the injected coarse field (periodic)."""
    f = fine_global(coarse, gx, gy, gz, fine, parent)
    out = np.empty((len(parent), 5, 20, 20, 20))
    for n, code in enumerate(np.asarray(parent)):
        g, o = divmod(int(code), 8)
        bx, by, bz = g % gx, (g // gx) % gy, g // (gx * gy)
        x0, y0, z0 = 32 * bx + 16 * (o & 1), 32 * by + 16 * ((o >> 1) & 1), 32 * bz + 16 * ((o >> 2) & 1)
        ix = np.arange(x0 - 2, x0 + 18) % f.shape[3]
        iy = np.arange(y0 - 2, y0 + 18) % f.shape[2]
        iz = np.arange(z0 - 2, z0 + 18) % f.shape[1]
        out[n] = f[:, iz][:, :, iy][:, :, :, ix]
    return out


def two_level_step(coarse, gx, gy, gz, fine, parent, faces, dt_c, dh_c, gamma, correct=True):
    """One coarse step and two fine sub-steps of dt_c / 2, then flux correction
    (unless ``correct`` is False) and restriction.  Fine ghost cells that fall on
    the coarse level come from the coarse state at the sub-step's start time
    (linear in time between the old and new coarse states).
    Returns (coarse, fine, coarse fluxes, summed fine fluxes)."""
    from oracle import amr
    coarse = np.asarray(coarse, dtype=np.float64)
    c_new, c_fl, _ = oracle.hydro_solve(oracle.pack_periodic(coarse, gx, gy, gz), dt_c, dh_c, gamma,
                                        want_fluxes=True)
    f = np.asarray(fine, dtype=np.float64)
    acc = None
    for s in (0, 1):
        c_t = coarse if s == 0 else 0.5 * (coarse + c_new)
        f, f_fl, _ = oracle.hydro_solve(fine_padded(c_t, gx, gy, gz, f, parent), 0.5 * dt_c,
                                        0.5 * dh_c, gamma, want_fluxes=True)
        acc = amr.flux_accumulate(acc, f_fl, 0.5 * dt_c)
    if correct:
        c_new = amr.flux_correct(c_new, c_fl, acc, faces, dt_c, dh_c)
    c_new = amr.restrict(c_new, f, parent)
    return c_new, f, c_fl, acc
