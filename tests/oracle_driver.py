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
