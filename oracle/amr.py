"""FP64 CPU oracle for the two steps that follow the solver in an AMR step --
TEST INFRASTRUCTURE (only tests/, the smoke check and the benchmark's CPU leg
may use it; it shares no code with the HIP library).

The paper's Sec. 1 builds on GAMER (Schive et al. 2010), an AMR code whose
levels are advanced with the solver and then made consistent:

  * restriction: a coarse cell covered by fine cells takes their volume
    average, U_C = (1/8) sum of its 2 x 2 x 2 children;
  * flux correction (conservative refluxing, Berger & Colella 1989): an
    unrefined coarse cell next to a coarse/fine face was updated with the
    coarse flux F_C over that face, dt_C * F_C / dh_C; it must instead use the
    fine fluxes over the same face, summed over the fine sub-steps s and
    averaged over the 2 x 2 fine faces that tile the coarse face:
        Phi = sum_s dt_s * (1/4) sum_{faces} F_f,s,
    so the cell below the face gains (dt_C F_C - Phi) / dh_C and the cell
    above it loses the same amount.

Everything is the plain definition in numpy float64; corrections are applied
record by record, x faces first, then y, then z.

Array layouts as in the main oracle: interior groups (n, 5, 16, 16, 16) with
index order [v][k][j][i]; flux planes (n, 3 dir, 3 plane, 5, 16, 16) with
planes at faces 0, 8, 16 and transverse (slow, fast) = (k, j) for x, (k, i)
for y, (j, i) for z.  Face records: the 24-byte layout described by fields
coarse_group, fine_group, dir, coarse_face (0, 1, 2: face 0, 8, 16 of the
coarse group along dir), side (0: the coarse cells lie below the face, the fine
group's face 0 covers it; 1: above, the fine group's face 16), qs, qf (which
8 x 8 quarter of the coarse plane, slow and fast).

Parity pins (tests/test_oracle_amr.py): restriction of linear fields and of
sums; a coarse/fine face in uniform flow changes nothing; and conservation of
all five totals through a two-level step (coarse step, two fine sub-steps,
correction, restriction) on periodic grids, which fails when the correction is
left out.
"""
import numpy as np


def restrict(coarse, fine, parent):
    """Copy of ``coarse`` whose cells covered by fine groups hold the mean of
    their 8 children.  parent[f] = coarse_group * 8 + octant (ox + 2 oy + 4 oz)."""
    out = np.array(coarse, dtype=np.float64, copy=True)
    fine = np.asarray(fine, dtype=np.float64)
    for f, code in enumerate(np.asarray(parent)):
        g, o = divmod(int(code), 8)
        ox, oy, oz = o & 1, (o >> 1) & 1, (o >> 2) & 1
        blk = np.zeros((5, 8, 8, 8))
        for a in (0, 1):
            for b in (0, 1):
                for c in (0, 1):
                    blk += fine[f][:, c::2, b::2, a::2]
        out[g, :, 8 * oz:8 * oz + 8, 8 * oy:8 * oy + 8, 8 * ox:8 * ox + 8] = blk / 8.0
    return out


def flux_accumulate(acc, fluxes, dt):
    """acc + dt * fluxes (acc None: zero), float64."""
    add = dt * np.asarray(fluxes, dtype=np.float64)
    return add if acc is None else np.asarray(acc, dtype=np.float64) + add


def flux_correct(coarse, coarse_fluxes, fine_acc, faces, dt_c, dh_c):
    """Copy of ``coarse`` with every face record's correction applied.
    ``fine_acc``: the fine groups' flux planes summed over sub-steps with their
    dt (flux_accumulate)."""
    out = np.array(coarse, dtype=np.float64, copy=True)
    cfl = np.asarray(coarse_fluxes, dtype=np.float64)
    acc = np.asarray(fine_acc, dtype=np.float64)
    for d in (0, 1, 2):
        for r in faces:
            if int(r["dir"]) != d:
                continue
            g, f = int(r["coarse_group"]), int(r["fine_group"])
            cf, side = int(r["coarse_face"]), int(r["side"])
            s0, f0 = 8 * int(r["qs"]), 8 * int(r["qf"])
            n = 8 * cf - 1 + side  # the coarse cells' index along d
            Fc = cfl[g, d, cf][:, s0:s0 + 8, f0:f0 + 8]
            Ff = acc[f, d, 2 * side]
            phi = (Ff[:, 0::2, 0::2] + Ff[:, 0::2, 1::2] + Ff[:, 1::2, 0::2] + Ff[:, 1::2, 1::2]) / 4.0
            delta = (dt_c * Fc - phi) / dh_c
            if side == 1:
                delta = -delta
            if d == 0:
                out[g, :, s0:s0 + 8, f0:f0 + 8, n] += delta
            elif d == 1:
                out[g, :, s0:s0 + 8, n, f0:f0 + 8] += delta
            else:
                out[g, :, n, s0:s0 + 8, f0:f0 + 8] += delta
    return out
