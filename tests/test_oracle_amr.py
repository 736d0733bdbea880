"""Pins of the AMR oracle (restriction, flux accumulation, flux correction)
against what the mathematics fixes -- CPU only.

  * restriction of a linear field gives the field at the coarse cell centre;
    it preserves totals; it leaves uncovered cells bitwise alone;
  * the face records of a refined set tile exactly the coarse/fine faces found
    by a brute-force neighbour test on the covered-cell mask;
  * a two-level step (coarse step, two fine sub-steps, correction,
    restriction) conserves all five totals on a periodic grid to rounding,
    and does not without the correction;
  * every corrected coarse cell equals a flux-form update written out from
    every face flux of both levels in global coordinates (the stage functions
    of the main oracle), with the fine fluxes over each coarse/fine face summed
    in time and averaged in area: an independent route to the same numbers,
    which catches a wrong cell, quarter, plane, orientation or sign.
"""
import numpy as np
import pytest

import oracle
from oracle import amr as oamr
from oracle_driver import fine_global, fine_padded, to_global, two_level_step
from paper_1007_3818_amd import amr, workloads as W

G53 = 5.0 / 3.0


def code(px, py, pz, gx, gy):
    return ((px // 2) + gx * ((py // 2) + gy * (pz // 2))) * 8 + (px % 2) + 2 * (py % 2) + 4 * (pz % 2)


# refined patches (patch coordinates of a 4 x 4 x 4-patch grid): an L-shaped
# set with a concave corner, crossing group boundaries, and one patch on the
# periodic wrap
PATCHES_2 = [(1, 1, 1), (2, 1, 1), (1, 2, 1), (1, 1, 2), (3, 2, 1), (0, 3, 3)]


def fine_origins(parent, gx, gy):
    """Fine-cell coordinates (x0, y0, z0) of each fine group's first cell."""
    out = []
    for c in parent:
        g, o = divmod(int(c), 8)
        bx, by, bz = g % gx, (g // gx) % gy, g // (gx * gy)
        out.append((32 * bx + 16 * (o & 1), 32 * by + 16 * ((o >> 1) & 1), 32 * bz + 16 * ((o >> 2) & 1)))
    return out


def inject(coarse, gx, gy, gz, parent):
    """Fine groups holding the coarse state copied into each child cell."""
    fg = fine_global(coarse, gx, gy, gz, np.zeros((0, 5, 16, 16, 16)), [])
    return np.stack([fg[:, z0:z0 + 16, y0:y0 + 16, x0:x0 + 16] for x0, y0, z0 in fine_origins(parent, gx, gy)])


def mask_global(m, gx, gy, gz):
    return to_global(np.repeat(m[:, None], 5, axis=1), gx, gy, gz)[0]


def patch_list(coords, gx, gy):
    return [divmod(code(px, py, pz, gx, gy), 8) for px, py, pz in coords]


def test_restrict_linear_and_sums():
    r = np.random.default_rng(1)
    gx = gy = gz = 2
    coarse = r.standard_normal((8, 5, 16, 16, 16))
    parent, _ = amr.refine(gx, gy, gz, patch_list(PATCHES_2, gx, gy))
    # fine field linear in the fine cell centres -> coarse centre values
    a = r.standard_normal((5, 4))
    fine = np.empty((len(parent), 5, 16, 16, 16))
    k, j, i = np.meshgrid(np.arange(16), np.arange(16), np.arange(16), indexing="ij")
    expect = coarse.copy()
    for n, c in enumerate(parent):
        g, o = divmod(int(c), 8)
        bx, by, bz = g % gx, (g // gx) % gy, g // (gx * gy)
        X = 32 * bx + 16 * (o & 1) + i + 0.5  # fine-cell centres, fine units
        Y = 32 * by + 16 * ((o >> 1) & 1) + j + 0.5
        Z = 32 * bz + 16 * ((o >> 2) & 1) + k + 0.5
        for v in range(5):
            fine[n, v] = a[v, 0] + a[v, 1] * X + a[v, 2] * Y + a[v, 3] * Z
        kc, jc, ic = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
        Xc = 2 * (16 * bx + 8 * (o & 1) + ic + 0.5)  # coarse centres, fine units
        Yc = 2 * (16 * by + 8 * ((o >> 1) & 1) + jc + 0.5)
        Zc = 2 * (16 * bz + 8 * ((o >> 2) & 1) + kc + 0.5)
        ox, oy, oz = o & 1, (o >> 1) & 1, (o >> 2) & 1
        for v in range(5):
            expect[g, v, 8 * oz:8 * oz + 8, 8 * oy:8 * oy + 8, 8 * ox:8 * ox + 8] = (
                a[v, 0] + a[v, 1] * Xc + a[v, 2] * Yc + a[v, 3] * Zc)
    out = oamr.restrict(coarse, fine, parent)
    np.testing.assert_allclose(out, expect, rtol=0, atol=1e-12)
    cov = amr.covered_mask(gx, gy, gz, parent)
    for v in range(5):
        cv = out[:, v]
        assert np.array_equal(cv[~cov], coarse[:, v][~cov])
        assert np.isclose(8 * np.sum(cv[cov]), np.sum(fine[:, v]), rtol=1e-13, atol=1e-9)


@pytest.mark.parametrize("g", [1, 2])
def test_face_records_tile_the_interface(g):
    """Each record's 64 coarse cells, expanded, are exactly the uncovered cells
    with a covered neighbour along that direction (brute force on the mask)."""
    gx = gy = gz = g
    coords = PATCHES_2 if g == 2 else [(0, 1, 1)]
    parent, faces = amr.refine(gx, gy, gz, patch_list(coords, gx, gy))
    cov = mask_global(amr.covered_mask(gx, gy, gz, parent), gx, gy, gz)  # (Z, Y, X)
    for d in range(3):
        axis = 2 - d
        below = np.zeros_like(cov)  # uncovered cells whose +d neighbour is covered
        above = np.zeros_like(cov)
        below |= ~cov & np.roll(cov, -1, axis=axis)
        above |= ~cov & np.roll(cov, 1, axis=axis)
        got_b = np.zeros_like(cov)
        got_a = np.zeros_like(cov)
        for r in faces[faces["dir"] == d]:
            gi, cf, side = int(r["coarse_group"]), int(r["coarse_face"]), int(r["side"])
            bx, by, bz = gi % gx, (gi // gx) % gy, gi // (gx * gy)
            n = 8 * cf - 1 + side
            s0, f0 = 8 * int(r["qs"]), 8 * int(r["qf"])
            tgt = got_b if side == 0 else got_a
            lo = [16 * bz, 16 * by, 16 * bx]  # Z, Y, X origins
            sl = [None, None, None]
            sl[axis] = slice(lo[axis] + n, lo[axis] + n + 1)
            slow_ax, fast_ax = {0: (0, 1), 1: (0, 2), 2: (1, 2)}[d]
            sl[slow_ax] = slice(lo[slow_ax] + s0, lo[slow_ax] + s0 + 8)
            sl[fast_ax] = slice(lo[fast_ax] + f0, lo[fast_ax] + f0 + 8)
            assert not tgt[tuple(sl)].any(), "a cell is listed twice"
            tgt[tuple(sl)] = True
            # the fine group sits across the face
            fg = int(r["fine_group"])
            assert 0 <= fg < len(parent)
        assert np.array_equal(got_b, below), d
        assert np.array_equal(got_a, above), d


def _state(g):
    st, dh = W.smooth_modes(n=16 * g, kmax=2, workload=2)
    return st.numpy(), dh


@pytest.mark.parametrize("g", [1, 2])
def test_two_level_step_conserves(g):
    gx = gy = gz = g
    coords = PATCHES_2 if g == 2 else [(0, 1, 1)]
    coarse, dh = _state(g)
    parent, faces = amr.refine(gx, gy, gz, patch_list(coords, gx, gy))
    fine = inject(coarse, gx, gy, gz, parent)
    # the initial fine state is the injected coarse state: composite totals agree
    assert np.allclose(oamr.restrict(coarse, fine, parent), coarse, rtol=4e-16, atol=0)
    dt = 0.4 * oracle.cfl_dt(coarse, dh, G53, 1.0)
    before = coarse.sum(axis=(0, 2, 3, 4))
    scale = np.abs(coarse).sum(axis=(0, 2, 3, 4))
    c1, _, _, _ = two_level_step(coarse, gx, gy, gz, fine, parent, faces, dt, dh, G53)
    err = np.abs(c1.sum(axis=(0, 2, 3, 4)) - before) / scale
    assert np.all(err < 1e-14), err
    c0, _, _, _ = two_level_step(coarse, gx, gy, gz, fine, parent, faces, dt, dh, G53, correct=False)
    err0 = np.abs(c0.sum(axis=(0, 2, 3, 4)) - before) / scale
    assert err0.max() > 1e-9, err0  # the correction matters


def _full_face_fluxes(padded, dt, dh):
    """Every face flux of every group, from the oracle's stage functions:
    list of (3, 5, 17, 16, 16) arrays."""
    out = []
    for U in padded:
        Wp = oracle.group_prim(U, G53)
        dW = oracle.group_slopes(Wp)
        Ub, _ = oracle.group_predict(U, Wp, dW, dt, dh, G53)
        Fl, _ = oracle.group_fluxes(Ub, G53)
        out.append(Fl)
    return out


def _global_faces(fl_list, origins, shape):
    """Scatter per-group face fluxes into global per-direction face arrays
    (5, Z, Y, X); face index X along x lies between cells X-1 and X."""
    NZ, NY, NX = shape
    G = [np.full((5, NZ, NY, NX), np.nan) for _ in range(3)]
    f = np.arange(17)
    t = np.arange(16)
    for Fl, (x0, y0, z0) in zip(fl_list, origins):
        # x faces: Fl[0][v][f][k][j]
        X = (x0 + f) % NX
        Y = (y0 + t) % NY
        Z = (z0 + t) % NZ
        G[0][:, Z[None, :, None], Y[None, None, :], X[:, None, None]] = Fl[0]
        # y faces: Fl[1][v][f][k][i]
        G[1][:, Z[None, :, None], ((y0 + f) % NY)[:, None, None], ((x0 + t) % NX)[None, None, :]] = Fl[1]
        # z faces: Fl[2][v][f][j][i]
        G[2][:, ((z0 + f) % NZ)[:, None, None], Y[None, :, None], ((x0 + t) % NX)[None, None, :]] = Fl[2]
    return G


def test_corrected_cells_match_flux_form_update():
    gx = gy = gz = 2
    coarse, dh = _state(2)
    parent, faces = amr.refine(gx, gy, gz, patch_list(PATCHES_2, gx, gy))
    r = np.random.default_rng(7)
    # a fine state that differs from the injected coarse one (so the two levels'
    # fluxes differ at every coarse/fine face)
    fine = inject(coarse, gx, gy, gz, parent)
    fine[:, 0] *= 1 + 0.02 * r.random(fine[:, 0].shape)
    fine[:, 4] *= 1 + 0.02 * r.random(fine[:, 4].shape)
    origins = fine_origins(parent, gx, gy)
    dt = 0.4 * oracle.cfl_dt(coarse, dh, G53, 1.0)
    c_new, f_new, c_fl, acc = two_level_step(coarse, gx, gy, gz, fine, parent, faces, dt, dh, G53)

    # coarse faces at every position, and the new coarse state without correction
    cpad = oracle.pack_periodic(coarse, gx, gy, gz)
    cfaces = _global_faces(_full_face_fluxes(cpad, dt, dh),
                           [(16 * (g % gx), 16 * ((g // gx) % gy), 16 * (g // (gx * gy))) for g in range(8)],
                           (32, 32, 32))
    # fine faces of both sub-steps, time-weighted
    ffaces = [np.zeros((5, 64, 64, 64)) for _ in range(3)]
    f = fine
    for s in (0, 1):
        c_t = coarse if s == 0 else 0.5 * (coarse + oracle.hydro_solve(cpad, dt, dh, G53)[0])
        fp = fine_padded(c_t, gx, gy, gz, f, parent)
        gl = _global_faces(_full_face_fluxes(fp, 0.5 * dt, 0.5 * dh), origins, (64, 64, 64))
        for d in range(3):
            ffaces[d] += 0.5 * dt * np.nan_to_num(gl[d], nan=0.0)
        f = oracle.hydro_solve(fp, 0.5 * dt, 0.5 * dh, G53)[0]

    cov = mask_global(amr.covered_mask(gx, gy, gz, parent), gx, gy, gz)
    U0 = to_global(coarse, gx, gy, gz)
    U1 = to_global(c_new, gx, gy, gz)
    scale = np.abs(U0).max(axis=(1, 2, 3))
    n_checked = 0
    for Z in range(32):
        for Y in range(32):
            for X in range(32):
                if cov[Z, Y, X]:
                    continue
                total = np.zeros(5)
                touches = False
                for d, (ex, ey, ez) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
                    for sgn, (fx, fy, fz, nx, ny, nz) in (
                            (-1, (X, Y, Z, X - ex, Y - ey, Z - ez)),
                            (+1, (X + ex, Y + ey, Z + ez, X + ex, Y + ey, Z + ez))):
                        fx, fy, fz = fx % 32, fy % 32, fz % 32
                        if cov[nz % 32, ny % 32, nx % 32]:
                            touches = True
                            xs = [2 * fx] if d == 0 else [2 * fx, 2 * fx + 1]
                            ys = [2 * fy] if d == 1 else [2 * fy, 2 * fy + 1]
                            zs = [2 * fz] if d == 2 else [2 * fz, 2 * fz + 1]
                            phi = sum(ffaces[d][:, z, y, x] for z in zs for y in ys for x in xs) / 4.0
                        else:
                            phi = dt * cfaces[d][:, fz, fy, fx]
                        total += sgn * phi
                if not touches:
                    continue
                n_checked += 1
                want = U0[:, Z, Y, X] - total / dh
                assert np.all(np.abs(U1[:, Z, Y, X] - want) <= 1e-13 * scale), (X, Y, Z)
    assert n_checked > 500
