"""Coarse/fine flux correction, flux accumulation and restriction on the GPU,
through the C ABI, against the AMR oracle.

Tolerances: FP64 1e-12 per cell (rho and E against the cell's own value, momenta against |m| + rho c_s);
FP32 1e-6
for the single kernels (one rounding per stored value), and for the whole
two-level step FP32 within 1e-5 in L1 per variable.  The invalid-record
counts are exact.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import amr as oamr
from oracle_driver import two_level_step
from paper_1007_3818_amd import amr, hydro, workloads as W
from parity import state_close

pytestmark = pytest.mark.gpu
G53 = 5.0 / 3.0

PATCHES = [(1, 1, 1), (2, 1, 1), (1, 2, 1), (1, 1, 2), (3, 2, 1), (0, 3, 3)]


def layout(gx=2, gy=2, gz=2, coords=PATCHES):
    pl = []
    for px, py, pz in coords:
        g = (px // 2) + gx * ((py // 2) + gy * (pz // 2))
        pl.append((g, (px % 2) + 2 * (py % 2) + 4 * (pz % 2)))
    return amr.refine(gx, gy, gz, pl)


def dev1(x, gpu):
    return torch.tensor([x], dtype=torch.float64, device=gpu)


def phys(r, n):
    """Random physical conserved states, independent per cell: rho and p
    log-normal, velocities standard normal (a restriction test needs states,
    not arbitrary numbers, for the per-cell comparison to mean anything)."""
    shp = (n, 16, 16, 16)
    rho = np.exp(0.5 * r.standard_normal(shp))
    u = r.standard_normal((3,) + shp)
    p = np.exp(0.5 * r.standard_normal(shp))
    m = rho * u
    E = p / (G53 - 1.0) + 0.5 * rho * (u ** 2).sum(axis=0)
    return torch.from_numpy(np.stack([rho, m[0], m[1], m[2], E], axis=1))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_flux_accumulate(gpu, dtype):
    r = np.random.default_rng(2)
    F1 = torch.from_numpy(r.standard_normal((7, 3, 3, 5, 16, 16))).to(dtype)
    F2 = torch.from_numpy(r.standard_normal((7, 3, 3, 5, 16, 16))).to(dtype)
    acc = hydro.flux_accumulate(F1.to(gpu), dev1(0.3, gpu))
    acc = hydro.flux_accumulate(F2.to(gpu), dev1(0.7, gpu), acc=acc)
    want = oamr.flux_accumulate(oamr.flux_accumulate(None, F1.double().numpy(), 0.3), F2.double().numpy(), 0.7)
    np.testing.assert_allclose(acc.cpu().numpy(), want, rtol=1e-15, atol=1e-15)
    acc = hydro.flux_accumulate(F2.to(gpu), dev1(0.5, gpu), acc=acc, reset=True)
    np.testing.assert_allclose(acc.cpu().numpy(), 0.5 * F2.double().numpy(), rtol=1e-15, atol=0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_restrict(gpu, dtype):
    r = np.random.default_rng(3)
    parent, _ = layout()
    coarse = phys(r, 8).to(dtype)
    fine = phys(r, len(parent)).to(dtype)
    want = oamr.restrict(coarse.double().numpy(), fine.double().numpy(), parent)
    c = coarse.to(gpu)
    bad = torch.zeros(1, dtype=torch.int32, device=gpu)
    hydro.restrict(fine.to(gpu), torch.from_numpy(parent).to(gpu), c, n_bad=bad)
    got = c.cpu().double().numpy()
    # The mean of eight children summed in another order differs by at most
    # 7u times the mean of |child| (u = 2^-53); for the positive rho and E that
    # is <= 7.8e-16 of the cell's value, and the momenta's mean |child| stays
    # within a few times |m| + rho c_s for these states.  FP32 adds one float
    # rounding of the double mean (6e-8).
    if dtype == torch.float64:
        state_close(got, want, 1e-14, "restrict fp64")
    else:
        state_close(got, want, 1e-7, "restrict fp32")
    cov = amr.covered_mask(2, 2, 2, parent)
    for v in range(5):
        assert np.array_equal(got[:, v][~cov], coarse[:, v].double().numpy()[~cov])
    assert int(bad.item()) == 0


def test_restrict_skips_and_counts_bad_parents(gpu):
    r = np.random.default_rng(4)
    coarse = phys(r, 2).to(gpu)
    before = coarse.clone()
    fine = phys(r, 3).to(gpu)
    parent = torch.tensor([-1, 2 * 8 + 3, 1 * 8 + 7], dtype=torch.int64, device=gpu)  # skip, bad, good
    bad = torch.zeros(1, dtype=torch.int32, device=gpu)
    hydro.restrict(fine, parent, coarse, n_bad=bad)
    assert int(bad.item()) == 1
    want = oamr.restrict(before.cpu().numpy(), fine.cpu().numpy()[2:], [15])
    state_close(coarse.cpu().numpy(), want, 1e-14, "one good parent")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_flux_correct_random_inputs(gpu, dtype):
    r = np.random.default_rng(5)
    parent, faces = layout()
    coarse = torch.from_numpy(1 + 0.1 * r.standard_normal((8, 5, 16, 16, 16))).to(dtype)
    cfl = torch.from_numpy(r.standard_normal((8, 3, 3, 5, 16, 16))).to(dtype)
    acc = torch.from_numpy(0.01 * r.standard_normal((len(parent), 3, 3, 5, 16, 16)))
    dt, dh = 0.013, 0.031
    want = oamr.flux_correct(coarse.double().numpy(), cfl.double().numpy(), acc.numpy(), faces, dt, dh)
    c = coarse.to(gpu)
    bad = torch.zeros(1, dtype=torch.int32, device=gpu)
    hydro.flux_correct(c, cfl.to(gpu), acc.to(gpu), amr.faces_to_device(faces, gpu), dev1(dt, gpu),
                       dev1(dh, gpu), n_bad=bad)
    assert int(bad.item()) == 0
    state_close(c.cpu().numpy(), want, 1e-12 if dtype == torch.float64 else 1e-6, f"flux correct {dtype}")
    # cells with no record are untouched
    changed = np.any(want != coarse.double().numpy(), axis=1)
    assert np.array_equal(np.any(c.cpu().double().numpy() != coarse.double().numpy(), axis=1), changed)


def test_flux_correct_skips_and_counts_bad_records(gpu):
    r = np.random.default_rng(6)
    parent, faces = layout()
    bad_faces = faces.copy()
    bad_faces[0]["coarse_group"] = 99       # out of range
    bad_faces[1]["fine_group"] = -1         # out of range
    bad_faces[2]["side"] = 2                # invalid
    bad_faces[3]["dir"] = 5                 # invalid direction (counted once)
    bad_faces[4]["coarse_face"] = 0
    bad_faces[4]["side"] = 0                # cell index -1
    bad_faces[5]["qs"] = 3                  # invalid quarter
    coarse = torch.from_numpy(1 + 0.1 * r.standard_normal((8, 5, 16, 16, 16)))
    cfl = torch.from_numpy(r.standard_normal((8, 3, 3, 5, 16, 16)))
    acc = torch.from_numpy(0.01 * r.standard_normal((len(parent), 3, 3, 5, 16, 16)))
    c = coarse.to(gpu)
    bad = torch.zeros(1, dtype=torch.int32, device=gpu)
    hydro.flux_correct(c, cfl.to(gpu), acc.to(gpu), amr.faces_to_device(bad_faces, gpu), dev1(0.01, gpu),
                       dev1(0.02, gpu), n_bad=bad)
    assert int(bad.item()) == 6
    want = oamr.flux_correct(coarse.numpy(), cfl.numpy(), acc.numpy(), faces[6:], 0.01, 0.02)
    state_close(c.cpu().numpy(), want, 1e-12, "good records only")


# ---------------------------------------------------------------- the whole step

def fine_padded_gpu(coarse, fine, parent, g):
    """Fine ghost fill on the GPU with torch indexing (a test helper: the
    product has no coarse-to-fine ghost interpolation): children of coarse
    cells take the coarse value, fine groups lie over them, periodic wrap."""
    n = 16 * g
    C = coarse.reshape(g, g, g, 5, 16, 16, 16).permute(3, 0, 4, 1, 5, 2, 6).reshape(5, n, n, n)
    Fg = C.repeat_interleave(2, 1).repeat_interleave(2, 2).repeat_interleave(2, 3).clone()
    origins = []
    for f, code in enumerate(parent.tolist()):
        gg, o = divmod(code, 8)
        x0 = 32 * (gg % g) + 16 * (o & 1)
        y0 = 32 * ((gg // g) % g) + 16 * ((o >> 1) & 1)
        z0 = 32 * (gg // (g * g)) + 16 * ((o >> 2) & 1)
        origins.append((x0, y0, z0))
        Fg[:, z0:z0 + 16, y0:y0 + 16, x0:x0 + 16] = fine[f]
    out = torch.empty((len(origins), 5, 20, 20, 20), dtype=fine.dtype, device=fine.device)
    N = 2 * n
    for f, (x0, y0, z0) in enumerate(origins):
        ix = torch.arange(x0 - 2, x0 + 18, device=fine.device) % N
        iy = torch.arange(y0 - 2, y0 + 18, device=fine.device) % N
        iz = torch.arange(z0 - 2, z0 + 18, device=fine.device) % N
        out[f] = Fg.index_select(1, iz).index_select(2, iy).index_select(3, ix)
    return out


def gpu_two_level_step(coarse, fine, parent_t, faces_t, dt, dh, g):
    dev = coarse.device
    dt_c, dh_c = dev1(dt, dev), dev1(dh, dev)
    dt_f, dh_f = dev1(0.5 * dt, dev), dev1(0.5 * dh, dev)
    nc = coarse.shape[0]
    cfl = torch.empty((nc, 3, 3, 5, 16, 16), dtype=coarse.dtype, device=dev)
    c_new = hydro.hydro_solve_batched(hydro.pack_periodic(coarse, g, g, g), None, dt_c, dh_c, G53,
                                      fluxes_out=cfl)
    f = fine
    acc = None
    ffl = torch.empty((fine.shape[0], 3, 3, 5, 16, 16), dtype=coarse.dtype, device=dev)
    for s in (0, 1):
        c_t = coarse if s == 0 else 0.5 * (coarse + c_new)
        f = hydro.hydro_solve_batched(fine_padded_gpu(c_t, f, parent_t, g), None, dt_f, dh_f, G53,
                                      fluxes_out=ffl)
        acc = hydro.flux_accumulate(ffl, dt_f, acc=acc, reset=(s == 0))
    bad = torch.zeros(1, dtype=torch.int32, device=dev)
    hydro.flux_correct(c_new, cfl, acc, faces_t, dt_c, dh_c, n_bad=bad)
    hydro.restrict(f, parent_t, c_new, n_bad=bad)
    assert int(bad.item()) == 0
    return c_new, f


def inject(coarse, parent, g):
    n = 16 * g
    C = coarse.reshape(g, g, g, 5, 16, 16, 16).transpose(3, 0, 4, 1, 5, 2, 6).reshape(5, n, n, n)
    Fg = C.repeat(2, 1).repeat(2, 2).repeat(2, 3)
    out = []
    for code in parent:
        gg, o = divmod(int(code), 8)
        x0 = 32 * (gg % g) + 16 * (o & 1)
        y0 = 32 * ((gg // g) % g) + 16 * ((o >> 1) & 1)
        z0 = 32 * (gg // (g * g)) + 16 * ((o >> 2) & 1)
        out.append(Fg[:, z0:z0 + 16, y0:y0 + 16, x0:x0 + 16])
    return np.stack(out)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_two_level_step_against_oracle(gpu, dtype):
    """Coarse step, two fine sub-steps, accumulation, correction, restriction:
    FP64 within 1e-12 of the oracle's two-level step; totals conserved on the
    GPU (gamer_conserved_sums) to 1e-13 in FP64; FP32 within 1e-5 in L1."""
    g = 2
    st, dh = W.smooth_modes(n=32, kmax=2, workload=2)
    coarse = st.to(dtype).double().numpy()
    parent, faces = layout()
    fine = inject(coarse, parent, g)
    r = np.random.default_rng(8)
    fine[:, 0] *= 1 + 0.02 * r.random(fine[:, 0].shape)  # the fine level differs from the coarse
    fine = torch.from_numpy(fine).to(dtype).double().numpy()
    dt = 0.4 * oracle.cfl_dt(coarse, dh, G53, 1.0)
    want_c, want_f, _, _ = two_level_step(coarse, g, g, g, fine, parent, faces, dt, dh, G53)
    c_gpu = torch.from_numpy(coarse).to(dtype).to(gpu)
    f_gpu = torch.from_numpy(fine).to(dtype).to(gpu)
    parent_t = torch.from_numpy(parent).to(gpu)
    # composite totals before the step: the fine groups restricted onto the coarse grid
    before = hydro.conserved_sums(hydro.restrict(f_gpu, parent_t, c_gpu.clone()), dh)
    got_c, got_f = gpu_two_level_step(c_gpu, f_gpu, parent_t, amr.faces_to_device(faces, gpu), dt, dh, g)
    if dtype == torch.float64:
        state_close(got_c.cpu().numpy(), want_c, 1e-12, "two-level coarse")
        state_close(got_f.cpu().numpy(), want_f, 1e-12, "two-level fine")
        after = hydro.conserved_sums(got_c, dh)
        scale = np.abs(coarse).sum(axis=(0, 2, 3, 4)) * dh ** 3
        assert np.all(np.abs(np.array(after) - np.array(before)) <= 1e-13 * scale), (before, after)
    else:
        for got, want in ((got_c, want_c), (got_f, want_f)):
            got = got.cpu().double().numpy()
            l1 = np.abs(got - want).sum(axis=(0, 2, 3, 4)) / np.abs(want).sum(axis=(0, 2, 3, 4))
            assert np.all(l1 < 1e-5), l1


def sphere_layout(g, radius=0.3):
    """The refined sphere the benchmark times on a grid of g^3 coarse groups:
    every 8^3 patch whose centre lies within `radius` of the box size from the
    box centre becomes a fine group."""
    npch = 2 * g
    c = (np.arange(npch) + 0.5) / npch - 0.5
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    sel = np.argwhere(X ** 2 + Y ** 2 + Z ** 2 < radius ** 2)  # (pz, py, px)
    patches = [((px // 2) + g * ((py // 2) + g * (pz // 2)), (px % 2) + 2 * (py % 2) + 4 * (pz % 2))
               for pz, py, px in sel]
    return amr.refine(g, g, g, patches)


@pytest.mark.timeout(400)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_bench_size_sphere(gpu, dtype):
    """Flux correction and restriction at the size the benchmark times: the
    256^3 grid (4096 coarse groups) with the refined sphere's 3648 fine groups
    and 1704 face records, each on the same input state, whole arrays against
    the oracle (on the same dtype-rounded inputs).  Coarse state: the smooth-mode flow; fine state:
    independent random physical states; fluxes: seeded random values."""
    g = 16
    parent, faces = sphere_layout(g)
    assert (len(parent), len(faces)) == (3648, 1704)
    st, dh = W.smooth_modes(n=256)
    r = np.random.default_rng(11)
    coarse = st.to(dtype)
    fine = phys(r, len(parent)).to(dtype)
    cfl = torch.from_numpy(0.1 * r.standard_normal((g ** 3, 3, 3, 5, 16, 16))).to(dtype)
    acc = torch.from_numpy(1e-3 * r.standard_normal((len(parent), 3, 3, 5, 16, 16)))
    dt = 0.05 * dh
    want = oamr.flux_correct(coarse.double().numpy(), cfl.double().numpy(), acc.numpy(), faces, dt, dh)
    c = coarse.to(gpu)
    bad = torch.zeros(1, dtype=torch.int32, device=gpu)
    hydro.flux_correct(c, cfl.to(gpu), acc.to(gpu), amr.faces_to_device(faces, gpu), dev1(dt, gpu),
                       dev1(dh, gpu), n_bad=bad)
    f64 = dtype == torch.float64
    state_close(c.cpu().numpy(), want, 1e-12 if f64 else 1e-6, f"sphere flux correct {dtype}")
    del cfl, acc
    # restriction of the same input state, checked on its own
    want2 = oamr.restrict(coarse.double().numpy(), fine.double().numpy(), parent)
    c = coarse.to(gpu)
    hydro.restrict(fine.to(gpu), torch.from_numpy(parent).to(gpu), c, n_bad=bad)
    state_close(c.cpu().numpy(), want2, 1e-14 if f64 else 1e-7, f"sphere restrict {dtype}")
    assert int(bad.item()) == 0
