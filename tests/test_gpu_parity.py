"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Tolerances (stated per test; the measures are in tests/parity.py):
  FP64: per cell, 1e-12 relative (rho and E against the cell's own |value|, each
        momentum component against the cell's |m| + rho c_s).
  FP32: the oracle runs on the float32-rounded input converted to double;
        smooth flow 1e-5 per cell; shocked runs L1 per variable.
  Flux planes: per value against |oracle| + the component's batch maximum.
  Integers (fallback counts) and the periodic ghost fill: exact.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle_driver import run_periodic
from paper_1007_3818_amd import hydro, workloads as W
from paper_1007_3818_amd.stepper import PeriodicGrid
from parity import flux_close, state_close

pytestmark = pytest.mark.gpu
G53 = 5.0 / 3.0


def padded_pair(state64, gx, gy, gz, dtype, dev):
    """GPU-packed input in `dtype` and the oracle's own packed input of the same
    (rounded) state in float64."""
    st = state64.to(dtype)
    gpu_pad = hydro.pack_periodic(st.to(dev), gx, gy, gz)
    ora_pad = oracle.pack_periodic(st.double().numpy(), gx, gy, gz)
    return gpu_pad, ora_pad


# ------------------------------------------------------------------ ghost fill

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_pack_periodic_bitwise(gpu, dtype):
    r = np.random.default_rng(11)
    gx, gy, gz = 3, 2, 2
    st = torch.from_numpy(r.standard_normal((gx * gy * gz, 5, 16, 16, 16)))
    gp, op = padded_pair(st, gx, gy, gz, dtype, gpu)
    assert np.array_equal(gp.cpu().double().numpy(), op)


# ------------------------------------------------------------------ exact cases

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_uniform_state_bitwise(gpu, dtype):
    W_ = [0.7, 0.3, -1.1, 2.0, 1.9]
    U = torch.tensor(oracle.cons_from_prim(W_, G53)).to(dtype)
    pad = U[None, :, None, None, None].expand(6, 5, 20, 20, 20).contiguous().to(gpu)
    flux = torch.empty((6, 3, 3, 5, 16, 16), dtype=dtype, device=gpu)
    out = hydro.hydro_solve(pad, 0.01, 0.1, G53, fluxes_out=flux)
    torch.cuda.synchronize()
    assert torch.equal(out.cpu(), pad[:, :, 2:18, 2:18, 2:18].cpu())


def test_zero_groups_is_noop(gpu):
    pad = torch.empty((0, 5, 20, 20, 20), dtype=torch.float64, device=gpu)
    out = hydro.hydro_solve(pad, 0.01, 0.1, G53)
    assert out.shape[0] == 0


# ------------------------------------------------------------------ one-step parity

def _cases():
    yield "sod", W.sod_x(), (2, 2, 2)
    yield "smooth48", W.smooth_modes(n=48), (3, 3, 3)
    yield "cosmo32", W.cosmo_like(n=32), (2, 2, 2)


@pytest.mark.parametrize("name", ["sod", "smooth48", "cosmo32"])
def test_one_step_fp64_parity(gpu, name):
    (st, dh), (gx, gy, gz) = next((c[1], c[2]) for c in _cases() if c[0] == name)
    gp, op = padded_pair(st, gx, gy, gz, torch.float64, gpu)
    dt = oracle.cfl_dt(st.numpy(), dh, G53, 0.5)
    ora, ofl, ocnt = oracle.hydro_solve(op, dt, dh, G53, want_fluxes=True)
    flux = torch.empty((gp.shape[0], 3, 3, 5, 16, 16), dtype=torch.float64, device=gpu)
    out = hydro.hydro_solve(gp, dt, dh, G53, fluxes_out=flux)
    torch.cuda.synchronize()
    state_close(out.cpu().numpy(), ora, 1e-12, f"{name} state")
    flux_close(flux.cpu().numpy().transpose(0, 3, 1, 2, 4, 5), ofl.transpose(0, 3, 1, 2, 4, 5), 1e-12,
               f"{name} fluxes")


@pytest.mark.parametrize("name", ["sod", "smooth48", "cosmo32"])
def test_fallback_counts_match(gpu, name):
    """Predictor and HLLE fallback counts (integers) equal the oracle's."""
    (st, dh), (gx, gy, gz) = next((c[1], c[2]) for c in _cases() if c[0] == name)
    gp, op = padded_pair(st, gx, gy, gz, torch.float64, gpu)
    dt = oracle.cfl_dt(st.numpy(), dh, G53, 0.5)
    _, _, ocnt = oracle.hydro_solve(op, dt, dh, G53)
    dt_dev = torch.tensor([dt], dtype=torch.float64, device=gpu)
    dh_dev = torch.tensor([dh], dtype=torch.float64, device=gpu)
    stats = torch.empty((gp.shape[0], 8), dtype=torch.float64, device=gpu)
    hydro.hydro_solve_batched(gp, None, dt_dev, dh_dev, G53, group_stats=stats)
    _, tot = hydro.step_reduce(stats, None, dh_dev, 0.5)
    t = tot.cpu().numpy()
    assert (int(t[5]), int(t[6])) == ocnt


@pytest.mark.parametrize("name", ["smooth48", "cosmo32"])
def test_one_step_fp32_parity(gpu, name):
    (st, dh), (gx, gy, gz) = next((c[1], c[2]) for c in _cases() if c[0] == name)
    gp, op = padded_pair(st, gx, gy, gz, torch.float32, gpu)
    dt = oracle.cfl_dt(st.float().double().numpy(), dh, G53, 0.5)
    ora, ofl, _ = oracle.hydro_solve(op, dt, dh, G53, want_fluxes=True)
    flux = torch.empty((gp.shape[0], 3, 3, 5, 16, 16), dtype=torch.float32, device=gpu)
    out = hydro.hydro_solve(gp, dt, dh, G53, fluxes_out=flux)
    torch.cuda.synchronize()
    if name == "smooth48":
        state_close(out.cpu().numpy(), ora, 1e-5, "fp32 smooth state")
        flux_close(flux.cpu().numpy().transpose(0, 3, 1, 2, 4, 5), ofl.transpose(0, 3, 1, 2, 4, 5),
              1e-4, "fp32 smooth fluxes")
    else:
        # Mach-10 log-normal flow: L1 of the relative difference per variable
        o = out.cpu().double().numpy()
        l1 = np.abs(o - ora).sum(axis=(0, 2, 3, 4)) / np.abs(ora).sum(axis=(0, 2, 3, 4))
        assert np.all(l1 < 1e-5), l1


def test_sod_fp32_l1(gpu):
    st, dh = W.sod_x()
    gp, op = padded_pair(st, 2, 2, 2, torch.float32, gpu)
    dt = oracle.cfl_dt(st.numpy(), dh, G53, 0.5)
    ora, _, _ = oracle.hydro_solve(op, dt, dh, G53)
    out = hydro.hydro_solve(gp, dt, dh, G53)
    l1 = np.abs(out.cpu().double().numpy() - ora).sum(axis=(0, 2, 3, 4)) / np.abs(ora).sum(axis=(0, 2, 3, 4)).clip(1e-300)
    assert np.all(l1[[0, 1, 4]] < 1e-6), l1


# ------------------------------------------------------------------ multi-step

def test_sod_ten_steps_fp64(gpu):
    """Workload 1: ten steps at CFL 0.5 with the device-resident time step."""
    st, dh = W.sod_x()
    ora, t_ora, _, counts = run_periodic(st.numpy(), 2, 2, 2, dh, G53, 0.5, steps=10)
    assert counts == (0, 0)
    grid = PeriodicGrid(st.to(gpu), 2, 2, 2, dh, G53, 0.5)
    grid.step(10)
    torch.cuda.synchronize()
    state_close(grid.current.cpu().numpy(), ora, 1e-12, "sod 10 steps")
    assert grid.time() == pytest.approx(t_ora, rel=1e-13)


def test_smooth_twenty_steps_fp64_and_graph(gpu):
    """20 steps of smooth flow, eager and replayed from a captured HIP graph:
    both match the oracle, and each other bitwise."""
    st, dh = W.smooth_modes(n=32)
    ora, t_ora, _, counts = run_periodic(st.numpy(), 2, 2, 2, dh, G53, 0.5, steps=20)
    eager = PeriodicGrid(st.to(gpu), 2, 2, 2, dh, G53, 0.5)
    eager.step(20)
    graph = PeriodicGrid(st.to(gpu), 2, 2, 2, dh, G53, 0.5).capture()
    for _ in range(9):  # two eager steps ran during capture; 9 replays of 2 steps
        graph.step(2)
        torch.cuda.synchronize()
    state_close(eager.current.cpu().numpy(), ora, 1e-12, "smooth 20 steps")
    assert torch.equal(eager.current, graph.current)
    assert eager.time() == graph.time() == pytest.approx(t_ora, rel=1e-13)


# ------------------------------------------------------------------ CFL, sums, stats

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_cfl_and_sums(gpu, dtype):
    st, dh = W.cosmo_like(n=32)
    st = st.to(dtype)
    host = st.double().numpy()
    dt_g = hydro.cfl_dt(st.to(gpu), dh, G53, 0.5)
    dt_o = oracle.cfl_dt(host, dh, G53, 0.5)
    # the signal speed is evaluated in the working precision with refined
    # (FP64) or hardware (FP32) reciprocal and square root
    assert dt_g == pytest.approx(dt_o, rel=4e-15 if dtype == torch.float64 else 1e-6)
    s_g = np.array(hydro.conserved_sums(st.to(gpu), dh))
    s_o = oracle.conserved_sums(host, dh)
    scale = dh ** 3 * np.abs(host).reshape(host.shape[0], 5, -1).sum(axis=(0, 2))
    assert np.all(np.abs(s_g - s_o) <= 1e-14 * scale)


def test_solver_stats_equal_group_stats(gpu):
    """The solver's fused epilogue and the stand-alone stats kernel agree bitwise
    on the sums and the signal speed of the same output."""
    st, dh = W.smooth_modes(n=32)
    gp = hydro.pack_periodic(st.to(gpu), 2, 2, 2)
    dt_dev = torch.tensor([1e-3], dtype=torch.float64, device=gpu)
    dh_dev = torch.tensor([dh], dtype=torch.float64, device=gpu)
    s1 = torch.empty((8, 8), dtype=torch.float64, device=gpu)
    out = hydro.hydro_solve_batched(gp, None, dt_dev, dh_dev, G53, group_stats=s1)
    s2 = hydro.group_stats(out, G53)
    assert torch.equal(s1[:, :6], s2[:, :6])


def test_determinism(gpu):
    st, dh = W.cosmo_like(n=32)
    gp = hydro.pack_periodic(st.to(gpu), 2, 2, 2)
    a = hydro.hydro_solve(gp, 1e-4, dh, G53)
    b = hydro.hydro_solve(gp, 1e-4, dh, G53)
    assert torch.equal(a, b)


# ------------------------------------------------------------------ batched levels

def test_batched_levels_fp64(gpu):
    """Groups of three levels with their own dt and dh in one launch: each group
    matches the oracle run with that group's dt and dh."""
    r = np.random.default_rng(12)
    st, dh0 = W.smooth_modes(n=32)
    P = oracle.pack_periodic(st.numpy(), 2, 2, 2)
    lev = r.integers(0, 3, size=P.shape[0]).astype(np.int8)
    dts = np.array([2e-3, 1e-3, 5e-4])
    dhs = np.array([dh0, dh0 / 2, dh0 / 4])
    out = hydro.hydro_solve_batched(torch.from_numpy(P).to(gpu), torch.from_numpy(lev).to(gpu),
                                    torch.from_numpy(dts).to(gpu), torch.from_numpy(dhs).to(gpu), G53)
    o = out.cpu().numpy()
    for L in range(3):
        sel = lev == L
        if sel.any():
            ora, _, _ = oracle.hydro_solve(P[sel], dts[L], dhs[L], G53)
            state_close(o[sel], ora, 1e-12, f"level {L}")


def test_step_reduce_per_level(gpu):
    st, dh = W.cosmo_like(n=32)
    gpu_st = st.to(gpu)
    stats = hydro.group_stats(gpu_st, G53)
    lev = torch.tensor([0, 1, 0, 2, 1, 0, 2, 2], dtype=torch.int8)
    dhs = torch.tensor([1.0, 0.5, 0.25], dtype=torch.float64)
    dt, tot = hydro.step_reduce(stats, lev.to(gpu), dhs.to(gpu), 0.5)
    host = st.numpy()
    for L in range(3):
        sel = (lev == L).numpy()
        want = oracle.cfl_dt(host[sel], float(dhs[L]), G53, 0.5)
        assert float(dt[L]) == pytest.approx(want, rel=4e-15)
    want = sum(oracle.conserved_sums(host[(lev == L).numpy()], float(dhs[L])) for L in range(3))
    np.testing.assert_allclose(tot[:5].cpu().numpy(), want, rtol=1e-13)


# ------------------------------------------------------------------ full size

def test_workload2_full_size_fp64_and_fp32(gpu):
    """256^3 smooth flow (4096 groups), the benchmark's input, one step: every
    group against the oracle in FP64, and FP32 within 1e-5."""
    st, dh = W.smooth_modes(n=256, device=gpu)
    dt = 0.5 * dh / 3.0  # fixed, well inside the CFL limit of this flow
    gp = hydro.pack_periodic(st, 16, 16, 16)
    out = hydro.hydro_solve(gp, dt, dh, G53).cpu().numpy()
    gp32 = hydro.pack_periodic(st.float(), 16, 16, 16)
    o32 = hydro.hydro_solve(gp32, dt, dh, G53)
    # the launch shapes the benchmark's tuner picks on this batch (FP32: a
    # persistent grid of 768 work-groups) give bitwise the same result
    dtd = torch.tensor([dt], dtype=torch.float64, device=gpu)
    dhd = torch.tensor([dh], dtype=torch.float64, device=gpu)
    assert torch.equal(hydro.hydro_solve_batched(gp32, None, dtd, dhd, G53, variant=0, grid=768), o32)
    del gp32
    out32 = o32.cpu().double().numpy()
    host = st.cpu().numpy()
    del gp
    ora, _, cnt = oracle.hydro_solve(oracle.pack_periodic(host, 16, 16, 16), dt, dh, G53)
    assert cnt == (0, 0)
    state_close(out, ora, 1e-12, "workload 2 fp64")
    ora32, _, _ = oracle.hydro_solve(oracle.pack_periodic(st.float().double().cpu().numpy(), 16, 16, 16),
                                     dt, dh, G53)
    state_close(out32, ora32, 1e-5, "workload 2 fp32")


# ------------------------------------------------------------------ tuning variants

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_variants_and_grids_agree(gpu, dtype):
    """Every compiled solver variant agrees with the default to rounding (FP32
    1e-6, FP64 1e-13 relative); within a variant, every launch grid gives
    bitwise the same output and stats."""
    from paper_1007_3818_amd.autotune import max_rel_diff
    st, dh = W.cosmo_like(n=48)
    gp = hydro.pack_periodic(st.to(dtype).to(gpu), 3, 3, 3)
    dt_dev = torch.tensor([2e-4], dtype=torch.float64, device=gpu)
    dh_dev = torch.tensor([dh], dtype=torch.float64, device=gpu)
    base = None
    for v in range(len(hydro.solver_variants(dtype))):
        ref_out, ref_st = None, None
        for grid in (0, 1, 4, 13, 100):
            stats = torch.empty((27, 8), dtype=torch.float64, device=gpu)
            out = hydro.hydro_solve_batched(gp, None, dt_dev, dh_dev, G53, group_stats=stats,
                                            variant=v, grid=grid)
            torch.cuda.synchronize()
            if ref_out is None:
                ref_out, ref_st = out.clone(), stats.clone()
            assert torch.equal(out, ref_out), (v, grid)
            assert torch.equal(stats, ref_st), (v, grid)
        if base is None:
            base = ref_out
        err = max_rel_diff(ref_out, base)
        assert err <= (1e-6 if dtype == torch.float32 else 1e-13), (v, err)


def test_autotune_picks_a_candidate(gpu, tmp_path, monkeypatch):
    from paper_1007_3818_amd import autotune
    monkeypatch.setenv("GAMER_TUNE_CACHE", str(tmp_path / "tune.json"))
    st, dh = W.smooth_modes(n=64)
    gp = hydro.pack_periodic(st.float().to(gpu), 4, 4, 4)
    dt_dev = torch.tensor([1e-3], dtype=torch.float64, device=gpu)
    dh_dev = torch.tensor([dh], dtype=torch.float64, device=gpu)
    r = autotune.tune(gp, dt_dev, dh_dev, G53, reps=2)
    assert (r["variant"], r["grid"]) in autotune.candidates(torch.float32, 64)
    assert not r["cached"]
    r2 = autotune.tune(gp, dt_dev, dh_dev, G53, reps=2)
    assert r2["cached"] and r2["variant"] == r["variant"] and r2["grid"] == r["grid"]


# ------------------------------------------------------------------ exact properties on the GPU

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_flux_planes_shared_bitwise(gpu, dtype):
    """Face 16 of a group and face 0 of its +d neighbour are the same face: the
    GPU writes the same bits for both, in every compiled variant (one code path
    computes a face state and a face flux wherever it sits in the group)."""
    gx = gy = gz = 3
    st, dh = W.cosmo_like(n=48)
    gp = hydro.pack_periodic(st.to(dtype).to(gpu), gx, gy, gz)
    dt_dev = torch.tensor([1e-4], dtype=torch.float64, device=gpu)
    dh_dev = torch.tensor([dh], dtype=torch.float64, device=gpu)

    def gid(x, y, z):
        return (x % gx) + gx * ((y % gy) + gy * (z % gz))

    for v in range(len(hydro.solver_variants(dtype))):
        fl = torch.empty((27, 3, 3, 5, 16, 16), dtype=dtype, device=gpu)
        hydro.hydro_solve_batched(gp, None, dt_dev, dh_dev, G53, fluxes_out=fl, variant=v)
        f = fl.cpu()
        for z in range(gz):
            for y in range(gy):
                for x in range(gx):
                    g = gid(x, y, z)
                    assert torch.equal(f[g, 0, 2], f[gid(x + 1, y, z), 0, 0]), (v, g, "x")
                    assert torch.equal(f[g, 1, 2], f[gid(x, y + 1, z), 1, 0]), (v, g, "y")
                    assert torch.equal(f[g, 2, 2], f[gid(x, y, z + 1), 2, 0]), (v, g, "z")


def test_sod_axes_agree_on_gpu(gpu):
    """Sod along x, y and z on the GPU (10 FP64 steps): the three solutions agree
    after permuting axes and momenta, to 1e-13 relative."""
    res = []
    for axis in range(3):
        st, dh = W.sod_x(axis=axis)
        grid = PeriodicGrid(st.to(gpu), 2, 2, 2, dh, G53, 0.5)
        grid.step(10)
        G = W.groups_to_global(grid.current.cpu(), 2, 2, 2).numpy()
        if axis == 1:
            G = G.transpose(0, 1, 3, 2)[[0, 2, 1, 3, 4]]
        elif axis == 2:
            G = G.transpose(0, 3, 2, 1)[[0, 3, 2, 1, 4]]
        res.append(G)
    for a in (1, 2):
        np.testing.assert_allclose(res[a], res[0], rtol=1e-13, atol=1e-13)
