"""GPU parity at the full sizes of workloads 3, 4 and 5, through the C ABI.

The GPU side packs ghost zones with its own kernel; the oracle builds the padded
inputs of the groups it checks with its own subset pack from the same seeded
state.  Tolerances as in test_gpu_parity: FP64 1e-12 relative per cell (the
measure of tests/parity.py); FP32 as stated per test.  The worst per-cell error
of each workload is printed.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1007_3818_amd import hydro, workloads as W
from parity import l1_rel, state_close

pytestmark = pytest.mark.gpu
G53 = 5.0 / 3.0


def test_workload3_three_level_batch(gpu):
    """Workload 3: 512 + 4096 + 20000 groups of a Sedov blast at dh = 1, 1/2, 1/4 in
    ONE launch with per-level dt read on the device.  Per-level dt against the
    oracle; groups around the blast and random others of every level against the
    oracle at their level's dt and dh, FP64 and FP32, with per-group fallback counts."""
    levels = W.sedov_amr(device=gpu)
    pads, inter, lev = [], [], []
    for L, (groups, dh, gx, ids) in enumerate(levels):
        idt = torch.as_tensor(ids, device=gpu)
        full = hydro.pack_periodic(groups, gx, gx, gx)
        pads.append(full[idt])
        del full
        inter.append(groups[idt])
        lev.append(torch.full((len(ids),), L, dtype=torch.int8))
    batch = torch.cat(pads)
    del pads
    interiors = torch.cat(inter)
    level = torch.cat(lev).to(gpu)
    n = batch.shape[0]
    assert n == 512 + 4096 + 20000
    dhs = [lv[1] for lv in levels]
    dh_dev = torch.tensor(dhs, dtype=torch.float64, device=gpu)

    # per-level CFL time steps
    dt_gpu, tot = hydro.step_reduce(hydro.group_stats(interiors, G53), level, dh_dev, 0.5)
    dt_ora = []
    for L, (groups, dh, gx, ids) in enumerate(levels):
        dt_ora.append(oracle.cfl_dt(groups[torch.as_tensor(ids, device=gpu)].cpu().numpy(), dh, G53, 0.5))
    np.testing.assert_allclose(dt_gpu.cpu().numpy(), dt_ora, rtol=4e-15)
    dt_dev = torch.tensor(dt_ora, dtype=torch.float64, device=gpu)

    stats = torch.empty((n, 8), dtype=torch.float64, device=gpu)
    out64 = hydro.hydro_solve_batched(batch, level, dt_dev, dh_dev, G53, group_stats=stats).cpu().numpy()
    out32 = hydro.hydro_solve_batched(batch.float(), level, dt_dev, dh_dev, G53).cpu().double().numpy()
    st = stats.cpu().numpy()

    rng = np.random.default_rng(3)
    offset = 0
    for L, (groups, dh, gx, ids) in enumerate(levels):
        c = gx // 2  # the blast cell is the lower corner of group (c, c, c)
        near = [(c - a) + gx * ((c - b) + gx * (c - e)) for a in (0, 1) for b in (0, 1) for e in (0, 1)]
        pick = sorted(set(near) | set(int(x) for x in rng.choice(ids, size=8, replace=False)))
        pos = np.searchsorted(ids, pick)
        assert np.array_equal(np.asarray(ids)[pos], pick)
        ref, _, cnt = oracle.hydro_solve(oracle.pack_periodic_subset(groups, gx, gx, gx, pick),
                                         dt_ora[L], dh, G53)
        state_close(out64[offset + pos], ref, 1e-12, f"level {L} fp64")
        assert (int(st[offset + pos, 6].sum()), int(st[offset + pos, 7].sum())) == cnt
        ref32, _, _ = oracle.hydro_solve(
            oracle.pack_periodic_subset(groups.float(), gx, gx, gx, pick), dt_ora[L], dh, G53)
        assert np.all(l1_rel(out32[offset + pos], ref32) < 1e-5), (L, l1_rel(out32[offset + pos], ref32))
        offset += len(ids)


def test_workload4_full_size(gpu):
    """Workload 4: 256^3 log-normal density with Mach-10 flow (4096 groups), one
    step at the CFL dt: every group against the oracle in FP64 per cell, fallback
    counts exact, FP32 within 1e-5 in L1 per variable; positivity: no output cell
    with rho <= 0, p <= 0 or a non-finite value in either precision (the oracle's
    own step has none either)."""
    st, dh = W.cosmo_like(n=256)
    host = st.numpy()
    dt = oracle.cfl_dt(host, dh, G53, 0.5)
    ref, _, cnt = oracle.hydro_solve(oracle.pack_periodic(host, 16, 16, 16), dt, dh, G53)
    dt_dev = torch.tensor([dt], dtype=torch.float64, device=gpu)
    dh_dev = torch.tensor([dh], dtype=torch.float64, device=gpu)
    stats = torch.empty((4096, 8), dtype=torch.float64, device=gpu)
    bad = torch.zeros(2, dtype=torch.int64, device=gpu)
    gp = hydro.pack_periodic(st.to(gpu), 16, 16, 16)
    out = hydro.hydro_solve_batched(gp, None, dt_dev, dh_dev, G53, group_stats=stats,
                                    bad_count=bad).cpu().numpy()
    assert oracle.max_speed(ref, G53) > 0  # finite: the oracle's step is physical everywhere
    state_close(out, ref, 1e-12, "workload 4 fp64")
    s = stats.cpu().numpy()
    assert (int(s[:, 6].sum()), int(s[:, 7].sum())) == cnt
    assert bad.cpu().tolist() == [0, 0]
    assert np.isfinite(s[:, 5]).all()
    h32 = st.float().double().numpy()
    ref32, _, _ = oracle.hydro_solve(oracle.pack_periodic(h32, 16, 16, 16), dt, dh, G53)
    bad32 = torch.zeros(2, dtype=torch.int64, device=gpu)
    stats32 = torch.empty((4096, 8), dtype=torch.float64, device=gpu)
    out32 = hydro.hydro_solve_batched(hydro.pack_periodic(st.float().to(gpu), 16, 16, 16), None, dt_dev, dh_dev,
                                      G53, group_stats=stats32, bad_count=bad32)
    l1 = l1_rel(out32.cpu().double().numpy(), ref32)
    print(f"[parity] workload 4 fp32: L1 per variable {l1}", flush=True)
    assert np.all(l1 < 1e-5)
    assert bad32.cpu().tolist() == [0, 0]
    assert np.isfinite(stats32.cpu().numpy()[:, 5]).all()


@pytest.mark.timeout(400)
def test_workload5_sampled_full_size(gpu):
    """Workload 5: 1024^3 (262144 groups), the largest single-GPU batch, in FP64
    (84 GB padded input) and FP32 (42 GB).  Sixteen groups (the corners of the
    grid, group 0 and its periodic neighbours, random others) against the oracle."""
    n = 1024
    g = n // 16
    st, dh = W.smooth_modes(n=n, kmax=8, workload=5, device=gpu)
    dt = 0.1 * dh
    rng = np.random.default_rng(5)
    corners = [x + g * (y + g * z) for x in (0, g - 1) for y in (0, g - 1) for z in (0, g - 1)]
    pick = sorted(set(corners) | set(int(x) for x in rng.choice(g ** 3, size=8, replace=False)))
    ref, _, cnt = oracle.hydro_solve(oracle.pack_periodic_subset(st, g, g, g, pick), dt, dh, G53)
    assert cnt == (0, 0)
    idx = torch.as_tensor(pick, device=gpu)
    gp = hydro.pack_periodic(st, g, g, g)
    out = hydro.hydro_solve(gp, dt, dh, G53)
    state_close(out[idx].cpu().numpy(), ref, 1e-12, "workload 5 fp64")
    del gp, out
    torch.cuda.empty_cache()
    s32 = st.float()
    ref32, _, _ = oracle.hydro_solve(oracle.pack_periodic_subset(s32, g, g, g, pick), dt, dh, G53)
    del st
    gp32 = hydro.pack_periodic(s32, g, g, g)
    out32 = hydro.hydro_solve(gp32, dt, dh, G53)
    state_close(out32[idx].cpu().numpy(), ref32, 1e-5, "workload 5 fp32")


@pytest.mark.timeout(400)
def test_workload5_sampled_periodic_and_mixed(gpu):
    """Workload 5 (1024^3, 262144 groups) through the fused periodic step (ghost
    cells read in place) as the benchmark times it: FP64, FP64 state with FP32
    arithmetic, and FP32.  The same sixteen sampled groups against the oracle,
    which pads them itself: FP64 per cell within 1e-12; the mixed and FP32
    steps per cell within 1e-5 (the FP32 one against the oracle on the
    float-rounded state)."""
    n = 1024
    g = n // 16
    st, dh = W.smooth_modes(n=n, kmax=8, workload=5, device=gpu)
    dt = 0.1 * dh
    rng = np.random.default_rng(5)
    corners = [x + g * (y + g * z) for x in (0, g - 1) for y in (0, g - 1) for z in (0, g - 1)]
    pick = sorted(set(corners) | set(int(x) for x in rng.choice(g ** 3, size=8, replace=False)))
    idx = torch.as_tensor(pick, device=gpu)
    dt_dev = torch.tensor([dt], dtype=torch.float64, device=gpu)
    dh_dev = torch.tensor([dh], dtype=torch.float64, device=gpu)
    ref, _, cnt = oracle.hydro_solve(oracle.pack_periodic_subset(st, g, g, g, pick), dt, dh, G53)
    assert cnt == (0, 0)
    out = torch.empty_like(st)
    hydro.hydro_solve_periodic(st, g, g, g, dt_dev, dh_dev, G53, out=out)
    state_close(out[idx].cpu().numpy(), ref, 1e-12, "workload 5 periodic fp64")
    hydro.hydro_solve_periodic(st, g, g, g, dt_dev, dh_dev, G53, out=out, compute=torch.float32)
    state_close(out[idx].cpu().numpy(), ref, 1e-5, "workload 5 periodic fp64 state, fp32 arithmetic")
    del out
    s32 = st.float()
    del st
    torch.cuda.empty_cache()
    ref32, _, _ = oracle.hydro_solve(oracle.pack_periodic_subset(s32, g, g, g, pick), dt, dh, G53)
    out32 = torch.empty_like(s32)
    hydro.hydro_solve_periodic(s32, g, g, g, dt_dev, dh_dev, G53, out=out32)
    state_close(out32[idx].cpu().numpy(), ref32, 1e-5, "workload 5 periodic fp32")
