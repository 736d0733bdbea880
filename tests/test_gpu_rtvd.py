"""The relaxing TVD scheme on the GPU, through the C ABI, against its oracle.

Bars: FP64 within 1e-12 per cell (rho and E against the cell's own value, momenta against |m| + rho c_s) for one
step in both sweep orders; FP32 within 1e-5 in L1 per variable (the oracle
runs on the float-rounded input); the periodic entry point (ghost cells read
in place) equal to the padded one, bitwise in FP64, and against the oracle on
grids one group thick along some axes; a uniform state kept
bitwise; ten alternating FP64 steps of a smooth flow within 1e-11 of the
oracle's ten steps; a batch spanning two rows of the x sweep's launch grid
equal, copy by copy, to its first copy.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1007_3818_amd import hydro, workloads as W
from parity import l1_rel, state_close

pytestmark = pytest.mark.gpu
G53 = 5.0 / 3.0


def pad3_gpu(state, gx, gy, gz):
    """Three-cell periodic ghost fill with torch indexing on the GPU (a test
    helper, independent of the oracle's numpy fill)."""
    G = state.reshape(gz, gy, gx, 5, 16, 16, 16).permute(3, 0, 4, 1, 5, 2, 6).reshape(
        5, gz * 16, gy * 16, gx * 16)
    out = torch.empty((gx * gy * gz, 5, 22, 22, 22), dtype=state.dtype, device=state.device)
    for g in range(gx * gy * gz):
        bx, by, bz = g % gx, (g // gx) % gy, g // (gx * gy)
        ix = torch.arange(16 * bx - 3, 16 * bx + 19, device=state.device) % G.shape[3]
        iy = torch.arange(16 * by - 3, 16 * by + 19, device=state.device) % G.shape[2]
        iz = torch.arange(16 * bz - 3, 16 * bz + 19, device=state.device) % G.shape[1]
        out[g] = G.index_select(1, iz).index_select(2, iy).index_select(3, ix)
    return out


def dev1(x, gpu):
    return torch.tensor([x], dtype=torch.float64, device=gpu)


CASES = {
    "sod": (lambda: W.sod_x(), (2, 2, 2)),
    "smooth48": (lambda: W.smooth_modes(n=48), (3, 3, 3)),
}


@pytest.mark.parametrize("name", ["sod", "smooth48"])
@pytest.mark.parametrize("order", [0, 1])
def test_one_step_fp64(gpu, name, order):
    (st, dh), (gx, gy, gz) = CASES[name][0](), CASES[name][1]
    host = st.numpy()
    dt = oracle.cfl_dt(host, dh, G53, 0.4)
    ref, bad = oracle.rtvd_solve(oracle.pack_periodic_rtvd(host, gx, gy, gz), dt, dh, G53, order)
    assert bad == 0
    s = st.to(gpu)
    out = hydro.rtvd_solve_batched(pad3_gpu(s, gx, gy, gz), None, dev1(dt, gpu), dev1(dh, gpu), G53, order)
    state_close(out.cpu().numpy(), ref, 1e-12, f"{name} order {order}")
    per = hydro.rtvd_solve_periodic(s, gx, gy, gz, dev1(dt, gpu), dev1(dh, gpu), G53, order)
    assert torch.equal(per, out)


@pytest.mark.parametrize("shape", [(1, 1, 1), (8, 1, 1), (1, 2, 4)])
def test_periodic_grid_shapes_fp64(gpu, shape):
    """Grids one group thick along some axes (the ghost cells then wrap into
    the group itself or its single neighbour), both sweep orders, against the
    oracle's three-cell ghost fill."""
    gx, gy, gz = shape
    st, dh = W.smooth_modes(n=16 if gx * gy * gz == 1 else 32)
    host = st.numpy()
    dt = oracle.cfl_dt(host, dh, G53, 0.4)
    for order in (0, 1):
        ref, bad = oracle.rtvd_solve(oracle.pack_periodic_rtvd(host, gx, gy, gz), dt, dh, G53, order)
        assert bad == 0
        out = hydro.rtvd_solve_periodic(st.to(gpu), gx, gy, gz, dev1(dt, gpu), dev1(dh, gpu), G53, order)
        state_close(out.cpu().numpy(), ref, 1e-12, f"{shape} order {order}")


@pytest.mark.parametrize("name", ["sod", "smooth48"])
def test_one_step_fp32(gpu, name):
    (st, dh), (gx, gy, gz) = CASES[name][0](), CASES[name][1]
    s32 = st.float()
    host = s32.double().numpy()
    dt = oracle.cfl_dt(host, dh, G53, 0.4)
    ref, _ = oracle.rtvd_solve(oracle.pack_periodic_rtvd(host, gx, gy, gz), dt, dh, G53, 0)
    out = hydro.rtvd_solve_periodic(s32.to(gpu), gx, gy, gz, dev1(dt, gpu), dev1(dh, gpu), G53, 0)
    assert np.all(l1_rel(out.cpu().numpy(), ref) < 1e-5), l1_rel(out.cpu().numpy(), ref)


def test_uniform_state_bitwise(gpu):
    U = torch.tensor(oracle.cons_from_prim([0.7, 0.3, -1.1, 2.0, 1.9], G53))
    for dtype in (torch.float64, torch.float32):
        st = U.to(dtype)[None, :, None, None, None].expand(8, 5, 16, 16, 16).contiguous().to(gpu)
        for order in (0, 1):
            out = hydro.rtvd_solve_periodic(st, 2, 2, 2, dev1(0.01, gpu), dev1(0.1, gpu), G53, order)
            assert torch.equal(out, st)


def test_ten_alternating_steps_fp64(gpu):
    st, dh = W.smooth_modes(n=32, kmax=2, workload=2)
    host = st.numpy()
    s = st.to(gpu)
    work = hydro.rtvd_workspace(8, torch.float64, gpu)
    for k in range(10):
        dt = oracle.cfl_dt(host, dh, G53, 0.4)
        host, _ = oracle.rtvd_step_periodic(host, 2, 2, 2, dt, dh, G53, order=k % 2)
        s = hydro.rtvd_solve_periodic(s, 2, 2, 2, dev1(dt, gpu), dev1(dh, gpu), G53, k % 2, work=work)
    state_close(s.cpu().numpy(), host, 1e-11, "ten steps")


def test_levels_read_on_device(gpu):
    """A batch of groups at two levels with their own dt and dh in one call."""
    st, dh = W.smooth_modes(n=32, kmax=2, workload=2)
    host = st.numpy()
    pad_h = oracle.pack_periodic_rtvd(host, 2, 2, 2)
    dts, dhs = [1e-3, 4e-4], [dh, 0.5 * dh]
    level = np.array([0, 1, 1, 0, 1, 0, 0, 1], dtype=np.int8)
    ref = np.empty((8, 5, 16, 16, 16))
    for L in (0, 1):
        sel = level == L
        ref[sel], _ = oracle.rtvd_solve(pad_h[sel], dts[L], dhs[L], G53, 1)
    out = hydro.rtvd_solve_batched(pad3_gpu(st.to(gpu), 2, 2, 2), torch.from_numpy(level).to(gpu),
                                   torch.tensor(dts, dtype=torch.float64, device=gpu),
                                   torch.tensor(dhs, dtype=torch.float64, device=gpu), G53, 1)
    state_close(out.cpu().numpy(), ref, 1e-12, "two levels")


def test_workspace_checked(gpu):
    st, dh = W.smooth_modes(n=32, kmax=2, workload=2)
    s = st.to(gpu)
    small = torch.empty(1024, dtype=torch.uint8, device=gpu)
    from paper_1007_3818_amd._native import GamerError
    with pytest.raises(GamerError):
        hydro.rtvd_solve_periodic(s, 2, 2, 2, dev1(1e-3, gpu), dev1(dh, gpu), G53, 0, work=small)


def test_batch_over_several_grid_rows(gpu):
    """The padded-input x sweep takes its group from a grid of 8192 groups per
    row: a batch of 8,208 groups (1,026 copies of one 2 x 2 x 2 grid's padded
    groups) spans two rows.  Every copy must equal the first bitwise, in both
    sweep orders (the first x sweep on 22 x 22 pencils, the last on 16 x 16),
    and the first copy must match the oracle within 1e-5 in L1 (FP32)."""
    st, dh = W.smooth_modes(n=32, kmax=2, workload=2)
    host32 = st.float().double().numpy()
    pad_h = oracle.pack_periodic_rtvd(host32, 2, 2, 2)
    dt = oracle.cfl_dt(host32, dh, G53, 0.4)
    reps = 1026
    pad = pad3_gpu(st.float().to(gpu), 2, 2, 2)
    big = pad.repeat(reps, 1, 1, 1, 1)
    print(f"[rtvd] batch of {big.shape[0]} padded groups (two grid rows of the x sweep)", flush=True)
    for order in (0, 1):
        out = hydro.rtvd_solve_batched(big, None, dev1(dt, gpu), dev1(dh, gpu), G53, order)
        first = out[:8]
        assert torch.equal(out.view(reps, 8, 5, 16, 16, 16), first.expand(reps, 8, 5, 16, 16, 16)), order
        ref, _ = oracle.rtvd_solve(pad_h, dt, dh, G53, order)
        l1 = l1_rel(first.cpu().double().numpy(), ref)
        print(f"[parity] rtvd {reps} x 8 groups order {order}: L1 per variable {l1}", flush=True)
        assert np.all(l1 < 1e-5), l1
        del out
