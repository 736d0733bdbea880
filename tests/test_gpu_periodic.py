"""The fused periodic step (ghost cells read from neighbouring groups in place)
through the C ABI.

Bar against the ghost-fill kernel followed by the batched step with the same
variant (state, fluxes, per-group stats), for every compiled variant, several
launch grids and several z-segment lengths (one work-group sweeping 1, 2, 3 or
all the groups of a column as one run of planes): FP64 bitwise; FP32 within 1e-6 relative (the periodic
kernel is its own instantiation, and the compiler may contract a float
multiply-add into an FMA in one and not in the other), fallback counts exact.
Against the oracle's own ghost fill + step: FP64 1e-12 per cell, relative to
the larger of the cell's own scale and the size of its update terms (the input
is a 64^3 log-normal flow with cells beside 1e4 times their own energy), FP32
1e-5 in L1 per variable.
Grids are deliberately non-cubic, and include one group wide axes, where a
group is its own periodic neighbour.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1007_3818_amd import hydro, workloads as W
from paper_1007_3818_amd.autotune import max_rel_diff
from paper_1007_3818_amd.stepper import PeriodicGrid
from parity import flux_close, l1_rel, state_close, update_terms

pytestmark = pytest.mark.gpu
G53 = 5.0 / 3.0


# 64 groups of the 4^3-group log-normal state, read as other group grids: every
# group is a valid state, and the group index order x + gx (y + gy z) of each
# shape defines who neighbours whom.
SHAPES = [(2, 4, 8), (8, 1, 8), (1, 1, 64), (4, 4, 4)]


def _state(dtype, dev):
    st, dh = W.cosmo_like(n=64)
    return st.to(dtype).to(dev), dh


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fused_equals_pack_then_solve(gpu, dtype):
    st, dh = _state(dtype, gpu)
    dt_dev = torch.tensor([1e-4], dtype=torch.float64, device=gpu)
    dh_dev = torch.tensor([dh], dtype=torch.float64, device=gpu)
    n = st.shape[0]
    for gx, gy, gz in SHAPES:
        pad = hydro.pack_periodic(st, gx, gy, gz)
        for v in range(len(hydro.solver_variants(dtype))):
            fl_a = torch.empty((n, 3, 3, 5, 16, 16), dtype=dtype, device=gpu)
            s_a = torch.empty((n, 8), dtype=torch.float64, device=gpu)
            a = hydro.hydro_solve_batched(pad, None, dt_dev, dh_dev, G53, fluxes_out=fl_a,
                                          group_stats=s_a, variant=v)
            for grid, zseg in ((0, None), (7, None), (256, None), (0, 2), (7, 3), (0, gz), (5, gz)):
                # zseg: groups of a column swept as one run of planes by one work-group
                fl_b = torch.full_like(fl_a, float("nan"))
                s_b = torch.full_like(s_a, float("nan"))
                b = hydro.hydro_solve_periodic(st, gx, gy, gz, dt_dev, dh_dev, G53, fluxes_out=fl_b,
                                               group_stats=s_b, variant=v, grid=grid, zseg=zseg)
                torch.cuda.synchronize()
                what = (gx, gy, gz, v, grid, zseg)
                if dtype == torch.float64:
                    assert torch.equal(a, b), what
                    assert torch.equal(fl_a, fl_b), what
                    assert torch.equal(s_a, s_b), what
                else:
                    assert max_rel_diff(b, a) <= 1e-6, what
                    assert max_rel_diff(fl_b.reshape(n * 9, 5, 16, 16, 1), fl_a.reshape(n * 9, 5, 16, 16, 1)) <= 1e-6, what
                    assert max_rel_diff(s_b[:, :5, None, None, None], s_a[:, :5, None, None, None]) <= 1e-6, what
                    assert torch.equal(s_b[:, 6:], s_a[:, 6:]), what


@pytest.mark.parametrize("shape", [(2, 4, 8), (1, 1, 64), (1, 1, 1)])
def test_fused_fp64_against_oracle(gpu, shape):
    gx, gy, gz = shape
    st, dh = W.cosmo_like(n=64)
    st = st[: gx * gy * gz].contiguous()
    host = st.numpy()
    dt = oracle.cfl_dt(host, dh, G53, 0.5)
    pad = oracle.pack_periodic(host, gx, gy, gz)
    ref, ofl, cnt = oracle.hydro_solve(pad, dt, dh, G53, want_fluxes=True)
    n = st.shape[0]
    dt_dev = torch.tensor([dt], dtype=torch.float64, device=gpu)
    dh_dev = torch.tensor([dh], dtype=torch.float64, device=gpu)
    fl = torch.empty((n, 3, 3, 5, 16, 16), dtype=torch.float64, device=gpu)
    stats = torch.empty((n, 8), dtype=torch.float64, device=gpu)
    out = hydro.hydro_solve_periodic(st.to(gpu), gx, gy, gz, dt_dev, dh_dev, G53, fluxes_out=fl,
                                     group_stats=stats)
    torch.cuda.synchronize()
    # this 64^3 log-normal flow has cells beside 1e4 times their own energy:
    # the bar is per cell, relative to the size of the cell's update terms
    state_close(out.cpu().numpy(), ref, 1e-12, f"{shape} state", terms=update_terms(pad, dt, dh))
    flux_close(fl.cpu().numpy().transpose(0, 3, 1, 2, 4, 5), ofl.transpose(0, 3, 1, 2, 4, 5), 1e-12,
               f"{shape} fluxes")
    s = stats.cpu().numpy()
    assert (int(s[:, 6].sum()), int(s[:, 7].sum())) == cnt


def test_fused_fp32_against_oracle(gpu):
    gx, gy, gz = 2, 4, 8
    st, dh = W.cosmo_like(n=64)
    s32 = st.float()
    host = s32.double().numpy()
    dt = oracle.cfl_dt(host, dh, G53, 0.5)
    ref, _, _ = oracle.hydro_solve(oracle.pack_periodic(host, gx, gy, gz), dt, dh, G53)
    dt_dev = torch.tensor([dt], dtype=torch.float64, device=gpu)
    dh_dev = torch.tensor([dh], dtype=torch.float64, device=gpu)
    out = hydro.hydro_solve_periodic(s32.to(gpu), gx, gy, gz, dt_dev, dh_dev, G53)
    assert np.all(l1_rel(out.cpu().numpy(), ref) < 1e-5), l1_rel(out.cpu().numpy(), ref)


def test_fused_full_size_matches_batched(gpu):
    """256^3 log-normal flow (4096 groups): the fused step is bitwise the packed
    one, and 64 sampled groups match the oracle in FP64."""
    st, dh = W.cosmo_like(n=256)
    g = 16
    host = st.numpy()
    dt = oracle.cfl_dt(host, dh, G53, 0.5)
    dt_dev = torch.tensor([dt], dtype=torch.float64, device=gpu)
    dh_dev = torch.tensor([dh], dtype=torch.float64, device=gpu)
    s = st.to(gpu)
    a = hydro.hydro_solve_batched(hydro.pack_periodic(s, g, g, g), None, dt_dev, dh_dev, G53)
    b = hydro.hydro_solve_periodic(s, g, g, g, dt_dev, dh_dev, G53)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    pick = sorted(int(x) for x in np.random.default_rng(41).choice(g ** 3, size=64, replace=False))
    ref, _, _ = oracle.hydro_solve(oracle.pack_periodic_subset(host, g, g, g, pick), dt, dh, G53)
    state_close(b[torch.as_tensor(pick, device=gpu)].cpu().numpy(), ref, 1e-12, "fused 256^3 fp64")


def test_binding_rejects_aliasing_and_bad_shape(gpu):
    st, dh = _state(torch.float64, gpu)
    dt_dev = torch.tensor([1e-4], dtype=torch.float64, device=gpu)
    dh_dev = torch.tensor([dh], dtype=torch.float64, device=gpu)
    with pytest.raises(ValueError):
        hydro.hydro_solve_periodic(st, 4, 4, 3, dt_dev, dh_dev, G53)
    from paper_1007_3818_amd._native import GamerError
    with pytest.raises(GamerError):
        hydro.hydro_solve_periodic(st, 4, 4, 4, dt_dev, dh_dev, G53, out=st)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_periodic_grid_paths_agree(gpu, dtype):
    """PeriodicGrid with and without the fused step: 6 steps of the Sod tube give
    the same state, time and totals (FP64 bitwise, FP32 to 1e-6), eagerly and
    from a captured graph."""
    st, dh = W.sod_x()
    st = st.to(dtype).to(gpu)
    a = PeriodicGrid(st, 2, 2, 2, dh, G53, 0.5, fused=False)
    a.step(6)
    b = PeriodicGrid(st, 2, 2, 2, dh, G53, 0.5, fused=True)
    b.step(6)
    c = PeriodicGrid(st, 2, 2, 2, dh, G53, 0.5, fused=True).capture()  # 2 eager steps
    c.step(4)
    torch.cuda.synchronize()
    for g in (b, c):
        if dtype == torch.float64:
            assert torch.equal(g.current, a.current)
            assert g.time() == a.time()
            assert torch.equal(g.totals, a.totals)
        else:
            assert max_rel_diff(g.current, a.current) <= 1e-6
            assert abs(g.time() - a.time()) <= 1e-6 * a.time()
            assert torch.equal(g.totals[5:], a.totals[5:])
    assert torch.equal(c.current, b.current)  # graph replay equals eager, bitwise
