"""The boundary's guard rails on the GPU, through the C ABI.

  * A level byte outside [0, n_levels) is never used as an index: the group is
    advanced with NaN dt and dh, so its output block and stats row are NaN, it is
    counted in bad_count_dev[1], and the other groups are unaffected.  The same
    holds in the CTU and relaxing-TVD steps; the reduction leaves such a group
    out of every level's dt and makes the totals NaN.
  * An output cell that is not physical (p <= 0 here) is counted in
    bad_count_dev[0], and the group's signal speed, hence the level's dt, is NaN
    (the oracle's CFL time step of the same output is NaN too).
  * The batched entry point launches on the stream passed to it.
Inputs are in-range arrays; a bad level byte or a negative pressure is data,
which the kernels handle without any data-dependent address.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1007_3818_amd import hydro, workloads as W
from parity import state_close

pytestmark = pytest.mark.gpu
G53 = 5.0 / 3.0

LEVELS = np.array([0, 1, 0, 5, 1, -3, 0, 1], dtype=np.int8)  # n_levels = 2: groups 3 and 5 are bad
BAD = LEVELS >= 2
BAD |= LEVELS < 0


def _batch():
    st, dh = W.smooth_modes(n=32)
    return oracle.pack_periodic(st.numpy(), 2, 2, 2), [2e-3, 1e-3], [dh, 0.5 * dh]


def _dev(a, gpu, dtype=torch.float64):
    return torch.as_tensor(np.asarray(a), dtype=dtype).to(gpu)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_bad_level_counted_and_isolated(gpu, dtype):
    P, dts, dhs = _batch()
    lev = torch.from_numpy(LEVELS).to(gpu)
    out = torch.full((8, 5, 16, 16, 16), 7.0, dtype=dtype, device=gpu)
    stats = torch.empty((8, 8), dtype=torch.float64, device=gpu)
    bad = torch.zeros(2, dtype=torch.int64, device=gpu)
    dt_dev, dh_dev = _dev(dts, gpu), _dev(dhs, gpu)
    hydro.hydro_solve_batched(_dev(P, gpu, dtype), lev, dt_dev, dh_dev, G53, out=out, group_stats=stats,
                              bad_count=bad)
    o = out.cpu().double().numpy()
    s = stats.cpu().numpy()
    b = bad.cpu().tolist()
    print(f"[boundary] {dtype}: bad counts {b}", flush=True)
    assert b == [2 * 16 ** 3, 2]  # every cell of the two skipped groups is NaN
    assert np.isnan(o[BAD]).all()
    assert np.isnan(s[BAD][:, :6]).all()
    for L in (0, 1):
        sel = LEVELS == L
        Pin = P[sel] if dtype == torch.float64 else P[sel].astype(np.float32).astype(np.float64)
        ref, _, _ = oracle.hydro_solve(Pin, dts[L], dhs[L], G53)
        state_close(o[sel], ref, 1e-12 if dtype == torch.float64 else 1e-5, f"level {L} beside bad groups")
    # the reduction: dt of each level from its good groups only, totals NaN
    dt_out, tot = hydro.step_reduce(stats, lev, dh_dev, 0.5)
    for L in (0, 1):
        want = oracle.cfl_dt(o[LEVELS == L], dhs[L], G53, 0.5)
        assert float(dt_out[L]) == pytest.approx(want, rel=4e-15 if dtype == torch.float64 else 1e-6)
    assert np.isnan(tot[:5].cpu().numpy()).all()


def test_bad_level_ctu_and_rtvd(gpu):
    P, dts, dhs = _batch()
    lev = torch.from_numpy(LEVELS).to(gpu)
    dt_dev, dh_dev = _dev(dts, gpu), _dev(dhs, gpu)
    bad = torch.zeros(2, dtype=torch.int64, device=gpu)
    out = hydro.ctu_solve_batched(_dev(P, gpu), lev, dt_dev, dh_dev, G53, bad_count=bad)
    o = out.cpu().numpy()
    assert bad.cpu().tolist() == [2 * 16 ** 3, 2]
    assert np.isnan(o[BAD]).all()
    for L in (0, 1):
        sel = LEVELS == L
        ref, _, _ = oracle.hydro_solve(P[sel], dts[L], dhs[L], G53, coupling="ctu")
        state_close(o[sel], ref, 1e-12, f"ctu level {L} beside bad groups")
    # relaxing TVD: three ghost cells per side
    st, dh = W.smooth_modes(n=32)
    R = oracle.pack_periodic_rtvd(st.numpy(), 2, 2, 2)
    out = hydro.rtvd_solve_batched(_dev(R, gpu), lev, dt_dev, dh_dev, G53, order=0)
    o = out.cpu().numpy()
    assert np.isnan(o[BAD]).all()
    for L in (0, 1):
        sel = LEVELS == L
        ref, _ = oracle.rtvd_solve(R[sel], dts[L], dhs[L], G53, 0)
        state_close(o[sel], ref, 1e-12, f"rtvd level {L} beside bad groups")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_nonphysical_output_counted_and_dt_nan(gpu, dtype):
    """A uniform flow with one interior cell of negative pressure: after a short
    step that cell is still not physical; it is counted, the group's signal speed
    is NaN and so is the level's dt; the other group is clean."""
    U = oracle.cons_from_prim([1.0, 0.5, 0.0, 0.0, 1.0], G53)
    pad = np.broadcast_to(U[None, :, None, None, None], (2, 5, 20, 20, 20)).copy()
    pad[1, 4, 10, 10, 10] = 0.5 * 0.25 - 0.1  # E below the kinetic energy: p < 0
    dt_dev, dh_dev = _dev([1e-4], gpu), _dev([0.1], gpu)
    stats = torch.empty((2, 8), dtype=torch.float64, device=gpu)
    bad = torch.zeros(2, dtype=torch.int64, device=gpu)
    out = hydro.hydro_solve_batched(_dev(pad, gpu, dtype), None, dt_dev, dh_dev, G53, group_stats=stats,
                                    bad_count=bad)
    b = bad.cpu().tolist()
    s = stats.cpu().numpy()
    print(f"[boundary] {dtype}: non-physical output cells {b[0]}", flush=True)
    assert b[0] >= 1 and b[1] == 0
    assert np.isfinite(s[0, 5]) and np.isnan(s[1, 5])
    dt_out, _ = hydro.step_reduce(stats, None, dh_dev, 0.5)
    assert np.isnan(float(dt_out[0]))
    o = out.cpu().double().numpy()
    assert np.isnan(oracle.cfl_dt(o, 0.1, G53, 0.5))
    assert np.isnan(hydro.cfl_dt(out, 0.1, G53, 0.5))
    # the clean group: a uniform state stays uniform bitwise
    assert np.array_equal(o[0], pad[0, :, 2:18, 2:18, 2:18].astype(o.dtype) if dtype == torch.float64
                          else pad[0, :, 2:18, 2:18, 2:18].astype(np.float32).astype(np.float64))


def test_explicit_stream_argument(gpu):
    """The batched step runs on the stream it is given (a second, default-priority
    stream here) and gives the same bits as on the default stream."""
    P, dts, dhs = _batch()
    p = _dev(P, gpu)
    dt_dev, dh_dev = _dev(dts[:1], gpu), _dev(dhs[:1], gpu)
    ref = hydro.hydro_solve_batched(p, None, dt_dev, dh_dev, G53)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        out = torch.empty_like(ref)
        hydro.hydro_solve_batched(p, None, dt_dev, dh_dev, G53, out=out)
    side.synchronize()
    assert torch.equal(out, ref)
