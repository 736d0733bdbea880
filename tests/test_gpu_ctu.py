"""The corner-transport-upwind (CTU) variant on the GPU, through the C ABI,
against the oracle's CTU step.

Bars: FP64 within 1e-12 relative per cell (tests/parity.py), flux planes per
value; fallback counts equal to the oracle's up to the number of the oracle's
decisions that sit within a relative margin of 1e-9 (about 4.5e6 ulp) of their
threshold, which a different rounding may take the other way (on these inputs
there are none, so the counts must be equal); FP32 within 1e-5 in L1 per
variable (oracle on the float-rounded input); a 1D state gives the default
path's result in FP64 to 1e-13 (the transverse fluxes cancel exactly; the two
are separate compilations); per-level dt and dh read on the device.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1007_3818_amd import hydro, workloads as W
from parity import flux_close, l1_rel, state_close, update_terms

pytestmark = pytest.mark.gpu
G53 = 5.0 / 3.0


def dev1(x, gpu):
    return torch.tensor([x], dtype=torch.float64, device=gpu)


CASES = {
    "smooth48": (lambda: W.smooth_modes(n=48), (3, 3, 3)),
    "cosmo32": (lambda: W.cosmo_like(n=32), (2, 2, 2)),
}


VARIANTS = [hydro.CTU_FUSED, hydro.CTU_PIPELINE]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", list(CASES))
def test_ctu_fp64(gpu, name, variant):
    (st, dh), (gx, gy, gz) = CASES[name][0](), CASES[name][1]
    host = st.numpy()
    dt = oracle.cfl_dt(host, dh, G53, 0.4)
    pad_h = oracle.pack_periodic(host, gx, gy, gz)
    (ref, ofl, cnt), borderline = oracle.borderline_decisions(
        lambda: oracle.hydro_solve(pad_h, dt, dh, G53, want_fluxes=True, coupling="ctu"), 1e-9)
    n = host.shape[0]
    pad = hydro.pack_periodic(st.to(gpu), gx, gy, gz)
    fl = torch.empty((n, 3, 3, 5, 16, 16), dtype=torch.float64, device=gpu)
    stats = torch.empty((n, 8), dtype=torch.float64, device=gpu)
    out = hydro.ctu_solve_batched(pad, None, dev1(dt, gpu), dev1(dh, gpu), G53, fluxes_out=fl,
                                  group_stats=stats, variant=variant)
    state_close(out.cpu().numpy(), ref, 1e-12, f"{name} v{variant} state")
    flux_close(fl.cpu().numpy().transpose(0, 3, 1, 2, 4, 5), ofl.transpose(0, 3, 1, 2, 4, 5), 1e-12,
               f"{name} fluxes")
    s = stats.cpu().numpy()
    got = (int(s[:, 6].sum()), int(s[:, 7].sum()))
    print(f"[parity] {name}: fallbacks gpu {got} oracle {cnt}, borderline decisions {borderline}")
    # a decision may differ only where the oracle's own decision is borderline
    assert abs(got[0] - cnt[0]) + abs(got[1] - cnt[1]) <= borderline, (got, cnt, borderline)
    scale = np.abs(ref).sum(axis=(0, 2, 3, 4))
    assert np.all(np.abs(s[:, :5].sum(axis=0) - ref.sum(axis=(0, 2, 3, 4))) <= 1e-12 * scale)


@pytest.mark.parametrize("variant", VARIANTS)
def test_ctu_fp32(gpu, variant):
    st, dh = W.cosmo_like(n=32)
    s32 = st.float()
    host = s32.double().numpy()
    dt = oracle.cfl_dt(host, dh, G53, 0.4)
    ref, _, _ = oracle.hydro_solve(oracle.pack_periodic(host, 2, 2, 2), dt, dh, G53, coupling="ctu")
    out = hydro.ctu_solve_batched(hydro.pack_periodic(s32.to(gpu), 2, 2, 2), None, dev1(dt, gpu),
                                  dev1(dh, gpu), G53, variant=variant)
    l1 = l1_rel(out.cpu().numpy(), ref)
    print(f"[parity] ctu fp32 v{variant}: L1 per variable {l1}", flush=True)
    assert np.all(l1 < 1e-5), l1


@pytest.mark.parametrize("variant", VARIANTS)
def test_ctu_one_dimensional_equals_default(gpu, variant):
    st, dh = W.sod_x(axis=1)
    pad = hydro.pack_periodic(st.to(gpu), 2, 2, 2)
    dt_dev, dh_dev = dev1(0.2 * dh, gpu), dev1(dh, gpu)
    a = hydro.ctu_solve_batched(pad, None, dt_dev, dh_dev, G53, variant=variant)
    b = hydro.hydro_solve_batched(pad, None, dt_dev, dh_dev, G53)
    from paper_1007_3818_amd.autotune import max_rel_diff
    assert max_rel_diff(a, b) <= 1e-13


@pytest.mark.parametrize("variant", VARIANTS)
def test_ctu_levels(gpu, variant):
    st, dh = W.smooth_modes(n=32, kmax=2, workload=2)
    host = st.numpy()
    pad_h = oracle.pack_periodic(host, 2, 2, 2)
    dts, dhs = [1e-3, 4e-4], [dh, 0.5 * dh]
    level = np.array([0, 1, 1, 0, 1, 0, 0, 1], dtype=np.int8)
    ref = np.empty((8, 5, 16, 16, 16))
    for L in (0, 1):
        sel = level == L
        ref[sel], _, _ = oracle.hydro_solve(pad_h[sel], dts[L], dhs[L], G53, coupling="ctu")
    out = hydro.ctu_solve_batched(hydro.pack_periodic(st.to(gpu), 2, 2, 2), torch.from_numpy(level).to(gpu),
                                  torch.tensor(dts, dtype=torch.float64, device=gpu),
                                  torch.tensor(dhs, dtype=torch.float64, device=gpu), G53, variant=variant)
    state_close(out.cpu().numpy(), ref, 1e-12, f"two levels v{variant}")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_ctu_fused_equals_pipeline(gpu, dtype):
    """The fused sweep and the pipeline compute the same arithmetic in another
    order of launches (the compiler may contract multiply-adds differently in
    the two): per cell relative to the larger of the cell's own scale and its
    update terms (the 48^3 log-normal flow has strong contrasts), FP64 within
    1e-13 and FP32 within 1e-5; the same fallback counts."""
    st, dh = W.cosmo_like(n=48)
    host = st.numpy()
    dt = oracle.cfl_dt(host, dh, G53, 0.4)
    pad = hydro.pack_periodic(st.to(dtype).to(gpu), 3, 3, 3)
    res = []
    for v in VARIANTS:
        fl = torch.empty((27, 3, 3, 5, 16, 16), dtype=dtype, device=gpu)
        stats = torch.empty((27, 8), dtype=torch.float64, device=gpu)
        out = hydro.ctu_solve_batched(pad, None, dev1(dt, gpu), dev1(dh, gpu), G53, fluxes_out=fl,
                                      group_stats=stats, variant=v)
        res.append((out.cpu().double().numpy(), fl.cpu().double().numpy(), stats.cpu().numpy()))
    (a, fa, sa), (b, fb, sb) = res
    tol = 1e-13 if dtype == torch.float64 else 1e-5
    terms = update_terms(pad.cpu().double().numpy(), dt, dh)
    state_close(a, b, tol, f"ctu fused vs pipeline {dtype}", terms=terms)
    flux_close(fa.transpose(0, 3, 1, 2, 4, 5), fb.transpose(0, 3, 1, 2, 4, 5), tol, "ctu fluxes fused vs pipeline")
    assert np.array_equal(sa[:, 6:], sb[:, 6:])
    print(f"[parity] ctu fused vs pipeline {dtype}: bitwise {np.array_equal(a, b)}, fallbacks "
          f"{sa[:, 6].sum():.0f} / {sa[:, 7].sum():.0f}", flush=True)
