"""The solver's method variants on the GPU, through the C ABI: characteristic
limiting (gamer_opts.limiting) and FP64 state with FP32 arithmetic
(gamer_hydro_solve_*_mixed).

Bars:
  * characteristic limiting: FP64 within 1e-12 of the oracle's characteristic
    limiting per cell (rho and E against the cell's own value, momenta against |m| + rho c_s), fallback counts exact, in every
    compiled variant; FP32 within 1e-5 in L1 per variable; the fused periodic
    step equal to ghost fill + batched step in FP64 within 1e-13 per cell (two
    instantiations that may contract multiply-adds differently), with equal
    fallback counts;
  * FP64 state, FP32 arithmetic: against the FP64 oracle within the FP32 bars
    (1e-5 relative on smooth flow, L1 1e-5 on the Mach-10 flow); within 1e-6 of
    the FP32 path on float-representable input; totals conserved over 20 steps
    to 1e-13 relative (the state is double), where the FP32 path drifts.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1007_3818_amd import hydro, workloads as W
from paper_1007_3818_amd.autotune import max_rel_diff
from parity import flux_close, l1_rel, state_close, update_terms

pytestmark = pytest.mark.gpu
G53 = 5.0 / 3.0


CASES = {
    "sod": (lambda: W.sod_x(), (2, 2, 2)),
    "smooth48": (lambda: W.smooth_modes(n=48), (3, 3, 3)),
    "cosmo32": (lambda: W.cosmo_like(n=32), (2, 2, 2)),
}


def dev1(x, gpu):
    return torch.tensor([x], dtype=torch.float64, device=gpu)


@pytest.mark.parametrize("name", list(CASES))
def test_characteristic_limiting_fp64(gpu, name):
    (st, dh), (gx, gy, gz) = CASES[name][0](), CASES[name][1]
    host = st.numpy()
    dt = oracle.cfl_dt(host, dh, G53, 0.5)
    ref, ofl, cnt = oracle.hydro_solve(oracle.pack_periodic(host, gx, gy, gz), dt, dh, G53, want_fluxes=True,
                                       limiting="characteristic")
    prim, _, _ = oracle.hydro_solve(oracle.pack_periodic(host, gx, gy, gz), dt, dh, G53)
    n = host.shape[0]
    pad = hydro.pack_periodic(st.to(gpu), gx, gy, gz)
    for v in range(len(hydro.solver_variants(torch.float64))):
        fl = torch.empty((n, 3, 3, 5, 16, 16), dtype=torch.float64, device=gpu)
        stats = torch.empty((n, 8), dtype=torch.float64, device=gpu)
        out = hydro.hydro_solve_batched(pad, None, dev1(dt, gpu), dev1(dh, gpu), G53, fluxes_out=fl,
                                        group_stats=stats, variant=v, limiting="characteristic")
        state_close(out.cpu().numpy(), ref, 1e-12, f"{name} v{v}")
        flux_close(fl.cpu().numpy().transpose(0, 3, 1, 2, 4, 5), ofl.transpose(0, 3, 1, 2, 4, 5), 1e-12,
              f"{name} v{v} fluxes")
        s = stats.cpu().numpy()
        assert (int(s[:, 6].sum()), int(s[:, 7].sum())) == cnt
        fstats = torch.empty((n, 8), dtype=torch.float64, device=gpu)
        fused = hydro.hydro_solve_periodic(st.to(gpu), gx, gy, gz, dev1(dt, gpu), dev1(dh, gpu), G53,
                                           variant=v, limiting="characteristic", group_stats=fstats)
        # The periodic and padded instantiations of the characteristic-limiting
        # kernel may contract different multiply-adds (measured: differences of
        # at most 2.2e-16 of a cell's own scale on the smooth flow, 1e-14 on the
        # log-normal one), so they agree to rounding, with exactly equal counts.
        state_close(fused.cpu().numpy(), out.cpu().numpy(), 1e-13, f"{name} v{v} periodic vs padded",
                    terms=update_terms(oracle.pack_periodic(host, gx, gy, gz), dt, dh))
        assert torch.equal(fstats[:, 6:], stats[:, 6:])
    if name == "cosmo32":  # the limitings differ where waves interact (not from the
        assert np.abs(ref - prim).max() > 1e-8  # piecewise-constant Sod start: all slopes vanish)


@pytest.mark.parametrize("name", ["sod", "cosmo32"])
def test_characteristic_limiting_fp32(gpu, name):
    (st, dh), (gx, gy, gz) = CASES[name][0](), CASES[name][1]
    s32 = st.float()
    host = s32.double().numpy()
    dt = oracle.cfl_dt(host, dh, G53, 0.5)
    ref, _, _ = oracle.hydro_solve(oracle.pack_periodic(host, gx, gy, gz), dt, dh, G53,
                                   limiting="characteristic")
    for v in range(len(hydro.solver_variants(torch.float32))):
        out = hydro.hydro_solve_batched(hydro.pack_periodic(s32.to(gpu), gx, gy, gz), None, dev1(dt, gpu),
                                        dev1(dh, gpu), G53, variant=v, limiting="characteristic")
        assert np.all(l1_rel(out.cpu().numpy(), ref) < 1e-5), (v, l1_rel(out.cpu().numpy(), ref))


@pytest.mark.parametrize("limiting", ["primitive", "characteristic"])
def test_mixed_precision_one_step(gpu, limiting):
    for name in ("smooth48", "cosmo32"):
        (st, dh), (gx, gy, gz) = CASES[name][0](), CASES[name][1]
        host = st.numpy()
        dt = oracle.cfl_dt(host, dh, G53, 0.5)
        ref, _, cnt = oracle.hydro_solve(oracle.pack_periodic(host, gx, gy, gz), dt, dh, G53, limiting=limiting)
        n = host.shape[0]
        for v in range(len(hydro.solver_variants(torch.float32))):
            stats = torch.empty((n, 8), dtype=torch.float64, device=gpu)
            out = hydro.hydro_solve_periodic(st.to(gpu), gx, gy, gz, dev1(dt, gpu), dev1(dh, gpu), G53,
                                             group_stats=stats, variant=v, limiting=limiting,
                                             compute=torch.float32)
            assert out.dtype == torch.float64
            if name == "smooth48":
                state_close(out.cpu().numpy(), ref, 1e-5, f"mixed {name} v{v}")
            else:
                assert np.all(l1_rel(out.cpu().numpy(), ref) < 1e-5), (v, l1_rel(out.cpu().numpy(), ref))
            # on float-representable input the arithmetic is the FP32 path's
            s32 = st.float().to(gpu)
            a = hydro.hydro_solve_periodic(s32.double(), gx, gy, gz, dev1(dt, gpu), dev1(dh, gpu), G53,
                                           variant=v, limiting=limiting, compute=torch.float32)
            b = hydro.hydro_solve_periodic(s32, gx, gy, gz, dev1(dt, gpu), dev1(dh, gpu), G53, variant=v,
                                           limiting=limiting)
            assert max_rel_diff(a, b.double()) <= 1e-6, (name, v)


def test_mixed_precision_conserves_in_double(gpu):
    """20 steps of the Mach-10 log-normal flow: FP64-state totals drift by
    <= 1e-13 relative; the FP32 path's totals by far more."""
    st, dh = W.cosmo_like(n=32)
    g = 2
    dt = dev1(0.5 * oracle.cfl_dt(st.numpy(), dh, G53, 0.5), gpu)
    dhd = dev1(dh, gpu)
    a = st.to(gpu)
    b = st.float().to(gpu)
    t0a = np.array(hydro.conserved_sums(a, dh))
    t0b = np.array(hydro.conserved_sums(b, dh))
    scale = np.abs(st.numpy()).sum(axis=(0, 2, 3, 4)) * dh ** 3
    for _ in range(20):
        a = hydro.hydro_solve_periodic(a, g, g, g, dt, dhd, G53, compute=torch.float32)
        b = hydro.hydro_solve_periodic(b, g, g, g, dt, dhd, G53)
    da = np.abs(np.array(hydro.conserved_sums(a, dh)) - t0a) / scale
    db = np.abs(np.array(hydro.conserved_sums(b, dh)) - t0b) / scale
    assert np.all(da <= 1e-13), da
    assert db.max() > 10 * max(da.max(), 1e-16), (da, db)


def test_mixed_batched_equals_periodic(gpu):
    st, dh = W.smooth_modes(n=48)
    s = st.to(gpu)
    dt, dhd = dev1(1e-3, gpu), dev1(dh, gpu)
    for v in range(len(hydro.solver_variants(torch.float32))):
        a = hydro.hydro_solve_batched(hydro.pack_periodic(s, 3, 3, 3), None, dt, dhd, G53, variant=v,
                                      compute=torch.float32)
        b = hydro.hydro_solve_periodic(s, 3, 3, 3, dt, dhd, G53, variant=v, compute=torch.float32)
        assert max_rel_diff(b, a) <= 1e-6, v
