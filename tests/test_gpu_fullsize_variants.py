"""The CTU and relaxing-TVD paths at the full size of the 256^3 smooth-flow
workload (4096 groups), through the entry points and launches the bench times,
against the oracle on sampled groups: the eight corner groups of the grid and
eight random ones, whose padded inputs the oracle assembles itself from the
same seeded state.  FP64 within 1e-12
per cell (rho and E against the cell's own value, momenta against |m| + rho c_s); FP32 within 1e-5 in L1 per variable against the oracle run on
the float-rounded state.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1007_3818_amd import hydro, workloads as W
from parity import l1_rel, state_close

pytestmark = pytest.mark.gpu
G53 = 5.0 / 3.0
N = 256
G = N // 16


def sample():
    rng = np.random.default_rng(2)
    corners = [x + G * (y + G * z) for x in (0, G - 1) for y in (0, G - 1) for z in (0, G - 1)]
    return sorted(set(corners) | set(int(x) for x in rng.choice(G ** 3, size=8, replace=False)))


def dev1(x, gpu):
    return torch.tensor([x], dtype=torch.float64, device=gpu)


@pytest.mark.timeout(300)
def test_ctu_full_size_sampled(gpu):
    st, dh = W.smooth_modes(n=N, device=gpu)
    dt = 0.05 * dh
    pick = sample()
    idx = torch.as_tensor(pick, device=gpu)
    for s, what in ((st, "fp64"), (st.float(), "fp32")):
        ref, _, cnt = oracle.hydro_solve(oracle.pack_periodic_subset(s, G, G, G, pick), dt, dh, G53,
                                         coupling="ctu")
        assert cnt == (0, 0)
        stats = torch.empty((G ** 3, 8), dtype=torch.float64, device=gpu)
        out = hydro.ctu_solve_batched(hydro.pack_periodic(s, G, G, G), None, dev1(dt, gpu), dev1(dh, gpu),
                                      G53, group_stats=stats)
        got = out[idx].cpu().double().numpy()
        if what == "fp64":
            state_close(got, ref, 1e-12, "ctu 256^3 fp64")
        else:
            assert np.all(l1_rel(got, ref) < 1e-5), l1_rel(got, ref)
        assert int(stats[:, 6].sum()) == 0 and int(stats[:, 7].sum()) == 0
        del out, stats
        torch.cuda.empty_cache()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("order", [0, 1])
def test_rtvd_full_size_sampled(gpu, order):
    st, dh = W.smooth_modes(n=N, device=gpu)
    dt = 0.05 * dh
    pick = sample()
    idx = torch.as_tensor(pick, device=gpu)
    for s, what in ((st, "fp64"), (st.float(), "fp32")):
        ref, bad = oracle.rtvd_solve(oracle.pack_periodic_rtvd_subset(s, G, G, G, pick), dt, dh, G53, order)
        assert bad == 0
        out = hydro.rtvd_solve_periodic(s, G, G, G, dev1(dt, gpu), dev1(dh, gpu), G53, order)
        got = out[idx].cpu().double().numpy()
        if what == "fp64":
            state_close(got, ref, 1e-12, f"rtvd 256^3 order {order} fp64")
        else:
            assert np.all(l1_rel(got, ref) < 1e-5), l1_rel(got, ref)
        del out
        torch.cuda.empty_cache()
