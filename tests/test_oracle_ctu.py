"""Pins of the oracle's corner-transport-upwind (CTU) coupling (CPU only).

  * a uniform state is kept bitwise; totals are conserved on a periodic grid;
  * on a state that varies along one axis only the transverse Roe fluxes
    cancel exactly, so CTU gives bitwise the default (Hancock) result, along
    every axis;
  * on a 3D flow it differs from the default coupling;
  * x <-> y mirror symmetry holds (to rounding);
  * an oblique density wave converges at second order, against the exact
    translated solution.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle_driver import from_global, to_global
from paper_1007_3818_amd import workloads as W

G53 = 5.0 / 3.0


def run(state, g, dh, coupling, steps=None, t_end=None, cfl=0.4):
    s = np.ascontiguousarray(state, dtype=np.float64)
    t, n = 0.0, 0
    while (steps is None or n < steps) and (t_end is None or t < t_end * (1 - 1e-14)):
        dt = oracle.cfl_dt(s, dh, G53, cfl)
        if t_end is not None:
            dt = min(dt, t_end - t)
        s, _ = oracle.step_periodic(s, *g, dt, dh, G53, coupling=coupling)
        t += dt
        n += 1
    return s, t


def test_uniform_and_conservative():
    U = oracle.cons_from_prim([0.7, 0.3, -1.1, 2.0, 1.9], G53)
    pad = np.broadcast_to(U[None, :, None, None, None], (2, 5, 20, 20, 20)).copy()
    out, _, cnt = oracle.hydro_solve(pad, 0.01, 0.1, G53, coupling="ctu")
    assert np.array_equal(out, pad[:, :, 2:18, 2:18, 2:18]) and cnt == (0, 0)
    st, dh = W.cosmo_like(n=32)
    s0 = st.numpy()
    s, _ = run(s0, (2, 2, 2), dh, "ctu", steps=4)
    a, b = oracle.conserved_sums(s0, dh), oracle.conserved_sums(s, dh)
    scale = dh ** 3 * np.abs(s0).reshape(s0.shape[0], 5, -1).sum(axis=(0, 2))
    assert np.all(np.abs(b - a) <= 1e-13 * scale)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_one_dimensional_states_equal_hancock(axis):
    st, dh = W.sod_x(axis=axis)
    s0 = st.numpy()
    a, _ = run(s0, (2, 2, 2), dh, "ctu", steps=5)
    b, _ = run(s0, (2, 2, 2), dh, "hancock", steps=5)
    assert np.array_equal(a, b)


def test_three_dimensional_flow_differs_and_mirror_symmetry():
    st, dh = W.smooth_modes(n=32, kmax=2, workload=2)
    s0 = st.numpy()
    dt = oracle.cfl_dt(s0, dh, G53, 0.4)
    a, _ = oracle.step_periodic(s0, 2, 2, 2, dt, dh, G53, coupling="ctu")
    b, _ = oracle.step_periodic(s0, 2, 2, 2, dt, dh, G53)
    assert np.abs(a - b).max() > 1e-8

    def mirror(groups):  # swap x and y (axes and momenta)
        G = to_global(groups, 2, 2, 2).transpose(0, 1, 3, 2)[[0, 2, 1, 3, 4]]
        return from_global(np.ascontiguousarray(G), 2, 2, 2)

    m, _ = oracle.step_periodic(mirror(s0), 2, 2, 2, dt, dh, G53, coupling="ctu")
    scale = np.abs(a).max(axis=(0, 2, 3, 4), keepdims=True)
    assert np.all(np.abs(mirror(m) - a) <= 1e-13 * scale)


def _oblique_wave(N):
    """rho = 1 + 0.2 sin(2 pi (x + y)), u = v = 1, p = 1 on an N x N x 16 box."""
    h = 1.0 / N
    x = (np.arange(N) + 0.5) * h
    X, Y = np.meshgrid(x, x, indexing="xy")  # [y][x]
    rho2 = 1 + 0.2 * np.sin(2 * np.pi * (X + Y))
    dims = (16, N, N)
    rho = torch.from_numpy(np.broadcast_to(rho2, dims).copy())
    one = torch.ones(dims, dtype=torch.float64)
    z = torch.zeros(dims, dtype=torch.float64)
    return from_global(W.conserved(rho, one, one, z, one, G53).numpy(), N // 16, N // 16, 1), x


def test_oblique_wave_second_order():
    t_end = 0.1
    errs = []
    for N in (32, 64):
        st, x = _oblique_wave(N)
        h = 1.0 / N
        s, t = run(st, (N // 16, N // 16, 1), h, "ctu", t_end=t_end)
        rho = to_global(s, N // 16, N // 16, 1)[0, 0]
        # exact cell average of sin(2 pi (x + y - 2t)) over each square cell
        X, Y = np.meshgrid(x, x, indexing="xy")
        k = 2 * np.pi
        avg = (np.sin(k * (X + Y - 2 * t)) * (np.sin(k * h / 2) / (k * h / 2)) ** 2)
        errs.append(np.abs(rho - (1 + 0.2 * avg)).mean())
    order = math.log2(errs[0] / errs[1])
    assert order >= 1.8, (order, errs)
