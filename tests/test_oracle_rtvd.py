"""Pins of the relaxing-TVD oracle (CPU only).

  * van Leer's limiter: closed-form values (zero at extrema, a at a = b,
    symmetric, bounded by twice the smaller difference);
  * a uniform state is kept bitwise; totals are conserved on a periodic grid;
  * the three-cell ghost fill is the wrapped global field (brute force);
  * a 1D state computed along x, along y and along z gives the same numbers
    after permuting axes and momenta (sweep order reversed for z), and the
    sweeps across a 1D state leave it bitwise unchanged;
  * Sod's shock tube converges to the exact solution (the L1 error falls with
    resolution and is small);
  * a smooth density wave converges at second order with alternating sweep
    orders (the symmetric splitting), moving either way;
  * on a 3D flow the two sweep orders differ, and order 1 on the x<->z mirror
    image of a state is the mirror image of order 0 on the state (to rounding:
    the kinetic energy sums the momenta in another order).
"""
import math

import numpy as np
import pytest
import torch

import exact_riemann as er
import oracle
from oracle_driver import from_global, to_global
from paper_1007_3818_amd import workloads as W

G53 = 5.0 / 3.0


def run_rtvd(state, gx, gy, gz, dh, gamma=G53, cfl=0.4, steps=None, t_end=None):
    """Alternate sweep orders step by step; dt from the oracle's CFL function."""
    s = np.ascontiguousarray(state, dtype=np.float64)
    t, n, bad = 0.0, 0, 0
    while (steps is None or n < steps) and (t_end is None or t < t_end * (1 - 1e-14)):
        dt = oracle.cfl_dt(s, dh, gamma, cfl)
        if t_end is not None:
            dt = min(dt, t_end - t)
        s, b = oracle.rtvd_step_periodic(s, gx, gy, gz, dt, dh, gamma, order=n % 2)
        bad += b
        t += dt
        n += 1
    return s, t, n, bad


def test_vanleer_closed_form():
    r = np.random.default_rng(1)
    for _ in range(200):
        a, b = r.standard_normal(2)
        v = oracle.vanleer(a, b)
        if a * b <= 0:
            assert v == 0.0
        else:
            assert np.isclose(v, 2 * a * b / (a + b), rtol=1e-15)
            assert abs(v) <= 2 * min(abs(a), abs(b)) * (1 + 1e-15)
            assert np.sign(v) == np.sign(a)
        assert oracle.vanleer(b, a) == v
        assert np.isclose(oracle.vanleer(a, a), a, rtol=2e-16, atol=0)


def test_uniform_state_bitwise_and_pencil_identity():
    U = oracle.cons_from_prim([0.7, 0.3, -1.1, 2.0, 1.9], G53)
    pad = np.broadcast_to(U[None, :, None, None, None], (2, 5, 22, 22, 22)).copy()
    for order in (0, 1):
        out, bad = oracle.rtvd_solve(pad, 0.01, 0.1, G53, order)
        assert bad == 0
        assert np.array_equal(out, pad[:, :, 3:19, 3:19, 3:19])
    pen = np.broadcast_to(U, (10, 5)).copy()
    for d in range(3):
        out, _ = oracle.rtvd_pencil(pen, d, 0.1, G53)
        assert np.array_equal(out, pen[3:7])


def test_pack_rtvd_brute_force():
    r = np.random.default_rng(2)
    gx, gy, gz = 3, 2, 2
    st = r.standard_normal((gx * gy * gz, 5, 16, 16, 16))
    pad = oracle.pack_periodic_rtvd(st, gx, gy, gz)
    G = to_global(st, gx, gy, gz)
    for _ in range(300):
        g = int(r.integers(gx * gy * gz))
        i, j, k = r.integers(-3, 19, 3)
        bx, by, bz = g % gx, (g // gx) % gy, g // (gx * gy)
        X, Y, Z = (16 * bx + i) % (16 * gx), (16 * by + j) % (16 * gy), (16 * bz + k) % (16 * gz)
        assert np.array_equal(pad[g, :, k + 3, j + 3, i + 3], G[:, Z, Y, X])
    # the subset pack (sampled full-size tests) gives the same padded groups,
    # from numpy or torch input
    ids = [0, 5, 11, 7]
    assert np.array_equal(oracle.pack_periodic_rtvd_subset(st, gx, gy, gz, ids), pad[ids])
    assert np.array_equal(oracle.pack_periodic_rtvd_subset(torch.from_numpy(st), gx, gy, gz, ids), pad[ids])


def test_conservation_periodic():
    st, dh = W.smooth_modes(n=32, kmax=2, workload=2)
    s0 = st.numpy()
    s, t, n, bad = run_rtvd(s0, 2, 2, 2, dh, steps=6)
    assert bad == 0
    a, b = oracle.conserved_sums(s0, dh), oracle.conserved_sums(s, dh)
    scale = dh ** 3 * np.abs(s0).reshape(s0.shape[0], 5, -1).sum(axis=(0, 2))
    assert np.all(np.abs(b - a) <= 1e-13 * scale), (b - a) / scale


def _sod(axis, n=32):
    st, dh = W.sod_x(*[(n // 16 if a == axis else 1) for a in range(3)], axis=axis)
    return st.numpy(), dh


def test_axes_agree_and_transverse_sweeps_are_identity():
    """Sod along x (orders 0 and 1), y (order 0) and z (order 1 reverses the
    roles of x and z): bitwise equal after permuting axes and momenta."""
    res = {}
    for axis, order in ((0, 0), (0, 1), (1, 0), (2, 1), (2, 0)):
        st, dh = _sod(axis)
        g = [2 if a == axis else 1 for a in range(3)]
        dt = 0.4 * dh
        s = st
        for k in range(3):
            s, bad = oracle.rtvd_step_periodic(s, *g, dt, dh, G53, order=order)
            assert bad == 0
        G = to_global(s, *g)
        if axis == 1:
            G = G.transpose(0, 1, 3, 2)[[0, 2, 1, 3, 4]]
        elif axis == 2:
            G = G.transpose(0, 3, 2, 1)[[0, 3, 2, 1, 4]]
        res[(axis, order)] = G
    base = res[(0, 0)]
    for key, G in res.items():
        assert np.array_equal(G, base), key


def test_sod_against_exact_solution():
    left, right = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    t_end = 0.1
    errs = []
    for n in (64, 128):
        st, dh = _sod(0, n)
        s, t, steps, bad = run_rtvd(st, n // 16, 1, 1, dh, t_end=t_end)
        assert bad == 0
        rho = to_global(s, n // 16, 1, 1)[0, 0, 0]
        x = (np.arange(n) + 0.5) * dh
        # the tube's first discontinuity sits at x = 0.5 (the periodic seam at 0 is far)
        ex = np.array([er.sample(left, right, G53, (xi - 0.5) / t_end)[0] for xi in x])
        win = (x > 0.25) & (x < 0.75)
        errs.append(np.abs(rho - ex)[win].mean())
    assert errs[1] < 0.75 * errs[0], errs
    assert errs[1] < 0.02, errs


def _wave_state(N, u0=1.0):
    x = (np.arange(N) + 0.5) / N
    rho1 = 1 + 0.2 * np.sin(2 * np.pi * x)
    dims = (16, 16, N)
    rho = torch.from_numpy(np.broadcast_to(rho1, dims).copy())
    u = torch.full(dims, u0, dtype=torch.float64)
    z = torch.zeros(dims, dtype=torch.float64)
    p = torch.ones(dims, dtype=torch.float64)
    return from_global(W.conserved(rho, u, z, z, p, G53).numpy(), N // 16, 1, 1)


@pytest.mark.parametrize("u0", [1.0, -1.0])
def test_second_order_convergence(u0):
    t_end = 0.2
    errs = []
    for N in (32, 64, 128):
        st = _wave_state(N, u0)
        s, t, n, bad = run_rtvd(st, N // 16, 1, 1, 1.0 / N, t_end=t_end)
        assert bad == 0
        line = to_global(s, N // 16, 1, 1)[0, 0, 0]
        x = (np.arange(N) + 0.5) / N
        h = 1.0 / N
        xs = x - u0 * t
        exact = 1 + 0.2 * (np.cos(2 * np.pi * (xs - h / 2)) - np.cos(2 * np.pi * (xs + h / 2))) / (2 * np.pi * h)
        errs.append(np.abs(line - exact).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders) >= 1.8, (orders, errs)


def test_sweep_order_mirror_symmetry():
    st, dh = W.smooth_modes(n=32, kmax=2, workload=2)
    s = st.numpy()
    dt = oracle.cfl_dt(s, dh, G53, 0.4)
    a, _ = oracle.rtvd_step_periodic(s, 2, 2, 2, dt, dh, G53, order=0)
    b, _ = oracle.rtvd_step_periodic(s, 2, 2, 2, dt, dh, G53, order=1)
    assert np.abs(a - b).max() > 1e-10  # the orders differ on a 3D flow

    def mirror(groups):  # swap x and z (axes and momenta)
        G = to_global(groups, 2, 2, 2).transpose(0, 3, 2, 1)[[0, 3, 2, 1, 4]]
        return from_global(np.ascontiguousarray(G), 2, 2, 2)

    c, _ = oracle.rtvd_step_periodic(mirror(s), 2, 2, 2, dt, dh, G53, order=1)
    m = mirror(c)
    scale = np.abs(a).max(axis=(0, 2, 3, 4), keepdims=True)
    assert np.all(np.abs(m - a) <= 1e-13 * scale)
    assert np.abs(a - b).max() > 1e3 * np.abs(m - a).max()
