"""Pin of the oracle's unsplit three-direction coupling (CPU only).

The paper applies MUSCL-Hancock unsplit in 3D.  In the conservative Hancock
predictor read here, every face state of a cell receives the same half-step
increment S = dt/(2dh) sum_d [F_d(U^{d,-}) - F_d(U^{d,+})], summed over all three
directions.  A wave travelling along one axis cannot tell whether the
transverse terms are there, since they vanish; a wave travelling obliquely
can: the scheme is second order only when each face state is advanced by the
flux differences of every direction.  So an oblique density wave,
rho = 1 + 0.2 sin(2 pi (x_a + x_b)) advected at unit velocity along both axes
of a coordinate plane with p = 1, must converge at second order against the
exact translated solution, along each of the three diagonal planes.
"""
import math

import numpy as np
import pytest
import torch

from oracle_driver import from_global, run_periodic, to_global
from paper_1007_3818_amd import workloads as W

G53 = 5.0 / 3.0


def _oblique_wave(N, plane):
    """Global (5, NZ, NY, NX) state of the wave in the (a, b) coordinate plane,
    N cells along a and b, 16 along the third axis, and the grid in groups."""
    a, b = plane
    n = [16, 16, 16]
    n[a] = n[b] = N
    dims = (n[2], n[1], n[0])  # (z, y, x)
    coords = [(np.arange(m) + 0.5) / m for m in n]
    Z, Y, X = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
    xyz = (X, Y, Z)
    rho = 1 + 0.2 * np.sin(2 * np.pi * (xyz[a] + xyz[b]))
    vel = [torch.zeros(dims, dtype=torch.float64) for _ in range(3)]
    vel[a] += 1.0
    vel[b] += 1.0
    U = W.conserved(torch.from_numpy(rho), *vel, torch.ones(dims, dtype=torch.float64), G53).numpy()
    g = (n[0] // 16, n[1] // 16, n[2] // 16)
    return from_global(U, *g), g, xyz, (a, b)


@pytest.mark.parametrize("plane", [(0, 1), (1, 2), (2, 0)], ids=["xy", "yz", "zx"])
def test_oblique_wave_second_order(plane):
    t_end = 0.1
    errs = []
    for N in (32, 64):
        st, g, xyz, (a, b) = _oblique_wave(N, plane)
        h = 1.0 / N
        s, t, n, counts = run_periodic(st, *g, h, G53, 0.5, t_end=t_end)
        assert counts == (0, 0)
        rho = to_global(s, *g)[0]
        # exact cell average of sin(k (x_a + x_b - 2t)) over a cell of side h in
        # the plane: the point value times sinc(k h / 2)^2 (uniform along the
        # third axis)
        k = 2 * np.pi
        exact = 1 + 0.2 * np.sin(k * (xyz[a] + xyz[b] - 2 * t)) * (np.sin(k * h / 2) / (k * h / 2)) ** 2
        errs.append(np.abs(rho - exact).mean())
    order = math.log2(errs[0] / errs[1])
    assert order >= 1.8, (order, errs)
