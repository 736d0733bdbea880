"""Seeded synthetic initial conditions shaped like the paper's hydro workloads.

This module only builds input states.  It holds none of the solver's
arithmetic and is the one piece of code that both the GPU path and the CPU
oracle consume (each then packs ghost zones and solves with its own code).

A uniform grid of Gx x Gy x Gz groups of 16^3 cells is stored as
``(G, 5, 16, 16, 16)`` conserved variables (rho, m_x, m_y, m_z, E), x fastest,
with group index g = gx + Gx (gy + Gy gz) and cell centres at (i + 1/2) dh.

Workloads (gamma = 5/3 throughout; random draws from numpy's PCG64 seeded
with 10073818 + workload number):
  1 ``sod_x``        Sod shock tube along x on a periodic 32^3 grid (8 groups).
  2 ``smooth_modes`` rho = 1 + 0.1 sum of 8 random Fourier modes, velocity of
                     8 modes per component scaled to rms |v| = 0.5 sqrt(gamma)
                     (Mach 0.5 at rho = p = 1), p = 1; 256^3 (4096 groups).
  3 ``sedov_amr``    three refinement levels (dh = 1, 1/2, 1/4) of a Sedov blast
                     (E = 1 in one cell, rho = 1, p = 1e-5), 512 + 4096 + 20000 groups.
  4 ``cosmo_like``   log-normal density from a Gaussian field with P(k) ~ k^-3,
                     rho = clip(exp(2 g), 1e-3, 1e4), velocity up to Mach 10,
                     p = 1e-2 rho^gamma; 256^3 (4096 groups).
  5 ``smooth_modes`` at 1024^3 (262144 groups) with wavenumbers up to 8.
The paper's own cosmological initial conditions are not available; workload 4
stands in for them.
"""
from __future__ import annotations

import math

import numpy as np
import torch

GAMMA = 5.0 / 3.0
SEED_BASE = 10073818
NI = 16


def rng(workload: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + workload))


def _to_groups(field: torch.Tensor, gx: int, gy: int, gz: int) -> torch.Tensor:
    """(5, NZ, NY, NX) global array -> (G, 5, 16, 16, 16) groups."""
    f = field.reshape(5, gz, NI, gy, NI, gx, NI)
    f = f.permute(1, 3, 5, 0, 2, 4, 6)  # gz, gy, gx, v, k, j, i
    return f.reshape(gx * gy * gz, 5, NI, NI, NI).contiguous()


def groups_to_global(groups: torch.Tensor, gx: int, gy: int, gz: int) -> torch.Tensor:
    """(G, 5, 16, 16, 16) -> (5, NZ, NY, NX)."""
    f = groups.reshape(gz, gy, gx, 5, NI, NI, NI).permute(3, 0, 4, 1, 5, 2, 6)
    return f.reshape(5, gz * NI, gy * NI, gx * NI).contiguous()


def conserved(rho, u, v, w, p, gamma=GAMMA) -> torch.Tensor:
    """Stack (rho, rho u, rho v, rho w, E) of an ideal gas, E = p/(gamma-1) + rho|u|^2/2."""
    e = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return torch.stack([rho, rho * u, rho * v, rho * w, e])


def sod_x(gx: int = 2, gy: int = 2, gz: int = 2, x0: float = 0.5, axis: int = 0,
          gamma: float = GAMMA, device="cpu"):
    """Workload 1: Sod tube on [0,1) along ``axis``: (rho, p) = (1, 1) where the cell
    centre coordinate is below x0, else (0.125, 0.1); v = 0.  Periodic, so a second,
    mirrored discontinuity sits at 0.  dh = 1 / (16 * groups along the axis)."""
    n = (gx, gy, gz)[axis] * NI
    dh = 1.0 / n
    shape = (gz * NI, gy * NI, gx * NI)
    c = (torch.arange(n, dtype=torch.float64, device=device) + 0.5) * dh
    left = c < x0
    view = [1, 1, 1]
    view[2 - axis] = n
    left = left.reshape(view).expand(shape)
    rho = torch.where(left, 1.0, 0.125).to(torch.float64)
    p = torch.where(left, 1.0, 0.1).to(torch.float64)
    z = torch.zeros(shape, dtype=torch.float64, device=device)
    return _to_groups(conserved(rho, z, z, z, p, gamma), gx, gy, gz), dh


def _pick_modes(r: np.random.Generator, count: int, kmax: int):
    """``count`` distinct integer wavevectors in {-kmax..kmax}^3 \\ {0}, no two equal up
    to sign (so the modes are orthogonal on the periodic unit cube), and phases."""
    seen, ks = set(), []
    while len(ks) < count:
        k = tuple(int(x) for x in r.integers(-kmax, kmax + 1, size=3))
        if k == (0, 0, 0) or k in seen or tuple(-x for x in k) in seen:
            continue
        seen.add(k)
        ks.append(k)
    phases = r.uniform(0.0, 2.0 * math.pi, size=count)
    return np.array(ks, dtype=np.int64), phases


def _mode_sum(ks, phases, nx, ny, nz, device, z_lo=0, z_hi=None):
    """sum_m sin(2 pi k_m . x + phi_m) at cell centres of an nx x ny x nz unit-cube grid,
    for z rows z_lo..z_hi.  Evaluated in float64 as Im(prod of 1D complex exponentials)."""
    z_hi = nz if z_hi is None else z_hi
    xs = (torch.arange(nx, dtype=torch.float64, device=device) + 0.5) / nx
    ys = (torch.arange(ny, dtype=torch.float64, device=device) + 0.5) / ny
    zs = (torch.arange(z_lo, z_hi, dtype=torch.float64, device=device) + 0.5) / nz
    return _mode_sum_at(ks, phases, xs, ys, zs)


def _mode_sum_at(ks, phases, xs, ys, zs):
    """The same sum on the tensor-product grid of the coordinates xs, ys, zs."""
    two_pi = 2.0 * math.pi
    out = torch.zeros((len(zs), len(ys), len(xs)), dtype=torch.float64, device=xs.device)
    for (kx, ky, kz), ph in zip(ks.tolist(), phases.tolist()):
        ax = two_pi * kx * xs
        ay = two_pi * ky * ys
        az = two_pi * kz * zs + ph
        # sin(a + b + c) = Im(e^{ia} e^{ib} e^{ic})
        ex = torch.complex(torch.cos(ax), torch.sin(ax))
        ey = torch.complex(torch.cos(ay), torch.sin(ay))
        ez = torch.complex(torch.cos(az), torch.sin(az))
        out += (ez[:, None, None] * ey[None, :, None] * ex[None, None, :]).imag
    return out


def _smooth_modes_draws(kmax, workload, gamma):
    r = rng(workload)
    rk, rph = _pick_modes(r, 8, kmax)
    vk = [_pick_modes(r, 8, kmax) for _ in range(3)]
    # each velocity component is a sum of 8 orthogonal unit sines: mean square 4,
    # so |v|^2 averages 12; scale to rms |v| = 0.5 sqrt(gamma)
    vscale = 0.5 * math.sqrt(gamma) / math.sqrt(12.0)
    return rk, rph, vk, vscale


def smooth_modes(n: int = 256, kmax: int = 4, workload: int = 2, gamma: float = GAMMA,
                 device="cpu", dtype=torch.float64):
    """Workloads 2 and 5: smooth periodic flow on an n^3 grid.  Returns (groups, dh)."""
    assert n % NI == 0
    rk, rph, vk, vscale = _smooth_modes_draws(kmax, workload, gamma)
    g = n // NI
    out = torch.empty((g * g * g, 5, NI, NI, NI), dtype=dtype, device=device)
    # build one z-slab of groups at a time to bound memory at large n
    for gzi in range(g):
        lo, hi = gzi * NI, (gzi + 1) * NI
        rho = 1.0 + 0.1 * _mode_sum(rk, rph, n, n, n, device, lo, hi)
        vel = [vscale * _mode_sum(k, ph, n, n, n, device, lo, hi) for k, ph in vk]
        p = torch.ones_like(rho)
        slab = conserved(rho, vel[0], vel[1], vel[2], p, gamma)
        out[gzi * g * g:(gzi + 1) * g * g] = _to_groups(slab, g, g, 1).to(dtype)
    return out, 1.0 / n


def smooth_modes_padded(ids, n: int = 1024, kmax: int = 8, workload: int = 5, gamma: float = GAMMA,
                        ghost: int = 2, device="cpu"):
    """The listed groups of the same flow with ``ghost`` periodic ghost cells per
    side, evaluated directly at their cell centres (wrapped into the unit cube),
    without building the whole grid: (len(ids), 5, 16 + 2 ghost, ...) float64.
    For inputs of large grids whose sample the CPU must process."""
    rk, rph, vk, vscale = _smooth_modes_draws(kmax, workload, gamma)
    g = n // NI
    m = NI + 2 * ghost
    out = torch.empty((len(ids), 5, m, m, m), dtype=torch.float64)
    loc = torch.arange(-ghost, NI + ghost, device=device)
    for t, gid in enumerate(ids):
        gid = int(gid)
        bx, by, bz = gid % g, (gid // g) % g, gid // (g * g)
        xs, ys, zs = ((((b * NI + loc) % n).to(torch.float64) + 0.5) / n for b in (bx, by, bz))
        rho = 1.0 + 0.1 * _mode_sum_at(rk, rph, xs, ys, zs)
        vel = [vscale * _mode_sum_at(k, ph, xs, ys, zs) for k, ph in vk]
        out[t] = conserved(rho, vel[0], vel[1], vel[2], torch.ones_like(rho), gamma).cpu()
    return out


def _gaussian_field(r: np.random.Generator, n: int, kmin: float, kmax: float, slope: float):
    """Unit-variance Gaussian random field on an n^3 periodic grid with power
    spectrum P(k) ~ k^slope for kmin <= |k| <= kmax (zero outside)."""
    noise = r.standard_normal((n, n, n))
    fk = np.fft.rfftn(noise)
    k1 = np.fft.fftfreq(n, 1.0 / n)
    kr = np.fft.rfftfreq(n, 1.0 / n)
    kk = np.sqrt(k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + kr[None, None, :] ** 2)
    amp = np.zeros_like(kk)
    band = (kk >= kmin) & (kk <= kmax)
    amp[band] = kk[band] ** (slope / 2.0)
    g = np.fft.irfftn(fk * amp, s=(n, n, n), axes=(0, 1, 2))
    g -= g.mean()
    return g / g.std()


def cosmo_like(n: int = 256, gamma: float = GAMMA, workload: int = 4, device="cpu",
               mach: float = 10.0):
    """Workload 4: high-contrast log-normal density, velocities up to Mach ``mach``."""
    r = rng(workload)
    g = _gaussian_field(r, n, 1.0, n / 2, -3.0)
    rho = np.clip(np.exp(2.0 * g), 1e-3, 1e4)
    p = 1e-2 * rho ** gamma
    cs = np.sqrt(gamma * p / rho)
    vf = [_gaussian_field(r, n, 1.0, n / 2, -3.0) for _ in range(3)]
    vmag = np.sqrt(vf[0] ** 2 + vf[1] ** 2 + vf[2] ** 2)
    scale = mach * cs / vmag.max()
    vel = [torch.from_numpy(scale * f) for f in vf]
    U = conserved(torch.from_numpy(rho), vel[0], vel[1], vel[2], torch.from_numpy(p), gamma)
    gg = n // NI
    return _to_groups(U, gg, gg, gg).to(device), 1.0 / n


def sedov_level(level: int, n_root: int = 128, gamma: float = GAMMA, device="cpu",
                rho0: float = 1.0, p0: float = 1e-5, e_blast: float = 1.0):
    """One uniform level of workload 3: domain [0, n_root)^3, dh = 2^-level,
    ambient (rho0, p0, v = 0) plus energy e_blast added to the cell whose lower
    corner is the domain centre.  Returns (groups, dh, gx)."""
    dh = 0.5 ** level
    n = n_root * 2 ** level
    shape = (n, n, n)
    rho = torch.full(shape, rho0, dtype=torch.float64, device=device)
    p = torch.full(shape, p0, dtype=torch.float64, device=device)
    z = torch.zeros(shape, dtype=torch.float64, device=device)
    U = conserved(rho, z, z, z, p, gamma)
    c = n // 2
    U[4, c, c, c] += e_blast / dh ** 3
    gx = n // NI
    return _to_groups(U, gx, gx, gx), dh, gx


def sedov_level2_selection(n_root: int = 128, count: int = 20000):
    """Indices of the ``count`` level-2 groups whose centres lie nearest the blast
    (ties broken by the lower group index)."""
    gx = n_root * 4 // NI
    idx = np.arange(gx ** 3)
    bx, by, bz = idx % gx, (idx // gx) % gx, idx // (gx * gx)
    centre = gx / 2.0
    d2 = (bx + 0.5 - centre) ** 2 + (by + 0.5 - centre) ** 2 + (bz + 0.5 - centre) ** 2
    order = np.lexsort((idx, d2))
    return np.sort(order[:count])


def sedov_amr(n_root: int = 128, count: int = 20000, gamma: float = GAMMA, device="cpu"):
    """Workload 3: the three uniform levels of the Sedov blast and the level-2
    groups kept in the batch.  Returns a list of (groups, dh, gx, ids) per level,
    where ``ids`` are the group indices of that level that enter the batch (all
    groups of levels 0 and 1, the ``count`` nearest the blast of level 2).  The
    batch is levels 0, 1, 2 in that order; each level is periodic within itself."""
    out = []
    for level in range(3):
        groups, dh, gx = sedov_level(level, n_root, gamma, device)
        ids = (np.arange(gx ** 3) if level < 2 else sedov_level2_selection(n_root, count))
        out.append((groups, dh, gx, ids))
    return out
