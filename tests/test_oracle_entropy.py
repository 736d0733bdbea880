"""Pins of the oracle's Harten-Hyman entropy fix (CPU only).

The fix changes the Roe flux only at transonic acoustic waves, where the plain
Roe flux would admit an expansion shock.  Two kinds of pin:

  * closed form: at constructed transonic pairs the oracle's flux equals the
    Roe flux assembled here from the textbook decomposition (Roe averages,
    eigenvalues and right eigenvectors of Toro 2009, Sec. 11.2; the wave
    strengths solved from K alpha = U_R - U_L with numpy), with the fixed
    modulus |lambda_k| -> (lambda_k^2 + delta_k^2) / (2 delta_k) and
    delta_k = max(0, lambda_k - lambda_left, lambda_right - lambda_k) from the
    speeds on the two sides of wave k (Harten & Hyman 1983; Toro 2009,
    Sec. 11.4.2).  Wave 1 has L and L* = L + alpha_1 K_1 on its sides, wave 5
    R* = R - alpha_5 K_5 and R.  One pair makes wave 1 transonic, its mirror
    image wave 5;
  * symmetry: the sonic rarefaction run and the run of its mirror image
    (x -> 1 - x, u -> -u) agree to rounding.  The two runs use waves 1 and 5
    respectively, so a fix that treats the two waves differently breaks it.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle_driver import from_global, run_periodic, to_global
from paper_1007_3818_amd import workloads as W


def cons(rho, u, v, w, p, g):
    return np.array([rho, rho * u, rho * v, rho * w, p / (g - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])


def prim(U, g):
    rho = U[0]
    u, v, w = U[1] / rho, U[2] / rho, U[3] / rho
    return rho, u, v, w, (g - 1.0) * (U[4] - 0.5 * rho * (u * u + v * v + w * w))


def flux_x(U, g):
    rho, u, v, w, p = prim(U, g)
    return np.array([U[1], U[1] * u + p, U[2] * u, U[3] * u, (U[4] + p) * u])


def decompose(L, R, g):
    """Roe averages, eigenvalues, right eigenvectors (rows) and wave strengths
    of the rotated pair (normal = component 1)."""
    rl, ul, vl, wl, pl = prim(L, g)
    rr, ur, vr, wr, pr = prim(R, g)
    sl, sr = math.sqrt(rl), math.sqrt(rr)

    def avg(a, b):
        return (sl * a + sr * b) / (sl + sr)

    u, v, w = avg(ul, ur), avg(vl, vr), avg(wl, wr)
    H = avg((L[4] + pl) / rl, (R[4] + pr) / rr)
    q2 = u * u + v * v + w * w
    a = math.sqrt((g - 1.0) * (H - 0.5 * q2))
    K = np.array([[1.0, u - a, v, w, H - u * a],
                  [1.0, u, v, w, 0.5 * q2],
                  [0.0, 0.0, 1.0, 0.0, v],
                  [0.0, 0.0, 0.0, 1.0, w],
                  [1.0, u + a, v, w, H + u * a]])
    alpha = np.linalg.solve(K.T, R - L)
    lam = np.array([u - a, u, u, u, u + a])
    return lam, K, alpha


def speeds(U, g):
    rho, u, v, w, p = prim(U, g)
    return u, math.sqrt(g * p / rho)


def roe_with_fix(L, R, g):
    """Roe flux of the rotated pair with the Harten-Hyman fix on waves 1 and 5;
    also returns (delta_1, delta_5) and the plain |lambda| for the checks."""
    lam, K, alpha = decompose(L, R, g)
    ab = np.abs(lam)
    uL, cL = speeds(L, g)
    uR, cR = speeds(R, g)
    us1, cs1 = speeds(L + alpha[0] * K[0], g)   # L*, right of wave 1
    us5, cs5 = speeds(R - alpha[4] * K[4], g)   # R*, left of wave 5
    d1 = max(0.0, lam[0] - (uL - cL), (us1 - cs1) - lam[0])
    d5 = max(0.0, lam[4] - (us5 + cs5), (uR + cR) - lam[4])
    fixed = ab.copy()
    if ab[0] < d1:
        fixed[0] = (lam[0] ** 2 + d1 ** 2) / (2.0 * d1)
    if ab[4] < d5:
        fixed[4] = (lam[4] ** 2 + d5 ** 2) / (2.0 * d5)
    diss = (alpha * fixed) @ K
    F = 0.5 * (flux_x(L, g) + flux_x(R, g)) - 0.5 * diss
    plain = 0.5 * (flux_x(L, g) + flux_x(R, g)) - 0.5 * (alpha * ab) @ K
    return F, plain, (d1, d5), ab


def rotate(U, d):
    n = [1 + d, 1 + (d + 1) % 3, 1 + (d + 2) % 3]
    return np.array([U[0], U[n[0]], U[n[1]], U[n[2]], U[4]])


def unrotate(Fr, d):
    F = np.empty(5)
    F[0], F[4] = Fr[0], Fr[4]
    F[1 + d], F[1 + (d + 1) % 3], F[1 + (d + 2) % 3] = Fr[1], Fr[2], Fr[3]
    return F


# Toro's sonic-point problem (left state moving at 0.75, gamma = 1.4) with
# transverse velocities added, and its mirror image; a second pair, whose
# left state is barely subsonic towards the right, and its mirror; primitives (rho, u_n, u_t1, u_t2, p) in the rotated frame
SONIC = ((1.0, 0.75, 0.3, -0.2, 1.0), (0.125, 0.0, 0.3, -0.2, 0.1))
WEAK = ((1.0, 1.0, -0.1, 0.4, 1.0), (0.5, 1.2, -0.1, 0.4, 0.4))


def mirrored(pair):
    (rl, ul, vl, wl, pl), (rr, ur, vr, wr, pr) = pair
    return (rr, -ur, vr, wr, pr), (rl, -ul, vl, wl, pl)


@pytest.mark.parametrize("pair,wave", [(SONIC, 0), (mirrored(SONIC), 4), (WEAK, 0), (mirrored(WEAK), 4)])
@pytest.mark.parametrize("d", [0, 1, 2])
def test_fix_value_closed_form(pair, wave, d):
    g = 1.4
    L, R = cons(*pair[0], g), cons(*pair[1], g)
    F, plain, deltas, ab = roe_with_fix(L, R, g)
    # the pair is transonic in the intended wave only: the fix is active there
    assert ab[wave] < deltas[wave // 4]
    other = 4 - wave
    assert not ab[other] < deltas[other // 4]
    # and it changes the flux by far more than rounding
    assert np.abs(F - plain).max() > 1e-5 * np.abs(F).max()
    # the oracle, for unrotated states along direction d
    UL, UR = unrotate(L, d), unrotate(R, d)
    Fo, hlle = oracle.roe_flux(UL, UR, d, g)
    assert not hlle
    np.testing.assert_allclose(rotate(Fo, d), F, rtol=1e-13, atol=1e-13 * np.abs(F).max())


def test_fix_inactive_away_from_sonic_points():
    """Where no acoustic wave is transonic the fix leaves Roe's flux alone."""
    g = 1.4
    r = np.random.default_rng(7)
    n_checked = 0
    for _ in range(400):
        pl = (math.exp(r.uniform(-2, 2)), r.uniform(-3, 3), r.uniform(-1, 1), r.uniform(-1, 1),
              math.exp(r.uniform(-2, 2)))
        pr = (pl[0] * math.exp(r.uniform(-0.3, 0.3)), pl[1] + r.uniform(-0.3, 0.3), pl[2], pl[3],
              pl[4] * math.exp(r.uniform(-0.3, 0.3)))
        L, R = cons(*pl, g), cons(*pr, g)
        F, plain, (d1, d5), ab = roe_with_fix(L, R, g)
        if ab[0] < d1 or ab[4] < d5:
            continue
        Fo, hlle = oracle.roe_flux(L, R, 0, g)
        if hlle:
            continue
        np.testing.assert_allclose(Fo, plain, rtol=1e-12, atol=1e-12 * np.abs(plain).max())
        n_checked += 1
    assert n_checked > 300


def _sonic_run(left, right, g=1.4, N=256, t_end=0.1):
    dh = 1.0 / N
    x = (np.arange(N) + 0.5) * dh
    prim_ = [np.where(x < 0.5, a, b) for a, b in zip(left, right)]
    dims = (16, 16, N)
    rho, u, p = (torch.from_numpy(np.broadcast_to(q, dims).copy()) for q in prim_)
    z = torch.zeros(dims, dtype=torch.float64)
    st = from_global(W.conserved(rho, u, z, z, p, g).numpy(), N // 16, 1, 1)
    s, t, n, counts = run_periodic(st, N // 16, 1, 1, dh, g, 0.5, t_end=t_end)
    return to_global(s, N // 16, 1, 1)[:, 0, 0, :], counts


def test_sonic_rarefaction_mirror_symmetry():
    """Toro's sonic rarefaction, left (1, 0.75, 1) | right (0.125, 0, 0.1), and its
    mirror image, left (0.125, 0, 0.1) | right (1, -0.75, 1): the second run equals
    the first reflected (x -> 1 - x, m_x -> -m_x) to rounding.  The first run's fan
    is carried by wave 1, the mirror's by wave 5."""
    a, ca = _sonic_run((1.0, 0.75, 1.0), (0.125, 0.0, 0.1))
    b, cb = _sonic_run((0.125, 0.0, 0.1), (1.0, -0.75, 1.0))
    assert ca == cb == (0, 0)
    ref = a[:, ::-1].copy()
    ref[1] = -ref[1]
    scale = np.abs(a).max(axis=1)
    moving = scale > 0  # the transverse momenta are zero throughout, in both runs
    assert np.array_equal(b[~moving], ref[~moving])
    err = np.abs(b - ref)[moving] / scale[moving, None]
    assert err.max() <= 1e-12, err.max()
