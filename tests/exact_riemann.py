"""Exact solution of the Riemann problem for the 1D Euler equations of an ideal gas.

Test helper, independent of both the oracle and the GPU path.  Follows the
construction in Toro (2009), Ch. 4: the star-region pressure p* is the root of
f(p) = f_L(p) + f_R(p) + (u_R - u_L), where f_K is the shock (Rankine-Hugoniot)
branch for p > p_K and the rarefaction (isentropic) branch otherwise; then
u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2, the star densities follow from the
shock or isentropic relations, and the self-similar solution is sampled at
xi = x / t.
"""
import math


def _fk(p, rho, pk, g):
    """f_K(p) and its derivative for one side."""
    c = math.sqrt(g * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    r = p / pk
    f = 2.0 * c / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho * c) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, g):
    """(p*, u*, rho*_L, rho*_R) for primitive states left/right = (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated")
    # two-rarefaction guess
    z = (g - 1.0) / (2.0 * g)
    p = ((cl + cr - 0.5 * (g - 1.0) * (ur - ul)) / (cl / pl ** z + cr / pr ** z)) ** (1.0 / z)
    p = max(p, 1e-12)
    for _ in range(200):
        fl, dfl = _fk(p, rl, pl, g)
        fr, dfr = _fk(p, rr, pr, g)
        f = fl + fr + (ur - ul)
        pn = p - f / (dfl + dfr)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= 1e-15 * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, g)
    fr, _ = _fk(p, rr, pr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    gg = (g - 1.0) / (g + 1.0)

    def rho_star(rho, pk):
        if p > pk:
            return rho * (p / pk + gg) / (gg * p / pk + 1.0)
        return rho * (p / pk) ** (1.0 / g)

    return p, u, rho_star(rl, pl), rho_star(rr, pr)


def wave_speeds(left, right, g):
    """Dict of the wave speeds: left/right head and tail (rarefaction) or shock speed."""
    rl, ul, pl = left
    rr, ur, pr = right
    p, u, rsl, rsr = star_state(left, right, g)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    out = {"contact": u}
    if p > pl:
        out["left_shock"] = ul - cl * math.sqrt((g + 1) / (2 * g) * p / pl + (g - 1) / (2 * g))
    else:
        out["left_head"] = ul - cl
        out["left_tail"] = u - cl * (p / pl) ** ((g - 1) / (2 * g))
    if p > pr:
        out["right_shock"] = ur + cr * math.sqrt((g + 1) / (2 * g) * p / pr + (g - 1) / (2 * g))
    else:
        out["right_head"] = ur + cr
        out["right_tail"] = u + cr * (p / pr) ** ((g - 1) / (2 * g))
    return out


def sample(left, right, g, xi):
    """Primitive state (rho, u, p) of the self-similar solution at xi = x/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    p, u, rsl, rsr = star_state(left, right, g)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    if xi <= u:  # left of the contact
        if p > pl:
            s = ul - cl * math.sqrt((g + 1) / (2 * g) * p / pl + (g - 1) / (2 * g))
            return (rl, ul, pl) if xi <= s else (rsl, u, p)
        head = ul - cl
        tail = u - cl * (p / pl) ** ((g - 1) / (2 * g))
        if xi <= head:
            return (rl, ul, pl)
        if xi >= tail:
            return (rsl, u, p)
        c = 2.0 / (g + 1) * (cl + 0.5 * (g - 1) * (ul - xi))
        uu = 2.0 / (g + 1) * (cl + 0.5 * (g - 1) * ul + xi)
        rho = rl * (c / cl) ** (2.0 / (g - 1))
        return (rho, uu, pl * (c / cl) ** (2.0 * g / (g - 1)))
    if p > pr:
        s = ur + cr * math.sqrt((g + 1) / (2 * g) * p / pr + (g - 1) / (2 * g))
        return (rr, ur, pr) if xi >= s else (rsr, u, p)
    head = ur + cr
    tail = u + cr * (p / pr) ** ((g - 1) / (2 * g))
    if xi >= head:
        return (rr, ur, pr)
    if xi <= tail:
        return (rsr, u, p)
    c = 2.0 / (g + 1) * (cr - 0.5 * (g - 1) * (ur - xi))
    uu = 2.0 / (g + 1) * (-cr + 0.5 * (g - 1) * ur + xi)
    rho = rr * (c / cr) ** (2.0 / (g - 1))
    return (rho, uu, pr * (c / cr) ** (2.0 * g / (g - 1)))
