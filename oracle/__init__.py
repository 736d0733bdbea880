"""FP64 CPU oracle for the MUSCL-Hancock + Roe group step -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``libgamer_oracle.so`` (plain C,
see ``gamer_oracle.c``) with numpy arrays on the host.  It shares no code with
the HIP library.

Array conventions (all float64, C-contiguous, x fastest):
  padded groups   (n, 5, 20, 20, 20)  conserved (rho, m_x, m_y, m_z, E)
  interior groups (n, 5, 16, 16, 16)
  flux planes     (n, 3, 3, 5, 16, 16)
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None

_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64
_PLL = ctypes.POINTER(ctypes.c_longlong)


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < max(os.path.getmtime(f) for f in _build.SRCS)):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        sig = {
            "gamer_oracle_set_threads": (None, [ctypes.c_int]),
            "gamer_oracle_get_threads": (ctypes.c_int, []),
            "gamer_oracle_prim_from_cons": (None, [_PD, _D, _PD]),
            "gamer_oracle_cons_from_prim": (None, [_PD, _D, _PD]),
            "gamer_oracle_phys_flux": (None, [_PD, ctypes.c_int, _D, _PD]),
            "gamer_oracle_limiter": (_D, [_D, _D, _D]),
            "gamer_oracle_group_prim": (None, [_PD, _D, _PD]),
            "gamer_oracle_group_slopes": (None, [_PD, _D, _PD]),
            "gamer_oracle_group_predict": (ctypes.c_longlong, [_PD, _PD, _PD, _D, _D, _D, _PD]),
            "gamer_oracle_group_fluxes": (ctypes.c_longlong, [_PD, _D, _PD]),
            "gamer_oracle_group_update": (None, [_PD, _PD, _D, _D, _PD, _PD]),
            "gamer_oracle_roe_flux": (ctypes.c_int, [_PD, _PD, ctypes.c_int, _D, _PD]),
            "gamer_oracle_roe_decompose": (None, [_PD, _PD, _D, _PD, _PD, _PD, _PD]),
            "gamer_oracle_hydro_solve": (ctypes.c_int, [_PD, _I64, _D, _D, _D, _D, _PD, _PD, _PLL]),
            "gamer_oracle_hydro_solve_lim": (ctypes.c_int, [_PD, _I64, _D, _D, _D, _D, ctypes.c_int, _PD,
                                                            _PD, _PLL]),
            "gamer_oracle_char_slope": (None, [_PD, _PD, _PD, ctypes.c_int, _D, _D, _PD]),
            "gamer_oracle_group_slopes_char": (None, [_PD, _D, _D, _PD]),
            "gamer_oracle_max_speed": (_D, [_PD, _I64, _D]),
            "gamer_oracle_cfl_dt": (_D, [_PD, _I64, _D, _D, _D]),
            "gamer_oracle_conserved_sums": (None, [_PD, _I64, _D, _PD]),
            "gamer_oracle_pack_periodic": (None, [_PD, ctypes.c_int, ctypes.c_int, ctypes.c_int, _PD]),
            "gamer_oracle_vanleer": (_D, [_D, _D]),
            "gamer_oracle_ctu_solve": (ctypes.c_int, [_PD, _I64, _D, _D, _D, _D, _PD, _PD, _PLL]),
            "gamer_oracle_rtvd_pencil": (ctypes.c_longlong, [_PD, ctypes.c_int, ctypes.c_int, _D, _D, _PD]),
            "gamer_oracle_rtvd_solve": (ctypes.c_int, [_PD, _I64, _D, _D, _D, ctypes.c_int, _PD, _PLL]),
            "gamer_oracle_margin_reset": (None, [_D]),
            "gamer_oracle_margin_hits": (ctypes.c_longlong, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_PD)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


THETA = 1.5  # generalised-minmod parameter of the default reading


def set_threads(n: int) -> None:
    _lib().gamer_oracle_set_threads(int(n))


def borderline_decisions(fn, tau):
    """Run ``fn()`` (a call into the oracle) on one thread and return (its result,
    the number of fallback decisions it took within a relative margin ``tau`` of
    their threshold; see gamer_oracle_margin_reset).  Test hook only."""
    L = _lib()
    threads = L.gamer_oracle_get_threads()
    L.gamer_oracle_set_threads(1)
    L.gamer_oracle_margin_reset(float(tau))
    try:
        res = fn()
        hits = int(L.gamer_oracle_margin_hits())
    finally:
        L.gamer_oracle_margin_reset(-1.0)
        L.gamer_oracle_set_threads(threads)
    return res, hits


def get_threads() -> int:
    return _lib().gamer_oracle_get_threads()


# --- single-state helpers ---------------------------------------------------

def prim_from_cons(U, gamma):
    U = _f64(U)
    W = np.empty(5)
    _lib().gamer_oracle_prim_from_cons(_p(U), gamma, _p(W))
    return W


def cons_from_prim(W, gamma):
    W = _f64(W)
    U = np.empty(5)
    _lib().gamer_oracle_cons_from_prim(_p(W), gamma, _p(U))
    return U


def phys_flux(U, d, gamma):
    U = _f64(U)
    F = np.empty(5)
    _lib().gamer_oracle_phys_flux(_p(U), int(d), gamma, _p(F))
    return F


def limiter(a, b, theta=THETA):
    return _lib().gamer_oracle_limiter(float(a), float(b), float(theta))


def roe_flux(UL, UR, d, gamma):
    """Roe flux along direction d between unrotated conserved states.
    Returns (F[5], hlle_used)."""
    UL, UR = _f64(UL), _f64(UR)
    F = np.empty(5)
    fb = _lib().gamer_oracle_roe_flux(_p(UL), _p(UR), int(d), gamma, _p(F))
    return F, bool(fb)


def roe_decompose(L, R, gamma):
    """Roe decomposition of rotated states (normal = component 1).
    Returns dict(avg=[u,v,w,H,a2,a], alpha[5], lam[5], K[5 wave, 5 comp])."""
    L, R = _f64(L), _f64(R)
    avg, alpha, lam, K = np.empty(6), np.empty(5), np.empty(5), np.empty((5, 5))
    _lib().gamer_oracle_roe_decompose(_p(L), _p(R), gamma, _p(avg), _p(alpha), _p(lam), _p(K))
    return dict(avg=avg, alpha=alpha, lam=lam, K=K)


# --- per-group stages -------------------------------------------------------

def group_prim(U, gamma):
    U = _f64(U)
    W = np.empty_like(U)
    _lib().gamer_oracle_group_prim(_p(U), gamma, _p(W))
    return W


def group_slopes(W, theta=THETA):
    W = _f64(W)
    dW = np.empty((3, 5, 18, 18, 18))
    _lib().gamer_oracle_group_slopes(_p(W), theta, _p(dW))
    return dW


def char_slope(Wc, a, b, d, gamma, theta=THETA):
    """Limited slope of one cell along d in characteristic variables, from the
    cell's primitive state and its one-sided primitive differences."""
    Wc, a, b = _f64(Wc), _f64(a), _f64(b)
    out = np.empty(5)
    _lib().gamer_oracle_char_slope(_p(Wc), _p(a), _p(b), int(d), gamma, theta, _p(out))
    return out


def group_slopes_char(W, gamma, theta=THETA):
    W = _f64(W)
    dW = np.empty((3, 5, 18, 18, 18))
    _lib().gamer_oracle_group_slopes_char(_p(W), gamma, theta, _p(dW))
    return dW


def group_predict(U, W, dW, dt, dh, gamma):
    U, W, dW = _f64(U), _f64(W), _f64(dW)
    Ub = np.empty((3, 2, 5, 18, 18, 18))
    n = _lib().gamer_oracle_group_predict(_p(U), _p(W), _p(dW), dt, dh, gamma, _p(Ub))
    return Ub, int(n)


def group_fluxes(Ub, gamma):
    Ub = _f64(Ub)
    Fl = np.empty((3, 5, 17, 16, 16))
    n = _lib().gamer_oracle_group_fluxes(_p(Ub), gamma, _p(Fl))
    return Fl, int(n)


def group_update(U, Fl, dt, dh, want_planes=False):
    U, Fl = _f64(U), _f64(Fl)
    out = np.empty((5, 16, 16, 16))
    planes = np.empty((3, 3, 5, 16, 16)) if want_planes else None
    _lib().gamer_oracle_group_update(_p(U), _p(Fl), dt, dh, _p(out), _p(planes))
    return (out, planes) if want_planes else out


# --- batch entry points -----------------------------------------------------

def hydro_solve(groups_in, dt, dh, gamma, theta=THETA, want_fluxes=False, limiting="primitive",
                coupling="hancock"):
    """One step on a batch.  Returns (groups_out, fluxes_or_None, (n_pred_fallback, n_hlle)).
    limiting: "primitive" or "characteristic" (variables the slopes are limited in);
    coupling: "hancock" (the unsplit Hancock predictor) or "ctu" (corner transport
    upwind, gamer_ctu.c; primitive limiting only)."""
    char = {"primitive": 0, "characteristic": 1}[limiting]
    if coupling == "ctu":
        if char:
            raise ValueError("the CTU variant limits primitive variables")
        return _ctu_solve(groups_in, dt, dh, gamma, theta, want_fluxes)
    if coupling != "hancock":
        raise ValueError(coupling)
    g = _f64(groups_in)
    assert g.ndim == 5 and g.shape[1:] == (5, 20, 20, 20), g.shape
    n = g.shape[0]
    out = np.empty((n, 5, 16, 16, 16))
    fl = np.empty((n, 3, 3, 5, 16, 16)) if want_fluxes else None
    counts = (ctypes.c_longlong * 2)()
    rc = _lib().gamer_oracle_hydro_solve_lim(_p(g), n, dt, dh, gamma, theta, char, _p(fl), _p(out),
                                             ctypes.cast(counts, _PLL))
    if rc != 0:
        raise ValueError("oracle hydro_solve rejected its arguments")
    return out, fl, (int(counts[0]), int(counts[1]))


def _ctu_solve(groups_in, dt, dh, gamma, theta, want_fluxes):
    g = _f64(groups_in)
    assert g.ndim == 5 and g.shape[1:] == (5, 20, 20, 20), g.shape
    n = g.shape[0]
    out = np.empty((n, 5, 16, 16, 16))
    fl = np.empty((n, 3, 3, 5, 16, 16)) if want_fluxes else None
    counts = (ctypes.c_longlong * 2)()
    rc = _lib().gamer_oracle_ctu_solve(_p(g), n, dt, dh, gamma, theta, _p(fl), _p(out),
                                       ctypes.cast(counts, _PLL))
    if rc != 0:
        raise ValueError("oracle ctu_solve rejected its arguments")
    return out, fl, (int(counts[0]), int(counts[1]))


def max_speed(groups, gamma):
    g = _f64(groups)
    return _lib().gamer_oracle_max_speed(_p(g), g.shape[0], gamma)


def cfl_dt(groups, dh, gamma, cfl):
    g = _f64(groups)
    assert g.shape[1:] == (5, 16, 16, 16)
    return _lib().gamer_oracle_cfl_dt(_p(g), g.shape[0], dh, gamma, cfl)


def conserved_sums(groups, dh):
    g = _f64(groups)
    s = np.empty(5)
    _lib().gamer_oracle_conserved_sums(_p(g), g.shape[0], dh, _p(s))
    return s


def pack_periodic(state, gx, gy, gz):
    """state (G, 5, 16, 16, 16) with g = gx + Gx (gy + Gy gz)  ->  (G, 5, 20, 20, 20)."""
    s = _f64(state)
    assert s.shape == (gx * gy * gz, 5, 16, 16, 16)
    out = np.empty((s.shape[0], 5, 20, 20, 20))
    _lib().gamer_oracle_pack_periodic(_p(s), gx, gy, gz, _p(out))
    return out


def pack_periodic_subset(state, gx, gy, gz, ids):
    """Padded groups (len(ids), 5, 20, 20, 20) for the listed groups of a periodic
    grid, assembled from the 3 x 3 x 3 neighbourhood of each group.  ``state`` is
    any array-like (G, 5, 16, 16, 16) indexable by group (numpy or torch)."""
    out = np.empty((len(ids), 5, 20, 20, 20))
    for n, g in enumerate(ids):
        g = int(g)
        bx, by, bz = g % gx, (g // gx) % gy, g // (gx * gy)
        block = np.empty((5, 48, 48, 48))
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    nb = ((bx + dx) % gx) + gx * (((by + dy) % gy) + gy * ((bz + dz) % gz))
                    q = state[nb]
                    q = q.detach().cpu().double().numpy() if hasattr(q, "detach") else np.asarray(q, np.float64)
                    block[:, 16 * (dz + 1):16 * (dz + 2), 16 * (dy + 1):16 * (dy + 2),
                          16 * (dx + 1):16 * (dx + 2)] = q
        out[n] = block[:, 14:34, 14:34, 14:34]
    return out


def step_periodic(state, gx, gy, gz, dt, dh, gamma, theta=THETA, limiting="primitive",
                  coupling="hancock"):
    """Ghost fill then one step of a uniform periodic grid held as groups."""
    out, _, counts = hydro_solve(pack_periodic(state, gx, gy, gz), dt, dh, gamma, theta,
                                 limiting=limiting, coupling=coupling)
    return out, counts


# --- relaxing TVD (gamer_rtvd.c) ----------------------------------------------

RG = 3  # ghost cells per side of the relaxing TVD scheme's seven-point stencil


def vanleer(a, b):
    return _lib().gamer_oracle_vanleer(float(a), float(b))


def rtvd_pencil(u, d, dtdx, gamma):
    """One relaxing-TVD update of a pencil u (n, 5) along direction d:
    returns (cells 3 .. n-4 as (n-6, 5), bad-cell count)."""
    u = _f64(u)
    n = u.shape[0]
    out = np.empty((n - 6, 5))
    bad = _lib().gamer_oracle_rtvd_pencil(_p(u), n, int(d), float(dtdx), float(gamma), _p(out))
    return out, int(bad)


def rtvd_solve(groups_in, dt, dh, gamma, order=0):
    """One relaxing-TVD step of padded groups (n, 5, 22, 22, 22) -> (n, 5, 16, 16, 16);
    order 0 sweeps x, y, z, order 1 z, y, x.  Returns (out, bad-cell count)."""
    g = _f64(groups_in)
    assert g.ndim == 5 and g.shape[1:] == (5, 22, 22, 22), g.shape
    n = g.shape[0]
    out = np.empty((n, 5, 16, 16, 16))
    bad = ctypes.c_longlong(0)
    rc = _lib().gamer_oracle_rtvd_solve(_p(g), n, dt, dh, gamma, int(order), _p(out), ctypes.byref(bad))
    if rc != 0:
        raise ValueError("oracle rtvd_solve rejected its arguments")
    return out, int(bad.value)


def pack_periodic_rtvd(state, gx, gy, gz):
    """Padded groups with three ghost cells per side, (G, 5, 22, 22, 22), from
    a periodic grid of groups (G, 5, 16, 16, 16): each padded cell is the cell
    at its wrapped global position (brute force over the global array)."""
    s = _f64(state)
    G = s.reshape(gz, gy, gx, 5, 16, 16, 16).transpose(3, 0, 4, 1, 5, 2, 6).reshape(
        5, gz * 16, gy * 16, gx * 16)
    out = np.empty((gx * gy * gz, 5, 22, 22, 22))
    for g in range(gx * gy * gz):
        bx, by, bz = g % gx, (g // gx) % gy, g // (gx * gy)
        ix = np.arange(16 * bx - RG, 16 * bx + 16 + RG) % G.shape[3]
        iy = np.arange(16 * by - RG, 16 * by + 16 + RG) % G.shape[2]
        iz = np.arange(16 * bz - RG, 16 * bz + 16 + RG) % G.shape[1]
        out[g] = G[:, iz][:, :, iy][:, :, :, ix]
    return out


def pack_periodic_rtvd_subset(state, gx, gy, gz, ids):
    """Padded groups (len(ids), 5, 22, 22, 22) with three ghost cells per side
    for the listed groups of a periodic grid, assembled from the 3 x 3 x 3
    neighbourhood of each group.  ``state`` as in pack_periodic_subset."""
    out = np.empty((len(ids), 5, 22, 22, 22))
    for n, g in enumerate(ids):
        g = int(g)
        bx, by, bz = g % gx, (g // gx) % gy, g // (gx * gy)
        block = np.empty((5, 48, 48, 48))
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    nb = ((bx + dx) % gx) + gx * (((by + dy) % gy) + gy * ((bz + dz) % gz))
                    q = state[nb]
                    q = q.detach().cpu().double().numpy() if hasattr(q, "detach") else np.asarray(q, np.float64)
                    block[:, 16 * (dz + 1):16 * (dz + 2), 16 * (dy + 1):16 * (dy + 2),
                          16 * (dx + 1):16 * (dx + 2)] = q
        out[n] = block[:, 16 - RG:32 + RG, 16 - RG:32 + RG, 16 - RG:32 + RG]
    return out


def rtvd_step_periodic(state, gx, gy, gz, dt, dh, gamma, order=0):
    out, bad = rtvd_solve(pack_periodic_rtvd(state, gx, gy, gz), dt, dh, gamma, order)
    return out, bad
