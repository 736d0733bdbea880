"""Torch-tensor front end of the C ABI (device memory and streams only).

Each function checks shapes, dtypes and devices, sets the library's stream to
torch's current stream and calls the entry point of the same name in
include/gamer_hydro.h.  All arithmetic happens in the HIP kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import _native

NI, NP, NV = 16, 20, 5


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    _native.check(_native.lib().gamer_set_stream(
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))


def _need(t, shape_tail, dtype, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape (n, {', '.join(map(str, shape_tail))}), got {tuple(t.shape)}")


def _f32(dtype):
    if dtype == torch.float32:
        return True
    if dtype == torch.float64:
        return False
    raise TypeError(f"unsupported dtype {dtype}")


def _bad_counter(bad_count):
    """Device address of a bad-cell counter pair: a GPU int64 tensor of two
    entries (cells not physical or not finite, groups with a level out of range),
    zeroed by the caller."""
    if bad_count is None:
        return None
    if (not isinstance(bad_count, torch.Tensor) or not bad_count.is_cuda or bad_count.dtype != torch.int64
            or bad_count.numel() < 2 or not bad_count.is_contiguous()):
        raise ValueError("bad_count must be a contiguous GPU int64 tensor of at least 2 entries")
    return bad_count.data_ptr()


def _opts(theta, variant, grid, limiting, bad_count=None, zseg=None):
    if (theta is None and variant is None and grid is None and limiting is None and bad_count is None
            and zseg is None):
        return None
    lim = {None: 0, "primitive": 0, "characteristic": 1}.get(limiting, limiting)
    return _native.GamerOpts(float(theta or 0.0), int(variant or 0), int(grid or 0), int(lim), int(zseg or 0),
                             _bad_counter(bad_count))


def _levels(level, dt_dev, dh_dev, n):
    if level is not None:
        if level.dtype != torch.int8 or not level.is_cuda or level.numel() != n:
            raise ValueError("level must be a GPU int8 tensor with one entry per group")
    for t, nm in ((dt_dev, "dt_dev"), (dh_dev, "dh_dev")):
        if t.dtype != torch.float64 or not t.is_cuda or t.dim() != 1:
            raise ValueError(f"{nm} must be a 1-D GPU float64 tensor")
    if dh_dev.numel() != dt_dev.numel():
        raise ValueError("dt_dev and dh_dev must have one entry per level")
    return dt_dev.numel()


def _solver_fn(name, dtype, compute):
    """Entry point for storage dtype and arithmetic dtype `compute` (None: the
    storage dtype; float32 with float64 storage: the mixed-precision path)."""
    f32 = _f32(dtype)
    if compute is None or compute == dtype:
        return getattr(_native.lib(), name + ("_f32" if f32 else ""))
    if dtype == torch.float64 and compute == torch.float32:
        return getattr(_native.lib(), name + "_mixed")
    raise TypeError(f"no {name} path storing {dtype} and computing in {compute}")


def hydro_solve(groups_in, dt, dh, gamma, out=None, fluxes_out=None):
    """One MUSCL-Hancock + Roe step of every padded group (same dt, dh)."""
    f32 = _f32(groups_in.dtype)
    _need(groups_in, (NV, NP, NP, NP), groups_in.dtype, "groups_in")
    n = groups_in.shape[0]
    if out is None:
        out = torch.empty((n, NV, NI, NI, NI), dtype=groups_in.dtype, device=groups_in.device)
    _need(out, (NV, NI, NI, NI), groups_in.dtype, "out")
    if fluxes_out is not None:
        _need(fluxes_out, (3, 3, NV, NI, NI), groups_in.dtype, "fluxes_out")
    _stream()
    fn = _native.lib().gamer_hydro_solve_f32 if f32 else _native.lib().gamer_hydro_solve
    _native.check(fn(_ptr(groups_in), n, float(dt), float(dh), float(gamma), _ptr(fluxes_out), _ptr(out)))
    return out


def hydro_solve_batched(groups_in, level, dt_dev, dh_dev, gamma, out=None, fluxes_out=None,
                        group_stats=None, theta=None, variant=None, grid=None, limiting=None,
                        compute=None, bad_count=None):
    """One launch over groups of uneven level; dt and dh read on the device.
    `variant` / `grid` select a compiled solver variant and a persistent grid,
    `limiting` "primitive" or "characteristic" (see gamer_opts); None keeps the
    defaults.  `compute=torch.float32` with float64 arrays selects the FP64-state,
    FP32-arithmetic path.  `bad_count`: GPU int64 [2] the step adds its counts of
    non-physical output cells and of groups with a level out of range to.  The
    launch goes to torch's current stream, passed as the call's stream argument."""
    fn = _solver_fn("gamer_hydro_solve_batched", groups_in.dtype, compute)
    _need(groups_in, (NV, NP, NP, NP), groups_in.dtype, "groups_in")
    n = groups_in.shape[0]
    if out is None:
        out = torch.empty((n, NV, NI, NI, NI), dtype=groups_in.dtype, device=groups_in.device)
    _need(out, (NV, NI, NI, NI), groups_in.dtype, "out")
    if fluxes_out is not None:
        _need(fluxes_out, (3, 3, NV, NI, NI), groups_in.dtype, "fluxes_out")
    if group_stats is not None:
        _need(group_stats, (8,), torch.float64, "group_stats")
    n_levels = _levels(level, dt_dev, dh_dev, n)
    opts = _opts(theta, variant, grid, limiting, bad_count)
    # torch's default stream has handle 0, which the call reads as "the thread's
    # current library stream": make that torch's current stream as well
    _stream()
    _native.check(fn(_ptr(groups_in), n, _ptr(level), _ptr(dt_dev), _ptr(dh_dev), n_levels,
                     float(gamma), _ptr(fluxes_out), _ptr(out), _ptr(group_stats),
                     ctypes.byref(opts) if opts is not None else None,
                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return out


def hydro_solve_periodic(state, gx, gy, gz, dt_dev, dh_dev, gamma, out=None, fluxes_out=None,
                         group_stats=None, theta=None, variant=None, grid=None, limiting=None,
                         compute=None, bad_count=None, zseg=None):
    """One step of a uniform periodic grid; ghost cells are read from the
    neighbouring groups in place (no padded copy).  `out` must not be `state`.
    zseg: groups of a column swept together by one work-group (None or 0: the
    library's choice); the results do not depend on it.  Other options as in
    hydro_solve_batched."""
    fn = _solver_fn("gamer_hydro_solve_periodic", state.dtype, compute)
    _need(state, (NV, NI, NI, NI), state.dtype, "state")
    n = state.shape[0]
    if n != gx * gy * gz:
        raise ValueError("state must hold gx*gy*gz groups")
    if out is None:
        out = torch.empty_like(state)
    _need(out, (NV, NI, NI, NI), state.dtype, "out")
    if fluxes_out is not None:
        _need(fluxes_out, (3, 3, NV, NI, NI), state.dtype, "fluxes_out")
    if group_stats is not None:
        _need(group_stats, (8,), torch.float64, "group_stats")
    for t, nm in ((dt_dev, "dt_dev"), (dh_dev, "dh_dev")):
        if t.dtype != torch.float64 or not t.is_cuda or t.numel() < 1:
            raise ValueError(f"{nm} must be a GPU float64 tensor")
    opts = _opts(theta, variant, grid, limiting, bad_count, zseg)
    _stream()
    _native.check(fn(_ptr(state), int(gx), int(gy), int(gz), _ptr(dt_dev), _ptr(dh_dev), float(gamma),
                     _ptr(fluxes_out), _ptr(out), _ptr(group_stats),
                     ctypes.byref(opts) if opts is not None else None))
    return out


def step_reduce(group_stats, level, dh_dev, cfl, dt_out=None, totals_out=None):
    """Per-level dt and conserved totals (+ fallback counts) from group stats, on the device."""
    _need(group_stats, (8,), torch.float64, "group_stats")
    n = group_stats.shape[0]
    n_levels = dh_dev.numel()
    dev = group_stats.device
    if dt_out is None:
        dt_out = torch.empty(n_levels, dtype=torch.float64, device=dev)
    if totals_out is None:
        totals_out = torch.empty(7, dtype=torch.float64, device=dev)
    _stream()
    _native.check(_native.lib().gamer_step_reduce(_ptr(group_stats), n, _ptr(level), _ptr(dh_dev),
                                                  n_levels, float(cfl), _ptr(dt_out), _ptr(totals_out)))
    return dt_out, totals_out


def group_stats(groups, gamma, out=None):
    f32 = _f32(groups.dtype)
    _need(groups, (NV, NI, NI, NI), groups.dtype, "groups")
    n = groups.shape[0]
    if out is None:
        out = torch.empty((n, 8), dtype=torch.float64, device=groups.device)
    _stream()
    fn = _native.lib().gamer_group_stats_f32 if f32 else _native.lib().gamer_group_stats
    _native.check(fn(_ptr(groups), n, float(gamma), _ptr(out)))
    return out


def cfl_dt(groups, dh, gamma, cfl, device_out=False):
    """dt = cfl dh / max(|u|+|v|+|w|+3 c_s); a float, or a 1-element GPU tensor."""
    f32 = _f32(groups.dtype)
    _need(groups, (NV, NI, NI, NI), groups.dtype, "groups")
    _stream()
    fn = _native.lib().gamer_cfl_dt_f32 if f32 else _native.lib().gamer_cfl_dt
    if device_out:
        out = torch.empty(1, dtype=torch.float64, device=groups.device)
        _native.check(fn(_ptr(groups), groups.shape[0], float(dh), float(gamma), float(cfl), _ptr(out), 1))
        return out
    host = ctypes.c_double(0.0)
    _native.check(fn(_ptr(groups), groups.shape[0], float(dh), float(gamma), float(cfl),
                     ctypes.cast(ctypes.byref(host), ctypes.c_void_p), 0))
    return host.value


def cfl_dt_noalloc(groups, dh, gamma, cfl, out=None):
    """gamer_cfl_dt_noalloc: the CFL time step of FP64 interior groups into a
    1-element float64 GPU tensor (``out``, or a new one), without any device
    allocation inside the library (at most NOALLOC_MAX_GROUPS groups)."""
    _need(groups, (NV, NI, NI, NI), torch.float64, "groups")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=groups.device)
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64
            and out.is_contiguous() and out.numel() >= 1 and out.device == groups.device):
        raise ValueError("out must be a contiguous float64 GPU tensor of at least 1 element on the groups' device")
    _stream()
    _native.check(_native.lib().gamer_cfl_dt_noalloc(_ptr(groups), groups.shape[0], float(dh), float(gamma),
                                                     float(cfl), _ptr(out)))
    return out


def conserved_sums(groups, dh, device_out=False):
    f32 = _f32(groups.dtype)
    _need(groups, (NV, NI, NI, NI), groups.dtype, "groups")
    _stream()
    fn = _native.lib().gamer_conserved_sums_f32 if f32 else _native.lib().gamer_conserved_sums
    if device_out:
        out = torch.empty(5, dtype=torch.float64, device=groups.device)
        _native.check(fn(_ptr(groups), groups.shape[0], float(dh), _ptr(out), 1))
        return out
    host = (ctypes.c_double * 5)()
    _native.check(fn(_ptr(groups), groups.shape[0], float(dh), ctypes.cast(host, ctypes.c_void_p), 0))
    return list(host)


def pack_periodic(state, gx, gy, gz, out=None):
    f32 = _f32(state.dtype)
    _need(state, (NV, NI, NI, NI), state.dtype, "state")
    if state.shape[0] != gx * gy * gz:
        raise ValueError("state must hold gx*gy*gz groups")
    if out is None:
        out = torch.empty((state.shape[0], NV, NP, NP, NP), dtype=state.dtype, device=state.device)
    _need(out, (NV, NP, NP, NP), state.dtype, "out")
    _stream()
    fn = _native.lib().gamer_pack_periodic_f32 if f32 else _native.lib().gamer_pack_periodic
    _native.check(fn(_ptr(state), int(gx), int(gy), int(gz), _ptr(out)))
    return out


# ---- corner-transport-upwind coupling --------------------------------------

def ctu_workspace(n_groups, dtype, device):
    """A workspace tensor of the size the CTU pipeline (variant 1) needs
    (256-byte aligned by torch's allocator)."""
    nbytes = _native.lib().gamer_ctu_workspace_bytes(int(n_groups), int(_f32(dtype)))
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


CTU_FUSED = 0     # one z-sweeping launch, intermediates on chip (default)
CTU_PIPELINE = 1  # three launches through a workspace


def ctu_solve_batched(groups_in, level, dt_dev, dh_dev, gamma, out=None, fluxes_out=None,
                      group_stats=None, theta=None, work=None, bad_count=None, variant=None):
    """One step of padded groups with corner-transport-upwind coupling.
    variant: CTU_FUSED (default) or CTU_PIPELINE, which takes `work` (allocated
    here when None)."""
    f32 = _f32(groups_in.dtype)
    _need(groups_in, (NV, NP, NP, NP), groups_in.dtype, "groups_in")
    n = groups_in.shape[0]
    if out is None:
        out = torch.empty((n, NV, NI, NI, NI), dtype=groups_in.dtype, device=groups_in.device)
    _need(out, (NV, NI, NI, NI), groups_in.dtype, "out")
    if fluxes_out is not None:
        _need(fluxes_out, (3, 3, NV, NI, NI), groups_in.dtype, "fluxes_out")
    if group_stats is not None:
        _need(group_stats, (8,), torch.float64, "group_stats")
    _levels(level, dt_dev, dh_dev, n)
    variant = CTU_FUSED if variant is None else int(variant)
    if variant == CTU_PIPELINE and work is None:
        work = ctu_workspace(n, groups_in.dtype, groups_in.device)
    if work is not None and (not isinstance(work, torch.Tensor) or not work.is_cuda
                             or not work.is_contiguous()):
        raise ValueError("work must be a contiguous GPU tensor")
    opts = _opts(theta, variant, None, None, bad_count)
    _stream()
    fn = _native.lib().gamer_ctu_solve_batched_f32 if f32 else _native.lib().gamer_ctu_solve_batched
    _native.check(fn(_ptr(groups_in), n, _ptr(level), _ptr(dt_dev), _ptr(dh_dev), dt_dev.numel(),
                     float(gamma), _ptr(fluxes_out), _ptr(out), _ptr(group_stats),
                     ctypes.byref(opts) if opts is not None else None, _ptr(work),
                     0 if work is None else work.numel() * work.element_size()))
    return out


# ---- the relaxing TVD scheme ----------------------------------------------

RP = 22  # padded cells per axis of the relaxing TVD scheme


def rtvd_workspace(n_groups, dtype, device):
    """A workspace tensor of the size the relaxing-TVD entry points need."""
    nbytes = _native.lib().gamer_rtvd_workspace_bytes(int(n_groups), int(_f32(dtype)))
    return torch.empty(max(nbytes, 16), dtype=torch.uint8, device=device)


def _work(work, n, dtype, device):
    if work is None:
        work = rtvd_workspace(n, dtype, device)
    if not isinstance(work, torch.Tensor) or not work.is_cuda or not work.is_contiguous():
        raise ValueError("work must be a contiguous GPU tensor")
    return work


def rtvd_solve_batched(groups_in, level, dt_dev, dh_dev, gamma, order=0, out=None, work=None):
    """One relaxing-TVD step of padded groups (n, 5, 22, 22, 22)."""
    f32 = _f32(groups_in.dtype)
    _need(groups_in, (NV, RP, RP, RP), groups_in.dtype, "groups_in")
    n = groups_in.shape[0]
    if out is None:
        out = torch.empty((n, NV, NI, NI, NI), dtype=groups_in.dtype, device=groups_in.device)
    _need(out, (NV, NI, NI, NI), groups_in.dtype, "out")
    _levels(level, dt_dev, dh_dev, n)
    work = _work(work, n, groups_in.dtype, groups_in.device)
    _stream()
    fn = _native.lib().gamer_rtvd_solve_batched_f32 if f32 else _native.lib().gamer_rtvd_solve_batched
    _native.check(fn(_ptr(groups_in), n, _ptr(level), _ptr(dt_dev), _ptr(dh_dev), dt_dev.numel(),
                     float(gamma), int(order), _ptr(work), work.numel() * work.element_size(), _ptr(out)))
    return out


def rtvd_solve_periodic(state, gx, gy, gz, dt_dev, dh_dev, gamma, order=0, out=None, work=None):
    """One relaxing-TVD step of a uniform periodic grid, ghost cells read in place."""
    f32 = _f32(state.dtype)
    _need(state, (NV, NI, NI, NI), state.dtype, "state")
    n = state.shape[0]
    if n != gx * gy * gz:
        raise ValueError("state must hold gx*gy*gz groups")
    if out is None:
        out = torch.empty_like(state)
    _need(out, (NV, NI, NI, NI), state.dtype, "out")
    for t, nm in ((dt_dev, "dt_dev"), (dh_dev, "dh_dev")):
        if t.dtype != torch.float64 or not t.is_cuda or t.numel() < 1:
            raise ValueError(f"{nm} must be a GPU float64 tensor")
    work = _work(work, n, state.dtype, state.device)
    _stream()
    fn = _native.lib().gamer_rtvd_solve_periodic_f32 if f32 else _native.lib().gamer_rtvd_solve_periodic
    _native.check(fn(_ptr(state), int(gx), int(gy), int(gz), _ptr(dt_dev), _ptr(dh_dev), float(gamma),
                     int(order), _ptr(work), work.numel() * work.element_size(), _ptr(out)))
    return out


# ---- two refinement levels ------------------------------------------------

def _dev_scalar(t, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or t.numel() < 1:
        raise ValueError(f"{name} must be a GPU float64 tensor")


def _counter(n_bad):
    if n_bad is None:
        return None
    if not isinstance(n_bad, torch.Tensor) or n_bad.dtype != torch.int32 or not n_bad.is_cuda:
        raise ValueError("n_bad must be a GPU int32 tensor")
    return _ptr(n_bad)


def flux_accumulate(fluxes, dt_dev, acc=None, reset=False):
    """acc = (reset or acc is None ? 0 : acc) + dt_dev[0] * fluxes, in float64."""
    f32 = _f32(fluxes.dtype)
    _need(fluxes, (3, 3, NV, NI, NI), fluxes.dtype, "fluxes")
    _dev_scalar(dt_dev, "dt_dev")
    if acc is None:
        acc = torch.empty(fluxes.shape, dtype=torch.float64, device=fluxes.device)
        reset = True
    _need(acc, (3, 3, NV, NI, NI), torch.float64, "acc")
    if acc.shape[0] != fluxes.shape[0]:
        raise ValueError("acc and fluxes must hold the same number of groups")
    _stream()
    fn = _native.lib().gamer_flux_accumulate_f32 if f32 else _native.lib().gamer_flux_accumulate
    _native.check(fn(_ptr(fluxes), fluxes.shape[0], _ptr(dt_dev), int(bool(reset)), _ptr(acc)))
    return acc


def flux_correct(coarse, coarse_fluxes, fine_acc, faces, dt_dev, dh_dev, n_bad=None):
    """Coarse/fine flux correction of ``coarse`` in place.  ``faces``: a GPU
    uint8 tensor (n, 24) of gamer_cf_face records (amr.faces_to_device)."""
    f32 = _f32(coarse.dtype)
    _need(coarse, (NV, NI, NI, NI), coarse.dtype, "coarse")
    _need(coarse_fluxes, (3, 3, NV, NI, NI), coarse.dtype, "coarse_fluxes")
    if coarse_fluxes.shape[0] != coarse.shape[0]:
        raise ValueError("coarse_fluxes must hold one entry per coarse group")
    _need(fine_acc, (3, 3, NV, NI, NI), torch.float64, "fine_acc")
    _need(faces, (24,), torch.uint8, "faces")
    _dev_scalar(dt_dev, "dt_dev")
    _dev_scalar(dh_dev, "dh_dev")
    _stream()
    fn = _native.lib().gamer_flux_correct_f32 if f32 else _native.lib().gamer_flux_correct
    _native.check(fn(_ptr(coarse), coarse.shape[0], _ptr(coarse_fluxes), _ptr(fine_acc), fine_acc.shape[0],
                     _ptr(faces), faces.shape[0], _ptr(dt_dev), _ptr(dh_dev), _counter(n_bad)))
    return coarse


def restrict(fine, parent, coarse, n_bad=None):
    """Restriction of fine groups onto ``coarse`` in place; parent: GPU int64
    [n_fine] of coarse_group * 8 + octant."""
    f32 = _f32(fine.dtype)
    _need(fine, (NV, NI, NI, NI), fine.dtype, "fine")
    _need(coarse, (NV, NI, NI, NI), fine.dtype, "coarse")
    if not isinstance(parent, torch.Tensor) or parent.dtype != torch.int64 or not parent.is_cuda \
            or parent.shape != (fine.shape[0],) or not parent.is_contiguous():
        raise ValueError("parent must be a contiguous GPU int64 tensor with one entry per fine group")
    _stream()
    fn = _native.lib().gamer_restrict_f32 if f32 else _native.lib().gamer_restrict
    _native.check(fn(_ptr(fine), _ptr(parent), fine.shape[0], _ptr(coarse), coarse.shape[0], _counter(n_bad)))
    return coarse


def solver_variants(dtype) -> list:
    """(threads per work-group, waves per SIMD) of the compiled solver variants."""
    f32 = int(_f32(dtype))
    L = _native.lib()
    out = []
    for v in range(L.gamer_solver_variants(f32)):
        th, wv = ctypes.c_int(0), ctypes.c_int(0)
        _native.check(L.gamer_solver_variant_shape(f32, v, ctypes.cast(ctypes.byref(th), ctypes.c_void_p),
                                                   ctypes.cast(ctypes.byref(wv), ctypes.c_void_p)))
        out.append((th.value, wv.value))
    return out
