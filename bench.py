#!/usr/bin/env python3
"""Throughput of the batched MUSCL-Hancock + Roe step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f32|f64|both]

A step is one pass of the whole hot path over one batch of ghost-padded groups
already resident in HBM: the fused solver launch (reconstruction, half-step
prediction, Roe fluxes, full-step update, per-group sums and signal-speed
maxima) followed by the reduction to the CFL time step and the conserved
totals.  The time step is read on the device.  Workload: 256^3 periodic smooth
flow (4096 groups of 16^3 + 2 ghost cells), seeded synthetic data.

Prints one JSON line.  `value` is FP32 cell-updates/s; the FP64 figures sit
under "fp64".  The roofline object is for the solver kernel of that precision:
algorithmic flops per launch (a per-cell count of the method's arithmetic,
times the cells per launch) over the kernel's mean duration from HIP events.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# ---- algorithmic work model (per group of 16^3 cells) ----------------------
CELLS = 16 ** 3
TOUCHED = 7360        # padded cells the five-point stencils read
FACE_STATE = 5632     # interior + one ghost layer across each face
FACES = 3 * 17 * 16 * 16
# arithmetic operations (+ - * / sqrt) per unit of each stage
FLOPS = {
    "prim": (12, TOUCHED),
    "slopes": (105, FACE_STATE),
    "predictor": (290, FACE_STATE),
    "roe": (219, FACES),
    "update": (35, CELLS),
    "cfl_sums": (24, CELLS),
}
FLOPS_PER_CELL = sum(f * n for f, n in FLOPS.values()) / CELLS

# the CTU coupling of the same method, counted the same way (per group): the
# one-direction predictor on the 5,824 cells of [-1,16]^3 with at most two
# coordinates outside the interior, the 16,320 transverse Roe fluxes the
# corrections use, two corrected states per final face, the final Roe fluxes
CTU_FLOPS = {
    "prim": (12, 7752),             # cells the one-direction stencils read
    "slopes": (105, 5824),
    "predictor": (285, 5824),       # per direction: face values 15, cons 24, fluxes 12,
                                    # increment 10, states 10, positivity 24
    "transverse_roe": (219, 16320),
    "corrections": (37, 2 * FACES),  # two transverse differences, the update, positivity
    "final_roe": (219, FACES),
    "update": (35, CELLS),
    "cfl_sums": (24, CELLS),
}
CTU_FLOPS_PER_CELL = sum(f * n for f, n in CTU_FLOPS.values()) / CELLS


def bytes_per_group(elem: int) -> int:
    # read the padded group once, write the interior, 8 doubles of stats
    return 5 * 20 ** 3 * elem + 5 * CELLS * elem + 8 * 8


PEAK = {"f32": 157.3e12, "f64": 78.6e12}  # MI355X vector FP32 / FP64, FLOP/s
HBM_PEAK = 8.0e12
GAMMA = 5.0 / 3.0
CFL = 0.5


def read_traffic(kernel_tag: str, variant: int, grid: int, n_groups: int):
    """HBM bytes per launch from the committed counter summary, when it was taken
    on the current kernel source, batch size and launch shape; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "solve_kernel_traffic.txt")
    if not os.path.exists(path):
        return None
    src = open(os.path.join(ROOT, "paper_1007_3818_amd", "csrc", "solver.hip"), "rb").read()
    digest = hashlib.sha256(src).hexdigest()[:16]
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("solver_sha256_16") != digest:
        return None
    if vals.get(f"shape_{kernel_tag}") != f"{variant} {grid} {n_groups}":
        return None
    v = vals.get(f"bytes_per_launch_{kernel_tag}")
    return float(v) if v else None


def progress(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def bench_dtype(tag, state, g, dh, steps, warmup, shape=None):
    import torch
    from paper_1007_3818_amd import autotune, hydro

    n_groups = g ** 3
    padded = hydro.pack_periodic(state, g, g, g)

    dev = padded.device
    out = torch.empty((n_groups, 5, 16, 16, 16), dtype=padded.dtype, device=dev)
    stats = torch.empty((n_groups, 8), dtype=torch.float64, device=dev)
    dh_dev = torch.full((1,), dh, dtype=torch.float64, device=dev)
    dt_dev = torch.empty(1, dtype=torch.float64, device=dev)
    totals = torch.empty(7, dtype=torch.float64, device=dev)
    # initial dt from the input's interior
    hydro.group_stats(padded[:, :, 2:18, 2:18, 2:18].contiguous(), GAMMA, out=stats)
    hydro.step_reduce(stats, None, dh_dev, CFL, dt_out=dt_dev, totals_out=totals)

    # pick the solver variant and launch grid for this batch on this device
    if shape is None:
        progress(f"{tag}: tuning launch shape")
        tuned = autotune.tune(padded, dt_dev, dh_dev, GAMMA, use_cache=False)
        variant, grid = tuned["variant"], tuned["grid"]
    else:
        variant, grid = shape
        tuned = {"table": []}
    progress(f"{tag}: timing variant {variant} grid {grid}")

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        hydro.hydro_solve_batched(padded, None, dt_dev, dh_dev, GAMMA, out=out, group_stats=stats,
                                  variant=variant, grid=grid)
        if ev is not None:
            ev[1].record()
        hydro.step_reduce(stats, None, dh_dev, CFL, dt_out=dt_dev, totals_out=totals)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for i in range(steps):
        step(evs[i])
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = t0.elapsed_time(t1) / steps
    k_each = sorted(a.elapsed_time(b) for a, b in evs)
    k_ms = sum(k_each) / steps
    k_median = k_each[len(k_each) // 2]
    cells = n_groups * CELLS
    elem = padded.element_size()
    flops = FLOPS_PER_CELL * cells
    traffic = read_traffic(tag, variant, grid, n_groups)
    roof = {
        "bound": "alu",
        "achieved": flops / (k_ms * 1e-3) / 1e12,
        "peak": PEAK[tag] / 1e12,
        "unit": "TFLOP/s",
        "frac": flops / (k_ms * 1e-3) / PEAK[tag],
        "traffic": traffic,
        # the instantiation as rocprofv3 names it: <storage, arithmetic, threads,
        # waves per SIMD, periodic input, characteristic limiting>
        "kernel": "solve_kernel<{0}, {0}, {1}, {2}, false, false>".format(
            "float" if tag == "f32" else "double", *hydro.solver_variants(padded.dtype)[variant]),
        "kernel_ms": k_ms,
        "kernel_ms_median": k_median,
        "flops_per_cell": FLOPS_PER_CELL,
        "algorithmic_bytes_per_cell": bytes_per_group(elem) / CELLS,
        "hbm_achieved_GBps": bytes_per_group(elem) * n_groups / (k_ms * 1e-3) / 1e9,
        "hbm_frac": bytes_per_group(elem) * n_groups / (k_ms * 1e-3) / HBM_PEAK,
    }
    tot = totals.cpu().tolist()
    dt_used = float(dt_dev.item())

    def timed_loop(one_step):
        # `out` holds a valid state after the timed steps; evolve it from there
        cur, nxt = out, torch.empty_like(out)
        for _ in range(warmup):
            one_step(cur, nxt)
            cur, nxt = nxt, cur
        torch.cuda.synchronize()
        t0.record()
        for _ in range(steps):
            one_step(cur, nxt)
            cur, nxt = nxt, cur
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / steps

    # the periodic grid advanced by the fused step (ghost cells read in place);
    # above the 256^3 grid the fused and mixed steps reuse the batched step's
    # tuned shape (tuning them would need two more state-sized arrays)
    retune = shape is None and n_groups <= 4096
    if retune:
        progress(f"{tag}: tuning the fused periodic step")
        ftuned = autotune.tune(out, dt_dev, dh_dev, GAMMA, use_cache=False, periodic=(g, g, g))
        fvariant, fgrid = ftuned["variant"], ftuned["grid"]
    else:
        fvariant, fgrid = variant, grid
    progress(f"{tag}: timing the fused periodic step, variant {fvariant} grid {fgrid}")

    def fused_step(cur, nxt):
        hydro.hydro_solve_periodic(cur, g, g, g, dt_dev, dh_dev, GAMMA, out=nxt, group_stats=stats,
                                   variant=fvariant, grid=fgrid)
        hydro.step_reduce(stats, None, dh_dev, CFL, dt_out=dt_dev, totals_out=totals)

    ms_fused = timed_loop(fused_step)

    # the same fused step, two steps per captured HIP graph, replayed
    graph = None
    if n_groups <= 4096:  # two more state-sized buffers
        from paper_1007_3818_amd.stepper import PeriodicGrid
        progress(f"{tag}: timing HIP graph replays of the fused periodic step")
        pg = PeriodicGrid(out, g, g, g, dh, GAMMA, cfl=CFL, variant=fvariant, grid=fgrid).capture()
        pg.step(2 * max(1, warmup // 2))
        pairs = max(1, steps // 2)
        torch.cuda.synchronize()
        t0.record()
        pg.step(2 * pairs)
        t1.record()
        torch.cuda.synchronize()
        ms_graph = t0.elapsed_time(t1) / (2 * pairs)
        graph = {"ms_per_step": ms_graph, "cell_updates_per_s": cells / (ms_graph * 1e-3),
                 "step": "fused periodic solve + reduce + device time accumulator, two steps per "
                         "captured graph"}
        del pg

    mixed = None
    if tag == "f64":
        # the same fused periodic step with FP64 state and FP32 arithmetic
        if retune:
            progress("f64: tuning the FP64-state, FP32-arithmetic periodic step")
            mt = autotune.tune(out, dt_dev, dh_dev, GAMMA, use_cache=False, periodic=(g, g, g),
                               compute=torch.float32)
            mvariant, mgrid = mt["variant"], mt["grid"]
        else:
            mvariant, mgrid = 0, (shape[1] if shape is not None else 0)

        def mixed_step(cur, nxt):
            hydro.hydro_solve_periodic(cur, g, g, g, dt_dev, dh_dev, GAMMA, out=nxt, group_stats=stats,
                                       variant=mvariant, grid=mgrid, compute=torch.float32)
            hydro.step_reduce(stats, None, dh_dev, CFL, dt_out=dt_dev, totals_out=totals)

        ms_mixed = timed_loop(mixed_step)
        mixed = {"ms_per_step": ms_mixed, "cell_updates_per_s": cells / (ms_mixed * 1e-3),
                 "variant": mvariant, "grid": mgrid,
                 "step": "fused periodic step, FP64 state, FP32 reconstruction/prediction/Riemann, "
                         "FP64 update + reduce"}

    progress(f"{tag}: timing ghost-fill kernel + batched step")

    def packed_step(cur, nxt):
        hydro.pack_periodic(cur, g, g, g, out=padded)
        hydro.hydro_solve_batched(padded, None, dt_dev, dh_dev, GAMMA, out=nxt, group_stats=stats,
                                  variant=variant, grid=grid)
        hydro.step_reduce(stats, None, dh_dev, CFL, dt_out=dt_dev, totals_out=totals)

    ms_full = timed_loop(packed_step)
    return {
        "value": cells / (ms_step * 1e-3),
        "ms_per_step": ms_step,
        "wall_s": wall,
        "solver_only_cell_updates_per_s": cells / (k_ms * 1e-3),
        "roofline": roof,
        "fallbacks": [int(tot[5]), int(tot[6])],
        "dt": dt_used,
        "tuning": {"variant": variant, "threads": hydro.solver_variants(padded.dtype)[variant][0],
                   "waves_per_simd": hydro.solver_variants(padded.dtype)[variant][1],
                   "grid": grid, "candidates": tuned["table"]},
        "periodic_fused": {"ms_per_step": ms_fused, "cell_updates_per_s": cells / (ms_fused * 1e-3),
                           "variant": fvariant, "grid": fgrid,
                           "step": "solve reading ghost cells from neighbouring groups + reduce, "
                                   "grid evolving"},
        "with_ghost_fill": {"ms_per_step": ms_full, "cell_updates_per_s": cells / (ms_full * 1e-3),
                            "step": "periodic ghost fill + batched solve + reduce, grid evolving"},
        **({"graph_replay": graph} if graph else {}),
        **({"fp64_state_fp32_arithmetic": mixed} if mixed else {}),
    }


def bench_amr(tag, state, g, dh, steps):
    """The coarse/fine kernels on a refined sphere of the same grid: patches
    whose centre lies within 0.3 of the box size from the centre become fine
    groups.  Per kernel: mean time over `steps` calls, algorithmic bytes, and
    the fraction of the HBM peak.  Values of the fine level do not change the
    work these kernels do, so the fine groups hold the injected coarse state and
    the fine fluxes are copies of coarse ones."""
    import numpy as np
    import torch
    from paper_1007_3818_amd import amr, hydro

    dev = state.device
    npch = 2 * g
    c = (np.arange(npch) + 0.5) / npch - 0.5
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    sel = np.argwhere(X ** 2 + Y ** 2 + Z ** 2 < 0.3 ** 2)  # (pz, py, px)
    patches = [((px // 2) + g * ((py // 2) + g * (pz // 2)), (px % 2) + 2 * (py % 2) + 4 * (pz % 2))
               for pz, py, px in sel]
    parent, faces = amr.refine(g, g, g, patches)
    nf, nr = len(parent), len(faces)
    elem = state.element_size()
    parent_t = torch.from_numpy(parent).to(dev)
    faces_t = amr.faces_to_device(faces, dev)
    coarse = state.clone()
    cfl = torch.empty((g ** 3, 3, 3, 5, 16, 16), dtype=state.dtype, device=dev)
    dt_dev = torch.full((1,), 1e-4, dtype=torch.float64, device=dev)
    dh_dev = torch.full((1,), dh, dtype=torch.float64, device=dev)
    hydro.hydro_solve_batched(hydro.pack_periodic(state, g, g, g), None, dt_dev, dh_dev, GAMMA,
                              fluxes_out=cfl)
    fine = coarse[torch.as_tensor(parent // 8, device=dev)].contiguous()
    ffl = cfl[torch.as_tensor(parent // 8, device=dev)].contiguous()
    acc = torch.zeros((nf, 3, 3, 5, 16, 16), dtype=torch.float64, device=dev)
    bad = torch.zeros(1, dtype=torch.int32, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(steps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / steps

    flux_vals = 3 * 3 * 5 * 16 * 16
    rows = {
        "flux_accumulate": (timed(lambda: hydro.flux_accumulate(ffl, dt_dev, acc=acc)),
                            nf * flux_vals * (elem + 16)),
        "flux_correct (3 launches)": (timed(lambda: hydro.flux_correct(coarse, cfl, acc, faces_t, dt_dev,
                                                                         dh_dev, n_bad=bad)),
                                      nr * 320 * (3 * elem + 32)),
        "restrict": (timed(lambda: hydro.restrict(fine, parent_t, coarse, n_bad=bad)),
                     nf * 5 * elem * (16 ** 3 + 8 ** 3)),
    }
    if int(bad.item()) != 0:
        raise RuntimeError("AMR kernels reported bad records")
    out = {"fine_groups": nf, "cf_face_records": nr}
    for k, (ms, b) in rows.items():
        out[k] = {"us": ms * 1e3, "algorithmic_bytes": b, "GBps": b / (ms * 1e-3) / 1e9,
                  "hbm_frac": b / (ms * 1e-3) / HBM_PEAK}
    return out


def bench_levels(tag, steps, warmup, variant, grid):
    """Workload 3: 512 + 4096 + 20000 groups of a Sedov blast at dh = 1, 1/2, 1/4 in
    one batched launch per step, each group reading its level's dt and dh on the
    device, then the per-level CFL reduce (the batch is not evolved: every step
    advances the same padded input)."""
    import torch
    from paper_1007_3818_amd import hydro, workloads

    dev = torch.device("cuda:0")
    dt_ = torch.float32 if tag == "f32" else torch.float64
    levels = workloads.sedov_amr(device=dev)
    pads, inter, lev = [], [], []
    for L, (groups, dh, gx, ids) in enumerate(levels):
        idt = torch.as_tensor(ids, device=dev)
        full = hydro.pack_periodic(groups.to(dt_), gx, gx, gx)
        pads.append(full[idt])
        del full
        inter.append(groups.to(dt_)[idt])
        lev.append(torch.full((len(ids),), L, dtype=torch.int8))
    batch = torch.cat(pads)
    del pads
    level = torch.cat(lev).to(dev)
    n = batch.shape[0]
    dh_dev = torch.tensor([lv[1] for lv in levels], dtype=torch.float64, device=dev)
    dt_dev = torch.empty(3, dtype=torch.float64, device=dev)
    stats = torch.empty((n, 8), dtype=torch.float64, device=dev)
    hydro.group_stats(torch.cat(inter), GAMMA, out=stats)
    del inter
    hydro.step_reduce(stats, level, dh_dev, CFL, dt_out=dt_dev)
    out = torch.empty((n, 5, 16, 16, 16), dtype=dt_, device=dev)
    totals = torch.empty(7, dtype=torch.float64, device=dev)

    def step():
        hydro.hydro_solve_batched(batch, level, dt_dev, dh_dev, GAMMA, out=out, group_stats=stats,
                                  variant=variant, grid=grid)
        hydro.step_reduce(stats, level, dh_dev, CFL, dt_out=dt_dev, totals_out=totals)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(steps):
        step()
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / steps
    del batch, out
    return {"groups": n, "levels": 3, "ms_per_step": ms, "cell_updates_per_s": n * CELLS / (ms * 1e-3),
            "variant": variant, "grid": grid,
            "step": "Sedov blast, 3 levels (512 + 4096 + 20000 groups), one batched launch with per-group "
                    "level dt/dh on the device + per-level CFL reduce"}


def bench_cosmo(tag, steps, warmup, variant, grid):
    """Workload 4: the high-contrast log-normal flow (256^3, 4096 groups, density
    1e-3..1e4, up to Mach 10), batched step + reduce, with the fallback counts of
    the first step (positivity guard of the predictor, HLLE in the Riemann solver)."""
    import torch
    from paper_1007_3818_amd import hydro, workloads

    dev = torch.device("cuda:0")
    dt_ = torch.float32 if tag == "f32" else torch.float64
    state, dh = workloads.cosmo_like(n=256, device=dev)
    padded = hydro.pack_periodic(state.to(dt_), 16, 16, 16)
    n = padded.shape[0]
    dh_dev = torch.full((1,), dh, dtype=torch.float64, device=dev)
    dt_dev = torch.empty(1, dtype=torch.float64, device=dev)
    stats = torch.empty((n, 8), dtype=torch.float64, device=dev)
    totals = torch.empty(7, dtype=torch.float64, device=dev)
    hydro.group_stats(state.to(dt_), GAMMA, out=stats)
    del state
    hydro.step_reduce(stats, None, dh_dev, CFL, dt_out=dt_dev)
    out = torch.empty((n, 5, 16, 16, 16), dtype=dt_, device=dev)

    def step():
        hydro.hydro_solve_batched(padded, None, dt_dev, dh_dev, GAMMA, out=out, group_stats=stats,
                                  variant=variant, grid=grid)
        hydro.step_reduce(stats, None, dh_dev, CFL, dt_out=dt_dev, totals_out=totals)

    step()
    first = totals.cpu().tolist()
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(steps):
        step()
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / steps
    del padded, out
    return {"ms_per_step": ms, "cell_updates_per_s": n * CELLS / (ms * 1e-3),
            "fallbacks_first_step": {"predictor_cells": int(first[5]), "hlle_faces": int(first[6])},
            "variant": variant, "grid": grid,
            "step": "log-normal density (sigma 2, clipped to 1e-3..1e4), velocities up to Mach 10, "
                    "batched step + reduce on the same padded input"}


def bench_ctu(tag, state, g, dh, steps, warmup):
    """The CTU-coupled step (three launches through a workspace) on the padded
    groups of the same grid, at the MUSCL-Hancock CFL time step."""
    import torch
    from paper_1007_3818_amd import hydro

    n = g ** 3
    dev = state.device
    padded = hydro.pack_periodic(state, g, g, g)
    dh_dev = torch.full((1,), dh, dtype=torch.float64, device=dev)
    dt_dev = torch.empty(1, dtype=torch.float64, device=dev)
    stats = torch.empty((n, 8), dtype=torch.float64, device=dev)
    hydro.group_stats(state, GAMMA, out=stats)
    hydro.step_reduce(stats, None, dh_dev, CFL, dt_out=dt_dev)
    work = hydro.ctu_workspace(n, state.dtype, dev)
    out = torch.empty_like(state)
    for _ in range(warmup):
        hydro.ctu_solve_batched(padded, None, dt_dev, dh_dev, GAMMA, out=out, group_stats=stats, work=work)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(steps):
        hydro.ctu_solve_batched(padded, None, dt_dev, dh_dev, GAMMA, out=out, group_stats=stats, work=work)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / steps
    del work, padded
    achieved = CTU_FLOPS_PER_CELL * n * CELLS / (ms * 1e-3)
    return {"ms_per_step": ms, "cell_updates_per_s": n * CELLS / (ms * 1e-3),
            "roofline": {"bound": "alu", "flops_per_cell": CTU_FLOPS_PER_CELL,
                         "achieved": achieved / 1e12, "peak": PEAK[tag] / 1e12, "unit": "TFLOP/s",
                         "frac": achieved / PEAK[tag], "scope": "whole step, three launches"},
            "step": "CTU coupling, padded input resident, three launches through a workspace"}


RTVD_VALUES_PER_GROUP = 16 ** 3 + 2 * (16 * 22 * 22) + 2 * (16 * 16 * 22) + 16 ** 3
# arithmetic of one sweep over a pencil of 22 cells (16 updated), counted as for
# the MUSCL-Hancock model: relaxed fluxes (48 per cell) at 22 cells, half step
# (35) and relaxed fluxes again at 20, second-order fluxes with the van Leer
# limiter (110 per face) at 17 faces, the update (15) at 16 cells; pencils per
# group and step: 22 x 22, 16 x 22 and 16 x 16
RTVD_FLOPS_PER_PENCIL = 22 * 48 + 20 * (35 + 48) + 17 * 110 + 16 * 15
RTVD_FLOPS_PER_CELL = RTVD_FLOPS_PER_PENCIL * (22 * 22 + 16 * 22 + 16 * 16) / CELLS


def bench_rtvd(tag, state, g, dh, steps, warmup):
    """The relaxing TVD scheme on the same periodic grid: one step = three
    sweep launches (ghost cells read in place by the first), alternating the
    sweep order.  Algorithmic bytes per group: read the state once, write and
    read the two intermediate blocks, write the result."""
    import torch
    from paper_1007_3818_amd import hydro

    n = g ** 3
    dev = state.device
    dh_dev = torch.full((1,), dh, dtype=torch.float64, device=dev)
    # the same CFL time step as the MUSCL-Hancock step (0.5 dh / max(|u|+|v|+|w|+3c)),
    # within the split scheme's per-direction limit
    stats = torch.empty((n, 8), dtype=torch.float64, device=dev)
    dt_dev = torch.empty(1, dtype=torch.float64, device=dev)
    hydro.group_stats(state, GAMMA, out=stats)
    hydro.step_reduce(stats, None, dh_dev, CFL, dt_out=dt_dev)
    work = hydro.rtvd_workspace(n, state.dtype, dev)
    cur, nxt = state.clone(), torch.empty_like(state)
    for k in range(warmup):
        hydro.rtvd_solve_periodic(cur, g, g, g, dt_dev, dh_dev, GAMMA, k % 2, out=nxt, work=work)
        cur, nxt = nxt, cur
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for k in range(steps):
        hydro.rtvd_solve_periodic(cur, g, g, g, dt_dev, dh_dev, GAMMA, k % 2, out=nxt, work=work)
        cur, nxt = nxt, cur
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / steps
    cells = n * CELLS
    if not bool(torch.isfinite(cur).all()):
        return {"error": "non-finite values after the timed steps", "ms_per_step": ms}
    b = RTVD_VALUES_PER_GROUP * 5 * state.element_size() * n
    flops = RTVD_FLOPS_PER_CELL * cells
    return {"ms_per_step": ms, "cell_updates_per_s": cells / (ms * 1e-3),
            "algorithmic_bytes_per_cell": b / cells, "hbm_GBps": b / (ms * 1e-3) / 1e9,
            "hbm_frac": b / (ms * 1e-3) / HBM_PEAK,
            "flops_per_cell": RTVD_FLOPS_PER_CELL, "alu_TFLOPs": flops / (ms * 1e-3) / 1e12,
            "alu_frac": flops / (ms * 1e-3) / PEAK[tag],
            "step": "three sweeps (x,y,z / z,y,x alternating), ghost cells read in place, CFL dt of "
                    "the initial state"}


def cpu_baseline(padded64_host, dh, dt):
    """The FP64 oracle on host cores: all groups of the workload, one step, with
    as many threads as the host offers (capped at 16)."""
    import oracle
    threads = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()))
    oracle.set_threads(threads)
    n = padded64_host.shape[0]
    t = time.perf_counter()
    ref, _, _ = oracle.hydro_solve(padded64_host, dt, dh, GAMMA)
    el = time.perf_counter() - t
    what = "all" if n == 4096 else "a sample of"
    # one core on a subset, the paper's single-core comparison
    oracle.set_threads(1)
    sub = padded64_host[:128]
    t = time.perf_counter()
    oracle.hydro_solve(sub, dt, dh, GAMMA)
    el1 = time.perf_counter() - t
    return {
        "value": n * CELLS / el,
        "unit": "cell-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{what} {n} groups of the workload, one FP64 step, {threads} OpenMP threads ({el:.2f} s)",
        "one_core": {"value": sub.shape[0] * CELLS / el1, "sample": f"first 128 groups, 1 thread ({el1:.2f} s)"},
    }, ref


def accuracy(state, g, dh, dt, ref64):
    """One step of each GPU path against the FP64 oracle on the same input (the
    oracle's step from the CPU leg; for FP32 the oracle is run again on the
    float-rounded input).  Errors per value relative to |oracle| + the
    variable's largest |oracle| (the parity tests' measure), and L1 relative
    per variable (largest over the five)."""
    import numpy as np
    import torch
    import oracle
    from paper_1007_3818_amd import hydro

    def errs(gpu, ref):
        gpu = np.asarray(gpu, dtype=np.float64)
        a = np.abs(ref)
        s = a.max(axis=(0, 2, 3, 4), keepdims=True)
        d = np.abs(gpu - ref)
        l1 = d.sum(axis=(0, 2, 3, 4)) / np.maximum(a.sum(axis=(0, 2, 3, 4)), 1e-300)
        return {"max_rel": float((d / (a + s)).max()), "l1_rel": float(l1.max())}

    dev = state.device
    dtd = torch.tensor([dt], dtype=torch.float64, device=dev)
    dhd = torch.tensor([dh], dtype=torch.float64, device=dev)
    out = {}
    p64 = hydro.pack_periodic(state, g, g, g)
    out["fp64"] = errs(hydro.hydro_solve_batched(p64, None, dtd, dhd, GAMMA).cpu().numpy(), ref64)
    out["fp64_state_fp32_arithmetic"] = errs(
        hydro.hydro_solve_batched(p64, None, dtd, dhd, GAMMA, compute=torch.float32).cpu().numpy(), ref64)
    del p64
    s32 = state.float()
    ref32, _, _ = oracle.hydro_solve(oracle.pack_periodic(s32.double().cpu().numpy(), g, g, g), dt, dh, GAMMA)
    out["fp32"] = errs(hydro.hydro_solve_batched(hydro.pack_periodic(s32, g, g, g), None, dtd, dhd, GAMMA)
                       .cpu().numpy(), ref32)
    out["fp32"]["oracle_input"] = "float-rounded input"
    out["fp32_vs_fp64_input"] = errs(
        hydro.hydro_solve_batched(hydro.pack_periodic(s32, g, g, g), None, dtd, dhd, GAMMA).cpu().numpy(), ref64)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", choices=["f32", "f64", "both"], default="both")
    ap.add_argument("--workload", type=int, choices=[2, 5], default=2,
                    help="2: smooth modes 256^3 (the metric's configuration); 5: 1024^3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-amr", action="store_true", help="skip the coarse/fine kernel timings")
    ap.add_argument("--no-rtvd", action="store_true", help="skip the relaxing TVD timings")
    ap.add_argument("--no-ctu", action="store_true", help="skip the CTU-coupled step timings")
    ap.add_argument("--no-levels", action="store_true", help="skip the three-level batch (workload 3)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (for counter scaling)")
    ap.add_argument("--variant", type=int, default=None,
                    help="use this compiled solver variant (with --grid) instead of tuning")
    ap.add_argument("--grid", type=int, default=0, help="launch grid with --variant (0: one per group)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU only; sharding across GPUs is "
                                   "described, not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1007_3818_amd import hydro, workloads

    dev = torch.device("cuda:0")
    progress("start")
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    n, kmax = (256, 4) if args.workload == 2 else (1024, 8)
    g = n // 16
    state, dh = workloads.smooth_modes(n=n, kmax=kmax, workload=args.workload, device=dev)
    n_groups = g ** 3
    progress(f"workload {args.workload} generated ({n_groups} groups)")
    shape = None if args.variant is None else (args.variant, args.grid)
    res = {}
    if args.dtype in ("f32", "both"):
        res["f32"] = bench_dtype("f32", state.float(), g, dh, args.steps, args.warmup, shape)
    if args.dtype in ("f64", "both"):
        res["f64"] = bench_dtype("f64", state, g, dh, args.steps, args.warmup, shape)
    extras = n_groups <= 4096  # the variants' workspaces are sized for the 256^3 grid
    if not args.no_rtvd and extras:
        for tag in list(res):
            progress(f"{tag}: relaxing TVD scheme")
            st = state.float() if tag == "f32" else state
            res[tag]["rtvd"] = bench_rtvd(tag, st, g, dh, args.steps, args.warmup)
    if not args.no_ctu and extras:
        for tag in list(res):
            progress(f"{tag}: CTU coupling")
            st = state.float() if tag == "f32" else state
            res[tag]["ctu"] = bench_ctu(tag, st, g, dh, max(args.steps // 5, 3), 1)
    if not args.no_amr and extras:
        for tag in list(res):
            progress(f"{tag}: coarse/fine correction and restriction kernels")
            st = state.float() if tag == "f32" else state
            res[tag]["amr"] = bench_amr(tag, st, g, dh, max(args.steps, 10))
    if extras and not args.no_levels:
        for tag in list(res):
            progress(f"{tag}: three-level batch (workload 3)")
            t = res[tag]["tuning"]
            res[tag]["levels_batch"] = bench_levels(tag, max(args.steps // 5, 5), 2, t["variant"], t["grid"])
            progress(f"{tag}: high-contrast flow (workload 4)")
            res[tag]["cosmo_batch"] = bench_cosmo(tag, max(args.steps // 5, 5), 2, t["variant"], t["grid"])
    main_tag = "f32" if "f32" in res else "f64"
    m = res[main_tag]
    line = {
        "metric": "cell-updates/s, FP32 vs FP64 MUSCL-Hancock+Roe; % of HBM/VALU roofline",
        "value": m["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_tag,
        "data": "synthetic",
        "config": {
            "workload": f"workload {args.workload}: smooth-mode flow {n}^3 periodic (|k| <= {kmax}), "
                        f"{n_groups} groups of 16^3 + 2 ghost cells, gamma 5/3, CFL 0.5",
            "groups": n_groups,
            "cells": n_groups * CELLS,
            "step": "batched solve (device dt) + CFL/totals reduce; padded input resident in HBM",
        },
        "roofline": m["roofline"],
    }
    for tag in ("f32", "f64"):
        if tag in res:
            line["fp32" if tag == "f32" else "fp64"] = {k: v for k, v in res[tag].items()}
    if not args.no_cpu_baseline:
        dt = res[main_tag]["dt"]
        import oracle  # only this leg runs the oracle
        if n_groups <= 4096:
            host_pad = oracle.pack_periodic(state.cpu().numpy(), g, g, g)
        else:  # a bounded sample of the large workload: its first 512 groups
            host_pad = oracle.pack_periodic_subset(state, g, g, g, range(512))
        progress("cpu baseline (oracle)")
        line["cpu_baseline"], ref = cpu_baseline(host_pad, dh, dt)
        if n_groups <= 4096:
            progress("one step of each path against the oracle")
            line["accuracy"] = accuracy(state, g, dh, dt, ref)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
