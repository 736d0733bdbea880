#!/usr/bin/env python3
"""Throughput of the batched MUSCL-Hancock + Roe step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f32|f64|both] [--workload 5|2]

A step is one pass of the whole hot path over one batch of ghost-padded groups
already resident in HBM: the fused solver launch (reconstruction, half-step
prediction, Roe fluxes, full-step update, per-group sums and signal-speed
maxima) followed by the reduction to the CFL time step and the conserved
totals.  The time step is read on the device.  Workload (default): the 1024^3
periodic smooth-mode flow, 262144 groups of 16^3 + 2 ghost cells, the largest
batch of the paper's workload shapes that fits one GPU; seeded synthetic data.
The 256^3 grid (4096 groups) runs afterwards for the variants that are sized
for it (relaxing TVD, CTU, coarse/fine kernels, the three-level and the
high-contrast batches).

Prints one JSON line.  `value` is FP32 cell-updates/s; the FP64 figures sit
under "fp64".  The roofline object is for the solver kernel of that precision:
algorithmic flops per launch (the operations the oracle performs per
cell-update on a sample of the workload, counted by an instrumented build of
it, times the cells per launch) over the kernel's mean duration from HIP
events on the stream it is launched on.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# ---- algorithmic work model ---------------------------------------------------
CELLS = 16 ** 3
# Floating-point operations (+ - * / sqrt) per cell-update as the FP64 oracle
# performs them, counted by running it compiled with a counting number type on
# 32 groups spread over each grid (the counts and the command that produces
# them: `python -m oracle.flopcount`; a CPU test recounts and compares).  The
# MUSCL-Hancock figure is one step plus the step's epilogue on the new state
# (the CFL signal-speed maximum and the conserved sums), which the GPU step
# also computes.  Per stage on the 1024^3 sample: prim 25.4, slopes 127.0,
# predictor 545.9, Roe fluxes 1131.6 (355 per face), update 35.0, CFL 20.0,
# sums 20.0.  The oracle converts to primitives inside every physical flux and
# Roe state, so these counts include recomputation a fused kernel avoids.
FLOP_SAMPLE_CELLS = 32 * CELLS
FLOPS_PER_CELL = {5: 249667972 / FLOP_SAMPLE_CELLS, 2: 249557240 / FLOP_SAMPLE_CELLS}
CTU_FLOPS_PER_CELL = (449795732 + 5242900) / FLOP_SAMPLE_CELLS   # CTU step + the same epilogue
RTVD_FLOPS_PER_CELL = 175112048 / FLOP_SAMPLE_CELLS              # three sweeps, no epilogue

# the smallest operation count of the method (each value it needs computed
# once, counted by hand from the oracle's formulas), reported beside the
# oracle's count: operations per unit and units per group
TOUCHED = 7360        # padded cells the five-point stencils read
FACE_STATE = 5632     # interior + one ghost layer across each face
FACES = 3 * 17 * 16 * 16
MIN_FLOPS = {
    "prim": (12, TOUCHED),
    "slopes": (105, FACE_STATE),
    "predictor": (290, FACE_STATE),
    "roe": (219, FACES),
    "update": (35, CELLS),
    "cfl_sums": (24, CELLS),
}
MIN_FLOPS_PER_CELL = sum(f * n for f, n in MIN_FLOPS.values()) / CELLS


def bytes_per_group(elem: int) -> int:
    # read the padded group once, write the interior, 8 doubles of stats
    return 5 * 20 ** 3 * elem + 5 * CELLS * elem + 8 * 8


PEAK = {"f32": 157.3e12, "f64": 78.6e12}  # MI355X vector FP32 / FP64, FLOP/s
HBM_PEAK = 8.0e12
GAMMA = 5.0 / 3.0
CFL = 0.5


SOLVER_SOURCES = ("solver.hip", "euler.h", "device_math.h", "internal.h")


def read_profile_values(name):
    """The `key = value` lines of a committed counter summary under profiles/,
    or None when it is missing or was taken on other solver sources."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in SOLVER_SOURCES:
        with open(os.path.join(ROOT, "paper_1007_3818_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    vals = {}
    for line in open(path):
        if " = " in line:
            k, v = line.strip().split(" = ", 1)
            vals[k] = v
    if vals.get("solver_sources_sha256_16") != h.hexdigest()[:16]:
        return None
    return vals


def read_traffic(tag, variant, grid, n_groups):
    """HBM bytes per launch of the batched solver from the committed counter
    summary, when it was taken on the current kernel sources, batch size and
    launch shape; else None."""
    vals = read_profile_values("solve_kernel_traffic_1024.md")
    if vals is None:
        return None
    if vals.get("n_groups") != str(n_groups) or vals.get("shape") != f"{variant} {grid}":
        return None
    v = vals.get(f"bytes_per_launch_{tag}")
    return float(v) if v else None


def read_valu_lane_instr(tag, variant):
    """VALU lane-instructions per cell-update of the default batched solver
    (variant 0) from the committed SQ counter summary, when it was taken on the
    current kernel sources; else None."""
    vals = read_profile_values("solve_kernel_counters_256.md")
    if vals is None or variant != 0:
        return None
    v = vals.get(f"valu_lane_instr_per_cell_{tag}")
    return float(v) if v else None


def progress(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def bench_dtype(tag, state, g, dh, steps, warmup, workload, shape=None, pick=None):
    """The batched step of one precision on the whole grid, timed, then the
    fused periodic, HIP-graph, FP64-state/FP32-arithmetic and ghost-fill steps.
    With `pick`, one more launch of the timed configuration at the input's own
    CFL time step keeps the new state of the picked groups (and the input
    groups the oracle needs to recompute them) for the accuracy check."""
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
    hydro.group_stats(state, GAMMA, out=stats)
    hydro.step_reduce(stats, None, dh_dev, CFL, dt_out=dt_dev, totals_out=totals)
    dt0 = float(dt_dev.item())

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
    fpc = FLOPS_PER_CELL[workload]
    flops = fpc * cells
    roof = {
        "bound": "alu",
        "achieved": flops / (k_ms * 1e-3) / 1e12,
        "peak": PEAK[tag] / 1e12,
        "unit": "TFLOP/s",
        "frac": flops / (k_ms * 1e-3) / PEAK[tag],
        # HBM bytes per launch from FETCH_SIZE / WRITE_SIZE counter runs, scaled by
        # a plain copy's counters; None unless taken on these sources and shape
        "traffic": read_traffic(tag, variant, grid, n_groups),
        # the instantiation as rocprofv3 names it: <storage, arithmetic, threads,
        # waves per SIMD, periodic input, characteristic limiting>
        "kernel": "solve_kernel<{0}, {0}, {1}, {2}, false, false>".format(
            "float" if tag == "f32" else "double", *hydro.solver_variants(padded.dtype)[variant]),
        "kernel_ms": k_ms,
        "kernel_ms_median": k_median,
        "launches_timed": steps,
        "flops_per_cell": fpc,
        "flops_source": "instrumented FP64 oracle, 32 sampled groups of this workload (python -m oracle.flopcount)",
        "min_flops_per_cell": MIN_FLOPS_PER_CELL,
        "frac_at_min_flops": MIN_FLOPS_PER_CELL * cells / (k_ms * 1e-3) / PEAK[tag],
        "algorithmic_bytes_per_cell": bytes_per_group(elem) / CELLS,
        "hbm_achieved_GBps": bytes_per_group(elem) * n_groups / (k_ms * 1e-3) / 1e9,
        "hbm_frac": bytes_per_group(elem) * n_groups / (k_ms * 1e-3) / HBM_PEAK,
    }
    # the share of the VALU issue ceiling (one wave64 instruction per 4 cycles per
    # SIMD, 1,024 SIMDs at 2.4 GHz, no packed FP32) at the counted instructions
    lane = read_valu_lane_instr(tag, variant)
    if lane is not None:
        ceiling = 1024 * 2.4e9 / 4 * 64 / lane  # cell-updates/s
        roof["valu_lane_instr_per_cell"] = lane
        roof["valu_issue_ceiling_cell_updates_per_s"] = ceiling
        roof["valu_issue_frac"] = cells / (k_ms * 1e-3) / ceiling
    tot = totals.cpu().tolist()
    dt_used = float(dt_dev.item())

    # the same step (solve + reduce) captured once in a HIP graph and replayed
    progress(f"{tag}: timing HIP graph replays of the batched step")
    gb = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(gb, stream=side):
            step()
    torch.cuda.current_stream().wait_stream(side)
    for _ in range(warmup):
        gb.replay()
    torch.cuda.synchronize()
    t0.record()
    for _ in range(steps):
        gb.replay()
    t1.record()
    torch.cuda.synchronize()
    ms_gb = t0.elapsed_time(t1) / steps
    graph_batched = {"ms_per_step": ms_gb, "cell_updates_per_s": n_groups * CELLS / (ms_gb * 1e-3),
                     "dt_after": float(dt_dev.item()),
                     "step": "the timed batched step (solve + reduce) captured in one HIP graph, replayed"}
    del gb

    sample = None
    if pick is not None:
        # the timed configuration once more, at the input's own CFL time step
        dt0_dev = torch.full((1,), dt0, dtype=torch.float64, device=dev)
        hydro.hydro_solve_batched(padded, None, dt0_dev, dh_dev, GAMMA, out=out, group_stats=stats,
                                  variant=variant, grid=grid)
        need = sorted({nb for p in pick for nb in neighbourhood(p, g)})
        sample = {"dt": dt0, "pick": list(pick),
                  "gpu": out[torch.as_tensor(pick, device=dev)].double().cpu().numpy(),
                  "inputs": dict(zip(need, state[torch.as_tensor(need, device=dev)].double().cpu().numpy()))}

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
        "_sample": sample,
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
        "graph_replay_batched": graph_batched,
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
    """The CTU-coupled step on the padded groups of the same grid, at the
    MUSCL-Hancock CFL time step: the fused z-sweep (one launch, the default) and
    the pipeline (three launches through a workspace)."""
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
    out = torch.empty_like(state)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    res = {}
    for name, variant in (("fused", hydro.CTU_FUSED), ("pipeline", hydro.CTU_PIPELINE)):
        work = hydro.ctu_workspace(n, state.dtype, dev) if variant == hydro.CTU_PIPELINE else None

        def run():
            hydro.ctu_solve_batched(padded, None, dt_dev, dh_dev, GAMMA, out=out, group_stats=stats, work=work,
                                    variant=variant)
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(steps):
            run()
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / steps
        del work
        achieved = CTU_FLOPS_PER_CELL * n * CELLS / (ms * 1e-3)
        res[name] = {"ms_per_step": ms, "cell_updates_per_s": n * CELLS / (ms * 1e-3),
                     "roofline": {"bound": "alu", "flops_per_cell": CTU_FLOPS_PER_CELL,
                                  "achieved": achieved / 1e12, "peak": PEAK[tag] / 1e12, "unit": "TFLOP/s",
                                  "frac": achieved / PEAK[tag]}}
    del padded
    res["step"] = ("CTU coupling, padded input resident: one z-sweeping launch with the intermediates "
                   "on chip (fused), or three launches through a workspace (pipeline)")
    return res


RTVD_VALUES_PER_GROUP = 16 ** 3 + 2 * (16 * 22 * 22) + 2 * (16 * 16 * 22) + 16 ** 3
# arithmetic of one sweep over a pencil of 22 cells (16 updated), counted as for
# the MUSCL-Hancock model: relaxed fluxes (48 per cell) at 22 cells, half step
# (35) and relaxed fluxes again at 20, second-order fluxes with the van Leer
# limiter (110 per face) at 17 faces, the update (15) at 16 cells; pencils per
# group and step: 22 x 22, 16 x 22 and 16 x 16


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


def neighbourhood(gid, g):
    """The 27 groups around group `gid` of a periodic g^3 grid of groups (itself included)."""
    bx, by, bz = gid % g, (gid // g) % g, gid // (g * g)
    return [((bx + dx) % g) + g * (((by + dy) % g) + g * ((bz + dz) % g))
            for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def sample_groups(g):
    """The accuracy sample: the eight corner groups of the grid and eight random others."""
    import numpy as np
    rng = np.random.default_rng(5)
    corners = [x + g * (y + g * z) for x in (0, g - 1) for y in (0, g - 1) for z in (0, g - 1)]
    return sorted(set(corners) | set(int(x) for x in rng.choice(g ** 3, size=8, replace=False)))


def host_threads():
    """The host cores this process may use: the CPU share the GPU machine gives one
    GPU (it exports OMP_NUM_THREADS), else the affinity mask."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def cpu_baseline(state, g, dh, dt):
    """The FP64 oracle on the host cores, on a bounded sample of the workload
    (10-30 s of CPU work): on a grid of more than 4096 groups the groups of the
    three lowest z-layers of groups (padded by the oracle's own periodic ghost
    fill of those layers and the layers just below and above them), else every
    group; one step; all host threads, then one thread on 128 groups (the
    paper's single-core comparison)."""
    import numpy as np
    import torch
    import oracle
    threads = host_threads()
    n_all = g ** 3
    if n_all <= 4096:
        pad = oracle.pack_periodic(state.double().cpu().numpy(), g, g, g)
        what = f"all {n_all} groups"
    else:
        nl = min(3, g - 2)  # sampled layers 0 .. nl-1, with layers -1 and nl for their ghost cells
        layers = [g - 1] + list(range(nl + 1))
        sub = torch.cat([state[z * g * g:(z + 1) * g * g].double().cpu() for z in layers]).numpy()
        pad = oracle.pack_periodic(sub, g, g, nl + 2)[g * g:(nl + 1) * g * g]
        del sub
        what = f"the {nl * g * g} groups of the {nl} lowest layers of groups (of {n_all})"
    pad = np.ascontiguousarray(pad)
    n = pad.shape[0]
    oracle.set_threads(threads)
    t = time.perf_counter()
    oracle.hydro_solve(pad, dt, dh, GAMMA)
    el = time.perf_counter() - t
    oracle.set_threads(1)
    sub = pad[:128]
    t = time.perf_counter()
    oracle.hydro_solve(sub, dt, dh, GAMMA)
    el1 = time.perf_counter() - t
    return {
        "value": n * CELLS / el,
        "unit": "cell-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{what}, one FP64 step, {threads} OpenMP threads ({el:.2f} s wall, "
                  f"about {el * threads:.0f} core-seconds)",
        "one_core": {"value": sub.shape[0] * CELLS / el1, "sample": f"first 128 groups, 1 thread ({el1:.2f} s)"},
    }


def cell_errors(gpu, ref):
    """Per-cell relative errors of conserved states (n, 5, 16, 16, 16): rho and E
    against the same cell's |oracle| value, each momentum component against the
    cell's |m| + rho c_s; NaN counts as infinite."""
    import numpy as np
    rho, E = ref[:, 0], ref[:, 4]
    m2 = (ref[:, 1:4] ** 2).sum(axis=1)
    p = (GAMMA - 1.0) * (E - 0.5 * m2 / rho)
    cs = np.sqrt(np.where(p > 0, GAMMA * p / rho, 0.0))
    ms = np.sqrt(m2) + np.abs(rho) * cs
    scale = np.stack([np.abs(rho), ms, ms, ms, np.abs(E)], axis=1)
    err = np.abs(np.asarray(gpu, np.float64) - ref) / scale
    return np.where(np.isnan(err), np.inf, err)


def accuracy(samples, g, dh):
    """The picked groups' new states from the timed launch configuration of each
    precision against the FP64 oracle run on the same input groups (for FP32 the
    float-rounded input; also against the FP64 input, which adds the input's
    rounding).  Worst per-cell error and the largest per-variable L1 relative."""
    import numpy as np
    import oracle
    out = {}

    def compare(gpu, ref):
        err = cell_errors(gpu, ref)
        l1 = np.abs(gpu - ref).sum(axis=(0, 2, 3, 4)) / np.abs(ref).sum(axis=(0, 2, 3, 4))
        return {"max_rel_per_cell": float(err.max()), "l1_rel": float(l1.max())}

    refs = {}
    for tag, smp in samples.items():
        pad = oracle.pack_periodic_subset(smp["inputs"], g, g, g, smp["pick"])
        ref, _, cnt = oracle.hydro_solve(pad, smp["dt"], dh, GAMMA)
        refs[tag] = ref
        r = compare(smp["gpu"], ref)
        r["oracle_input"] = "same input" if tag == "f64" else "float-rounded input"
        r["oracle_fallbacks"] = list(cnt)
        r["groups"] = len(smp["pick"])
        r["bar"] = 1e-12 if tag == "f64" else 1e-5
        r["within_bar"] = bool(r["max_rel_per_cell"] <= r["bar"])
        out[tag] = r
    if "f32" in samples and "f64" in samples:
        # the FP32 result against the oracle on the FP64 input (input rounding included)
        s32, s64 = samples["f32"], samples["f64"]
        pad = oracle.pack_periodic_subset(s64["inputs"], g, g, g, s32["pick"])
        ref, _, _ = oracle.hydro_solve(pad, s32["dt"], dh, GAMMA)
        out["f32_vs_fp64_input"] = compare(s32["gpu"], ref)
    return out


def counter_pass(args, dev):
    """The launches a counter run measures, with few other dispatches."""
    import torch
    from paper_1007_3818_amd import hydro, workloads

    if args.dtype == "both":
        raise SystemExit("--counter-pass takes --dtype f32 or f64")
    n, kmax = (256, 4) if args.workload == 2 else (1024, 8)
    g = n // 16
    progress(f"generating workload {args.workload} on the host")
    st, dh = workloads.smooth_modes(n=n, kmax=kmax, workload=args.workload, device="cpu")
    st = (st.float() if args.dtype == "f32" else st).to(dev)
    progress("plain 1 GiB device copy")
    a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    pad = hydro.pack_periodic(st, g, g, g)
    stats = torch.empty((g ** 3, 8), dtype=torch.float64, device=dev)
    dh_dev = torch.full((1,), dh, dtype=torch.float64, device=dev)
    dt_dev = torch.empty(1, dtype=torch.float64, device=dev)
    hydro.group_stats(st, GAMMA, out=stats)
    hydro.step_reduce(stats, None, dh_dev, CFL, dt_out=dt_dev)
    # the relaxing TVD and the fused periodic step read the grid in place
    pad_state = st if args.counter_kernel in ("rtvd", "periodic") else None
    del st
    out = torch.empty((g ** 3, 5, 16, 16, 16), dtype=pad.dtype, device=dev)
    v = args.variant or 0
    for k in range(args.counter_pass):
        if args.counter_kernel == "solve":
            hydro.hydro_solve_batched(pad, None, dt_dev, dh_dev, GAMMA, out=out, group_stats=stats, variant=v,
                                      grid=args.grid)
        elif args.counter_kernel == "periodic":
            hydro.hydro_solve_periodic(pad_state if k % 2 == 0 else out, g, g, g, dt_dev, dh_dev, GAMMA,
                                       out=out if k % 2 == 0 else pad_state, group_stats=stats, variant=v,
                                       grid=args.grid)
        elif args.counter_kernel == "ctu":
            hydro.ctu_solve_batched(pad, None, dt_dev, dh_dev, GAMMA, out=out, group_stats=stats,
                                    variant=hydro.CTU_FUSED)
        else:
            hydro.rtvd_solve_periodic(out if k % 2 else pad_state, g, g, g, dt_dev, dh_dev, GAMMA, k % 2,
                                      out=pad_state if k % 2 else out)
        torch.cuda.synchronize()
        progress(f"{args.counter_kernel} {k + 1} of {args.counter_pass}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", choices=["f32", "f64", "both"], default="both")
    ap.add_argument("--workload", type=int, choices=[2, 5], default=5,
                    help="5: smooth modes 1024^3, 262144 groups (default); 2: 256^3, 4096 groups")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle legs (CPU baseline and accuracy)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip every 256^3 leg after the main workload")
    ap.add_argument("--no-amr", action="store_true", help="skip the coarse/fine kernel timings")
    ap.add_argument("--no-rtvd", action="store_true", help="skip the relaxing TVD timings")
    ap.add_argument("--no-ctu", action="store_true", help="skip the CTU-coupled step timings")
    ap.add_argument("--no-levels", action="store_true", help="skip the three-level and high-contrast batches")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (for counter scaling)")
    ap.add_argument("--counter-pass", type=int, default=0, metavar="N",
                    help="for a counter run: generate the workload on the host (a counter run serialises "
                         "every dispatch, and the device generator issues thousands), copy it over, run a "
                         "plain 1 GiB device copy, then N batched solves of --dtype at --variant/--grid, "
                         "and exit without timing")
    ap.add_argument("--counter-kernel", choices=["solve", "periodic", "ctu", "rtvd"], default="solve",
                    help="with --counter-pass: the batched solver (default), the fused periodic step, the "
                         "fused CTU step or the relaxing-TVD step (alternating sweep orders)")
    ap.add_argument("--variant", type=int, default=None,
                    help="use this compiled solver variant (with --grid) instead of tuning")
    ap.add_argument("--grid", type=int, default=0, help="launch grid with --variant (0: one per group)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; how the batch would be sharded over "
                                   "several GPUs is described in the design notes, not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1007_3818_amd import workloads

    dev = torch.device("cuda:0")
    progress("start")
    if args.counter_pass > 0:
        counter_pass(args, dev)
        return
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
    pick = sample_groups(g) if not args.no_cpu_baseline else None
    res, samples = {}, {}
    if args.dtype in ("f32", "both"):
        res["f32"] = bench_dtype("f32", state.float(), g, dh, args.steps, args.warmup, args.workload, shape, pick)
        torch.cuda.empty_cache()
    if args.dtype in ("f64", "both"):
        res["f64"] = bench_dtype("f64", state, g, dh, args.steps, args.warmup, args.workload, shape, pick)
        torch.cuda.empty_cache()
    for tag in res:
        smp = res[tag].pop("_sample")
        if smp is not None:
            samples[tag] = smp
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
            line["fp32" if tag == "f32" else "fp64"] = res[tag]
    if not args.no_cpu_baseline:
        import oracle  # noqa: F401  (only the oracle legs below use it)
        progress("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(state, g, dh, res[main_tag]["dt"])
        progress("sampled groups of the timed launches against the oracle")
        line["accuracy"] = accuracy(samples, g, dh)
    # the 256^3 grid: the legs whose workspaces are sized for it
    if not args.no_extras:
        if args.workload == 2:
            st2, dh2, g2, ext = state, dh, g, res
        else:
            del state
            torch.cuda.empty_cache()
            st2, dh2 = workloads.smooth_modes(n=256, kmax=4, workload=2, device=dev)
            g2 = 16
            ext = {}
            for tag in res:
                s2 = st2.float() if tag == "f32" else st2
                progress(f"{tag}: workload 2 (256^3) batched and fused steps")
                r2 = bench_dtype(tag, s2, g2, dh2, args.steps, args.warmup, 2)
                r2.pop("_sample")
                ext[tag] = r2
            line["workload2_256"] = {("fp32" if t == "f32" else "fp64"): v for t, v in ext.items()}
        tuned = {tag: (ext[tag]["tuning"]["variant"], ext[tag]["tuning"]["grid"]) for tag in ext}
        for tag in list(ext):
            st = st2.float() if tag == "f32" else st2
            where = ext[tag]
            if not args.no_rtvd:
                progress(f"{tag}: relaxing TVD scheme")
                where["rtvd"] = bench_rtvd(tag, st, g2, dh2, args.steps, args.warmup)
            if not args.no_ctu:
                progress(f"{tag}: CTU coupling")
                where["ctu"] = bench_ctu(tag, st, g2, dh2, max(args.steps // 5, 3), 1)
            if not args.no_amr:
                progress(f"{tag}: coarse/fine correction and restriction kernels")
                where["amr"] = bench_amr(tag, st, g2, dh2, max(args.steps, 10))
            if not args.no_levels:
                v, gr = tuned[tag]
                progress(f"{tag}: three-level batch (workload 3)")
                where["levels_batch"] = bench_levels(tag, max(args.steps // 5, 5), 2, v, gr)
                progress(f"{tag}: high-contrast flow (workload 4)")
                where["cosmo_batch"] = bench_cosmo(tag, max(args.steps // 5, 5), 2, v, gr)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
