"""Launch-shape tuner for the batched solver.

For a given batch (precision, group count) it times every compiled solver
variant (work-group size, register budget) with one work-group per group and
with persistent grids of 1-4 work-groups per CU, checks that all candidates
agree with the first to rounding (the compiler may contract to FMA
differently under different register budgets; each variant is deterministic),
and returns (and caches) the fastest.

The cache is a JSON file keyed by device name, precision and the group count
rounded up to a power of two; ``GAMER_TUNE_CACHE`` overrides its path.
"""
from __future__ import annotations

import json
import os

import torch

from . import hydro


def cache_path() -> str:
    return os.environ.get("GAMER_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "gamer_hydro", "tune.json")


def _key(dtype, n_groups: int, periodic: bool = False, compute=None) -> str:
    name = torch.cuda.get_device_name(0)
    bucket = 1 << max(0, (int(n_groups) - 1).bit_length())
    kind = "|periodic" if periodic else ""
    prec = "f32" if dtype == torch.float32 else "f64"
    if compute is not None and compute != dtype:
        prec += "-f32compute"
    return f"{name}|{prec}|{bucket}{kind}"


def candidates(dtype, n_groups: int):
    """(variant, grid) pairs for arithmetic dtype `dtype`."""
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    grids = [0] + [n_cu * k for k in (1, 2, 3, 4) if n_cu * k < n_groups]
    # compiled variants x grids
    return [(v, g) for v in range(len(hydro.solver_variants(dtype))) for g in grids]


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(table):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # an unwritable cache only costs re-tuning


def max_rel_diff(a: torch.Tensor, b: torch.Tensor, chunk: int = 2048) -> float:
    """max |a - b| / (|b| + max over the batch of |b| per variable), in double,
    a chunk of groups at a time (no full-size temporaries)."""
    n = b.shape[0]
    scale = None
    for i in range(0, n, chunk):
        m = b[i:i + chunk].double().abs().amax(dim=(0, 2, 3, 4), keepdim=True)
        scale = m if scale is None else torch.maximum(scale, m)
    worst = 0.0
    for i in range(0, n, chunk):
        ac, bc = a[i:i + chunk].double(), b[i:i + chunk].double()
        den = bc.abs() + scale
        diff = (ac - bc).abs()
        rel = torch.where(den > 0, diff / torch.where(den > 0, den, torch.ones_like(den)),
                          torch.where(diff > 0, torch.full_like(diff, float("inf")), torch.zeros_like(diff)))
        worst = max(worst, float(rel.max()))
    return worst


def tune(padded: torch.Tensor, dt_dev: torch.Tensor, dh_dev: torch.Tensor, gamma: float,
         level=None, reps: int = 5, use_cache: bool = True, periodic=None, compute=None) -> dict:
    """Return {"variant", "grid", "ms", "table"} for this batch.  With
    ``periodic=(gx, gy, gz)``, ``padded`` is instead the interior state of a
    periodic grid and the fused periodic step is tuned; ``compute`` as in
    hydro.hydro_solve_batched."""
    key = _key(padded.dtype, padded.shape[0], periodic is not None, compute)
    cdt = compute if compute is not None else padded.dtype
    if use_cache:
        hit = _load().get(key)
        if hit is not None:
            return dict(hit, cached=True)
    n = padded.shape[0]
    out = torch.empty((n, 5, 16, 16, 16), dtype=padded.dtype, device=padded.device)

    def run(v, g):
        if periodic is None:
            hydro.hydro_solve_batched(padded, level, dt_dev, dh_dev, gamma, out=out, variant=v, grid=g,
                                      compute=compute)
        else:
            hydro.hydro_solve_periodic(padded, *periodic, dt_dev, dh_dev, gamma, out=out, variant=v,
                                       grid=g, compute=compute)

    ref = None
    table = []
    for v, g in candidates(cdt, n):
        run(v, g)
        torch.cuda.synchronize()
        if ref is None:
            ref = out.clone()
        else:
            err = max_rel_diff(out, ref)
            if not err <= (1e-6 if cdt == torch.float32 else 1e-13):
                raise RuntimeError(f"solver variant {v} grid {g} differs from variant 0 by {err:.3e}: "
                                   "refusing to tune")
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            run(v, g)
        ev[1].record()
        torch.cuda.synchronize()
        th, wv = hydro.solver_variants(cdt)[v]
        table.append({"variant": v, "threads": th, "waves_per_simd": wv,
                      "grid": g, "ms": ev[0].elapsed_time(ev[1]) / reps})
    best = min(table, key=lambda r: r["ms"])
    result = {"variant": best["variant"], "grid": best["grid"], "ms": best["ms"], "table": table}
    if use_cache:
        t = _load()
        t[key] = result
        _save(t)
    return dict(result, cached=False)
