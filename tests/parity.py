"""Comparison measures of the GPU parity tests (test side only).

States are compared per cell:
  * density and total energy relative to |oracle| of the same cell;
  * each momentum component relative to |m| + rho c_s of the same cell, the
    momentum a sound wave carries there (a component that is zero, such as the
    transverse momentum of a one-dimensional problem, is still held to the
    cell's own scale, not to a batch-wide one).
c_s = sqrt(gamma p / rho) from the oracle's cell (0 if the oracle's p <= 0).
A NaN on either side fails the comparison.

Flux planes are compared per value relative to |oracle| plus the largest
|oracle| of that flux component over the batch: a face flux has no state of
its own to scale with, and its error reaches a cell only through the update,
which the state comparison covers per cell.
"""
import numpy as np

G53 = 5.0 / 3.0
NAMES = ("rho", "m_x", "m_y", "m_z", "E")


def cell_errors(gpu, ora, gamma=G53):
    """Per-cell relative errors (same shape as the inputs, (n, 5, ...))."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ora = np.asarray(ora, dtype=np.float64)
    assert gpu.shape == ora.shape and ora.shape[1] == 5, (gpu.shape, ora.shape)
    rho, E = ora[:, 0], ora[:, 4]
    m2 = (ora[:, 1:4] ** 2).sum(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        p = (gamma - 1.0) * (E - 0.5 * m2 / rho)
        cs = np.sqrt(np.where((rho > 0) & (p > 0), gamma * p / rho, 0.0))
    mscale = np.sqrt(m2) + np.abs(rho) * cs
    scale = np.stack([np.abs(rho), mscale, mscale, mscale, np.abs(E)], axis=1)
    d = np.abs(gpu - ora)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(scale > 0, d / np.where(scale > 0, scale, 1.0), np.where(d == 0, 0.0, np.inf))


def worst(err):
    """(largest error, (group, variable, cell index)) of an error array; NaN wins."""
    if err.size == 0:
        return 0.0, None
    flat = np.where(np.isnan(err), np.inf, err)
    k = int(np.argmax(flat))
    idx = np.unravel_index(k, err.shape)
    return float(err.flat[k]), (int(idx[0]), NAMES[idx[1]], tuple(int(i) for i in idx[2:]))


def state_close(gpu, ora, rtol, what="", gamma=G53):
    """Per-cell comparison of conserved states; prints and returns the worst error."""
    e, where = worst(cell_errors(gpu, ora, gamma))
    print(f"[parity] {what}: worst per-cell error {e:.3e} at {where} (bar {rtol:.0e})", flush=True)
    assert e <= rtol, f"{what}: per-cell relative error {e:.3e} at {where} > {rtol:.1e}"
    return e


def flux_close(gpu, ora, rtol, what=""):
    """Flux-plane comparison, per value relative to |oracle| + the component's
    largest |oracle| over the batch (axis 1 indexes the component)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ora = np.asarray(ora, dtype=np.float64)
    assert gpu.shape == ora.shape
    axes = tuple(i for i in range(ora.ndim) if i != 1)
    denom = np.abs(ora) + np.abs(ora).max(axis=axes, keepdims=True)
    d = np.abs(gpu - ora)
    err = np.where(denom > 0, d / np.where(denom > 0, denom, 1.0), np.where(d == 0, 0.0, np.inf))
    e = float(np.where(np.isnan(err), np.inf, err).max()) if err.size else 0.0
    assert e <= rtol, f"{what}: flux relative error {e:.3e} > {rtol:.1e}"
    return e


def l1_rel(gpu, ora):
    """L1 of the difference relative to the L1 of the oracle, per variable."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ora = np.asarray(ora, dtype=np.float64)
    axes = tuple(i for i in range(ora.ndim) if i != 1)
    den = np.abs(ora).sum(axis=axes)
    num = np.abs(gpu - ora).sum(axis=axes)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)
