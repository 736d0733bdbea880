"""Host-side bookkeeping for two refinement levels of patch groups.

A coarse level is a periodic grid of gx x gy x gz groups of 16^3 cells (group
index x + gx (y + gy z)); each group is 2 x 2 x 2 patches of 8^3 cells.
Refining a coarse patch replaces it by one fine group of 16^3 cells at half
the spacing, as in GAMER's patch-based AMR (Schive et al. 2010, cited in the
paper's Sec. 1), where the children of a patch form one patch group.

``refine`` lists, for such a set of refined patches,
  * the parent code of every fine group: coarse_group * 8 + octant, octant =
    ox + 2 oy + 4 oz (which patch of the coarse group it covers), and
  * the coarse/fine interface faces: one record per 8 x 8 coarse-cell patch
    face that separates an unrefined coarse patch from a fine group, in the
    layout of ``gamer_cf_face`` (``CF_FACE_DTYPE``).

These are the inputs of the flux-correction and restriction entry points.
Nothing here does arithmetic of the method.
"""
from __future__ import annotations

import numpy as np

# struct gamer_cf_face: int64 coarse_group, int64 fine_group, int8 dir,
# int8 coarse_face, int8 side, int8 qs, int8 qf, int8 reserved[3]  (24 bytes)
CF_FACE_DTYPE = np.dtype([
    ("coarse_group", "<i8"),
    ("fine_group", "<i8"),
    ("dir", "i1"),
    ("coarse_face", "i1"),
    ("side", "i1"),
    ("qs", "i1"),
    ("qf", "i1"),
    ("reserved", "i1", (3,)),
])
assert CF_FACE_DTYPE.itemsize == 24


def _patch_to_code(px, py, pz, gx, gy):
    g = (px // 2) + gx * ((py // 2) + gy * (pz // 2))
    return g * 8 + (px % 2) + 2 * (py % 2) + 4 * (pz % 2)


def refine(gx: int, gy: int, gz: int, patches) -> tuple[np.ndarray, np.ndarray]:
    """``patches``: iterable of (coarse_group, octant) to refine, in the order of
    the fine groups.  Returns (parent int64 [n_fine], faces CF_FACE_DTYPE [n])."""
    npx, npy, npz = 2 * gx, 2 * gy, 2 * gz
    parent = []
    coords = []
    for g, o in patches:
        g, o = int(g), int(o)
        if not (0 <= g < gx * gy * gz and 0 <= o < 8):
            raise ValueError(f"bad patch ({g}, {o})")
        bx, by, bz = g % gx, (g // gx) % gy, g // (gx * gy)
        coords.append((2 * bx + (o & 1), 2 * by + ((o >> 1) & 1), 2 * bz + ((o >> 2) & 1)))
        parent.append(g * 8 + o)
    if len(set(parent)) != len(parent):
        raise ValueError("a patch is refined twice")
    refined = set(coords)
    faces = []
    for f, (px, py, pz) in enumerate(coords):
        for d in range(3):
            for side in (0, 1):
                # side 0: the unrefined cells lie below the fine group's lower face;
                # side 1: above its upper face
                q = [px, py, pz]
                q[d] += -1 if side == 0 else 1
                q[0] %= npx
                q[1] %= npy
                q[2] %= npz
                if tuple(q) in refined:
                    continue
                code = _patch_to_code(q[0], q[1], q[2], gx, gy)
                g, o = divmod(code, 8)
                oc = ((o & 1), (o >> 1) & 1, (o >> 2) & 1)
                # the face's index within the coarse group along d: the neighbour
                # patch's upper face (side 0) or lower face (side 1)
                face_cells = 8 * oc[d] + (8 if side == 0 else 0)
                # transverse (slow, fast) axes of a plane: (z, y) for x, (z, x) for y,
                # (y, x) for z
                slow, fast = {0: (2, 1), 1: (2, 0), 2: (1, 0)}[d]
                faces.append((g, f, d, face_cells // 8, side, oc[slow], oc[fast], (0, 0, 0)))
    return np.asarray(parent, dtype=np.int64), np.array(faces, dtype=CF_FACE_DTYPE)


def covered_mask(gx: int, gy: int, gz: int, parent) -> np.ndarray:
    """Boolean (G, 16, 16, 16) of coarse cells covered by a fine group."""
    m = np.zeros((gx * gy * gz, 16, 16, 16), dtype=bool)
    for code in np.asarray(parent):
        g, o = divmod(int(code), 8)
        ox, oy, oz = o & 1, (o >> 1) & 1, (o >> 2) & 1
        m[g, 8 * oz:8 * oz + 8, 8 * oy:8 * oy + 8, 8 * ox:8 * ox + 8] = True
    return m


def faces_to_device(faces: np.ndarray, device) -> "torch.Tensor":
    """Face records as the (n, 24) uint8 GPU tensor the flux-correction entry
    point takes (the bytes of the gamer_cf_face array)."""
    import torch
    faces = np.ascontiguousarray(faces, dtype=CF_FACE_DTYPE)
    raw = faces.view(np.uint8).reshape(-1, CF_FACE_DTYPE.itemsize)
    return torch.from_numpy(raw.copy()).to(device)
