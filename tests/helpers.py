"""Test-side conversions between the oracle's full tensors and the HIP packed layout.

Packed layout (the library's internal storage): (c, *grid) with c components,
small strain Mandel [11,22,33,r2*23,r2*13,r2*12] (2D [11,22,r2*12]), finite
strain F row-major.  Oracle layout: (*grid, d, d).
"""

import numpy as np

R2 = np.sqrt(2.0)


def mandel_pairs(d):
    return [(0, 0), (1, 1), (0, 1)] if d == 2 else [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def pack(full, small):
    d = full.shape[-1]
    if not small:
        return np.moveaxis(full.reshape(full.shape[:-2] + (d * d,)), -1, 0).copy()
    comps = []
    for i, j in mandel_pairs(d):
        comps.append(full[..., i, i] if i == j else R2 * 0.5 * (full[..., i, j] + full[..., j, i]))
    return np.stack(comps, axis=0)


def unpack(packed, small, d):
    grid = packed.shape[1:]
    if not small:
        return np.moveaxis(packed, 0, -1).reshape(grid + (d, d)).copy()
    full = np.zeros(grid + (d, d))
    for k, (i, j) in enumerate(mandel_pairs(d)):
        if i == j:
            full[..., i, i] = packed[k]
        else:
            full[..., i, j] = full[..., j, i] = packed[k] / R2
    return full


def rel(a, b):
    """Relative 2-norm difference ||a - b|| / ||b|| (reading R18's field metric)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def relmax(a, b):
    """Element-wise difference: max |a - b| / max |b|.  A relative 2-norm can hide one wrong
    entry among many; this cannot."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def field_err(a, b):
    """The larger of the relative 2-norm and the element-wise max difference."""
    return max(rel(a, b), relmax(a, b))


def lame_fields(phase, table, density=None, p=3.0):
    table = np.asarray(table, dtype=np.float64)
    lam = table[phase, 0]
    mu = table[phase, 1]
    if density is not None:
        s = np.asarray(density) ** p
        lam, mu = lam * s, mu * s
    return lam, mu


def ncomp(kin, d):
    return (3 if d == 2 else 6) if kin == "small" else d * d
