"""FP64 oracle of the breathing-motion view of a temperature image.

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU
baseline leg, never by the product package; shares no code with the HIP
library.

The simulated temperature image is deformed by the inverse breathing
motion (Eq. (eq:breathing)): the temperature shown at position x is the
reference temperature at x + u(x, t), u = beta(t) v(x) with v a
displacement field in metres and beta a breathing surrogate.  Reading
(the paper does not say): T_ref between voxel centres is the trilinear
interpolant of the voxel values, and sample positions outside the grid
are clamped to its extent (the outer layer is held at 37 degC)."""
from __future__ import annotations

import numpy as np


def warp(T: np.ndarray, v: np.ndarray, spacing, beta: float) -> np.ndarray:
    """T [nx, ny, nz] (degC), v [3, nx, ny, nz] metres, spacing (dx, dy, dz)
    metres; returns T_ref(x + beta v(x)) at every voxel centre, FP64."""
    T = np.asarray(T, dtype=np.float64)
    shape = T.shape
    idx = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    lo, fr = [], []
    for a in range(3):
        p = idx[a] + float(beta) * np.asarray(v[a], dtype=np.float64) / spacing[a]
        p = np.clip(p, 0.0, shape[a] - 1.0)
        i0 = np.minimum(np.floor(p), shape[a] - 2).astype(np.int64)
        lo.append(i0)
        fr.append(p - i0)
    out = np.zeros(shape)
    for cx in (0, 1):
        wx = fr[0] if cx else 1.0 - fr[0]
        for cy in (0, 1):
            wy = fr[1] if cy else 1.0 - fr[1]
            for cz in (0, 1):
                wz = fr[2] if cz else 1.0 - fr[2]
                out += wx * wy * wz * T[lo[0] + cx, lo[1] + cy, lo[2] + cz]
    return out
