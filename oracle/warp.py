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


def warp(T: np.ndarray, v: np.ndarray, spacing, beta: float, v2=None,
         beta2: float = 0.0) -> np.ndarray:
    """T [nx, ny, nz] (degC), v [3, nx, ny, nz] metres, spacing (dx, dy, dz)
    metres; returns T_ref(x + u(x)) at every voxel centre, FP64, with the
    displacement u = beta v, or u = beta v + beta2 v2 given a second field
    (the keyframe form of the motion model: two consecutive phase fields
    weighted 1 - a and a; or a regression on two surrogate signals)."""
    T = np.asarray(T, dtype=np.float64)
    shape = T.shape
    idx = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    lo, fr = [], []
    for a in range(3):
        u = float(beta) * np.asarray(v[a], dtype=np.float64)
        if v2 is not None:
            u = u + float(beta2) * np.asarray(v2[a], dtype=np.float64)
        p = idx[a] + u / spacing[a]
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
