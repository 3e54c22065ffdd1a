"""Small case builders shared by the tests (inputs only, no method arithmetic)."""
from __future__ import annotations

import numpy as np

from paper_1907_05709_amd import workloads as W


def box_case(shape=(20, 18, 16), spacing=(1e-3, 1e-3, 1e-3), k=0.52, rho=1060.0,
             c=3600.0, h=24306.0, q_met=0.0, dt=0.05, n_steps=100, needle=None,
             t_boundary=37.0):
    """Homogeneous box: class 0 = held outer layer, class 1 = tissue."""
    labels = np.ones(shape, dtype=np.uint8)
    labels[0, :, :] = labels[-1, :, :] = 0
    labels[:, 0, :] = labels[:, -1, :] = 0
    labels[:, :, 0] = labels[:, :, -1] = 0
    tissue = [W.Tissue(k, rho, c, 0.0, 0.0, t_boundary, fixed=1, tissue=0),
              W.Tissue(k, rho, c, h, q_met)]
    if needle is None:
        needle = W.straight_needle([0, 0, 2e-3], [0, 0, 1], 4e-3, 5.0, max(spacing))
    return W.Case("box", tuple(shape), tuple(spacing), labels, tissue, needle, dt,
                  n_steps, 0)


def interior(a):
    return a[1:-1, 1:-1, 1:-1]


def voxel_grid(case):
    ax = W.voxel_axes(case.shape, case.spacing)
    return np.meshgrid(*ax, indexing="ij")
