"""Pins of the FP64 breathing-warp oracle (Eq. (eq:breathing)) against what
the mathematics fixes: the identity at beta = 0, exact integer shifts along
each axis (sign, axis order and per-axis spacing), exact reproduction of an
affine temperature (the trilinear interpolant of an affine field is that
field), clamping at the grid walls, and scipy's independent order-1 spline
interpolation at the same clamped positions."""
from __future__ import annotations

import numpy as np
import pytest

from oracle.warp import warp
from paper_1907_05709_amd import workloads as W

SHAPE = (9, 11, 13)
SPACING = (0.7e-3, 1.1e-3, 0.5e-3)


def _T(seed=1):
    return np.random.default_rng(seed).uniform(30.0, 120.0, SHAPE)


def test_zero_surrogate_is_the_identity():
    T = _T()
    v = np.random.default_rng(2).normal(0.0, 3e-3, (3,) + SHAPE)
    assert np.array_equal(warp(T, v, SPACING, 0.0), T)


@pytest.mark.parametrize("axis,k,beta", [(0, 2, 1.0), (1, -3, 1.0), (2, 4, 0.5)])
def test_integer_shift_along_each_axis(axis, k, beta):
    """v = k/beta voxels along one axis: the output is T shifted by k voxels,
    the positions beyond the wall take the wall's value."""
    T = _T(3)
    v = np.zeros((3,) + SHAPE)
    v[axis] = k / beta * SPACING[axis]
    out = warp(T, v, SPACING, beta)
    n = SHAPE[axis]
    src = np.clip(np.arange(n) + k, 0, n - 1)
    ref = np.take(T, src, axis=axis)
    assert np.allclose(out, ref, rtol=0, atol=1e-12)


def test_affine_temperature_is_reproduced():
    """Trilinear interpolation is exact on affine fields: at every clamped
    sample position p the output equals a + b . p."""
    a, b = 40.0, np.array([1.5, -0.75, 2.25])
    idx = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in SHAPE], indexing="ij")
    T = a + b[0] * idx[0] + b[1] * idx[1] + b[2] * idx[2]
    v = np.random.default_rng(4).normal(0.0, 2e-3, (3,) + SHAPE)
    beta = 0.8
    out = warp(T, v, SPACING, beta)
    p = [np.clip(idx[i] + beta * v[i] / SPACING[i], 0, SHAPE[i] - 1) for i in range(3)]
    ref = a + b[0] * p[0] + b[1] * p[1] + b[2] * p[2]
    assert np.abs(out - ref).max() < 1e-11


def test_matches_scipy_order_one_interpolation():
    from scipy.ndimage import map_coordinates
    T = _T(5)
    v = np.random.default_rng(6).normal(0.0, 1.5e-3, (3,) + SHAPE)
    beta = 0.6
    out = warp(T, v, SPACING, beta)
    idx = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in SHAPE], indexing="ij")
    p = np.stack([np.clip(idx[i] + beta * v[i] / SPACING[i], 0, SHAPE[i] - 1) for i in range(3)])
    ref = map_coordinates(T, p, order=1, mode="nearest")
    assert np.abs(out - ref).max() < 1e-10


def test_synthetic_breathing_field_is_smooth_and_bounded():
    """The synthetic displacement keeps the map x -> x + v(x) invertible
    (|dv/dx| well below 1 per axis) and vanishes on the walls normal to z."""
    shape, spacing = (48, 40, 64), (0.8e-3, 0.8e-3, 0.8e-3)
    v = W.breathing_field(shape, spacing).astype(np.float64)
    assert np.abs(v).max() <= 5e-3 * 1.0001
    for a in range(3):
        g = np.gradient(v[a], spacing[a], axis=a)
        assert np.abs(g).max() < 0.6
    assert np.abs(v[:, :, :, 0]).max() == 0.0 and np.abs(v[:, :, :, -1]).max() < 1e-9
    assert W.breathing_surrogate(0.0) == 0.0 and abs(W.breathing_surrogate(2.0) - 1.0) < 1e-12


def test_two_fields_match_scipy_and_reduce_to_one():
    """The two-field displacement beta v + beta2 v2: scipy's order-1
    interpolation at the clamped combined positions; beta2 = 0 is the
    one-field view bit for bit; equal fields add their weights."""
    from scipy.ndimage import map_coordinates
    T = _T(8)
    rng = np.random.default_rng(9)
    v = rng.normal(0.0, 1.5e-3, (3,) + SHAPE)
    v2 = rng.normal(0.0, 1.5e-3, (3,) + SHAPE)
    b1, b2 = 0.7, 0.4
    out = warp(T, v, SPACING, b1, v2, b2)
    idx = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in SHAPE], indexing="ij")
    p = np.stack([np.clip(idx[i] + (b1 * v[i] + b2 * v2[i]) / SPACING[i], 0, SHAPE[i] - 1)
                  for i in range(3)])
    assert np.abs(out - map_coordinates(T, p, order=1, mode="nearest")).max() < 1e-10
    assert np.array_equal(warp(T, v, SPACING, b1, v2, 0.0), warp(T, v, SPACING, b1))
    assert np.abs(warp(T, v, SPACING, b1, v, b2) - warp(T, v, SPACING, b1 + b2)).max() < 1e-10
