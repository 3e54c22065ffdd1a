"""Edge cases on the GPU against the oracle: the smallest grids the method
admits (one free voxel, thin slabs), a grid without a source (equilibrium
must hold exactly), zero steps, a grid whose every voxel is held, and
shapes the library must reject."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

import parity
from oracle import oracle as O
from paper_1907_05709_amd import workloads as W

pytestmark = pytest.mark.gpu


def _plans(shape):
    plans = [dict(kernel=1), dict(kernel=2, depth=1, z_vec=1, tile_y=4, tile_x=4),
             dict(kernel=2, depth=2, tile_y=8, tile_x=4)]
    if shape[2] % 2 == 0:
        plans.append(dict(kernel=2, depth=1, z_vec=2, tile_y=4, tile_x=4))
    return plans


@pytest.mark.parametrize("shape", [(3, 3, 3), (3, 5, 4), (4, 3, 66), (5, 6, 3), (70, 3, 3)])
def test_minimum_grids_match_oracle_on_every_kernel(shape):
    """3^3 has a single free voxel; the others are one free voxel thick along
    one axis.  Every kernel must agree bitwise and match the oracle."""
    case = W.random_tissue_case(4700 + sum(shape), shape=shape, n_classes=4, n_tines=1,
                                n_steps=40)
    # interior voxels in the free classes 1 and 2 (class 3 is fixed), so the
    # tine has free voxels to heat
    labels = case.labels.copy()
    rng = np.random.default_rng(sum(shape))
    inner = labels[1:-1, 1:-1, 1:-1]
    inner[...] = rng.integers(1, 3, size=inner.shape)
    case = dataclasses.replace(case, labels=labels)
    ost, _, _ = O.run(case)
    ref = None
    for kw in _plans(shape):
        g, T, mask, om, _, _ = parity.gpu_run(case, **kw)
        parity.compare(case, T, mask, om, ost)
        hi, lo = g.raw_state()
        if ref is None:
            ref = (hi, lo, om)
        else:
            assert np.array_equal(hi, ref[0]) and np.array_equal(lo, ref[1])
            assert np.array_equal(om, ref[2])
        g.close()


def test_grid_without_source_stays_at_equilibrium():
    """No needle, no metabolic heat, T_a = 37 degC: every increment is exactly
    zero, so the temperature stays 37 degC bitwise while damage accrues at
    the 37 degC Arrhenius rate."""
    case = W.case_homogeneous(n=16, n_steps=200)
    none = W.Needle(np.array([0], np.int32), np.zeros((0, 3)), np.zeros(0),
                    case.needle.sigma, "none")
    case = dataclasses.replace(case, needle=none)
    ost, _, _ = O.run(case)
    g, T, mask, om, _, d = parity.gpu_run(case)
    assert np.all(T == 37.0)
    parity.compare(case, T, mask, om, ost)
    assert d["mono_violations"] == 0 and d["injected_J"] == 0.0
    assert d["t_min_C"] == d["t_max_C"] == 37.0
    g.close()


def test_zero_steps_is_a_no_op():
    from paper_1907_05709_amd import rfa
    case = W.random_tissue_case(4800, shape=(9, 7, 11), n_classes=4, n_tines=2, n_steps=5)
    g = rfa.Grid(case.shape, case.spacing)
    g.load_case(case)
    g.step(5, case.dt)
    before = (g.raw_state(), g.damage(), g.step_count())
    g.step(0, case.dt)
    after = (g.raw_state(), g.damage(), g.step_count())
    for a, b in zip(before[0] + before[1][:2], after[0] + after[1][:2]):
        assert np.array_equal(a, b)
    assert before[2] == after[2] == 5
    g.close()


def test_grid_with_every_voxel_held_does_not_change():
    """Every voxel in the fixed, non-tissue class at its fixed temperature:
    the step must leave the state bitwise unchanged and accrue no damage.
    A tine then has no free voxel to heat: both the oracle and the library
    reject it (its normalisation would divide by zero)."""
    from paper_1907_05709_amd import rfa
    case = W.random_tissue_case(4900, shape=(12, 9, 70), n_classes=4, n_tines=1, n_steps=30)
    labels = np.zeros_like(case.labels)        # class 0: fixed at 37 degC, not tissue
    needle = case.needle
    none = W.Needle(np.array([0], np.int32), np.zeros((0, 3)), np.zeros(0), needle.sigma, "none")
    case = dataclasses.replace(case, labels=labels, needle=none)
    ost, _, _ = O.run(case)
    g, T, mask, om, _, d = parity.gpu_run(case)
    assert np.all(T == 37.0) and np.all(om == 0.0) and not mask.any()
    parity.compare(case, T, mask, om, ost)
    assert d["mono_violations"] == 0
    with pytest.raises(ValueError):
        O.run(dataclasses.replace(case, needle=needle))
    with pytest.raises(rfa.RfaError) as e:
        g.set_needle(needle)
    assert e.value.status == rfa.RFA_ERR_ARG
    g.close()


@pytest.mark.parametrize("shape", [(2, 5, 5), (5, 2, 5), (5, 5, 2), (0, 5, 5)])
def test_grids_thinner_than_three_voxels_are_rejected(shape):
    from paper_1907_05709_amd import rfa
    with pytest.raises(rfa.RfaError) as e:
        rfa.Grid(shape, (1e-3, 1e-3, 1e-3))
    assert e.value.status == rfa.RFA_ERR_ARG


def test_insulating_vessel_class_exchanges_no_heat():
    """Eq. (2675-eq6)'s zero-flux reading: a held vessel class with K = 0.
    Its temperature leaves every free voxel bitwise unchanged on every
    kernel, and the state matches the oracle."""
    from helpers import box_case
    case = box_case(shape=(16, 14, 18), h=0.0, n_steps=60)
    labels = case.labels.copy()
    labels[5:9, 4:8, 2:5] = 2
    wall = dataclasses.replace(case.tissue[0], k=0.0)
    free = labels == 1
    for kw in _plans(case.shape):
        T_free = []
        for t in (20.0, 80.0):
            c = dataclasses.replace(case, labels=labels, tissue=[
                wall, case.tissue[1], W.Tissue(0.0, 1060.0, 3600.0, 0.0, 0.0, t, fixed=1,
                                               tissue=0)])
            ost, _, _ = O.run(c)
            g, T, mask, om, _, _ = parity.gpu_run(c, **kw)
            parity.compare(c, T, mask, om, ost)
            assert np.all(T[labels == 2] == t)
            T_free.append(g.raw_state()[0][free])
            g.close()
        assert np.array_equal(T_free[0], T_free[1])


def test_overflowing_state_reports_a_numeric_error():
    """A state whose next step overflows FP32 (two adjacent free voxels at
    +3e38 and -3e38 degC: their difference is beyond the float range) makes
    the diagnosed step return RFA_ERR_NUMERIC instead of a silent NaN image;
    the step without diagnostics does not check.  No fault: the kernels only
    compute with infinities."""
    from paper_1907_05709_amd import rfa
    case = W.case_homogeneous(n=12, n_steps=1)
    T0 = np.full(case.shape, 37.0)
    T0[5, 6, 6], T0[6, 6, 6] = 3e38, -3e38
    g = rfa.Grid(case.shape, case.spacing)
    g.load_case(case)
    g.set_temperature(T0)
    with pytest.raises(rfa.RfaError) as e:
        g.step(1, case.dt, diag=True)
    assert e.value.status == rfa.RFA_ERR_NUMERIC
    assert "non-finite" in str(e.value)
    assert not np.isfinite(g.temperature()).all()
    g.close()
