"""Parity at the benchmark workloads' full sizes, in the launch shapes that
bench.py times.

The oracle cannot follow the 256^3 umbrella workload for its 6000 steps
within a test, so that grid is compared with the oracle over its first
steps (every voxel, full size, the bench's launch plan) and with the
reference kernel bitwise; the 64-grid planning sweep is checked bitwise
against its grids stepped alone; the 128^3 differentiation workload's
per-tine gradients are checked against central differences of the GPU
forward at full size."""
from __future__ import annotations

import numpy as np
import pytest

import bench
import parity
from oracle import oracle as O
from paper_1907_05709_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_umbrella_256_bench_plan_matches_oracle_and_reference():
    from paper_1907_05709_amd import rfa
    n_steps = 24
    case = W.case_umbrella(n_steps=n_steps)
    zv, ty, xc = bench.PLANS[3]
    g = rfa.Grid(case.shape, case.spacing, depth=1, z_vec=zv, tile_y=ty, tile_x=xc)
    ref = rfa.Grid(case.shape, case.spacing, kernel=1)
    for x in (g, ref):
        x.load_case(case)
    plan = g.plan()
    assert (plan["z_vec"], plan["tile_y"], plan["tile_x"]) == (zv, ty, xc)
    d = g.step(n_steps, case.dt, diag=True)
    ref.step(n_steps, case.dt, diag=False)
    T = g.temperature()
    mask, om, _ = g.damage()
    for a1, a2 in zip(g.raw_state(), ref.raw_state()):
        assert np.array_equal(a1, a2)
    ost, _, _ = O.run(case, n_steps=n_steps)
    err = parity.compare(case, T, mask, om, ost)
    print(f"umbrella 256^3 x {n_steps}: max|dT| = {err:.3e} K, Tmax = {T.max():.2f}")
    assert d["mono_violations"] == 0 and T.min() >= 37.0 - 1e-9
    g.close()
    ref.close()


def test_one_gpu_slab_bench_plan_matches_oracle_and_reference():
    """The 256x34x256 y slab (one GPU's share of the 256^3 case) in the bench's
    launch plan: every voxel against the oracle over 300 steps, bitwise
    against the reference kernel."""
    import dataclasses
    from paper_1907_05709_amd import rfa
    n_steps = 300
    case, _ = bench.workload(7)
    case = dataclasses.replace(case, n_steps=n_steps)
    zv, ty, xc = bench.PLANS[7]
    g = rfa.Grid(case.shape, case.spacing, depth=1, z_vec=zv, tile_y=ty, tile_x=xc)
    ref = rfa.Grid(case.shape, case.spacing, kernel=1)
    for x in (g, ref):
        x.load_case(case)
    plan = g.plan()
    assert (plan["z_vec"], plan["tile_y"], plan["tile_x"]) == (zv, ty, xc)
    d = g.step(n_steps, case.dt, diag=True)
    ref.step(n_steps, case.dt, diag=False)
    T = g.temperature()
    mask, om, _ = g.damage()
    for a1, a2 in zip(g.raw_state(), ref.raw_state()):
        assert np.array_equal(a1, a2)
    ost, _, _ = O.run(case, n_steps=n_steps)
    err = parity.compare(case, T, mask, om, ost)
    print(f"y slab 256x34x256 x {n_steps}: max|dT| = {err:.3e} K, Tmax = {T.max():.2f}")
    assert d["mono_violations"] == 0
    g.close()
    ref.close()


def test_planning_sweep_batch_equals_grids_stepped_alone():
    from paper_1907_05709_amd import rfa
    n_steps = 9
    cases = W.planning_sweep(64, n_steps=n_steps)
    singles, batched = [], []
    for c in cases:
        for lst in (singles, batched):
            g = rfa.Grid(c.shape, c.spacing)
            g.load_case(c)
            lst.append(g)
    b = rfa.Batch(batched, [c.dt for c in cases])
    assert b.plan()["groups"] > 1
    b.step(n_steps)
    for g, c in zip(singles, cases):
        g.step(n_steps, c.dt, diag=False)
    for g1, g2 in zip(singles, batched):
        for a1, a2 in zip(g1.raw_state(), g2.raw_state()):
            assert np.array_equal(a1, a2)
    b.close()
    for g in singles + batched:
        g.close()


def test_differentiation_128_gradients_match_central_differences():
    import torch
    from paper_1907_05709_amd import rfa
    from paper_1907_05709_amd.autograd import coverage_loss
    case = W.case_differentiation()
    m, every = 16, 50
    g = rfa.Grid(case.shape, case.spacing, device=True)
    g.load_case(case)
    g.set_perfusion_bspline(np.zeros((m, m, m), np.float32))
    labels = torch.from_numpy(case.labels).cuda()
    vox = float(np.prod(case.spacing))

    def loss(powers):
        g.set_tine_powers(powers)
        g.reset_state()
        g.forward_checkpointed(case.n_steps, case.dt, every)
        _, om, _ = g.damage()
        return om, coverage_loss(om, labels, vox)

    P = case.needle.power.copy()
    om, L0 = loss(P)
    om = om.clone().requires_grad_(True)
    (w,) = torch.autograd.grad(coverage_loss(om, labels, vox), om)
    dP, _, _ = g.adjoint(w.float(), len(P), m)
    for k in np.argsort(-np.abs(dP))[:2]:
        # The FP32 forward's rounding puts a floor of ~1e-7 L under the loss
        # differences; at this size a 1e-2 relative step keeps that floor
        # below the tolerance while the central difference's truncation
        # error stays ~1e-4 relative (the 32^3 tests use 1e-3).
        h = 1e-2 * P[k]
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (float(loss(Pp)[1]) - float(loss(Pm)[1])) / (2 * h)
        print(f"tine {k}: adjoint {dP[k]:.6e}  central difference {fd:.6e}")
        assert abs(dP[k] - fd) <= 1e-3 * abs(fd) + 1e-7 * float(L0) / h
    g.close()
