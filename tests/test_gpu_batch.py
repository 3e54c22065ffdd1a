"""Batched stepping (one launch per step over all grids' tiles, step loop
replayed from a hipGraph) against independent single-grid runs and the
FP64 oracle."""
from __future__ import annotations

import math

import numpy as np
import pytest

import parity
from oracle import oracle as O
from paper_1907_05709_amd import workloads as W

pytestmark = pytest.mark.gpu


def small_sweep(n_inst=5, n_min=20, n_max=70, seed=4100):
    cases = []
    for i in range(n_inst):
        c = W.case_planning_instance(i, n_min=n_min, n_max=n_max, base_seed=seed)
        cases.append(c)
    return cases


def grid_for(case, **kw):
    from paper_1907_05709_amd import rfa
    g = rfa.Grid(case.shape, case.spacing, t_death=case.t_death, A=case.arrhenius_a,
                 Ea=case.arrhenius_ea, R=case.gas_r, omega_cap=case.omega_cap, **kw)
    g.load_case(case)
    return g


def state(g):
    hi, lo = g.raw_state()
    m, om, _ = g.damage()
    return hi, lo, m, om


@pytest.mark.parametrize("group_voxels,layout", [(-1, "tiles"), (120_000, "tiles"), (0, "tiles"),
                                                 (-1, "flat"), (120_000, "flat"), (0, "flat")])
def test_batch_bitwise_equals_single_grids_and_replays(group_voxels, layout):
    """Default grouping, several small groups (each runs all its steps before
    the next), and all grids in lockstep; work items as 2.5-D tiles and as
    flat plane segments."""
    from paper_1907_05709_amd import rfa
    cases = small_sweep()
    assert len({c.shape for c in cases}) > 2          # uneven grids
    singles = [grid_for(c) for c in cases]
    batched = [grid_for(c) for c in cases]
    b = rfa.Batch(batched, [c.dt for c in cases])
    plan = b.set_plan(0, 0, 0, group_voxels, layout)
    assert plan["layout"] == layout
    if group_voxels == 120_000:
        assert plan["groups"] > 1
    elif group_voxels == 0:
        assert plan["groups"] == 1
    schedule = [37, 12, 37, 1]                        # odd counts, replayed graph
    for n in schedule:
        for g, c in zip(singles, cases):
            g.step(n, c.dt, diag=False)
        b.step(n)
    ms, vs = b.last_time()
    assert vs == sum(c.n_voxels for c in cases) and ms > 0
    for g1, g2 in zip(singles, batched):
        for a1, a2 in zip(state(g1), state(g2)):
            assert np.array_equal(a1, a2)
        assert g1.step_count() == g2.step_count() == sum(schedule)
    b.close()
    for g in singles + batched:
        g.close()


@pytest.mark.parametrize("workgroups,layout", [(0, "tiles"), (7, "tiles"), (0, "flat"),
                                               (7, "flat")])
def test_batch_mixed_perfusion_fields_and_persistent_plan(workgroups, layout):
    """Grids with a perfusion multiplier field run in their own launch; the
    persistent schedule (few work-groups walking the item list) and the
    one-work-group-per-item schedule give the same bits as single grids."""
    from paper_1907_05709_amd import rfa
    cases = small_sweep(n_inst=5, seed=4600)
    rng = np.random.default_rng(4601)
    fields = [None if i % 2 else rng.uniform(0.5, 2.0, c.shape).astype(np.float32)
              for i, c in enumerate(cases)]
    singles = [grid_for(c) for c in cases]
    batched = [grid_for(c) for c in cases]
    for g1, g2, f in zip(singles, batched, fields):
        if f is not None:
            g1.set_perfusion(f)
            g2.set_perfusion(f)
    dts = [0.9 * min(c.dt, g.dt_max()) for c, g in zip(cases, singles)]
    b = rfa.Batch(batched, dts)
    b.set_plan(0, 0, workgroups, -1, layout)
    plan = b.plan()
    if workgroups:
        assert plan["workgroups"] <= 2 * workgroups
    else:
        assert plan["workgroups"] == plan["items"]
    for n in (9, 4):
        for g, dt in zip(singles, dts):
            g.step(n, dt, diag=False)
        b.step(n)
    for g1, g2 in zip(singles, batched):
        for a1, a2 in zip(state(g1), state(g2)):
            assert np.array_equal(a1, a2)
    b.close()
    for g in singles + batched:
        g.close()


def test_batch_tune_leaves_states_unchanged():
    """The tuner times candidate plans on the live grids and restores them:
    stepping on after tuning must match grids that were never tuned."""
    from paper_1907_05709_amd import rfa
    cases = small_sweep(n_inst=4, seed=4650)
    singles = [grid_for(c) for c in cases]
    batched = [grid_for(c) for c in cases]
    b = rfa.Batch(batched, [c.dt for c in cases])
    b.step(5)
    for g, c in zip(singles, cases):
        g.step(5, c.dt, diag=False)
    plan = b.tune(reps=3)
    assert plan["layout"] in ("flat", "tiles") and plan["groups"] >= 1
    assert [g.step_count() for g in batched] == [5] * len(cases)
    b.step(7)
    for g, c in zip(singles, cases):
        g.step(7, c.dt, diag=False)
    for g1, g2 in zip(singles, batched):
        for a1, a2 in zip(state(g1), state(g2)):
            assert np.array_equal(a1, a2)
    b.close()
    for g in singles + batched:
        g.close()


def test_batch_resyncs_after_a_grid_is_stepped_alone():
    from paper_1907_05709_amd import rfa
    cases = small_sweep(n_inst=3, seed=4200)
    singles = [grid_for(c) for c in cases]
    batched = [grid_for(c) for c in cases]
    b = rfa.Batch(batched, [c.dt for c in cases])
    b.step(10)
    batched[1].step(3, cases[1].dt, diag=False)      # outside the batch
    b.step(10)
    for i, (g, c) in enumerate(zip(singles, cases)):
        g.step(10, c.dt, diag=False)
        if i == 1:
            g.step(3, c.dt, diag=False)
        g.step(10, c.dt, diag=False)
    for g1, g2 in zip(singles, batched):
        for a1, a2 in zip(state(g1), state(g2)):
            assert np.array_equal(a1, a2)
    b.close()
    for g in singles + batched:
        g.close()


@pytest.mark.parametrize("group_voxels,layout", [(-1, "tiles"), (100_000, "tiles"),
                                                 (-1, "flat")])
def test_batch_diagnostics_match_single_grids(group_voxels, layout):
    from paper_1907_05709_amd import rfa
    cases = small_sweep(n_inst=4, seed=4300)
    singles = [grid_for(c) for c in cases]
    batched = [grid_for(c) for c in cases]
    b = rfa.Batch(batched, [c.dt for c in cases])
    b.set_plan(0, 0, 0, group_voxels, layout)
    d_b = b.step(70, diag=True)                       # crosses a reduction boundary
    for g, c, db in zip(singles, cases, d_b):
        ds = g.step(70, c.dt, diag=True)
        assert ds["mono_violations"] == db["mono_violations"] == 0
        assert ds["energy_J"] == db["energy_J"]
        # per-step sums are FP32 work-group partials in a different order:
        # compare against the energy budget, not the (possibly ~0) value
        scale = abs(db["injected_J"]) + abs(db["perfusion_J"]) + abs(db["boundary_J"])
        for k in ("perfusion_J", "boundary_J"):
            assert abs(ds[k] - db[k]) <= 1e-6 * scale, (k, ds[k], db[k], scale)
        assert abs(db["residual_J"]) <= 1e-6 * scale   # energy balance to FP32 partial-sum rounding
    b.close()
    for g in singles + batched:
        g.close()


def test_batch_instance_matches_oracle():
    from paper_1907_05709_amd import rfa
    cases = small_sweep(n_inst=3, n_min=24, n_max=40, seed=4400)
    grids = [grid_for(c) for c in cases]
    b = rfa.Batch(grids, [c.dt for c in cases])
    b.step(150)
    for g, c in zip(grids, cases):
        ost, _, _ = O.run(c, n_steps=150)
        T = g.temperature()
        mask, om, _ = g.damage()
        parity.compare(c, T, mask, om, ost)
    b.close()
    for g in grids:
        g.close()


def test_batch_rejects_unstable_dt_and_bad_args():
    from paper_1907_05709_amd import rfa
    cases = small_sweep(n_inst=2, seed=4500)
    grids = [grid_for(c) for c in cases]
    with pytest.raises(rfa.RfaError) as e:
        rfa.Batch(grids, [cases[0].dt, 10.0 * grids[1].dt_max()])
    assert e.value.status == rfa.RFA_ERR_UNSTABLE
    with pytest.raises(rfa.RfaError) as e:
        rfa.Batch([grids[0], grids[0]], [cases[0].dt, cases[0].dt])
    assert e.value.status == rfa.RFA_ERR_ARG
    b = rfa.Batch(grids, [c.dt for c in cases])
    before = b.plan()
    assert (before["layout"], before["tile_y"]) == ("flat", 8)   # default for nz <= 256
    for bad in (dict(tile_y=6), dict(tile_x=-1), dict(workgroups=-2), dict(layout=3),
                dict(layout="flat", tile_y=4)):
        with pytest.raises(rfa.RfaError) as e:
            b.set_plan(**bad)
        assert e.value.status == rfa.RFA_ERR_ARG
    assert b.plan() == before
    b.close()
    # flat segments of 8 waves cover grids up to nz = 256; 16 waves up to 512
    deep = W.random_tissue_case(4501, shape=(6, 5, 300), n_classes=3, n_tines=1, n_steps=4)
    gd = grid_for(deep)
    b = rfa.Batch([grids[0], gd], [cases[0].dt, deep.dt])
    before = b.plan()
    assert (before["layout"], before["tile_y"]) == ("tiles", 4)
    with pytest.raises(rfa.RfaError) as e:
        b.set_plan(tile_y=8, layout="flat")
    assert e.value.status == rfa.RFA_ERR_ARG
    assert b.plan() == before
    assert b.set_plan(tile_y=16, layout="flat")["layout"] == "flat"
    b.close()
    gd.close()
    for g in grids:
        g.close()
