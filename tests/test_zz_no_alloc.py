"""rfa_damage_noalloc (the allocation-free damage outputs) against
rfa_damage, through the C ABI: identical masks, damage integrals and dead
volumes on two grids in a row (the second smaller), on host and device
pointers, with the counters cleared between calls; host masks beyond the
scratch limit are refused."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1907_05709_amd import workloads as W

pytestmark = pytest.mark.gpu


def _stepped(case, n_steps, device=False):
    from paper_1907_05709_amd import rfa
    g = rfa.Grid(case.shape, case.spacing, device=device)
    g.load_case(case)
    g.step(n_steps, case.dt, diag=False)
    return g


def _same(a, b):
    for x, y in zip(a, b):
        if hasattr(x, "cpu"):
            x, y = x.cpu().numpy(), y.cpu().numpy()
        assert np.array_equal(x, y)


def test_noalloc_damage_equals_damage_on_two_grids_in_a_row():
    """A 64^3 grid, then a smaller 40^3 one (the scratch keeps the first
    call's contents): every output equal to rfa_damage's, twice per grid
    (the dead counters start from zero on every call)."""
    for n, seed, steps in ((64, 2030, 400), (40, 2031, 250)):
        case = W.case_straight(n=n, n_steps=0, seed=seed)
        g = _stepped(case, steps)
        ref = g.damage()
        assert (ref[0] & 1).any() and (ref[0] & 2).any()
        for _ in range(2):
            _same(g.damage_noalloc(), ref)
        # outputs left out are not written and do not change the others
        m, o, d = g.damage_noalloc(want_omega=False)
        assert o is None and np.array_equal(m, ref[0]) and np.array_equal(d, ref[2])
        g.close()


def test_noalloc_damage_on_device_pointers():
    """Device grids: the mask goes straight to the caller's tensor; without
    dead volumes the call only enqueues work on the grid's stream."""
    import torch
    for n, seed in ((56, 2032), (36, 2033)):
        case = W.case_straight(n=n, n_steps=0, seed=seed)
        g = _stepped(case, 300, device=True)
        ref = g.damage()
        _same(g.damage_noalloc(), ref)
        m, o, d = g.damage_noalloc(want_dead=False)
        torch.cuda.synchronize()
        assert d is None
        _same((m, o), ref[:2])
        g.close()


def test_noalloc_damage_refuses_host_masks_beyond_the_scratch():
    from paper_1907_05709_amd import rfa
    shape = (257, 256, 256)                       # 16.8 Mi voxels > 16 Mi
    g = rfa.Grid(shape, (0.5e-3,) * 3)
    labels = np.ones(shape, np.uint8)
    g.set_tissue(labels, W.standard_tissue())
    with pytest.raises(rfa.RfaError) as e:
        g.damage_noalloc()
    assert e.value.status == rfa.RFA_ERR_ARG
    _, _, d = g.damage_noalloc(want_mask=False, want_omega=False)
    _, _, dref = g.damage()
    assert np.array_equal(d, dref)
    g.close()
