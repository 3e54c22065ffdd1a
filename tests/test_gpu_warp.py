"""Breathing-motion warp (Eq. (eq:breathing)) on the GPU against the FP64
oracle, element by element, at the project's temperature tolerance:
max |T_view - T_oracle| <= 1e-4 K.

Where the kernel's error comes from (eps = 2^-24), printed beside each
check: the output is rounded once (<= eps |T|); the lerps act on corner
excesses over the cell's nearest corner (<= ~10 eps D, D the largest such
excess, a few K); the fraction within the cell is rounded to float once per
axis (<= eps / 2 voxel times the neighbour difference G_a along that axis);
sample positions are float-float (~2^-47 relative).  Below 1024 degC a cell
reads the lo word of its nearest corner only (each dropped lo word is at
most ulp(hi) / 2 <= 3.1e-5 K); hotter cells read all eight.  On voxel
centres (zero surrogate, integer shifts, positions clamped to a wall) the
view is the float-float state rounded once to float, bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from oracle.warp import warp as warp_oracle
from paper_1907_05709_amd import workloads as W

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -24


GATE = 1e-4


def bound(T):
    """Rounding estimate of the kernel's view (see the module docstring),
    with D <= 3 max_a G_a for the excesses over a cell's first corner."""
    G = [np.abs(np.diff(T, axis=a)).max() if T.shape[a] > 1 else 0.0 for a in range(3)]
    return EPS * (np.abs(T).max() + 10 * 3 * max(G) + 0.5 * sum(G))


def rounded_state(hi, lo):
    """The float-float state 37 + hi + lo rounded to float as the kernel
    does on a voxel centre: 37 + hi split exactly, then one rounding."""
    hi = hi.astype(np.float32)
    lo = lo.astype(np.float32)
    c = np.float32(37.0)
    s = c + hi
    bv = s - c
    e = (c - (s - bv)) + (hi - bv)
    return s + (e + lo)


def _grid(shape, spacing, device=False):
    from paper_1907_05709_amd import rfa
    case = W.random_tissue_case(6100, shape=shape, n_classes=3, n_tines=1, n_steps=5)
    g = rfa.Grid(shape, spacing, device=device)
    labels = case.labels
    if device:
        import torch
        labels = torch.from_numpy(np.ascontiguousarray(labels)).cuda()
    g.set_tissue(labels, case.tissue)
    return g


@pytest.mark.parametrize("shape,beta", [((37, 29, 70), 0.7), ((3, 3, 3), 1.0),
                                        ((5, 130, 4), -0.4), ((64, 64, 65), 1.0)])
def test_warp_matches_oracle(shape, beta):
    """Ragged shapes (several work-groups plus a partial one), the smallest
    grid, a thin slab and a negative surrogate."""
    spacing = (0.8e-3, 0.9e-3, 0.7e-3)
    T = W.hot_field(shape, spacing, peak_c=600.0, sigma_m=2e-3, seed=6200 + shape[0])
    v = W.breathing_field(shape, spacing, amplitude_m=3e-3, seed=6300 + shape[1])
    g = _grid(shape, spacing)
    g.set_temperature(T)
    out = g.warp(v, beta)
    ref = warp_oracle(T, v, spacing, beta)
    err = np.abs(out.astype(np.float64) - ref).max()
    print(shape, beta, "max err", err, "rounding estimate", bound(T))
    assert out.dtype == np.float32 and err <= GATE
    g.close()


@pytest.mark.parametrize("beta", [1.0, 0.0])
def test_hot_cells_read_every_lo_word(beta):
    """A needle-hot core above 1024 degC (cells there read all eight lo
    words) in a cooler periphery (nearest corner's lo word only): within the
    gate everywhere, and bit for bit the rounded state on voxel centres."""
    shape, spacing = (40, 37, 66), (0.6e-3, 0.7e-3, 0.5e-3)
    T = W.hot_field(shape, spacing, peak_c=1500.0, sigma_m=4e-3, seed=6250)
    assert T.max() > 1300.0 and np.mean(T < 1000.0) > 0.5
    v = W.breathing_field(shape, spacing, amplitude_m=3e-3, seed=6251)
    g = _grid(shape, spacing)
    g.set_temperature(T)
    out = g.warp(v, beta)
    ref = warp_oracle(T, v, spacing, beta)
    err = np.abs(out.astype(np.float64) - ref).max()
    print("hot core max err", err, "rounding estimate", bound(T))
    assert err <= GATE
    if beta == 0.0:
        hi, lo = g.raw_state()
        assert np.array_equal(out, rounded_state(hi, lo))
    g.close()


def test_zero_surrogate_returns_the_rounded_temperature():
    shape, spacing = (20, 17, 33), (1e-3, 1e-3, 1e-3)
    T = W.hot_field(shape, spacing, seed=6400)
    v = W.breathing_field(shape, spacing, seed=6401)
    g = _grid(shape, spacing)
    g.set_temperature(T)
    out = g.warp(v, 0.0)
    hi, lo = g.raw_state()
    assert np.array_equal(out, rounded_state(hi, lo))
    assert np.abs(out - T).max() <= 2.0 * EPS * np.abs(T).max()
    g.close()


def test_displacement_beyond_the_walls_samples_the_walls():
    """Every sample position far outside the grid: the view is the wall
    voxel of each row (z pushed past the top, x past the bottom)."""
    shape, spacing = (9, 10, 12), (1e-3, 1e-3, 1e-3)
    T = W.hot_field(shape, spacing, sigma_m=3e-3, seed=6500)
    v = np.zeros((3,) + shape, np.float32)
    v[2] = 1.0
    v[0] = -0.5
    g = _grid(shape, spacing)
    g.set_temperature(T)
    out = g.warp(v, 1.0)
    ref = warp_oracle(T, v, spacing, 1.0)
    wall = np.broadcast_to(T[0:1, :, -1:], shape)
    assert np.allclose(ref, wall, rtol=0, atol=1e-9)
    assert np.abs(out - ref).max() <= 2.0 * EPS * np.abs(T).max()
    hi, lo = g.raw_state()     # on the walls the view is the rounded wall voxel, exactly
    assert np.array_equal(out, np.broadcast_to(rounded_state(hi, lo)[0:1, :, -1:], shape))
    g.close()


def test_warp_of_a_simulated_ablation_matches_oracle():
    """End to end: the oracle's state after the simulation, warped by the
    oracle, against the library's state warped by the kernel (the step
    parity bound, 1e-4 K, carries through the convex interpolation)."""
    from paper_1907_05709_amd import rfa
    O.build(force=False)
    case = W.random_tissue_case(6600, shape=(40, 36, 48), n_classes=5, n_tines=2, n_steps=200)
    ost, _, _ = O.run(case)
    T_o = ost.T
    v = W.breathing_field(case.shape, case.spacing, amplitude_m=4e-3, seed=6601)
    beta = W.breathing_surrogate(1.3)
    g = rfa.Grid(case.shape, case.spacing)
    g.load_case(case)
    g.step(case.n_steps, case.dt)
    out = g.warp(v, beta)
    ref = warp_oracle(T_o, v, case.spacing, beta)
    err = np.abs(out.astype(np.float64) - ref).max()
    print("max err", err, "rounding estimate", bound(T_o))
    assert err <= GATE
    g.close()


def test_full_size_device_warp_matches_oracle():
    """256^3 at 0.5 mm with a 12 mm field, device pointers and the launch the
    benchmark times, every voxel against the oracle."""
    import torch
    shape, spacing = (256, 256, 256), (0.5e-3,) * 3
    T = W.hot_field(shape, spacing)
    v = W.breathing_field(shape, spacing, amplitude_m=12e-3)
    g = _grid(shape, spacing, device=True)
    g.set_temperature(torch.from_numpy(T).cuda())
    out, ms = g.warp(torch.from_numpy(v).cuda(), 1.0, timed=True)
    out = out.cpu().numpy()
    ref = warp_oracle(T, v, spacing, 1.0)
    err = np.abs(out.astype(np.float64) - ref).max()
    at = np.unravel_index(np.abs(out.astype(np.float64) - ref).argmax(), shape)
    print("max err", err, "at", at, "T there", ref[at], "rounding estimate", bound(T),
          "kernel ms", ms)
    assert err <= GATE and ms > 0
    g.close()


def test_warp_beyond_buffer_offsets_matches_oracle():
    """A grid whose rows are longer than 2^24 voxels takes the kernel's
    path without buffer descriptors (64-bit addresses, full-width index
    products): same tolerance, same exact voxel centres."""
    shape, spacing = (3, 3, (1 << 24) + 1), (1e-3, 1e-3, 1e-3)
    rng = np.random.default_rng(6950)
    z = np.arange(shape[2], dtype=np.float64)
    T = np.empty(shape)
    T[:] = 37.0 + 600.0 * np.exp(-((z - 0.5 * shape[2]) / 40.0) ** 2)
    T[1] += 3.0
    T[:, 1] += 1.5
    v = np.zeros((3,) + shape, np.float32)
    v[2] = rng.uniform(-3e-3, 3e-3, shape).astype(np.float32)
    v[0] = rng.uniform(-0.4e-3, 0.4e-3, shape).astype(np.float32)
    g = _grid(shape, spacing)
    g.set_temperature(T)
    out = g.warp(v, 0.8)
    ref = warp_oracle(T, v, spacing, 0.8)
    err = np.abs(out.astype(np.float64) - ref).max()
    print("long rows max err", err)
    assert err <= GATE
    del ref
    hi, lo = g.raw_state()
    assert np.array_equal(g.warp(v, 0.0), rounded_state(hi, lo))
    g.close()


def test_warp_rejects_bad_arguments():
    from paper_1907_05709_amd import rfa
    shape = (6, 7, 8)
    g = rfa.Grid(shape, (1e-3,) * 3)
    v = np.zeros((3,) + shape, np.float32)
    with pytest.raises(rfa.RfaError) as e:        # no tissue yet
        g.warp(v, 1.0)
    assert e.value.status == rfa.RFA_ERR_STATE
    g.close()
    g = _grid(shape, (1e-3,) * 3)
    v[1, 2, 3, 4] = np.nan
    with pytest.raises(rfa.RfaError) as e:
        g.warp(v, 1.0)
    assert e.value.status == rfa.RFA_ERR_ARG
    v[1, 2, 3, 4] = 0.0
    with pytest.raises(rfa.RfaError) as e:
        g.warp(v, float("inf"))
    assert e.value.status == rfa.RFA_ERR_ARG
    with pytest.raises(ValueError):
        g.warp(v[:2], 1.0)
    g.close()


def test_integer_shift_is_exact_and_host_equals_device():
    """With a power-of-two spacing and beta = 1 the shift of k voxels is
    exact and every sample sits on a voxel centre (inside, or clamped to a
    wall), so the view is the rounded state shifted by k, bit for bit; host
    and device pointers give the same bits."""
    import torch
    shape, d = (12, 10, 33), 2.0 ** -10
    spacing = (d, d, d)
    T = W.hot_field(shape, spacing, sigma_m=2e-3, seed=6700)
    v = np.zeros((3,) + shape, np.float32)
    v[0] = -2 * d
    v[2] = 3 * d
    g = _grid(shape, spacing)
    g.set_temperature(T)
    out = g.warp(v, 1.0)
    hi, lo = g.raw_state()
    xs = np.clip(np.arange(shape[0]) - 2, 0, shape[0] - 1)
    zs = np.clip(np.arange(shape[2]) + 3, 0, shape[2] - 1)
    ref = rounded_state(hi, lo)[xs][:, :, zs]
    assert np.array_equal(out, ref)
    assert np.abs(out - warp_oracle(T, v, spacing, 1.0)).max() <= GATE
    gd = _grid(shape, spacing, device=True)
    gd.set_temperature(torch.from_numpy(T).cuda())
    outd = gd.warp(torch.from_numpy(v).cuda(), 1.0).cpu().numpy()
    assert np.array_equal(outd, out)
    g.close()
    gd.close()


@pytest.mark.parametrize("device", [False, True])
def test_keyframe_warp_matches_oracle(device):
    """Two consecutive phase fields blended 1 - a and a (the keyframe form),
    on a ragged grid, host and device pointers."""
    import torch
    shape, spacing = (29, 34, 66), (0.8e-3, 0.7e-3, 0.9e-3)
    T = W.hot_field(shape, spacing, peak_c=700.0, sigma_m=2.5e-3, seed=6800)
    v1 = W.breathing_field(shape, spacing, amplitude_m=4e-3, seed=6801)
    v2 = W.breathing_field(shape, spacing, amplitude_m=6e-3, seed=6802)
    a = 0.3
    g = _grid(shape, spacing, device=device)
    if device:
        g.set_temperature(torch.from_numpy(T).cuda())
        out = g.warp(torch.from_numpy(v1).cuda(), 1 - a, v2=torch.from_numpy(v2).cuda(),
                     beta2=a).cpu().numpy()
    else:
        g.set_temperature(T)
        out = g.warp(v1, 1 - a, v2=v2, beta2=a)
    ref = warp_oracle(T, v1, spacing, 1 - a, v2, a)
    err = np.abs(out.astype(np.float64) - ref).max()
    print("keyframe max err", err, "rounding estimate", bound(T))
    assert err <= GATE
    g.close()


def test_second_field_with_zero_weight_is_the_one_field_view():
    shape, spacing = (17, 21, 40), (1e-3, 1e-3, 1e-3)
    T = W.hot_field(shape, spacing, seed=6900)
    v1 = W.breathing_field(shape, spacing, amplitude_m=3e-3, seed=6901)
    v2 = W.breathing_field(shape, spacing, amplitude_m=5e-3, seed=6902)
    g = _grid(shape, spacing)
    g.set_temperature(T)
    assert np.array_equal(g.warp(v1, 0.8, v2=v2, beta2=0.0), g.warp(v1, 0.8))
    from paper_1907_05709_amd import rfa
    bad = v2.copy()
    bad[2, 3, 4, 5] = np.inf
    with pytest.raises(rfa.RfaError) as e:
        g.warp(v1, 0.8, v2=bad, beta2=0.5)
    assert e.value.status == rfa.RFA_ERR_ARG
    with pytest.raises(rfa.RfaError) as e:
        g.warp(v1, 0.8, v2=v2, beta2=float("nan"))
    assert e.value.status == rfa.RFA_ERR_ARG
    g.close()
