"""Discrete adjoint on the GPU (checkpoint + recompute) against the FP64
oracle's discrete adjoint and against central finite differences of the GPU
forward; the autograd bridge against direct adjoint calls.

Loss: soft undertreatment of the tumour + 0.1 x healthy-liver damage volume
(cm^3), d = sigmoid(4 ln Omega).  Gradients with respect to the per-tine
powers and a B-spline perfusion-correction lattice."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_05709_amd import workloads as W

pytestmark = pytest.mark.gpu

N_STEPS, DT, EVERY, M = 60, 0.2, 7, 8
# Element-wise gradient tolerances.  Against the oracle's FP64 discrete
# adjoint: 1e-3 relative plus 1e-5 of the largest component (the FP32
# adjoint's rounding, ~1e-5 relative, is amplified where a component is a
# sum of contributions of both signs; a tine whose gradient is 1 % of the
# largest is then held to 2e-3).  Against central differences of the FP32
# forward: 1e-3 relative plus 3e-4 of the largest component, the
# differences' own rounding noise.  The loss of the FP32 forward carries
# ~3e-9 of rounding noise, i.e. noise / (2 h) in a difference quotient:
# with a step of 1e-3 of a tine's power that is ~1.5e-4 of the largest
# tine gradient (measured at 32^3 and 128^3); a control value's step of
# 1e-3 is 10^3 times smaller relative to its gradient scale, so control
# values use Richardson's extrapolation of central differences at steps
# 1e-2 and 2e-2 (O(h^4) truncation), whose noise is 10x smaller.
ORACLE_RTOL, ORACLE_FLOOR = 1e-3, 1e-5
FD_RTOL, FD_FLOOR = 1e-3, 3e-4


def within(got, want, rtol, floor, scale):
    return np.abs(got - want) <= rtol * np.abs(want) + floor * scale


def coverage(case, omega):
    """Loss and dL/dOmega in FP64 (numpy), same definition as the autograd
    helper."""
    lab = case.labels
    om = np.clip(omega.astype(np.float64), 0.0, None)
    om4 = om ** 4
    d = om4 / (1.0 + om4)
    tum = lab == W.LABEL_TUMOUR
    liv = lab == W.LABEL_LIVER
    V = np.prod(case.spacing) * 1e6
    L = (1.0 - d[tum]).mean() + 0.1 * d[liv].sum() * V
    dd = 4.0 * om ** 3 / (1.0 + om4) ** 2
    w = np.zeros_like(om)
    w[tum] = -dd[tum] / tum.sum()
    w[liv] += 0.1 * V * dd[liv]
    return L, w


@pytest.fixture(scope="module")
def setup():
    O.build(force=False)
    case = W.case_differentiation(n=32, dx=2e-3, n_steps=N_STEPS, dt=DT, seed=5001)
    rng = np.random.default_rng(5)
    ctrl = (0.3 * rng.standard_normal((M, M, M))).astype(np.float32)
    return case, ctrl


def gpu_grid(case, ctrl, **plan):
    from paper_1907_05709_amd import rfa
    g = rfa.Grid(case.shape, case.spacing, **plan)
    g.load_case(case)
    g.set_perfusion_bspline(ctrl)
    return g


def gpu_loss(g, case, powers):
    g.set_tine_powers(powers)
    g.reset_state()
    g.forward_checkpointed(N_STEPS, DT, EVERY)
    _, om, _ = g.damage()
    return coverage(case, om)


@pytest.mark.parametrize("zero_tine", [False, True])
def test_adjoint_matches_oracle_discrete_adjoint(setup, zero_tine):
    """Every gradient component against the oracle's FP64 adjoint; with a
    tine switched off (zero power) its gradient comes from voxels where the
    RF increment is 0, outside the flagged source support."""
    import copy
    case, ctrl = setup
    g = gpu_grid(case, ctrl)
    P = case.needle.power.copy()
    if zero_tine:
        P[3] = 0.0
        case = copy.deepcopy(case)
        case.needle.power = P.copy()
    L, w = gpu_loss(g, case, P)
    dP, dc, dperf = g.adjoint(w.astype(np.float32), len(P), M, want_dperf=True)
    # oracle: same inputs, FP64 throughout
    f = O.bspline_field(case.shape, ctrl.astype(np.float64))
    q, gt, _ = O.source(case, per_tine=True)
    dq, dperf_o = O.adjoint(case, w, n_steps=N_STEPS, dt=DT, q=q, perf=f)
    dP_o = np.tensordot(gt, dq, axes=([1, 2, 3], [0, 1, 2]))
    dc_o = O.bspline_grad(f, dperf_o, M)
    # element by element: every tine, every control value, every voxel's
    # perfusion gradient (ORACLE_RTOL relative plus ORACLE_FLOOR of the
    # largest component)
    rel_p = np.abs(dP - dP_o) / np.abs(dP_o)
    rel_c = np.abs(dc - dc_o) / np.abs(dc_o)
    wc = np.unravel_index(rel_c.argmax(), rel_c.shape)
    big = np.abs(dperf_o) > 1e-3 * np.abs(dperf_o).max()
    rel_f = np.abs(dperf[big] - dperf_o[big]) / np.abs(dperf_o[big])
    print("dP gpu", dP, "\ndP oracle", dP_o)
    print(f"worst tine rel {rel_p.max():.2e} (tine {rel_p.argmax()}, |dP| "
          f"{np.abs(dP_o[rel_p.argmax()]) / np.abs(dP_o).max():.3f} of the largest); worst "
          f"control value rel {rel_c.max():.2e} at {wc} ({dc[wc]:.4e} vs {dc_o[wc]:.4e}); "
          f"worst voxel dL/dperf rel {rel_f.max():.2e} over the {int(big.sum())} voxels above "
          f"1e-3 of the largest")
    assert within(dP, dP_o, ORACLE_RTOL, ORACLE_FLOOR, np.abs(dP_o).max()).all()
    assert within(dc, dc_o, ORACLE_RTOL, ORACLE_FLOOR, np.abs(dc_o).max()).all()
    assert within(dperf, dperf_o, ORACLE_RTOL, ORACLE_FLOOR, np.abs(dperf_o).max()).all()
    g.close()


def test_adjoint_matches_central_differences(setup):
    case, ctrl = setup
    g = gpu_grid(case, ctrl)
    P = case.needle.power.copy()
    L0, w = gpu_loss(g, case, P)
    dP, dc, _ = g.adjoint(w.astype(np.float32), len(P), M)
    # every tine, central differences with a step of 1e-3 relative
    worst = 0.0
    for k in range(len(P)):
        h = 1e-3 * P[k]
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (gpu_loss(g, case, Pp)[0] - gpu_loss(g, case, Pm)[0]) / (2 * h)
        print("tine", k, dP[k], fd)
        worst = max(worst, abs(dP[k] - fd) / abs(fd))
        assert within(dP[k], fd, FD_RTOL, FD_FLOOR, np.abs(dP).max())
    print(f"worst tine against central differences: {worst:.2e}")
    # control values: the three largest gradients, and the two largest among
    # the control values of the lattice's end spans (index 0, 1, M - 2 or
    # M - 1 along some axis: the knot spans clamped at the grid's faces),
    # step 1e-3 max(|c|, 1)
    mags = np.abs(dc)
    flat = list(np.argsort(-mags.ravel())[:3])
    ii = np.indices(dc.shape)
    outer = ((ii <= 1) | (ii >= M - 2)).any(axis=0).ravel()
    cand = np.flatnonzero(outer)
    edge = list(cand[np.argsort(-mags.ravel()[cand])[:2]])
    assert mags.ravel()[edge].min() > 1e-3 * mags.max()
    flat += edge
    def central(idx, h):
        cp, cm = ctrl.copy(), ctrl.copy()
        cp[idx] += np.float32(h)
        cm[idx] -= np.float32(h)
        hh = float(cp[idx]) - float(cm[idx])
        g.set_perfusion_bspline(cp)
        Lp = gpu_loss(g, case, P)[0]
        g.set_perfusion_bspline(cm)
        Lm = gpu_loss(g, case, P)[0]
        return (Lp - Lm) / hh

    worst = 0.0
    for j in flat:
        idx = np.unravel_index(j, dc.shape)
        h = 1e-2 * max(abs(float(ctrl[idx])), 1.0)
        f1, f2 = central(idx, h), central(idx, 2 * h)
        fd = (4.0 * f1 - f2) / 3.0
        print("ctrl", idx, dc[idx], fd, "(steps h, 2h:", f1, f2, ")")
        worst = max(worst, abs(dc[idx] - fd) / abs(fd))
        assert within(dc[idx], fd, FD_RTOL, FD_FLOOR, np.abs(dc).max())
    print(f"worst control value against central differences: {worst:.2e}")
    g.set_perfusion_bspline(ctrl)
    g.close()


@pytest.mark.parametrize("shape", [(37, 29, 70), (21, 45, 130), (19, 23, 67), (9, 40, 258)])
def test_tiled_adjoint_bitwise_equals_reference(shape):
    """The tiled adjoint kernel (x-march, LDS plane, predicated stores) and
    the one-thread-per-voxel reference share the per-voxel update: the same
    gradients bit for bit, on ragged tiles (odd and even nz, a ragged last
    z tile) with a perfusion field."""
    from paper_1907_05709_amd import rfa
    case = W.random_tissue_case(77, shape=shape, n_classes=5, n_tines=2, n_steps=30)
    field = np.random.default_rng(78).uniform(0.5, 2.0, shape).astype(np.float32)
    w = np.random.default_rng(79).standard_normal(shape).astype(np.float32)
    outs = []
    for kernel in (1, 2):
        g = rfa.Grid(case.shape, case.spacing, kernel=kernel)
        g.load_case(case)
        g.set_perfusion(field)
        dt = 0.9 * min(case.dt, g.dt_max())
        g.reset_state()
        g.forward_checkpointed(30, dt, 7)
        outs.append(g.adjoint(w, 2, 0, want_dperf=True))
        g.close()
    (dP1, _, f1), (dP2, _, f2) = outs
    assert np.abs(dP1).max() > 0 and np.abs(f1).max() > 0
    assert np.array_equal(dP1, dP2) and np.array_equal(f1, f2)


# the automatic plan, and the wide kernel (two z voxels per lane), whose
# recompute steps skip the damage integral and class bytes
@pytest.mark.parametrize("plan", [{}, dict(z_vec=2, tile_y=4, tile_x=8)])
def test_checkpoint_spacing_does_not_change_gradients(setup, plan):
    case, ctrl = setup
    g = gpu_grid(case, ctrl, **plan)
    if plan:
        assert g.plan()["z_vec"] == 2 and g.plan()["depth"] == 1
    P = case.needle.power.copy()
    g.set_tine_powers(P)
    out = []
    for every in (EVERY, N_STEPS, 1, 0):   # 0: the whole trajectory kept, no recomputation
        g.reset_state()
        g.forward_checkpointed(N_STEPS, DT, every)
        _, om, _ = g.damage()
        _, w = coverage(case, om)
        out.append(g.adjoint(w.astype(np.float32), len(P), M, want_dperf=True))
        # the forward writes the last segment's trajectory itself; a second
        # adjoint of the same forward recomputes that segment too
        again = g.adjoint(w.astype(np.float32), len(P), M, want_dperf=True)
        for a, b in zip(out[-1], again):
            assert np.array_equal(a, b)
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    for a, b in zip(out[0], out[2]):
        assert np.array_equal(a, b)
    for a, b in zip(out[0], out[3]):
        assert np.array_equal(a, b)
    g.close()


def test_autograd_function_and_state_checks(setup):
    import torch
    from paper_1907_05709_amd import rfa
    from paper_1907_05709_amd.autograd import RfaFunction, coverage_loss
    case, ctrl = setup
    g = rfa.Grid(case.shape, case.spacing, device=True)
    g.load_case(case)
    labels = torch.from_numpy(case.labels).cuda()
    p = torch.tensor(case.needle.power, dtype=torch.float64, requires_grad=True)
    c = torch.tensor(ctrl, dtype=torch.float32, requires_grad=True)
    om = RfaFunction.apply(p, c, g, N_STEPS, DT, EVERY)
    loss = coverage_loss(om, labels, float(np.prod(case.spacing)))
    loss.backward()
    # the same gradients through the direct calls
    h = gpu_grid(case, ctrl)
    L, w = gpu_loss(h, case, case.needle.power.copy())
    dP, dc, _ = h.adjoint(w.astype(np.float32), len(case.needle.power), M)
    assert abs(float(loss) - L) <= 1e-9 * abs(L)
    assert np.allclose(p.grad.numpy(), dP, rtol=1e-5, atol=0)
    assert np.allclose(c.grad.numpy(), dc, rtol=1e-4, atol=1e-6 * np.abs(dc).max())
    # the grid changed since the forward: no adjoint
    h.step(1, DT, diag=False)
    with pytest.raises(rfa.RfaError) as e:
        h.adjoint(w.astype(np.float32), len(case.needle.power), M)
    assert e.value.status == rfa.RFA_ERR_STATE
    torch.cuda.synchronize()
    g.close()
    h.close()


def test_projected_adam_plan_optimisation_lowers_the_loss(setup):
    """The downstream use of the gradients: a few projected Adam steps on the
    tine powers (fixed total power) and the perfusion lattice lower the
    coverage loss, every iterate stays feasible."""
    import torch
    from paper_1907_05709_amd import rfa
    from paper_1907_05709_amd.autograd import optimise_plan
    case, ctrl = setup
    g = rfa.Grid(case.shape, case.spacing, device=True)
    g.load_case(case)
    labels = torch.from_numpy(case.labels).cuda()
    vox = float(np.prod(case.spacing))
    P0 = case.needle.power.copy()
    total = float(P0.sum())
    P, c, losses = optimise_plan(g, labels, vox, P0, ctrl, N_STEPS, DT, iters=6,
                                 lr_power=0.1 * total / len(P0), lr_ctrl=0.05,
                                 total_power=total)
    print("coverage loss per iteration:", [f"{x:.5f}" for x in losses])
    assert min(losses[1:]) < losses[0]
    assert bool((P >= 0).all()) and abs(float(P.sum()) - total) <= 1e-9 * total
    assert float(c.abs().max()) <= 30.0
    g.close()


def test_adjoint_kernel_timing_counts_the_kept_trajectory_launches(setup):
    from paper_1907_05709_amd import rfa
    case, ctrl = setup
    g = rfa.Grid(case.shape, case.spacing, time_kernels=16)
    g.load_case(case)
    g.set_perfusion_bspline(ctrl)
    assert g.adjoint_kernel_stats() == (0.0, 0)
    P = case.needle.power.copy()
    _, w = gpu_loss(g, case, P)      # checkpointed: not timed
    g.adjoint(w.astype(np.float32), len(P), M)
    assert g.adjoint_kernel_stats() == (0.0, 0)
    g.reset_state()
    g.forward_checkpointed(N_STEPS, DT, 0)
    g.adjoint(w.astype(np.float32), len(P), M)
    ms, n = g.adjoint_kernel_stats()
    assert n == N_STEPS and ms > 0.0
    assert g.adjoint_kernel_stats() == (0.0, 0)
    g.close()
