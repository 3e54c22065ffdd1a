"""torch.autograd bridge: damage integral as a function of tine powers and a
B-spline perfusion-correction lattice.

RfaFunction.apply(powers, ctrl, grid, n_steps, dt, ckpt_every) resets the
grid, sets the powers (W, one per tine) and the perfusion multiplier
f = exp(B ctrl), runs the forward (ckpt_every = 0: keeping every step's
temperature in device memory; k > 0: a checkpoint every k steps) and returns
Omega^N (the Arrhenius damage integral per voxel) as a tensor on the grid's
device.  backward() runs the library's discrete adjoint (from the kept
trajectory, or recomputing each segment from its checkpoint) and returns
dL/dpowers and dL/dctrl.  All computation
is in librfa.so; this module only moves arguments.
"""
from __future__ import annotations

import numpy as np
import torch

from . import rfa


class RfaFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, powers, ctrl, grid, n_steps: int, dt: float, ckpt_every: int):
        if not grid.device:
            raise ValueError("RfaFunction needs a device grid (device=True)")
        grid.set_tine_powers(powers.detach().double().cpu().numpy())
        grid.set_perfusion_bspline(ctrl.detach().float().cpu().numpy())
        grid.reset_state()
        grid.forward_checkpointed(int(n_steps), float(dt), int(ckpt_every))
        omega = grid.omega()
        ctx.grid = grid
        ctx.n_tines = int(powers.numel())
        ctx.m = int(ctrl.shape[0])
        ctx.pdev, ctx.pdtype = powers.device, powers.dtype
        ctx.cdev, ctx.cdtype = ctrl.device, ctrl.dtype
        return omega

    @staticmethod
    def backward(ctx, grad_omega):
        dP, dc, _ = ctx.grid.adjoint(grad_omega.contiguous().float(), ctx.n_tines, ctx.m)
        gP = torch.from_numpy(dP).to(ctx.pdev, ctx.pdtype)
        gc = torch.from_numpy(dc).to(ctx.cdev, ctx.cdtype)
        return gP, gc, None, None, None, None


def coverage_loss(omega, labels, voxel_m3: float, tumour: int = 2, liver: int = 1,
                  healthy_weight: float = 0.1):
    """Soft undertreatment of the tumour plus healthy_weight x healthy-liver
    damage volume in cm^3, with the damaged fraction d = sigmoid(4 ln Omega)
    = Omega^4 / (1 + Omega^4).  omega, labels: tensors of the grid's shape."""
    om = omega.double().clamp_min(0.0)
    # sigmoid(4 ln Omega) written without the logarithm (Omega may be 0)
    d = 1.0 / (1.0 + torch.where(om > 0, om, torch.ones_like(om)).pow(-4.0))
    d = torch.where(om > 0, d, torch.zeros_like(d))
    # masked sums rather than boolean indexing: no device-to-host sync
    tum = (labels == tumour).double()
    liv = (labels == liver).double()
    u = ((1.0 - d) * tum).sum() / tum.sum().clamp_min(1.0)  # 0 without tumour voxels
    dv = (d * liv).sum() * (voxel_m3 * 1e6)
    return u + healthy_weight * dv


def optimise_plan(grid, labels, voxel_m3: float, powers, ctrl, n_steps: int, dt: float,
                  iters: int = 10, lr_power: float = 1.0, lr_ctrl: float = 0.1,
                  total_power=None, ckpt_every: int = 0):
    """Projected Adam on the per-tine powers (W) and the B-spline perfusion
    lattice for coverage_loss: after each update the powers are clipped at
    0 and, with total_power, scaled back to that total; the lattice is
    clipped to the library's |ctrl| <= 30.  Every iteration is one forward
    and one adjoint in librfa.so (grid: a device grid with its tissue and
    needle set).  Returns the final powers and lattice and the loss of every
    iteration (evaluated before that iteration's update)."""
    p = torch.as_tensor(np.asarray(powers), dtype=torch.float64).clone().requires_grad_(True)
    c = torch.as_tensor(np.asarray(ctrl), dtype=torch.float32).clone().requires_grad_(True)
    opt = torch.optim.Adam([{"params": [p], "lr": lr_power}, {"params": [c], "lr": lr_ctrl}])
    losses = []
    for _ in range(int(iters)):
        opt.zero_grad()
        omega = RfaFunction.apply(p, c, grid, n_steps, dt, ckpt_every)
        loss = coverage_loss(omega, labels, voxel_m3)
        loss.backward()
        opt.step()
        with torch.no_grad():
            p.clamp_(min=0.0)
            if total_power is not None and float(p.sum()) > 0.0:
                p.mul_(float(total_power) / p.sum())
            c.clamp_(-30.0, 30.0)
        losses.append(float(loss))
    return p.detach(), c.detach(), losses
