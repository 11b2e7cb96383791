"""torch.autograd functions over the placer's objective (Eq. 2), with the library's
hand-written adjoint kernels as their backward.

    obj = PlacementObjective(placer, gamma)          # placer: hybro.Placer
    wl = obj.wirelength(x, y)                         # WA wirelength, Eq. 3
    n = obj.density_energy(x, y)                      # electrostatic energy (the D term)
    f = obj.objective(x, y, lam)                      # WL + lam * N
    f.backward()                                      # x.grad, y.grad

x and y are device tensors of the movable cells' lower-left coordinates (the placer's
precision).  The forward pass evaluates on a scratch slot of the placer and its launches
already produce the gradient (per-pin WA adjoint reduced to cells, and the density adjoint:
the exact derivative sum_b psi_b dq_ib/dx_i by default, or the field force); backward scales
it by the incoming gradient.  Forward values are returned as 0-d tensors.
"""
from __future__ import annotations

import torch


def _eval(pl, slot, x, y, gamma, lam, grad_mode):
    pl.set_positions(slot, x.detach().contiguous(), y.detach().contiguous())
    (wl, en, _), gx, gy = pl.eval(slot, gamma, lam=lam, grads=True, grad_mode=grad_mode)
    return float(wl[0]), float(en[0]), gx[0], gy[0]


class _Objective(torch.autograd.Function):
    """f = WL + lam * N at (x, y); lam = 0 gives the wirelength alone."""

    @staticmethod
    def forward(ctx, x, y, pl, slot, gamma, lam, grad_mode):
        wl, en, gx, gy = _eval(pl, slot, x, y, gamma, lam, grad_mode)
        ctx.save_for_backward(gx, gy)
        return x.new_tensor(wl + lam * en if lam != 0.0 else wl)

    @staticmethod
    def backward(ctx, go):
        gx, gy = ctx.saved_tensors
        return go * gx, go * gy, None, None, None, None, None


class _Density(torch.autograd.Function):
    """N at (x, y), with its gradient from one density-only evaluation (the library's density
    adjoint launch with lambda = 1; the net sweep does not run)."""

    @staticmethod
    def forward(ctx, x, y, pl, slot, gamma, grad_mode):
        from .hybro import HP_GRAD_DENSITY_ONLY
        _, en, gx, gy = _eval(pl, slot, x, y, gamma, 1.0, grad_mode | HP_GRAD_DENSITY_ONLY)
        ctx.save_for_backward(gx.clone(), gy.clone())
        return x.new_tensor(en)

    @staticmethod
    def backward(ctx, go):
        gx, gy = ctx.saved_tensors
        return go * gx, go * gy, None, None, None, None


class PlacementObjective:
    """Differentiable wirelength, density energy and objective on one placer's netlist."""

    def __init__(self, placer, gamma: float, grad_mode: int = 1):
        self.pl = placer
        self.gamma = float(gamma)
        self.grad_mode = int(grad_mode)
        self.slot = placer.new_slot()

    def wirelength(self, x, y):
        return _Objective.apply(x, y, self.pl, self.slot, self.gamma, 0.0, self.grad_mode)

    def density_energy(self, x, y):
        return _Density.apply(x, y, self.pl, self.slot, self.gamma, self.grad_mode)

    def objective(self, x, y, lam: float):
        return _Objective.apply(x, y, self.pl, self.slot, self.gamma, float(lam), self.grad_mode)

    def close(self):
        if self.slot is not None:
            self.pl.free_slot(self.slot)
            self.slot = None
