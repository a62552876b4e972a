"""torch.autograd.Function over the library's differentiable energy.

forward(system, pos, lam, params) -> V[W]: the total potential energy of
each walker (the extended potential of the method's "Theory" section,
lambda-scaled soft-core LJ and shifted-force Coulomb of its "Alchemical
pathway" section, plus restraints), evaluated by the HIP kernels.
backward: the kernels recompute every pair term (nothing is stored by the
forward pass) and return g_w dV/dx, g_w dV/dlambda and
g_w dV/d(epsilon, sigma, q) of the solute atoms.

pos [N][3], lam [W] and params [S][3] are float64 GPU tensors; params are
the solute atoms' (epsilon, sigma, q) in increasing atom order.  Each call
installs its configuration in the system (positions, lambda and solute
parameters replace the system's).
"""
from __future__ import annotations

import torch


class AlchemicalEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, system, pos, lam, params):
        pos, lam, params = pos.detach().contiguous(), lam.detach().contiguous(), params.detach().contiguous()
        e = system.energy(pos, lam, params)
        ctx.system = system
        ctx.save_for_backward(pos, lam, params)
        return e

    @staticmethod
    def backward(ctx, grad_e):
        pos, lam, params = ctx.saved_tensors
        need = ctx.needs_input_grad
        gp = torch.empty_like(pos) if need[1] else None
        gl = torch.empty_like(lam) if need[2] else None
        gq = torch.empty_like(params) if need[3] else None
        ctx.system.energy_backward(grad_e.detach().to(torch.float64).contiguous(), pos, lam, params,
                                   gp, gl, gq)
        return None, gp, gl, gq


def energy(system, pos, lam, params):
    """V[W] with gradients to pos, lam and params through the HIP backward kernel."""
    return AlchemicalEnergy.apply(system, pos, lam, params)
