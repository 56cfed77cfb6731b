"""phi(m) as a differentiable torch function.

`HelmholtzMisfit.apply(m, grid, omegas, d_obs, sources, receivers, ...)`
returns the misfit phi of eq. (phi) (plus the regularisation term of
eq. (Gamma) when alpha or mu is non-zero) as a 0-d FP64 tensor on the device
of m.  Its backward is the adjoint-state gradient of the appendix "Gradient of
phi" (Algorithm 3): both come from one call of helm_misfit_grad, which
factors A(m, omega) once per frequency and uses the factors for the forward
and the adjoint solves.  Gradients flow to m only.
"""
from __future__ import annotations

import torch

from . import helm


class HelmholtzMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m, grid, omegas, d_obs, sources, receivers, alpha=0.0, mu=0.0, precision="fp64", tol=0.0):
        if not (isinstance(m, torch.Tensor) and m.is_cuda and m.dtype == torch.float64):
            raise TypeError("m must be a float64 CUDA tensor")
        if m.numel() != grid.N:
            raise ValueError(f"m has {m.numel()} entries, the grid {grid.N}")
        mf = m.detach().reshape(-1).contiguous()
        phi, g, _ = helm.misfit_grad(grid, mf, omegas, d_obs, sources, receivers, alpha, mu, precision, tol)
        ctx.save_for_backward(g.reshape(m.shape))
        return torch.tensor(phi, dtype=torch.float64, device=m.device)

    @staticmethod
    def backward(ctx, gphi):
        (g,) = ctx.saved_tensors
        return (gphi * g,) + (None,) * 9


def misfit(m, grid, omegas, d_obs, sources, receivers, alpha=0.0, mu=0.0, precision="fp64", tol=0.0):
    """phi(m) with autograd support (see HelmholtzMisfit)."""
    return HelmholtzMisfit.apply(m, grid, omegas, d_obs, sources, receivers, alpha, mu, precision, tol)
