"""torch.autograd bridge for the wettability gradient.

``WettabilityLoss.apply(xi, lattice, rho0, region, nsteps, every)`` sets the
per-voxel adhesion parameter ``xi`` (Eqs. 13-15), starts from the equilibrium
of the densities ``rho0``, runs ``nsteps`` steps with a checkpoint every
``every`` steps and returns the smooth non-wetting saturation of ``region``
(a 0-d float64 tensor); ``OutletFluxLoss`` (same arguments) returns the
component-1 flux sum rho1 u_x over ``region`` instead.  Its backward runs the library's hand-written adjoint
(checkpoint, recompute and reverse sweep, all in HIP kernels) and returns
dL/dxi.  Everything runs in libmclbm.so; this module only moves tensors.
"""
import torch


class WettabilityLoss(torch.autograd.Function):

    @staticmethod
    def forward(ctx, xi, lattice, rho0, region, nsteps, every):
        lattice.set_geometry(lattice.solid, xi.detach())
        lattice.init_equilibrium(rho0)
        ckpt = lattice.step_checkpointed(nsteps, every)
        loss = lattice.loss_snw(region)
        ctx.lattice, ctx.region, ctx.nsteps, ctx.every = lattice, region, nsteps, every
        ctx.ckpt = ckpt
        ctx.xi_dtype, ctx.xi_shape = xi.dtype, xi.shape
        return torch.tensor(loss, dtype=torch.float64, device=xi.device)

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.lattice.gradient_snw(ctx.nsteps, ctx.every, ctx.ckpt, ctx.region)
        g = (g * grad_out).to(ctx.xi_dtype).reshape(ctx.xi_shape)
        return g, None, None, None, None, None


class OutletFluxLoss(torch.autograd.Function):

    @staticmethod
    def forward(ctx, xi, lattice, rho0, region, nsteps, every):
        lattice.set_geometry(lattice.solid, xi.detach())
        lattice.init_equilibrium(rho0)
        ckpt = lattice.step_checkpointed(nsteps, every)
        loss = lattice.loss_flux(region)
        ctx.lattice, ctx.region, ctx.nsteps, ctx.every = lattice, region, nsteps, every
        ctx.ckpt = ckpt
        ctx.xi_dtype, ctx.xi_shape = xi.dtype, xi.shape
        return torch.tensor(loss, dtype=torch.float64, device=xi.device)

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.lattice.gradient_flux(ctx.nsteps, ctx.every, ctx.ckpt, ctx.region)
        g = (g * grad_out).to(ctx.xi_dtype).reshape(ctx.xi_shape)
        return g, None, None, None, None, None
