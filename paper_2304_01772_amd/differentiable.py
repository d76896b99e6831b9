"""Equilibrium Ising observables as a differentiable PyTorch function.

``ising_observables(Jx, Jy, h, ...)`` samples one L x L periodic Ising replica
per entry of the coupling tensors with the library's checkerboard Metropolis
sweep (Methods, Algorithm 1; Eq. (1) read as H = -Jx sum_h ss' - Jy sum_v ss'
- h sum s) and returns the sample means of the energy per site and of
|m| = |M|/N over the recorded sweeps after burn-in.

Its backward pass is the fluctuation (covariance) estimator of the gradient
of an equilibrium expectation, d<O>/dtheta = <dO/dtheta> - beta Cov(O,
dH/dtheta) with dH/dJx = -Bx, dH/dJy = -By, dH/dh = -M, evaluated by the
library's backward kernel over the statistics that the forward pass
recorded, and contracted there with the incoming gradient.  This replaces
the logistic relaxation of the paper's differentiable chain (Algorithm 2) by
an estimator that is exact in expectation and leaves the integer chain
unchanged.
"""
import torch

from .sampler import Sampler

__all__ = ["IsingObservables", "ising_observables"]


class IsingObservables(torch.autograd.Function):
    """forward(Jx, Jy, h, L, beta, n_sweeps, burn_in, seed, rid0) ->
    (e, absm), each [R] float64 on the device; backward -> (dJx, dJy, dh)."""

    @staticmethod
    def forward(ctx, Jx, Jy, h, L, beta, n_sweeps, burn_in, seed, rid0):
        R = Jx.numel()
        if Jy.numel() != R or h.numel() != R:
            raise ValueError("Jx, Jy and h must have one entry per replica")
        if not 0 <= burn_in < n_sweeps:
            raise ValueError("need 0 <= burn_in < n_sweeps")
        jx = Jx.detach().double().cpu().tolist()
        jy = Jy.detach().double().cpu().tolist()
        hh = h.detach().double().cpu().tolist()
        reps = [dict(model=0, Lx=int(L), Ly=int(L), q=2, Jx=jx[i], Jy=jy[i], h=hh[i],
                     beta=float(beta), rid=int(rid0) + i) for i in range(R)]
        smp = Sampler(reps, int(seed), init=True)
        stats = smp.sweep(int(n_sweeps), 1)
        means, _, _ = smp.grad(stats, int(burn_in))
        ctx.smp, ctx.stats, ctx.burn_in = smp, stats, int(burn_in)
        ctx.dtypes = (Jx.dtype, Jy.dtype, h.dtype)
        ctx.device = Jx.device
        return means[:, 0].clone(), means[:, 1].clone()

    @staticmethod
    def backward(ctx, g_e, g_absm):
        smp = ctx.smp
        R = smp.R
        if g_e is None:
            g_e = torch.zeros(R, dtype=torch.float64, device=smp.device)
        if g_absm is None:
            g_absm = torch.zeros(R, dtype=torch.float64, device=smp.device)
        gout = torch.stack([g_e.to(smp.device, torch.float64),
                            g_absm.to(smp.device, torch.float64)], dim=1).contiguous()
        _, _, dtheta = smp.grad(ctx.stats, ctx.burn_in, grad_out=gout)
        smp.close()
        ctx.smp = ctx.stats = None
        d = [dtheta[:, k].to(ctx.device, ctx.dtypes[k]) for k in range(3)]
        return d[0], d[1], d[2], None, None, None, None, None, None


def ising_observables(Jx, Jy, h, L=64, beta=1.0, n_sweeps=2000, burn_in=500, seed=1, rid0=0):
    """(<e>, <|m|>) per replica with covariance-estimator gradients with
    respect to Jx, Jy and h (tensors of shape [R])."""
    return IsingObservables.apply(Jx, Jy, h, L, beta, n_sweeps, burn_in, seed, rid0)
