"""Differentiable Monte Carlo (Methods, Algorithm 2) on the library's kernels.

``RelaxedIsing`` is a ``torch.autograd.Function``: its forward runs the
relaxed checkerboard chain (``spinmc_dmc_forward``) on continuous spins with
one coupling per bond, its backward replays the chain in reverse
(``spinmc_dmc_backward``) and returns the gradients with respect to the
initial spins and the two coupling fields.  ``optimise_couplings`` is the
paper's spin-pattern optimisation (Results): Adam (``spinmc_adam``) on the
couplings so that the relaxed chain drives the lattice to a target pattern,
followed by the algorithm's last step, the discretisation s -> sign(s).
"""
import ctypes as C

import torch

from ._lib import DmcParams, check, lib

__all__ = ["RelaxedIsing", "relaxed_ising", "optimise_couplings", "discretize",
           "pathwise_energy_gradient", "gradient_vs_temperature"]


def _p(t):
    return C.c_void_p(t.data_ptr())


def _params(R, Lx, Ly, n_sweeps, beta, alpha, h, seed, t0, rid0):
    p = DmcParams()
    p.R, p.Lx, p.Ly, p.n_sweeps = int(R), int(Lx), int(Ly), int(n_sweeps)
    p.beta, p.alpha, p.h = float(beta), float(alpha), float(h)
    p.seed, p.t0, p.rid0 = int(seed), int(t0), int(rid0)
    return p


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class RelaxedIsing(torch.autograd.Function):
    """forward(s0, Jx, Jy, beta, alpha, h, n_sweeps, seed, t0, rid0) ->
    final spins [R, Ly, Lx] (FP32 device tensors in and out)."""

    @staticmethod
    def forward(ctx, s0, Jx, Jy, beta, alpha, h, n_sweeps, seed, t0, rid0):
        R, Ly, Lx = s0.shape
        if Jx.shape != s0.shape or Jy.shape != s0.shape:
            raise ValueError("s0, Jx and Jy must all be [R, Ly, Lx]")
        p = _params(R, Lx, Ly, n_sweeps, beta, alpha, h, seed, t0, rid0)
        L = lib()
        n_save = L.spinmc_dmc_save_floats(C.byref(p))
        if n_save < 0:
            check(n_save)
        s = s0.detach().to(torch.float32).contiguous().clone()
        jx = Jx.detach().to(torch.float32).contiguous()
        jy = Jy.detach().to(torch.float32).contiguous()
        save = torch.empty(max(n_save, 1), dtype=torch.float32, device=s.device)
        check(L.spinmc_dmc_forward(C.byref(p), _p(s), _p(jx), _p(jy), _p(save), _stream()))
        ctx.p = p
        ctx.save_for_backward(s, jx, jy, save)
        return s.clone()

    @staticmethod
    def backward(ctx, g):
        s_final, jx, jy, save = ctx.saved_tensors
        p = ctx.p
        L = lib()
        s = s_final.clone()
        gs = g.to(torch.float32).contiguous().clone()
        gjx = torch.zeros_like(jx)
        gjy = torch.zeros_like(jy)
        work = torch.empty(max(L.spinmc_dmc_work_floats(C.byref(p)), 1), dtype=torch.float32,
                           device=s.device)
        check(L.spinmc_dmc_backward(C.byref(p), _p(s), _p(jx), _p(jy), _p(save), _p(gs),
                                    _p(gjx), _p(gjy), _p(work), _stream()))
        return gs, gjx, gjy, None, None, None, None, None, None, None


def relaxed_ising(s0, Jx, Jy, beta=1.0, alpha=10.0, h=0.0, n_sweeps=10, seed=1, t0=0, rid0=0):
    """Final spins of the relaxed chain, differentiable in s0, Jx and Jy."""
    return RelaxedIsing.apply(s0, Jx, Jy, beta, alpha, h, n_sweeps, seed, t0, rid0)


def discretize(s):
    """The algorithm's last step: -1 where s < 0, +1 elsewhere."""
    return torch.where(s < 0, -torch.ones_like(s), torch.ones_like(s))


def optimise_couplings(target, s0, Jx, Jy, steps=200, lr=1e-3, beta=1.0, alpha=10.0, h=0.0,
                       n_sweeps=10, seed=1, log=None):
    """Spin-pattern optimisation: Adam on (Jx, Jy) minimising the mean squared
    difference between the relaxed chain's final spins and the target
    pattern (+-1); every step reuses the same random numbers (same seed and
    sweep counter).  Returns (Jx, Jy, loss history, discretised final spins)."""
    L = lib()
    params = torch.stack([Jx, Jy]).to(torch.float32).contiguous().clone()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    target = target.to(torch.float32)
    hist = []
    for step in range(1, steps + 1):
        jx = params[0].clone().requires_grad_(True)
        jy = params[1].clone().requires_grad_(True)
        s = relaxed_ising(s0, jx, jy, beta, alpha, h, n_sweeps, seed)
        loss = ((s - target) ** 2).mean()
        loss.backward()
        grad = torch.stack([jx.grad, jy.grad]).contiguous()
        check(L.spinmc_adam(_p(params), _p(grad), _p(m), _p(v), params.numel(), step, lr, 0.9,
                            0.999, 1e-8, _stream()))
        hist.append(float(loss.detach()))
        if log and (step % 50 == 0 or step == steps):
            log(f"step {step}: loss {hist[-1]:.5f}")
    with torch.no_grad():
        s = relaxed_ising(s0, params[0], params[1], beta, alpha, h, n_sweeps, seed)
    return params[0], params[1], hist, discretize(s)


def pathwise_energy_gradient(L=4, R=4096, beta=0.44, alpha=10.0, n_sweeps=1, burn_in=50,
                             seed=1, device="cuda"):
    """The differentiable chain's estimate of d<e>/dJ for uniform couplings
    J = Jx = Jy (e = H/N): R replicas of L x L start from random +-1 spins,
    run burn_in relaxed sweeps, are discretised, then run n_sweeps more
    relaxed sweeps with every bond coupling a leaf; the derivative of the
    final energy per site (explicit in J and through the chain) summed over
    all bonds.  Returns (per-replica values [R] float64, mean, standard
    error).  For comparison with the fluctuation estimator (covariance of e
    with dH/dJ) and exact enumeration: the relaxed chain is a different
    Markov chain, so this is not an unbiased estimate of the equilibrium
    derivative."""
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    s = (torch.randint(0, 2, (R, L, L), generator=g).to(torch.float32) * 2 - 1).to(device)
    one = torch.ones((R, L, L), dtype=torch.float32, device=device)
    with torch.no_grad():
        s = discretize(relaxed_ising(s, one, one, beta, alpha, 0.0, burn_in, seed, 0))
    Jx = one.clone().requires_grad_(True)
    Jy = one.clone().requires_grad_(True)
    sf = relaxed_ising(s, Jx, Jy, beta, alpha, 0.0, n_sweeps, seed, burn_in)
    N = L * L
    e = -(sf * (Jx * torch.roll(sf, -1, 2) + Jy * torch.roll(sf, -1, 1))).sum(dim=(1, 2)) / N
    e.sum().backward()
    d = (Jx.grad.sum(dim=(1, 2)) + Jy.grad.sum(dim=(1, 2))).double()
    mean = float(d.mean())
    se = float(d.std() / R ** 0.5) if R > 1 else float("nan")
    return d, mean, se


def gradient_vs_temperature(target, s0, Jx, Jy, temperatures, alpha=10.0, n_sweeps=10, seed=1):
    """Mean |dL/dJ| over all bonds and replicas of the spin-pattern loss
    L = mean((s_final - target)^2) at each temperature T = 1/beta, from the
    same start and the same random numbers (Results, optimisation of the
    exchange parameters: the gradients are small at high and at low T and
    largest in between).  Returns a list of floats."""
    out = []
    target = target.to(torch.float32)
    for T in temperatures:
        jx = Jx.detach().to(torch.float32).clone().requires_grad_(True)
        jy = Jy.detach().to(torch.float32).clone().requires_grad_(True)
        s = relaxed_ising(s0, jx, jy, 1.0 / float(T), alpha, 0.0, n_sweeps, seed)
        ((s - target) ** 2).mean().backward()
        out.append(float(torch.cat([jx.grad.abs().flatten(), jy.grad.abs().flatten()]).mean()))
    return out
