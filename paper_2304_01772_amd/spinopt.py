"""Spin-value optimisation (Results, optimisation of the spin values) on the
library's kernels: three ways to find low-energy states of an Ising lattice
with one coupling per bond (J = 1 everywhere, or J = +-1 with mean zero, the
spin-glass case), compared step by step.

* ``mc``: one Metropolis sweep per step at an annealed inverse temperature
  beta_k -- the relaxed chain (``spinmc_dmc_forward``) in its hard limit,
  discretised;
* ``gradient``: s <- discretize(s - eta dH/ds) at every site at once
  (``spinmc_dmc_energy`` for dH/ds, ``spinmc_dmc_discretize``);
* ``dmc``: the relaxed chain moves the spins (n sweeps at beta_k), the
  reverse replay (``spinmc_dmc_backward``) gives the gradient of the final
  energy with respect to the chain's input, and the quantised step
  s <- discretize(s_chain - eta g) follows (Algorithm 2 with the spins as
  the optimised parameters).

Every step runs in the HIP kernels; the energies are FP64 sums per replica.
"""
import ctypes as C

import numpy as np
import torch

from ._lib import DmcParams, check, lib

__all__ = ["SpinOptimiser", "ALPHA_HARD", "spin_glass_couplings"]

ALPHA_HARD = 1e9  # q is 0 or 1 in FP32 unless P and r agree to ~1e-8


def _p(t):
    return C.c_void_p(t.data_ptr())


def spin_glass_couplings(R, Ly, Lx, seed, device="cuda"):
    """J = +-1 per bond with equal probability (mean zero): (Jx, Jy)."""
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    J = torch.randint(0, 2, (2, R, Ly, Lx), generator=g).to(torch.float32) * 2 - 1
    return J[0].to(device).contiguous(), J[1].to(device).contiguous()


class SpinOptimiser:
    """Buffers and steps for R replicas of Ly x Lx spins with fixed per-bond
    couplings Jx, Jy (FP32 [R, Ly, Lx] device tensors) and field h."""

    def __init__(self, Jx, Jy, h=0.0, seed=1, rid0=0):
        if Jx.shape != Jy.shape or Jx.dim() != 3:
            raise ValueError("Jx and Jy must both be [R, Ly, Lx]")
        self.Jx = Jx.to(torch.float32).contiguous()
        self.Jy = Jy.to(torch.float32).contiguous()
        self.R, self.Ly, self.Lx = self.Jx.shape
        self.N = self.Ly * self.Lx
        self.h, self.seed, self.rid0 = float(h), int(seed), int(rid0)
        self.L = lib()
        dev = self.Jx.device
        self.e = torch.empty(self.R, dtype=torch.float64, device=dev)
        self.g = torch.empty_like(self.Jx)
        self.gJx = torch.empty_like(self.Jx)
        self.gJy = torch.empty_like(self.Jx)
        self._save = {}
        self._work = None

    def _params(self, n_sweeps=0, beta=1.0, alpha=1.0, t0=0):
        p = DmcParams()
        p.R, p.Lx, p.Ly, p.n_sweeps = self.R, self.Lx, self.Ly, int(n_sweeps)
        p.beta, p.alpha, p.h = float(beta), float(alpha), self.h
        p.seed, p.t0, p.rid0 = self.seed, int(t0), self.rid0
        return p

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def _save_buf(self, p):
        n = p.n_sweeps
        if n not in self._save:
            k = self.L.spinmc_dmc_save_floats(C.byref(p))
            if k < 0:
                check(k)
            self._save[n] = torch.empty(max(k, 1), dtype=torch.float32, device=self.Jx.device)
        return self._save[n]

    def energy(self, s, grad=False):
        """H per replica (FP64 [R], a view of an internal buffer) and, if
        grad, dH/ds (FP32, an internal buffer)."""
        s = s.contiguous()
        p = self._params()
        check(self.L.spinmc_dmc_energy(C.byref(p), _p(s), _p(self.Jx), _p(self.Jy), _p(self.e),
                                       _p(self.g) if grad else None, self._stream()))
        return self.e, (self.g if grad else None)

    def _chain(self, s, beta, alpha, n_sweeps, t0):
        """The relaxed chain from s (not modified); returns (final spins,
        params, save buffer)."""
        p = self._params(n_sweeps, beta, alpha, t0)
        sc = s.contiguous().clone()
        save = self._save_buf(p)
        check(self.L.spinmc_dmc_forward(C.byref(p), _p(sc), _p(self.Jx), _p(self.Jy), _p(save),
                                        self._stream()))
        return sc, p, save

    def _discretize(self, base, g, eta, out):
        check(self.L.spinmc_dmc_discretize(base.numel(), _p(base), _p(g) if g is not None else None,
                                           float(eta), _p(out), self._stream()))
        return out

    def mc_step(self, s, beta, k):
        """One annealed Metropolis sweep (counter k), discretised."""
        sc, _, _ = self._chain(s, beta, ALPHA_HARD, 1, k)
        return self._discretize(sc, None, 0.0, sc)

    def gradient_step(self, s, eta):
        _, g = self.energy(s, grad=True)
        return self._discretize(s.contiguous(), g, eta, torch.empty_like(s))

    def dmc_step(self, s, beta, alpha, n_sweeps, eta, k):
        """Relaxed chain (counter k n_sweeps), reverse replay of the final
        energy's gradient, quantised step on the chain's output."""
        sc, p, save = self._chain(s, beta, alpha, n_sweeps, k * n_sweeps)
        _, g = self.energy(sc, grad=True)
        if self._work is None:
            self._work = torch.empty(max(self.L.spinmc_dmc_work_floats(C.byref(p)), 1),
                                     dtype=torch.float32, device=self.Jx.device)
        replay = sc.clone()  # the replay restores it to s
        gs = g.clone()
        check(self.L.spinmc_dmc_backward(C.byref(p), _p(replay), _p(self.Jx), _p(self.Jy),
                                         _p(save), _p(gs), _p(self.gJx), _p(self.gJy),
                                         _p(self._work), self._stream()))
        return self._discretize(sc, gs, eta, sc)

    def run(self, method, s0, steps, betas=None, alpha=10.0, n_sweeps=1, eta=1.0):
        """Energy per site after every step (numpy float64 [steps + 1, R],
        row 0 the start) and the final spins."""
        s = s0.to(torch.float32).contiguous().clone()
        hist = torch.empty((steps + 1, self.R), dtype=torch.float64, device=s.device)
        hist[0] = self.energy(s)[0] / self.N
        for k in range(steps):
            if method == "mc":
                s = self.mc_step(s, betas[k], k)
            elif method == "gradient":
                s = self.gradient_step(s, eta)
            elif method == "dmc":
                s = self.dmc_step(s, betas[k], alpha, n_sweeps, eta, k)
            else:
                raise ValueError(f"unknown method {method!r}")
            hist[k + 1] = self.energy(s)[0] / self.N
        return hist.cpu().numpy(), s

    def compare(self, s0, steps, beta0=0.3, beta1=3.0, alpha=20.0, n_sweeps=1, eta_dmc=0.05,
                eta_grad=1.0):
        """The three methods from the same start over the same linear beta
        schedule: {method: (energy history, best energy per replica)}."""
        betas = list(np.linspace(beta0, beta1, steps))
        out = {}
        for m, kw in (("mc", dict(betas=betas)), ("gradient", dict(eta=eta_grad)),
                      ("dmc", dict(betas=betas, alpha=alpha, n_sweeps=n_sweeps, eta=eta_dmc))):
            hist, _ = self.run(m, s0, steps, **kw)
            out[m] = (hist, hist.min(axis=0))
        return out
