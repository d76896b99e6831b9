"""Spin-value optimisation (Results, optimisation of the spin values) --
TEST INFRASTRUCTURE ONLY.

FP64 reference of the three ways the paper compares to find low-energy
states of an Ising lattice with one coupling per bond (J = 1 everywhere, or
J = +-1 drawn with mean zero, the spin-glass case):

  energy      H(s) = -sum_{y,x} s[y,x] (Jx[y,x] s[y,x+1] + Jy[y,x] s[y+1,x])
                     - h sum s      (periodic; the convention of ``dmc``)
              dH/ds = -(local field) = -(sum over the four bonds of J s_n + h)
  Monte Carlo anneal   one Metropolis sweep per step at inverse temperature
              beta_k: the relaxed chain of ``dmc`` in its hard limit
              (alpha = ALPHA_HARD, where q is 0 or 1 unless P and r agree to
              ~1e-8), counter t0 = k, discretised;
  gradient    s <- discretize(s - eta dH/ds), every site at once;
  DMC         s_c = relaxed chain (n sweeps at beta_k, alpha, counter
              t0 = k n) from s, L = H(s_c), g = dL/ds by reverse mode
              through the chain, s <- discretize(s_c - eta g): the chain
              moves the spins and the gradient through it moves them further
              (Algorithm 2 with the spins as the optimised parameters and the
              quantisation as its last step).

Readings where the paper is silent: the three rules above (its text names
the methods, the annealing towards T = 0 and the quantisation, not the
update formulas); the energy is reported per site after every step, for the
discretised state.

Pins (tests/test_oracle_spinopt.py): closed forms of the energy (uniform
and checkerboard states, a lattice with a single coupled bond), the energy
of uniform couplings against the integer bond sums of the C oracle,
dH/ds against central finite differences, the fixed points and one-defect
repair of the gradient step, the beta = 0 Monte Carlo sweep (every spin
flips), and the DMC step with eta = 0 reducing to the discretised relaxed
chain.
"""
import numpy as np
import torch

from . import dmc

ALPHA_HARD = 1e9


def _t(a):
    return a if torch.is_tensor(a) else torch.tensor(np.asarray(a, np.float64))


def energy(s, Jx, Jy, h=0.0):
    """H per replica (float64 [R]) and dH/ds (float64 [R, Ly, Lx])."""
    s, Jx, Jy = _t(s).double(), _t(Jx).double(), _t(Jy).double()
    right = torch.roll(s, -1, dims=2)
    down = torch.roll(s, -1, dims=1)
    H = -(s * (Jx * right + Jy * down)).sum(dim=(1, 2)) - h * s.sum(dim=(1, 2))
    grad = -dmc.local_field(s, Jx, Jy, h)
    return H, grad


def discretize_step(base, g, eta):
    """discretize(base - eta g): -1 where the value is < 0, +1 elsewhere."""
    v = _t(base).double() - eta * _t(g).double()
    return torch.where(v < 0, -torch.ones_like(v), torch.ones_like(v))


def mc_anneal_step(s, Jx, Jy, h, beta, seed, rids, k):
    """One Metropolis sweep (hard-limit relaxed chain) at beta, counter k,
    discretised (q can miss 0 and 1 only where P and r agree to ~1e-8, so
    this changes a spin with probability below 2^-24 per update)."""
    sc = dmc.forward(_t(s).double(), _t(Jx).double(), _t(Jy).double(), h, beta, ALPHA_HARD,
                     seed, rids, k, 1)
    return discretize_step(sc, torch.zeros_like(sc), 0.0)


def gradient_step(s, Jx, Jy, h, eta):
    _, g = energy(s, Jx, Jy, h)
    return discretize_step(s, g, eta)


def dmc_step(s, Jx, Jy, h, beta, alpha, n_sweeps, eta, seed, rids, k):
    """One DMC step: relaxed chain, gradient of the final energy with
    respect to the chain's input, quantised update of the chain's output."""
    s0 = _t(s).double().clone().requires_grad_(True)
    sc = dmc.forward(s0, _t(Jx).double(), _t(Jy).double(), h, beta, alpha, seed, rids,
                     k * n_sweeps, n_sweeps)
    H, _ = energy(sc, Jx, Jy, h)
    H.sum().backward()
    return discretize_step(sc.detach(), s0.grad, eta)


def run(method, s, Jx, Jy, h, steps, betas=None, alpha=None, n_sweeps=1, eta=1.0, seed=1,
        rids=None):
    """Energy per site after every step, float64 [steps + 1, R] (row 0: the
    start), and the final state."""
    s = _t(s).double()
    R, Ly, Lx = s.shape
    rids = list(range(R)) if rids is None else rids
    hist = [energy(s, Jx, Jy, h)[0] / (Ly * Lx)]
    for k in range(steps):
        if method == "mc":
            s = mc_anneal_step(s, Jx, Jy, h, betas[k], seed, rids, k)
        elif method == "gradient":
            s = gradient_step(s, Jx, Jy, h, eta)
        elif method == "dmc":
            s = dmc_step(s, Jx, Jy, h, betas[k], alpha, n_sweeps, eta, seed, rids, k)
        else:
            raise ValueError(method)
        hist.append(energy(s, Jx, Jy, h)[0] / (Ly * Lx))
    return torch.stack(hist).numpy(), s.detach()
