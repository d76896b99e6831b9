"""Differentiable Monte Carlo (Algorithm 2) -- TEST INFRASTRUCTURE ONLY.

FP64 reference of the relaxed checkerboard chain of the paper's
differentiable Monte Carlo (Methods, Algorithm 2) for the Ising model on an
L x L periodic lattice with continuous spins s in [-1, 1] and one coupling
per bond: Jx[y, x] couples (y, x) with (y, x + 1), Jy[y, x] couples (y, x)
with (y + 1, x); h is a uniform field (Eq. (1) with the sign convention of
the rest of this package: H = -sum_bonds J s s' - h sum s).

One colour pass (colour c = (x + y) & 1, pass index p = 2t + c, colour 0
first) updates every site of colour c at once from the current spins:

    hloc = sum over the four bonds of J * s_neighbour + h
    dE   = 2 s hloc                   (the proposal flips the spin, s' = -s)
    P    = exp(-beta dE)               (no clipping at 1, as the algorithm states;
                                        the exponent is capped at EXP_CAP)
    r    = uniform in [0, 1)
    q    = 1 / (1 + exp(-alpha (P - r)))
    s   <- q s' + (1 - q) s = s (1 - 2 q)

Readings where the paper is silent (the same readings bind the HIP path):
  - r comes from Philox4x32-10 with key (seed lo, seed hi), counter
    (k >> 2, p, rid, 3), word k & 3, where k = y (Lx/2) + (x >> 1) is the
    within-colour site index; r = (word >> 8) 2^-24 (24 bits, exact in
    FP32 and FP64);
  - the proposal of the Ising model is the flip;
  - gradients are those of the relaxed chain as computed (reverse mode
    through every pass), here by torch.autograd over plain FP64 ops.

Pins (tests/test_oracle_dmc.py): beta = 0 and alpha = 0 closed forms; the
alpha -> infinity limit samples the Metropolis distribution (4x4 exact
enumeration within 3 sigma); global spin-flip symmetry at h = 0; gradients
against central finite differences of the forward.
"""
import numpy as np
import torch

from . import chain

TAG_DMC = 3
# P = exp(min(-beta dE, EXP_CAP)): beyond the cap q is exactly 1 in FP32 and
# FP64 for any alpha >= 2e-33 (or alpha = 0, where q = 1/2 anyway), so no
# forward value changes; only the infinite P of an overflowing exponent, and
# the 0 * inf in its gradient, are avoided (FP32 overflows at 88.7).
EXP_CAP = 80.0


def uniforms(Lx, Ly, seed, rids, p):
    """r for every site of colour p & 1 in pass p: float64 [R, Ly, Lx],
    zero on the other colour."""
    W = Lx // 2
    n_sites = Ly * W
    n_blocks = (n_sites + 3) // 4
    words = chain.philox_grid(n_blocks, p, rids, TAG_DMC, seed).reshape(len(rids), -1)[:, :n_sites]
    r = (words >> np.uint32(8)).astype(np.float64) * 2.0 ** -24
    c = p & 1
    out = np.zeros((len(rids), Ly, Lx))
    k = np.arange(n_sites)
    y = k // W
    x = 2 * (k % W) + ((y + c) & 1)
    out[:, y, x] = r
    return torch.tensor(out, dtype=torch.float64)


def colour_mask(Lx, Ly, c):
    y = torch.arange(Ly).view(-1, 1)
    x = torch.arange(Lx).view(1, -1)
    return ((x + y) % 2) == c


def local_field(s, Jx, Jy, h):
    """sum over the four bonds of J * s_neighbour, plus h; tensors [R, Ly, Lx]."""
    right = torch.roll(s, -1, dims=2)
    left = torch.roll(s, 1, dims=2)
    down = torch.roll(s, -1, dims=1)
    up = torch.roll(s, 1, dims=1)
    return (Jx * right + torch.roll(Jx, 1, dims=2) * left + Jy * down
            + torch.roll(Jy, 1, dims=1) * up + h)


def forward(s0, Jx, Jy, h, beta, alpha, seed, rids, t0, n_sweeps):
    """Relaxed chain from spins s0 [R, Ly, Lx] for n_sweeps sweeps starting at
    sweep counter t0; returns the final spins.  Differentiable with respect
    to s0, Jx, Jy (and h if it is a tensor)."""
    R, Ly, Lx = s0.shape
    s = s0
    for t in range(t0, t0 + n_sweeps):
        for c in (0, 1):
            p = 2 * t + c
            m = colour_mask(Lx, Ly, c)
            hloc = local_field(s, Jx, Jy, h)
            P = torch.exp(torch.clamp(-beta * 2.0 * s * hloc, max=EXP_CAP))
            r = uniforms(Lx, Ly, seed, rids, p)
            q = 1.0 / (1.0 + torch.exp(-alpha * (P - r)))
            s = torch.where(m, s * (1.0 - 2.0 * q), s)
    return s


def forward_backward(s0, Jx, Jy, h, beta, alpha, seed, rids, t0, n_sweeps, g_final):
    """Final spins and the gradients of sum(g_final * s_final) with respect to
    (s0, Jx, Jy, h): numpy float64 arrays."""
    s0 = torch.tensor(np.asarray(s0, np.float64), requires_grad=True)
    Jx = torch.tensor(np.asarray(Jx, np.float64), requires_grad=True)
    Jy = torch.tensor(np.asarray(Jy, np.float64), requires_grad=True)
    hh = torch.tensor(float(h), dtype=torch.float64, requires_grad=True)
    s = forward(s0, Jx, Jy, hh, beta, alpha, seed, rids, t0, n_sweeps)
    (s * torch.tensor(np.asarray(g_final, np.float64))).sum().backward()
    return (s.detach().numpy(), s0.grad.numpy(), Jx.grad.numpy(), Jy.grad.numpy(),
            float(hh.grad))


def discretize(s):
    """The algorithm's last step: s -> -1 if s < 0 else +1."""
    return np.where(np.asarray(s) < 0, -1, 1).astype(np.int8)
