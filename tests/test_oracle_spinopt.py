"""Pins of the spin-value optimisation oracle: the energy with per-bond
couplings against closed forms and the C oracle's integer bond sums, its
gradient against finite differences, and the three update rules against
their fixed points and special cases."""
import numpy as np
import torch

from oracle import chain as orc
from oracle import dmc
from oracle import spinopt as so


def _pm1(rng, *shape):
    return rng.choice([-1.0, 1.0], size=shape)


def test_energy_closed_forms():
    """Uniform state: H = -N (Jx + Jy) - h N; checkerboard: H = +N (Jx + Jy)
    - 0 (the field cancels on an even torus)."""
    R, Ly, Lx, a, b, h = 1, 6, 8, 0.7, -0.3, 0.25
    Jx = np.full((R, Ly, Lx), a)
    Jy = np.full((R, Ly, Lx), b)
    N = Ly * Lx
    up = np.ones((R, Ly, Lx))
    H, _ = so.energy(up, Jx, Jy, h)
    assert abs(float(H[0]) - (-N * (a + b) - h * N)) < 1e-12
    y, x = np.meshgrid(np.arange(Ly), np.arange(Lx), indexing="ij")
    cb = np.where((x + y) % 2 == 0, 1.0, -1.0)[None]
    H, _ = so.energy(cb, Jx, Jy, h)
    assert abs(float(H[0]) - N * (a + b)) < 1e-12


def test_single_bond_energy_names_the_right_neighbour():
    """Only Jx[y0, x0] = J coupled: H = -J s(y0, x0) s(y0, x0 + 1); only
    Jy[y0, x0]: H = -J s(y0, x0) s(y0 + 1, x0) (periodic wrap included)."""
    rng = np.random.default_rng(0)
    Ly, Lx, J = 4, 6, 1.7
    for (y0, x0) in [(1, 2), (3, 5), (0, 0)]:
        s = _pm1(rng, 1, Ly, Lx)
        Z = np.zeros((1, Ly, Lx))
        Jb = Z.copy()
        Jb[0, y0, x0] = J
        H, _ = so.energy(s, Jb, Z, 0.0)
        assert float(H[0]) == -J * s[0, y0, x0] * s[0, y0, (x0 + 1) % Lx]
        H, _ = so.energy(s, Z, Jb, 0.0)
        assert float(H[0]) == -J * s[0, y0, x0] * s[0, (y0 + 1) % Ly, x0]


def test_uniform_couplings_match_the_integer_bond_sums():
    """For uniform couplings H = -(Jx Bx + Jy By + h M) with M, Bx, By from
    the C oracle's statistics of the same state."""
    rng = np.random.default_rng(1)
    Ly, Lx, a, b, h = 8, 10, 0.9, 0.4, -0.2
    for _ in range(5):
        s = _pm1(rng, 1, Ly, Lx)
        M, Bx, By = orc.ising_stats(s[0].astype(np.int8))[:3]
        H, _ = so.energy(s, np.full(s.shape, a), np.full(s.shape, b), h)
        assert abs(float(H[0]) + (a * Bx + b * By + h * M)) < 1e-12


def test_energy_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    R, Ly, Lx, h = 2, 4, 6, 0.1
    s = rng.uniform(-1, 1, size=(R, Ly, Lx))
    Jx = rng.uniform(-1, 1, size=(R, Ly, Lx))
    Jy = rng.uniform(-1, 1, size=(R, Ly, Lx))
    _, g = so.energy(s, Jx, Jy, h)
    eps = 1e-6
    for idx in [(0, 0, 0), (1, 3, 5), (0, 2, 3), (1, 0, 5)]:
        sp, sm = s.copy(), s.copy()
        sp[idx] += eps
        sm[idx] -= eps
        fd = (float(so.energy(sp, Jx, Jy, h)[0][idx[0]])
              - float(so.energy(sm, Jx, Jy, h)[0][idx[0]])) / (2 * eps)
        assert abs(fd - float(g[idx])) < 1e-8


def test_discretize_step():
    base = np.array([[[0.5, -0.5, 0.0, 0.0]]])
    g = np.array([[[1.0, -1.0, 0.0, 1e-3]]])
    out = so.discretize_step(base, g, 1.0).numpy()
    assert out.tolist() == [[[-1.0, 1.0, 1.0, -1.0]]]  # 0 -> +1, as the paper's step function


def test_gradient_step_fixed_point_and_defect_repair():
    """J = 1: the uniform state is a fixed point; a single flipped spin is
    flipped back in one step and no other spin moves (its neighbours see a
    field of 2 along their spin)."""
    Ly, Lx = 6, 6
    J = np.ones((1, Ly, Lx))
    up = np.ones((1, Ly, Lx))
    assert torch.equal(so.gradient_step(up, J, J, 0.0, 1.0), torch.tensor(up))
    d = up.copy()
    d[0, 2, 3] = -1
    assert torch.equal(so.gradient_step(d, J, J, 0.0, 1.0), torch.tensor(up))
    # a small step (eta |grad| <= 1 everywhere) never flips a +-1 spin
    assert torch.equal(so.gradient_step(d, J, J, 0.0, 0.2), torch.tensor(d))


def test_mc_sweep_at_infinite_temperature_flips_every_spin():
    """beta = 0: P = 1 > r always, so the hard-limit sweep flips every spin."""
    rng = np.random.default_rng(3)
    s = _pm1(rng, 2, 4, 6)
    J = rng.choice([-1.0, 1.0], size=s.shape)
    out = so.mc_anneal_step(s, J, J, 0.0, 0.0, 9, [0, 1], 4).numpy()
    assert np.array_equal(out, -s)


def test_mc_anneal_energy_never_rises_at_zero_temperature_limit():
    """At very large beta only moves with dE <= 0 are taken (P = exp(-beta dE)
    < r for dE > 0 unless r is tiny), so the energy does not increase."""
    rng = np.random.default_rng(4)
    s = _pm1(rng, 3, 8, 8)
    J = rng.choice([-1.0, 1.0], size=(2, 3, 8, 8))
    hist, _ = so.run("mc", s, J[0], J[1], 0.0, 10, betas=[40.0] * 10, seed=5)
    assert np.all(np.diff(hist, axis=0) <= 1e-12)


def test_dmc_step_without_gradient_is_the_discretised_chain():
    rng = np.random.default_rng(5)
    s = _pm1(rng, 2, 6, 6)
    J = rng.choice([-1.0, 1.0], size=(2, 2, 6, 6))
    out = so.dmc_step(s, J[0], J[1], 0.0, 0.8, 6.0, 3, 0.0, 11, [0, 1], 2)
    chain = dmc.forward(torch.tensor(s), torch.tensor(J[0]), torch.tensor(J[1]), 0.0, 0.8, 6.0,
                        11, [0, 1], 6, 3)
    assert torch.equal(out, torch.where(chain < 0, -1.0, 1.0).double())
