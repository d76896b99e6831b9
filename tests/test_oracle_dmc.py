"""Pins of the differentiable-Monte-Carlo oracle (relaxed chain of the
paper's Algorithm 2): closed forms at beta = 0 and alpha = 0, the hard limit
alpha -> infinity against exact 4x4 enumeration, the spin-flip symmetry, and
reverse-mode gradients against finite differences of the forward."""
import math

import numpy as np
import pytest
import torch

import exact
from oracle import chain as orc
from oracle import dmc


def _rng_state(rng, R, Ly, Lx):
    return rng.uniform(-1.0, 1.0, size=(R, Ly, Lx))


def test_uniforms_follow_the_counter_layout():
    """r at (y, x) of colour c in pass p is word k & 3 of the Philox block
    (k >> 2, p, rid, 3), k = y Lx/2 + x >> 1, scaled by 2^-24 after >> 8."""
    Lx, Ly, seed, rids, p = 8, 6, 0x1234_5678_9ABC, [7, 3000000000], 13
    r = dmc.uniforms(Lx, Ly, seed, rids, p).numpy()
    c = p & 1
    for ri, rid in enumerate(rids):
        for y in range(Ly):
            for x in range(Lx):
                if (x + y) % 2 != c:
                    assert r[ri, y, x] == 0.0
                    continue
                k = y * (Lx // 2) + (x >> 1)
                w = orc.philox4x32_10([k >> 2, p, rid, 3], [seed & 0xFFFFFFFF, seed >> 32])[k & 3]
                assert r[ri, y, x] == (int(w) >> 8) * 2.0 ** -24


def test_beta_zero_is_a_site_by_site_closed_form():
    """beta = 0 makes P = 1: every site of a pass becomes s (1 - 2 q) with
    q = 1 / (1 + exp(-alpha (1 - r))), whatever its neighbours."""
    rng = np.random.default_rng(1)
    R, Ly, Lx, alpha, seed, rids = 2, 4, 6, 2.5, 99, [1, 2]
    s0 = _rng_state(rng, R, Ly, Lx)
    J = rng.uniform(0.2, 1.0, size=(R, Ly, Lx))
    out = dmc.forward(torch.tensor(s0), torch.tensor(J), torch.tensor(J), 0.3, 0.0, alpha, seed,
                      rids, 5, 1).numpy()
    want = s0.copy()
    for c in (0, 1):
        r = dmc.uniforms(Lx, Ly, seed, rids, 2 * 5 + c).numpy()
        q = 1.0 / (1.0 + np.exp(-alpha * (1.0 - r)))
        m = dmc.colour_mask(Lx, Ly, c).numpy()
        want = np.where(m, want * (1.0 - 2.0 * q), want)
    np.testing.assert_allclose(out, want, rtol=1e-15, atol=0)


def test_alpha_zero_sets_every_spin_to_zero():
    """alpha = 0 makes q = 1/2, so one sweep maps every spin to 0."""
    rng = np.random.default_rng(2)
    s0 = _rng_state(rng, 1, 4, 4)
    J = np.full((1, 4, 4), 0.7)
    out = dmc.forward(torch.tensor(s0), torch.tensor(J), torch.tensor(J), 0.1, 0.8, 0.0, 3, [0],
                      0, 1).numpy()
    assert np.all(out == 0.0)


def test_global_spin_flip_symmetry_at_zero_field():
    """With h = 0, flipping every initial spin flips every final spin."""
    rng = np.random.default_rng(3)
    R, Ly, Lx = 3, 6, 4
    s0 = _rng_state(rng, R, Ly, Lx)
    Jx, Jy = rng.uniform(-1, 1, size=(2, R, Ly, Lx))
    args = (0.0, 0.7, 4.0, 11, [4, 5, 6], 2, 3)
    a = dmc.forward(torch.tensor(s0), torch.tensor(Jx), torch.tensor(Jy), *args).numpy()
    b = dmc.forward(torch.tensor(-s0), torch.tensor(Jx), torch.tensor(Jy), *args).numpy()
    assert np.array_equal(a, -b)


def test_hard_limit_samples_the_metropolis_distribution():
    """alpha -> infinity turns q into the accept indicator [r < P], i.e. the
    Metropolis rule: spins stay at +-1, and on the 4x4 torus the replica
    averages of <e> and <|m|> agree with exact enumeration within 3 sigma."""
    R, L, J, beta, burn, n = 256, 4, 1.0, 0.44, 300, 1500
    rng = np.random.default_rng(4)
    s = torch.tensor(rng.choice([-1.0, 1.0], size=(R, L, L)))
    Jt = torch.full((R, L, L), J, dtype=torch.float64)
    rids = list(range(R))
    e_acc = np.zeros(R)
    m_acc = np.zeros(R)
    for t in range(n):
        s = dmc.forward(s, Jt, Jt, 0.0, beta, 1e12, 77, rids, t, 1)
        if t >= burn:
            sn = s.numpy()
            assert np.all(np.abs(sn) == 1.0)
            B = (sn * np.roll(sn, -1, 2)).sum((1, 2)) + (sn * np.roll(sn, -1, 1)).sum((1, 2))
            e_acc += -J * B / (L * L)
            m_acc += np.abs(sn.sum((1, 2))) / (L * L)
    e = e_acc / (n - burn)
    m = m_acc / (n - burn)
    ex = exact.ising_exact(L, L, J, J, 0.0, beta)
    for est, ref in ((e, ex["e"]), (m, ex["absm"])):
        se = est.std(ddof=1) / math.sqrt(R)
        assert abs(est.mean() - ref) <= 3 * se, (est.mean(), ref, se)


@pytest.mark.parametrize("alpha,beta", [(3.0, 0.5), (0.5, 1.2)])
def test_gradients_match_finite_differences(alpha, beta):
    """Reverse-mode gradients of sum(g * s_final) with respect to the initial
    spins, both coupling fields and h equal central differences of the
    forward (FP64, step 1e-6)."""
    rng = np.random.default_rng(5)
    R, Ly, Lx, seed, rids, t0, n = 2, 4, 4, 123, [9, 10], 1, 3
    s0 = _rng_state(rng, R, Ly, Lx)
    Jx = rng.uniform(0.1, 0.9, size=(R, Ly, Lx))
    Jy = rng.uniform(0.1, 0.9, size=(R, Ly, Lx))
    h = 0.05
    g = rng.normal(size=(R, Ly, Lx))
    _, gs0, gJx, gJy, gh = dmc.forward_backward(s0, Jx, Jy, h, beta, alpha, seed, rids, t0, n, g)

    def f(s0_, Jx_, Jy_, h_):
        out = dmc.forward(torch.tensor(s0_), torch.tensor(Jx_), torch.tensor(Jy_), h_, beta,
                          alpha, seed, rids, t0, n).numpy()
        return float((out * g).sum())

    eps = 1e-6
    for arr, grad, name in ((s0, gs0, "s0"), (Jx, gJx, "Jx"), (Jy, gJy, "Jy")):
        for idx in [(0, 0, 0), (1, 2, 3), (0, 3, 1), (1, 1, 2)]:
            a_p, a_m = arr.copy(), arr.copy()
            a_p[idx] += eps
            a_m[idx] -= eps
            args_p = dict(s0=s0, Jx=Jx, Jy=Jy)
            args_m = dict(s0=s0, Jx=Jx, Jy=Jy)
            args_p[name], args_m[name] = a_p, a_m
            fd = (f(args_p["s0"], args_p["Jx"], args_p["Jy"], h)
                  - f(args_m["s0"], args_m["Jx"], args_m["Jy"], h)) / (2 * eps)
            assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, grad[idx])
    fd_h = (f(s0, Jx, Jy, h + eps) - f(s0, Jx, Jy, h - eps)) / (2 * eps)
    assert abs(fd_h - gh) <= 1e-6 * max(1.0, abs(fd_h))


def test_exponent_cap_changes_no_forward_value(monkeypatch):
    """At beta = 1000 the exponent -beta dE reaches thousands: with the cap
    the forward equals the uncapped one (q is exactly 1 past the cap) and
    the gradients stay finite."""
    rng = np.random.default_rng(6)
    R, Ly, Lx, beta, alpha = 2, 4, 6, 1000.0, 10.0
    s0 = _rng_state(rng, R, Ly, Lx)
    J = rng.uniform(0.2, 1.0, size=(R, Ly, Lx))
    g = rng.normal(size=(R, Ly, Lx))
    capped, gs0, gJx, gJy, gh = dmc.forward_backward(s0, J, J, 0.0, beta, alpha, 4, [0, 1], 0, 2,
                                                     g)
    for a in (gs0, gJx, gJy, np.array(gh)):
        assert np.all(np.isfinite(a))
    monkeypatch.setattr(dmc, "EXP_CAP", float("inf"))
    plain = dmc.forward(torch.tensor(s0), torch.tensor(J), torch.tensor(J), 0.0, beta, alpha, 4,
                        [0, 1], 0, 2).numpy()
    assert np.array_equal(capped, plain)
