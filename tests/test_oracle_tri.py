"""Pins of the triangular-lattice Ising oracle (the six-neighbour lattice of
the Methods' triangular kernels): bond statistics against an independent
energy, one sweep against a brute-force prediction, the infinite-temperature
and zero-temperature limits, and long chains against exact enumeration of a
3 x 6 torus (ferromagnetic and frustrated antiferromagnetic)."""
import math

import numpy as np
import pytest

import exact
from oracle import chain as orc

NB6 = [(0, -1), (0, 1), (-1, 0), (1, 0), (-1, 1), (1, -1)]


def _energy(s, J, h):
    """H = -J sum over the bonds (each once) - h sum s, by explicit loops."""
    Ly, Lx = s.shape
    H = 0.0
    for y in range(Ly):
        for x in range(Lx):
            for dy, dx in [(0, 1), (1, 0), (1, -1)]:
                H -= J * s[y, x] * s[(y + dy) % Ly, (x + dx) % Lx]
            H -= h * s[y, x]
    return H


def _key(seed):
    return [seed & 0xFFFFFFFF, seed >> 32]


def test_statistics_give_the_energy():
    rng = np.random.default_rng(0)
    for Ly, Lx in ((3, 3), (6, 9), (9, 6)):
        s = rng.choice([-1, 1], size=(Ly, Lx)).astype(np.int8)
        M, Bh, Bv, Bd = orc.tri_stats(s)[:4]
        J, h = 0.7, -0.2
        assert abs(-(J * (Bh + Bv + Bd) + h * M) - _energy(s.astype(float), J, h)) < 1e-12
        assert M == s.sum()


def test_one_sweep_matches_bruteforce():
    """Three colour passes c = (x + 2y) mod 3, each from the pass-start
    state: flip iff W < ceil(2^32 exp(-beta dE)) (dE <= 0: always), W word
    k & 3 of Philox (k >> 2, 3t + c, rid, 0), k = y Lx/3 + x/3."""
    rng = np.random.default_rng(1)
    Ly, Lx, J, h, beta, seed, rid, t = 6, 9, 0.8, 0.1, 0.6, 0xABCDEF123, 4, 7
    s = rng.choice([-1, 1], size=(Ly, Lx)).astype(np.int8)
    want = s.copy()
    for c in range(3):
        p = 3 * t + c
        cur = want.copy()
        for y in range(Ly):
            for x in range(Lx):
                if (x + 2 * y) % 3 != c:
                    continue
                k = y * (Lx // 3) + x // 3
                W = int(orc.philox4x32_10([k >> 2, p, rid, 0], _key(seed))[k & 3])
                E0 = _energy(cur.astype(float), J, h)
                trial = cur.copy()
                trial[y, x] = -trial[y, x]
                dE = _energy(trial.astype(float), J, h) - E0
                if dE <= 1e-12 or W < math.ceil(math.ldexp(math.exp(-beta * dE), 32)):
                    want[y, x] = -cur[y, x]
    got, _ = orc.tri_run(s, J, h, beta, seed, rid, t, 1)
    assert np.array_equal(got, want)


def test_infinite_temperature_flips_every_spin():
    rng = np.random.default_rng(2)
    s = rng.choice([-1, 1], size=(6, 6)).astype(np.int8)
    got, _ = orc.tri_run(s, 1.0, 0.3, 0.0, 5, 0, 0, 1)
    assert np.array_equal(got, -s)


def test_zero_temperature_never_raises_the_energy():
    rng = np.random.default_rng(3)
    s = rng.choice([-1, 1], size=(9, 9)).astype(np.int8)
    _, st = orc.tri_run(s, 1.0, 0.0, 60.0, 6, 0, 0, 40, 1)
    E = -(st[:, 1] + st[:, 2] + st[:, 3]).astype(float)
    assert np.all(np.diff(E) <= 0)


@pytest.mark.parametrize("J,beta", [(1.0, 0.25), (-1.0, 0.8)])
def test_long_chains_match_exact_enumeration(J, beta):
    """3 x 6 torus (2^18 states): replica means of <e> and <|m|> within 3
    sigma of the exact values; J < 0 is the frustrated antiferromagnet."""
    Ly, Lx, R, burn, n = 3, 6, 64, 1000, 10000
    ex = exact.tri_exact(Ly, Lx, J, 0.0, beta)
    e = np.zeros(R)
    m = np.zeros(R)
    for r in range(R):
        s0 = orc.ising_init(Lx, Ly, 9, r)
        _, st = orc.tri_run(s0.reshape(Ly, Lx), J, 0.0, beta, 9, r, 0, burn + n, 1)
        st = st[burn:].astype(float)
        e[r] = (-J * (st[:, 1] + st[:, 2] + st[:, 3])).mean() / (Ly * Lx)
        m[r] = np.abs(st[:, 0]).mean() / (Ly * Lx)
    for est, ref in ((e, ex["e"]), (m, ex["absm"])):
        se = est.std(ddof=1) / math.sqrt(R)
        assert abs(est.mean() - ref) <= 3 * se, (est.mean(), ref, se)
