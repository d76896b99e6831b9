"""Pins of the chain / square / simple-cubic Ising oracle (the 1D, 2D and 3D
convolutions of the Methods in one natural layout): the periodic chain
against its transfer-matrix solution, cubic tori against exact enumeration,
the square case's statistics against the square-lattice oracle, one sweep
against a brute-force prediction, and the beta = 0 limit."""
import itertools
import math

import numpy as np
import pytest

import exact
from oracle import chain as orc


def _key(seed):
    return [seed & 0xFFFFFFFF, seed >> 32]


def _neighbours(Lz, Ly, Lx, z, y, x):
    out = [(z, y, (x - 1) % Lx), (z, y, (x + 1) % Lx)]
    if Ly > 1:
        out += [(z, (y - 1) % Ly, x), (z, (y + 1) % Ly, x)]
    if Lz > 1:
        out += [((z - 1) % Lz, y, x), ((z + 1) % Lz, y, x)]
    return out


def _energy(s, J, h):
    """H = -J sum over forward bonds (one per present direction and site)
    - h sum s, by explicit loops."""
    Lz, Ly, Lx = s.shape
    H = 0.0
    for z, y, x in itertools.product(range(Lz), range(Ly), range(Lx)):
        H -= J * s[z, y, x] * s[z, y, (x + 1) % Lx]
        if Ly > 1:
            H -= J * s[z, y, x] * s[z, (y + 1) % Ly, x]
        if Lz > 1:
            H -= J * s[z, y, x] * s[(z + 1) % Lz, y, x]
        H -= h * s[z, y, x]
    return H


def _chain_exact_e(N, J, h, beta):
    """<e> of the periodic chain from Z = l+^N + l-^N (transfer matrix),
    by a central difference of ln Z in beta."""
    def lnZ(b):
        a = math.exp(b * J) * math.cosh(b * h)
        r = math.sqrt(math.exp(2 * b * J) * math.sinh(b * h) ** 2 + math.exp(-2 * b * J))
        return math.log((a + r) ** N + (a - r) ** N)
    d = 1e-6
    return -(lnZ(beta + d) - lnZ(beta - d)) / (2 * d) / N


def _enum(Lz, Ly, Lx, J, h, beta):
    n = Lz * Ly * Lx
    idx = np.arange(2 ** n, dtype=np.int64)
    st = (2 * ((idx[:, None] >> np.arange(n)[None, :]) & 1) - 1).reshape(-1, Lz, Ly, Lx)
    M = st.sum(axis=(1, 2, 3))
    B = (st * np.roll(st, -1, axis=3)).sum(axis=(1, 2, 3))
    if Ly > 1:
        B = B + (st * np.roll(st, -1, axis=2)).sum(axis=(1, 2, 3))
    if Lz > 1:
        B = B + (st * np.roll(st, -1, axis=1)).sum(axis=(1, 2, 3))
    E = -(J * B + h * M)
    a = -beta * E
    w = np.exp(a - a.max())
    p = w / w.sum()
    return float((p * E).sum() / n), float((p * np.abs(M)).sum() / n)


def _chains(Lz, Ly, Lx, J, h, beta, R=64, burn=500, n=20000):
    e, m = np.zeros(R), np.zeros(R)
    N = Lz * Ly * Lx
    for r in range(R):
        s0 = orc.hc_init(Lx, Ly, Lz, 17, r)
        _, st = orc.hc_run(s0, J, h, beta, 17, r, 0, burn + n, 1)
        st = st[burn:].astype(float)
        e[r] = (-(J * (st[:, 1] + st[:, 2] + st[:, 3]) + h * st[:, 0])).mean() / N
        m[r] = np.abs(st[:, 0]).mean() / N
    return e, m


def test_chain_matches_the_transfer_matrix():
    N, J, h, beta = 10, 1.0, 0.1, 0.6
    want = _chain_exact_e(N, J, h, beta)
    e_enum, _ = _enum(1, 1, N, J, h, beta)
    assert abs(want - e_enum) < 1e-8  # the enumeration helper agrees
    e, _ = _chains(1, 1, N, J, h, beta)
    se = e.std(ddof=1) / math.sqrt(len(e))
    assert abs(e.mean() - want) <= 3 * se, (e.mean(), want, se)


@pytest.mark.parametrize("shape,J,beta", [((2, 2, 4), 1.0, 0.2), ((2, 4, 2), -0.7, 0.5)])
def test_cubic_torus_matches_enumeration(shape, J, beta):
    Lz, Ly, Lx = shape
    we, wm = _enum(Lz, Ly, Lx, J, 0.0, beta)
    e, m = _chains(Lz, Ly, Lx, J, 0.0, beta)
    for est, ref in ((e, we), (m, wm)):
        se = est.std(ddof=1) / math.sqrt(len(est))
        assert abs(est.mean() - ref) <= 3 * se, (est.mean(), ref, se)


def test_square_case_statistics_equal_the_square_oracle():
    rng = np.random.default_rng(0)
    for Ly, Lx in ((4, 6), (8, 8)):
        s = rng.choice([-1, 1], size=(1, Ly, Lx)).astype(np.int8)
        assert np.array_equal(orc.hc_stats(s)[:3], orc.ising_stats(s[0])[:3])
        assert orc.hc_stats(s)[3] == 0


def test_statistics_give_the_energy():
    rng = np.random.default_rng(1)
    for shape in ((2, 4, 6), (4, 2, 2), (1, 1, 8)):
        s = rng.choice([-1, 1], size=shape).astype(np.int8)
        M, Bx, By, Bz = orc.hc_stats(s)[:4]
        assert abs(-(0.8 * (Bx + By + Bz) + 0.3 * M) - _energy(s.astype(float), 0.8, 0.3)) < 1e-12


def test_one_sweep_matches_bruteforce():
    rng = np.random.default_rng(2)
    Lz, Ly, Lx, J, h, beta, seed, rid, t = 4, 2, 6, 0.9, -0.1, 0.5, 0x1234ABCD5678, 3, 11
    s = rng.choice([-1, 1], size=(Lz, Ly, Lx)).astype(np.int8)
    want = s.copy()
    for c in (0, 1):
        cur = want.copy()
        for z, y, x in itertools.product(range(Lz), range(Ly), range(Lx)):
            if (x + y + z) & 1 != c:
                continue
            k = ((z * Ly + y) * Lx + x) >> 1
            W = int(orc.philox4x32_10([k >> 2, 2 * t + c, rid, 0], _key(seed))[k & 3])
            S = sum(int(cur[q]) for q in _neighbours(Lz, Ly, Lx, z, y, x))
            dE = 2 * cur[z, y, x] * (J * S + h)
            if dE <= 0 or W < math.ceil(math.ldexp(math.exp(-beta * dE), 32)):
                want[z, y, x] = -cur[z, y, x]
    got, _ = orc.hc_run(s, J, h, beta, seed, rid, t, 1)
    assert np.array_equal(got, want)


def test_infinite_temperature_flips_every_spin():
    rng = np.random.default_rng(3)
    s = rng.choice([-1, 1], size=(2, 4, 4)).astype(np.int8)
    got, _ = orc.hc_run(s, 1.0, 0.2, 0.0, 5, 0, 0, 1)
    assert np.array_equal(got, -s)
