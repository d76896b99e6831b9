"""Pins of the multispin-coded Ising oracle (32 replicas per uint32 word,
shared random numbers): with Jx = Jy every bit follows the natural-layout
chain of the chain / square / cubic oracle (pinned by enumeration) from the
same start and stream; anisotropic couplings against a brute-force sweep;
the initial words and the statistics bit by bit."""
import math

import numpy as np

from oracle import chain as orc


def _key(seed):
    return [seed & 0xFFFFFFFF, seed >> 32]


def test_each_bit_is_the_square_natural_layout_chain():
    Ly, Lx, J, h, beta, seed, rid = 6, 8, 0.8, 0.1, 0.5, 77, 9
    w0 = orc.msc_init(Lx, Ly, seed, rid)
    w, st = orc.msc_run(w0, J, J, h, beta, seed, rid, 3, 5, 1)
    bits0 = orc.msc_unpack(w0)
    bits = orc.msc_unpack(w)
    for b in range(32):
        want, _ = orc.hc_run(bits0[b][None], J, h, beta, seed, rid, 3, 5)
        assert np.array_equal(bits[b], want[0]), b
    # statistics of every bit are those of its unpacked lattice
    for b in range(32):
        assert np.array_equal(st[-1, b, :3], orc.ising_stats(bits[b])[:3])


def test_initial_words():
    Ly, Lx, seed, rid = 4, 6, 0x1234567890, 5
    w = orc.msc_init(Lx, Ly, seed, rid)
    assert np.array_equal(orc.msc_unpack(w)[0], orc.ising_init(Lx, Ly, seed, rid).reshape(Ly, Lx))
    for n in (0, 5, 23):
        for b in (0, 7, 31):
            word = orc.philox4x32_10([n >> 2, b, rid, 2], _key(seed))[n & 3]
            assert ((int(w.reshape(-1)[n]) >> b) & 1) == (1 if word < 2 ** 31 else 0)


def test_anisotropic_sweep_matches_bruteforce():
    rng = np.random.default_rng(3)
    Ly, Lx, Jx, Jy, h, beta, seed, rid, t = 4, 6, 1.1, -0.4, 0.05, 0.7, 12345, 2, 4
    w0 = rng.integers(0, 2 ** 32, size=(Ly, Lx), dtype=np.uint64).astype(np.uint32)
    s = orc.msc_unpack(w0).astype(int)
    for c in (0, 1):
        new = s.copy()
        for y in range(Ly):
            for x in range(Lx):
                if (x + y) & 1 != c:
                    continue
                k = (y * Lx + x) >> 1
                W = int(orc.philox4x32_10([k >> 2, 2 * t + c, rid, 0], _key(seed))[k & 3])
                for b in range(32):
                    sv = s[b, y, x]
                    Sx = s[b, y, (x - 1) % Lx] + s[b, y, (x + 1) % Lx]
                    Sy = s[b, (y - 1) % Ly, x] + s[b, (y + 1) % Ly, x]
                    dE = 2 * sv * (np.float32(Jx) * Sx + np.float32(Jy) * Sy + np.float32(h))
                    T = 2 ** 32 if dE <= 0 else math.ceil(math.ldexp(math.exp(-beta * dE), 32))
                    if W < T:
                        new[b, y, x] = -sv
        s = new
    got, _ = orc.msc_run(w0, Jx, Jy, h, beta, seed, rid, t, 1)
    assert np.array_equal(orc.msc_unpack(got), s.astype(np.int8))
