"""One-sweep predictions of the oracle chain from brute-force energies.

For every colour pass the test recomputes, independently of the oracle:
  * the energy change of each proposal from two full-lattice energies
    (Eq. (1), Eq. (2), Eq. (3)), not from a local formula;
  * the Metropolis rule of Algorithm 1 in its plain form: accept when
    dE <= 0, else when the uniform W / 2^32 < exp(-beta dE);
  * all sites of the colour at once, from the pass-start state (the
    checkerboard argument), whereas the oracle updates them in place.
The uniform W and the proposals follow the documented counter layout of the
Philox streams (Philox itself is pinned in test_oracle_philox.py).
A dropped term, a wrong sign, a transposed axis or a wrong colour order in
the oracle changes at least one site here.
"""
import math

import numpy as np
import pytest

from exact import ising_energy, potts_energy

MASK16 = 0xFFFF


def _key(seed):
    return [seed & 0xFFFFFFFF, seed >> 32]


def _u(orc, a, p, rid, tag, seed):
    return [int(v) for v in orc.philox4x32_10([a, p, rid, tag], _key(seed))]


def _metropolis(W, dE, beta):
    return dE <= 0 or W < math.ldexp(math.exp(-beta * dE), 32)


def predict_ising(orc, s, Jx, Jy, h, beta, seed, rid, t):
    s = s.astype(np.int8).copy()
    Ly, Lx = s.shape
    for c in (0, 1):
        p = 2 * t + c
        E0, _ = ising_energy(s, Jx, Jy, h)
        new = s.copy()
        for y in range(Ly):
            for x in range(Lx):
                if (x + y) % 2 != c:
                    continue
                k = y * (Lx // 2) + x // 2
                w = _u(orc, k >> 3, p, rid, 0, seed)
                hw = k & 7
                ra = (w[hw >> 1] >> (16 * (hw & 1))) & MASK16
                f = _u(orc, k, p, rid, 1, seed)
                W = (ra << 16) | (f[0] & MASK16)
                trial = s.copy()
                trial[y, x] = -trial[y, x]
                E1, _ = ising_energy(trial, Jx, Jy, h)
                if _metropolis(W, E1 - E0, beta):
                    new[y, x] = -s[y, x]
        s = new
    return s


@pytest.mark.parametrize("shape,Jx,Jy,h,beta,seed,rid,t", [
    ((6, 8), 1.0, 1.0, 0.0, 0.44, 1, 0, 0),
    ((8, 6), 0.7, 1.3, 0.2, 0.6, 99, 5, 17),
    ((4, 10), 1.1, 0.4, -0.3, 0.9, 2 ** 40 + 3, 1023, 123456),
    ((10, 20), 0.5, 0.5, 0.05, 0.3, 7, 3, 2),
])
def test_ising_sweep_matches_bruteforce(orc, shape, Jx, Jy, h, beta, seed, rid, t):
    rng = np.random.default_rng(seed % 1000)
    s0 = (2 * rng.integers(0, 2, size=shape) - 1).astype(np.int8)
    Jx, Jy, h = (float(np.float32(v)) for v in (Jx, Jy, h))
    want = predict_ising(orc, s0, Jx, Jy, h, beta, seed, rid, t)
    got, _ = orc.ising_run(s0, Jx, Jy, h, beta, seed, rid, t, 1)
    assert np.array_equal(got, want)


def test_ising_flip_frequencies_follow_metropolis(orc):
    """From one fixed state, over many chain seeds, each site of colour 0
    flips in its first pass with probability min(1, exp(-beta dE))."""
    rng = np.random.default_rng(3)
    s0 = (2 * rng.integers(0, 2, size=(4, 8)) - 1).astype(np.int8)
    Jx, Jy, h, beta = 1.0, 0.5, 0.1, 0.5
    E0, _ = ising_energy(s0, Jx, Jy, h)
    n = 3000
    flips = np.zeros(s0.shape)
    for seed in range(n):
        # half a sweep: run one sweep and look at colour-0 sites only, which
        # colour 1 never changes
        got, _ = orc.ising_run(s0, Jx, Jy, h, beta, seed + 1, 0, 0, 1)
        flips += (got != s0)
    for y in range(4):
        for x in range(8):
            if (x + y) % 2:
                continue
            trial = s0.copy()
            trial[y, x] *= -1
            dE = ising_energy(trial, Jx, Jy, h)[0] - E0
            p = min(1.0, math.exp(-beta * dE))
            sd = math.sqrt(max(p * (1 - p), 1e-12) / n)
            assert abs(flips[y, x] / n - p) < 5 * sd + 1e-9


def _potts_offset(rp, fb, m):
    prod = rp * m
    if (prod & MASK16) < (65536 % m):
        return (fb * m) >> 32
    return prod >> 16


def predict_potts(orc, s, q, J, h, beta, seed, rid, t):
    s = s.astype(np.uint8).copy()
    Ly, Lx = s.shape
    for c in (0, 1):
        p = 2 * t + c
        E0, _ = potts_energy(s, J, h)
        new = s.copy()
        for y in range(Ly):
            for x in range(Lx):
                if (x + y) % 2 != c:
                    continue
                k = y * (Lx // 2) + x // 2
                word = _u(orc, k >> 2, p, rid, 0, seed)[k & 3]
                f = _u(orc, k, p, rid, 1, seed)
                W = ((word >> 16) << 16) | (f[0] & MASK16)
                off = _potts_offset(word & MASK16, f[1], q - 1)
                s2 = (int(s[y, x]) + 1 + off) % q
                assert s2 != s[y, x]
                trial = s.copy()
                trial[y, x] = s2
                E1, _ = potts_energy(trial, J, h)
                if _metropolis(W, E1 - E0, beta):
                    new[y, x] = s2
        s = new
    return s


@pytest.mark.parametrize("shape,q,J,h,beta,seed,rid,t", [
    ((6, 8), 3, 1.0, 0.0, 1.0, 1, 0, 0),
    ((8, 6), 4, 1.0, 0.15, 1.2, 5, 9, 31),
    ((4, 8), 8, 0.75, -0.1, 1.5, 123, 77, 4),
    ((6, 6), 2, 1.0, 0.0, 0.8, 3, 1, 0),
])
def test_potts_sweep_matches_bruteforce(orc, shape, q, J, h, beta, seed, rid, t):
    rng = np.random.default_rng(seed)
    s0 = rng.integers(0, q, size=shape).astype(np.uint8)
    J, h = float(np.float32(J)), float(np.float32(h))
    want = predict_potts(orc, s0, q, J, h, beta, seed, rid, t)
    got, _ = orc.potts_run(s0, q, J, h, beta, seed, rid, t, 1)
    assert np.array_equal(got, want)


def test_potts_proposal_offsets_exactly_uniform():
    """Lemire's multiply-shift with rejection: over all 2^16 prefixes the
    accepted ones give every offset in [0, m) equally often."""
    for m in range(1, 12):
        counts = np.zeros(m, np.int64)
        rej = 0
        for rp in range(65536):
            prod = rp * m
            if (prod & MASK16) < (65536 % m):
                rej += 1
                continue
            counts[prod >> 16] += 1
        assert rej == 65536 % m
        assert np.all(counts == counts[0])


# ------------------------------------------------------------------ CPM
MOORE = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]


def cpm_energy(ids, J, ctype, A, lam, area):
    """Eq. (3): adhesion over unordered Moore pairs between different ids,
    plus lambda (a - A)^2 over cells (not the medium), with given areas."""
    Ly, Lx = ids.shape
    H = 0.0
    for dy, dx in [(0, 1), (1, 0), (1, 1), (1, -1)]:
        nb = np.roll(np.roll(ids, -dy, axis=0), -dx, axis=1)
        diff = ids != nb
        H += float(J[ctype[ids[diff]], ctype[nb[diff]]].astype(np.float64).sum())
    cells = np.arange(1, len(A))
    H += lam * float(((area[cells].astype(np.float64) - A[cells]) ** 2).sum())
    return H


def predict_cpm(orc, ids, J, ctype, A, lam, T, seed, rid, t):
    ids = ids.copy()
    Ly, Lx = ids.shape
    for c in range(4):
        p = 4 * t + c
        snap = np.bincount(ids.reshape(-1), minlength=len(A))
        E0 = cpm_energy(ids, J, ctype, A, lam, snap)
        new = ids.copy()
        for y in range(Ly):
            for x in range(Lx):
                if 2 * (y & 1) + (x & 1) != c:
                    continue
                k = (y >> 1) * (Lx // 2) + (x >> 1)
                word = _u(orc, k >> 2, p, rid, 0, seed)[k & 3]
                dy, dx = MOORE[word & 7]
                s, tg = ids[y, x], ids[(y + dy) % Ly, (x + dx) % Lx]
                if s == tg:
                    continue
                f = _u(orc, k, p, rid, 1, seed)
                W = ((word >> 16) << 16) | (f[0] & MASK16)
                trial = ids.copy()
                trial[y, x] = tg
                a1 = snap.copy()
                a1[tg] += 1
                a1[s] -= 1
                dH = cpm_energy(trial, J, ctype, A, lam, a1) - E0
                if dH <= 0 or W < math.ldexp(math.exp(-dH / T), 32):
                    new[y, x] = tg
        ids = new
    return ids


def _cpm_case(seed, L=(8, 10), n_cells=5):
    rng = np.random.default_rng(seed)
    Ly, Lx = L
    ids = rng.integers(0, n_cells + 1, size=(Ly, Lx)).astype(np.int32)
    ctype = np.concatenate([[0], rng.integers(1, 3, size=n_cells)]).astype(np.int8)
    A = np.concatenate([[0], rng.integers(5, 15, size=n_cells)]).astype(np.int32)
    return ids, ctype, A


@pytest.mark.parametrize("seed,lam,T,Jset", [
    (1, 1.0, 10.0, "sorting"),
    (2, 0.5, 3.0, "halves"),
    (3, 0.0, 1.0, "sorting"),
    (4, 2.0, 25.0, "halves"),
])
def test_cpm_mcs_matches_bruteforce(orc, seed, lam, T, Jset):
    ids, ctype, A = _cpm_case(seed)
    if Jset == "sorting":
        J = np.array([[0, 16, 16], [16, 2, 11], [16, 11, 16]], np.float32)
    else:
        J = np.array([[0, 3.5, 4.5], [3.5, 1.5, 2.0], [4.5, 2.0, 0.5]], np.float32)
    want = predict_cpm(orc, ids, J, ctype, A, lam, T, seed, 2, 5)
    got, area, _ = orc.cpm_run(ids, J, ctype, A, lam, T, seed, 2, 5, 1)
    assert np.array_equal(got, want)
    assert np.array_equal(area, np.bincount(got.reshape(-1), minlength=len(A)))


# ------------------------------------------------ CPM, 5 x 5 neighbourhood
# the 24 offsets within Chebyshev distance 2, row-major, and the 12 that
# count each unordered pair once
N24 = [(dy, dx) for dy in range(-2, 3) for dx in range(-2, 3) if (dy, dx) != (0, 0)]
F12 = [(0, 1), (0, 2), (1, -2), (1, -1), (1, 0), (1, 1), (1, 2), (2, -2), (2, -1), (2, 0),
       (2, 1), (2, 2)]


def cpm_energy5(ids, J, ctype, A, lam, area):
    """Eq. (3) with the second shell: adhesion over unordered pairs at
    Chebyshev distance <= 2 between different ids, plus the area term."""
    H = 0.0
    for dy, dx in F12:
        nb = np.roll(np.roll(ids, -dy, axis=0), -dx, axis=1)
        diff = ids != nb
        H += float(J[ctype[ids[diff]], ctype[nb[diff]]].astype(np.float64).sum())
    cells = np.arange(1, len(A))
    H += lam * float(((area[cells].astype(np.float64) - A[cells]) ** 2).sum())
    return H


def predict_cpm5(orc, ids, J, ctype, A, lam, T, seed, rid, t):
    """Nine passes c = 3 (y % 3) + x % 3; neighbour by Lemire's
    multiply-shift of the low 16 bits into 24 with rejection, then 24 times
    word 1 of the fallback block shifted by 32."""
    ids = ids.copy()
    Ly, Lx = ids.shape
    for c in range(9):
        p = 9 * t + c
        snap = np.bincount(ids.reshape(-1), minlength=len(A))
        E0 = cpm_energy5(ids, J, ctype, A, lam, snap)
        new = ids.copy()
        for y in range(Ly):
            for x in range(Lx):
                if 3 * (y % 3) + x % 3 != c:
                    continue
                k = (y // 3) * (Lx // 3) + x // 3
                word = _u(orc, k >> 2, p, rid, 0, seed)[k & 3]
                f = _u(orc, k, p, rid, 1, seed)
                l = (word & MASK16) * 24
                j = l >> 16 if (l & MASK16) >= 65536 % 24 else (f[1] * 24) >> 32
                dy, dx = N24[j]
                s, tg = ids[y, x], ids[(y + dy) % Ly, (x + dx) % Lx]
                if s == tg:
                    continue
                W = ((word >> 16) << 16) | (f[0] & MASK16)
                trial = ids.copy()
                trial[y, x] = tg
                a1 = snap.copy()
                a1[tg] += 1
                a1[s] -= 1
                dH = cpm_energy5(trial, J, ctype, A, lam, a1) - E0
                if dH <= 0 or W < math.ldexp(math.exp(-dH / T), 32):
                    new[y, x] = tg
        ids = new
    return ids


def test_lemire_choice_of_24_is_exactly_uniform():
    counts = np.zeros(24, np.int64)
    rej = 0
    for u in range(65536):
        l = u * 24
        if (l & MASK16) < 65536 % 24:
            rej += 1
        else:
            counts[l >> 16] += 1
    assert rej == 16 and np.all(counts == 2730)


@pytest.mark.parametrize("seed,lam,T,shape", [
    (11, 1.0, 10.0, (6, 12)), (12, 0.5, 3.0, (12, 6)), (13, 2.0, 25.0, (6, 6))])
def test_cpm5_mcs_matches_bruteforce(orc, seed, lam, T, shape):
    ids, ctype, A = _cpm_case(seed, L=shape, n_cells=6)
    J = np.array([[0, 16, 16], [16, 2, 11], [16, 11, 14]], np.float32)
    want = predict_cpm5(orc, ids, J, ctype, A, lam, T, seed, 3, 4)
    got, area, _ = orc.cpm_run(ids, J, ctype, A, lam, T, seed, 3, 4, 1, nrange=2)
    assert np.array_equal(got, want)
    assert np.array_equal(area, np.bincount(got.reshape(-1), minlength=len(A)))


def test_cpm5_energy_statistic_matches_bruteforce(orc):
    rng = np.random.default_rng(14)
    J = np.array([[0, 3.5, 4.5], [3.5, 1.5, 2.0], [4.5, 2.0, 0.5]], np.float32)
    S = orc.cpm_scale(J, 0.5)
    for shape in ((6, 6), (12, 18)):
        ids, ctype, A = _cpm_case(int(rng.integers(1 << 30)), L=shape, n_cells=7)
        area = np.bincount(ids.reshape(-1), minlength=len(A))
        st = orc.cpm_stats(ids, J, ctype, A, 0.5, nrange=2)
        H = (int(st[11]) << 32) | (int(st[10]) & 0xFFFFFFFF)
        assert H == round(cpm_energy5(ids, J, ctype, A, 0.5, area) * S)
        # the boundary bonds stay von Neumann: the same as for range 1
        assert np.array_equal(st[:10], orc.cpm_stats(ids, J, ctype, A, 0.5)[:10])


def test_cpm5_rejects_shapes_off_the_3x3_sublattice(orc):
    ids, ctype, A = _cpm_case(15, L=(8, 12), n_cells=3)
    J = np.array([[0, 1], [1, 0]], np.float32)
    with pytest.raises(Exception):
        orc.cpm_run(ids, J, np.minimum(ctype, 1), A, 1.0, 5.0, 1, 0, 0, 1, nrange=2)


def test_cpm5_neighbour_fallback_path(orc):
    """A seed whose Monte Carlo step meets the rejected branch of the
    neighbour choice (probability 16/65536 per attempt): the oracle still
    equals the brute-force prediction there."""
    Ly, Lx, rid, t = 6, 6, 1, 0
    hit = None
    for seed in range(1, 5000):
        for c in range(9):
            for blk in range(((Ly // 3) * (Lx // 3) + 3) // 4):
                for word in _u(orc, blk, 9 * t + c, rid, 0, seed):
                    if ((word & MASK16) * 24) & MASK16 < 16:
                        hit = seed
                        break
                if hit:
                    break
            if hit:
                break
        if hit:
            break
    assert hit is not None
    ids, ctype, A = _cpm_case(hit, L=(Ly, Lx), n_cells=5)
    J = np.array([[0, 16, 16], [16, 2, 11], [16, 11, 14]], np.float32)
    want = predict_cpm5(orc, ids, J, ctype, A, 1.0, 50.0, hit, rid, t)
    got, _, _ = orc.cpm_run(ids, J, ctype, A, 1.0, 50.0, hit, rid, t, 1, nrange=2)
    assert np.array_equal(got, want)


def test_pass_rows_on_threads_change_no_bit(orc):
    """Large square lattices split a colour pass's rows over threads: the
    chain (states and recorded statistics) equals the one-thread chain."""
    n_thr = orc.num_threads()
    try:
        out = {}
        for k in (1, max(n_thr, 4)):
            orc.set_num_threads(k)
            s = orc.ising_init(256, 256, 9, 3)
            a = orc.ising_run(s, 0.9, 1.1, 0.02, 0.44, 9, 3, 5, 6, 2)
            s = orc.potts_init(512, 128, 5, 9, 4)
            b = orc.potts_run(s, 5, 1.0, 0.01, 1.2, 9, 4, 5, 6, 3)
            out[k] = (a, b)
        (a1, b1), (a2, b2) = out[1], out[max(n_thr, 4)]
        for u, v in ((a1, a2), (b1, b2)):
            assert np.array_equal(u[0], v[0]) and np.array_equal(u[1], v[1])
    finally:
        orc.set_num_threads(n_thr)
