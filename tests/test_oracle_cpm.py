"""Cellular Potts oracle: invariants, limits and the sorting trend.

The snapshot-area chain (areas read from the start of each colour pass) is a
deliberate reading for a parallel update; beyond the brute-force one-step
test in test_oracle_onestep.py it has no exact pin, so these tests check what
must hold for any correct implementation of Eq. (3) with copy moves.
"""
import math

import numpy as np
import pytest

import synth
from test_oracle_onestep import MOORE, _u


def _case(seed, L=16, n_cells=12):
    rng = np.random.default_rng(seed)
    ids = rng.integers(0, n_cells + 1, size=(L, L)).astype(np.int32)
    ctype = np.concatenate([[0], rng.integers(1, 3, size=n_cells)]).astype(np.int8)
    A = np.concatenate([[0], np.full(n_cells, 16)]).astype(np.int32)
    J = np.array([[0, 16, 16], [16, 2, 11], [16, 11, 16]], np.float32)
    return ids, ctype, A, J


def test_scale_choice(orc):
    assert orc.cpm_scale(np.array([[0, 16], [16, 2]], np.float32), 1.0) == 1
    assert orc.cpm_scale(np.array([[0, 1.5], [1.5, 2]], np.float32), 1.0) == 2
    assert orc.cpm_scale(np.array([[0, 1.25], [1.25, 2]], np.float32), 0.5) == 4
    with pytest.raises(ValueError):
        orc.cpm_scale(np.array([[0, 0.1], [0.1, 0]], np.float32), 1.0)


def test_area_bookkeeping_and_no_new_ids(orc):
    ids, ctype, A, J = _case(1)
    before = set(np.unique(ids))
    out, area, stats = orc.cpm_run(ids, J, ctype, A, 1.0, 10.0, 3, 0, 0, 20, 5)
    assert area.sum() == ids.size
    assert np.array_equal(area, np.bincount(out.reshape(-1), minlength=len(A)))
    assert set(np.unique(out)) <= before
    assert stats.shape == (4, 16)


def test_resume_is_bit_identical(orc):
    ids, ctype, A, J = _case(2)
    full, _, _ = orc.cpm_run(ids, J, ctype, A, 1.0, 10.0, 3, 7, 0, 12)
    half, _, _ = orc.cpm_run(ids, J, ctype, A, 1.0, 10.0, 3, 7, 0, 5)
    rest, _, _ = orc.cpm_run(half, J, ctype, A, 1.0, 10.0, 3, 7, 5, 7)
    assert np.array_equal(full, rest)


def test_zero_temperature_limit_rejects_every_uphill_move(orc):
    """T -> 0: a copy is taken only when its energy change is <= 0, so a
    site whose chosen neighbour differs keeps its id whenever copying would
    cost energy; at T -> infinity every such copy is taken."""
    ids, ctype, A, J = _case(3)
    L = ids.shape[0]
    for T, want_all in [(1e-9, False), (1e12, True)]:
        out, _, _ = orc.cpm_run(ids, J, ctype, A, 1.0, T, 5, 1, 0, 1)
        # first pass only touches colour 0; compare its sites
        snap = np.bincount(ids.reshape(-1), minlength=len(A))
        copied = 0
        for y in range(0, L, 2):
            for x in range(0, L, 2):
                k = (y >> 1) * (L // 2) + (x >> 1)
                word = _u(orc, k >> 2, 0, 1, 0, 5)[k & 3]
                dy, dx = MOORE[word & 7]
                s, t = ids[y, x], ids[(y + dy) % L, (x + dx) % L]
                if s == t:
                    continue
                # energy change of this single copy (snapshot areas)
                dH = 0.0
                for my, mx in MOORE:
                    m = ids[(y + my) % L, (x + mx) % L]
                    dH += J[ctype[t], ctype[m]] * (t != m) - J[ctype[s], ctype[m]] * (s != m)
                if t != 0:
                    dH += 2 * (snap[t] - A[t]) + 1
                if s != 0:
                    dH += -2 * (snap[s] - A[s]) + 1
                later_pass_changed = False  # colour-0 sites are not touched again
                took = out[y, x] == t and not later_pass_changed
                if want_all:
                    # the remaining passes never rewrite colour-0 sites
                    assert out[y, x] == t
                else:
                    assert took == (dH <= 0)
                copied += took
        assert copied > 0


@pytest.mark.slow
def test_cell_sorting_trend(orc):
    """Differential adhesion (Results, cellular Potts; J_am = J_bm = 16 >
    J_ab = 11 > J_aa = 2): the light (a) cells cluster, so the a-medium
    and a-b boundaries shrink while a-a contacts grow over the run."""
    ids, ctype, A, J, prm = synth.cpm_sorting(n_rep=1, L=96, n_cells=36, side=10, slot=14,
                                              offset=4, seed=11)
    A = np.where(np.arange(len(A)) == 0, 0, 100).astype(np.int32)
    ids0 = ids[0]

    def boundary(z):
        st = orc.cpm_stats(z, J, ctype, A, 1.0)
        # pair index for (a, b) with a <= b among 3 types: a*3 - a(a-1)/2 + (b-a)
        return {"mm": st[0], "ma": st[1], "mb": st[2], "aa": st[3], "ab": st[4], "bb": st[5]}

    b0 = boundary(ids0)
    out, _, _ = orc.cpm_run(ids0, J, ctype, A, 1.0, 10.0, 4, 0, 0, 400)
    b1 = boundary(out)
    assert b1["aa"] > b0["aa"]
    assert b1["ma"] < b0["ma"]
    assert math.isfinite(float(b1["ab"]))


# ------------------------------------------- statistics against a recount
def _pair_slots(n_types):
    """Unordered type pairs (a <= b) in the order a = 0, 1, ...; b = a ...:
    the position of a pair in this list is its statistics slot."""
    return [(a, b) for a in range(n_types) for b in range(a, n_types)]


def _recount_boundary(ids, ctype, n_types):
    """Results, Fig. 6 boundary lengths: every von Neumann bond (right and
    down neighbour on the torus, so each bond once) whose two ids differ,
    tallied by the unordered pair of the two cells' types."""
    slots = {p: i for i, p in enumerate(_pair_slots(n_types))}
    out = np.zeros(10, np.int64)
    Ly, Lx = ids.shape
    for y in range(Ly):
        for x in range(Lx):
            for ny, nx in ((y, (x + 1) % Lx), ((y + 1) % Ly, x)):
                a, b = int(ids[y, x]), int(ids[ny, nx])
                if a == b:
                    continue
                ta, tb = sorted((int(ctype[a]), int(ctype[b])))
                out[slots[(ta, tb)]] += 1
    return out


@pytest.mark.parametrize("n_types,shape,seed", [(2, (6, 8), 21), (3, (12, 10), 22),
                                                 (4, (8, 16), 23), (4, (12, 18), 24)])
def test_boundary_counts_equal_a_recount(orc, n_types, shape, seed):
    """The ten boundary slots of the CPM statistics equal a plain recount of
    von Neumann bonds between different ids by unordered type pair, for both
    neighbourhood ranges (the boundary measure does not depend on the range
    of the adhesion energy)."""
    rng = np.random.default_rng(seed)
    n_cells = 9
    ids = rng.integers(0, n_cells + 1, size=shape).astype(np.int32)
    # clusters as well as noise: copy a shifted block so that equal-id bonds occur
    ids[: shape[0] // 2, : shape[1] // 2] = ids[0, 0]
    ctype = np.concatenate([[0], rng.integers(1, n_types, size=n_cells)]).astype(np.int8)
    if n_types > 2:
        ctype[1:n_types] = np.arange(1, n_types)  # every type present
    A = np.concatenate([[0], rng.integers(3, 12, size=n_cells)]).astype(np.int32)
    J = rng.integers(0, 9, size=(n_types, n_types)).astype(np.float32)
    J = np.triu(J) + np.triu(J, 1).T
    want = _recount_boundary(ids, ctype, n_types)
    assert want.sum() > 0
    for nrange in (1, 2):
        if nrange == 2 and (shape[0] % 6 or shape[1] % 6):
            continue
        st = orc.cpm_stats(ids, J, ctype, A, 1.0, nrange=nrange)
        assert np.array_equal(st[:10].astype(np.int64), want), (nrange, st[:10], want)


def test_boundary_slot_of_each_type_pair(orc):
    """The bonds of an interface between two cells of given types land in
    the slot of that unordered pair and nowhere else (both orders of the two
    types, the medium included)."""
    n_types = 4
    J = np.zeros((4, 4), np.float32)
    slots = _pair_slots(n_types)
    for ta in range(n_types):
        for tb in range(n_types):
            # a 2 x 4 torus, left half one id, right half another: two vertical
            # interfaces crossed by two rows each, 4 bonds.  A type-0 side is
            # the medium (id 0); the other sides are cells 1 and 2.
            left = 0 if ta == 0 else 1
            right = 0 if (tb == 0 and ta != 0) else 2
            ids = np.array([[left, left, right, right]] * 2, np.int32)
            ctype = np.array([0, ta, tb], np.int8)
            A = np.array([0, 4, 4], np.int32)
            st = orc.cpm_stats(ids, J, ctype, A, 0.0)
            want = np.zeros(10, np.int64)
            want[slots.index(tuple(sorted((ta, tb))))] = 4
            assert np.array_equal(st[:10].astype(np.int64), want), (ta, tb, st[:10])


@pytest.mark.parametrize("J,lam", [
    (np.array([[0, 16, 16], [16, 2, 11], [16, 11, 16]], np.float32), 1.0),
    (np.array([[0, 3.5, 4.5], [3.5, 1.5, 2.0], [4.5, 2.0, 0.5]], np.float32), 0.5),
    (np.array([[0, 1.25, 2.0, 0.75], [1.25, 0.5, 1.0, 3.0], [2.0, 1.0, 0.25, 1.5],
               [0.75, 3.0, 1.5, 2.0]], np.float32), 1.5),
])
def test_range1_energy_statistic_matches_bruteforce(orc, J, lam):
    """Eq. (3) with the Moore neighbourhood: the fixed-point energy statistic
    H S equals the brute-force energy (adhesion over unordered Moore pairs of
    different ids plus the area term over cells) times the scale S."""
    from test_oracle_onestep import cpm_energy
    rng = np.random.default_rng(31)
    S = orc.cpm_scale(J, lam)
    n_types = J.shape[0]
    for shape in ((4, 6), (8, 8), (10, 14)):
        n_cells = 7
        ids = rng.integers(0, n_cells + 1, size=shape).astype(np.int32)
        ctype = np.concatenate([[0], rng.integers(1, n_types, size=n_cells)]).astype(np.int8)
        A = np.concatenate([[0], rng.integers(2, 20, size=n_cells)]).astype(np.int32)
        area = np.bincount(ids.reshape(-1), minlength=n_cells + 1)
        st = orc.cpm_stats(ids, J, ctype, A, lam)
        H = (int(st[11]) << 32) | (int(st[10]) & 0xFFFFFFFF)
        if H >= 1 << 63:
            H -= 1 << 64
        want = cpm_energy(ids, J, ctype, A, lam, area) * S
        assert H == round(want), (shape, H, want)
