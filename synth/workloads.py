"""Workload manifests (parameter draws and initial states), seeded.

Each manifest mirrors a workload shape of the paper's experiments: square
periodic lattices, batches of replicas over temperatures (Methods, batched
tensors), Potts lattices with several q, and a cell-sorting CPM setup
(Results, cellular Potts).  Everything is synthetic; nothing here computes an
energy, an acceptance or an observable.
"""
import numpy as np

__all__ = [
    "single_ising", "batched_ising_potts", "differentiation", "cpm_sorting", "cpm_paper_aggregate",
    "surrogate_points", "random_ising", "random_potts", "ISING", "POTTS", "CPM",
]

ISING, POTTS, CPM = 0, 1, 2


def single_ising():
    """One 32x32 periodic Ising lattice, J=1, h=0, beta=0.44, 1000 sweeps,
    Philox initial state (seed 1, replica 0), statistics every sweep."""
    return dict(model=ISING, Lx=32, Ly=32, Jx=1.0, Jy=1.0, h=0.0, beta=0.44, rid=0, seed=1,
                n_sweeps=1000, record_every=1)


def batched_ising_potts(n_ising=1024, n_potts=512, ising_L=256, seed=1002,
                        potts_L=(64, 128, 256, 512, 1024), potts_q=(3, 4, 6, 8)):
    """Batched Ising + q-Potts: ``n_ising`` Ising replicas of ising_L^2 with
    beta on a 64-point grid over [0.30, 0.60] (n_ising/64 replicas each), then
    ``n_potts`` Potts lattices with L and q drawn uniformly from the given
    sets and beta ~ U[0.9, 1.1] * ln(1 + sqrt q).  Returns a list of replica
    dicts; replica ids are 0..R-1 in order.  Chain seed 2."""
    rng = np.random.default_rng(seed)
    reps = []
    grid = np.linspace(0.30, 0.60, 64)
    per = max(1, n_ising // 64)
    for r in range(n_ising):
        reps.append(dict(model=ISING, Lx=ising_L, Ly=ising_L, q=2, Jx=1.0, Jy=1.0, h=0.0,
                         beta=float(grid[min(r // per, 63)]), rid=r))
    Ls = rng.choice(np.array(potts_L), size=n_potts)
    qs = rng.choice(np.array(potts_q), size=n_potts)
    fac = rng.uniform(0.9, 1.1, size=n_potts)
    for i in range(n_potts):
        q = int(qs[i])
        reps.append(dict(model=POTTS, Lx=int(Ls[i]), Ly=int(Ls[i]), q=q, Jx=1.0, Jy=1.0, h=0.0,
                         beta=float(fac[i] * np.log1p(np.sqrt(q))), rid=n_ising + i))
    return reps


def differentiation(n=256, L=128, seed=1003):
    """256 replicas of 128x128 Ising with per-replica FP32 couplings
    J ~ U(0.3, 0.6) and fields h ~ U(-0.05, 0.05), beta = 1, chain seed 3."""
    rng = np.random.default_rng(seed)
    J = rng.uniform(0.3, 0.6, size=n).astype(np.float32)
    h = rng.uniform(-0.05, 0.05, size=n).astype(np.float32)
    return [dict(model=ISING, Lx=L, Ly=L, q=2, Jx=float(J[i]), Jy=float(J[i]), h=float(h[i]),
                 beta=1.0, rid=i) for i in range(n)]


def cpm_sorting(n_rep=8, L=512, n_cells=1000, side=14, seed=1004, slot=14, offset=4):
    """Cell-sorting CPM setup: ``n_cells`` square side x side cells placed on
    a grid of slots (pitch ``slot``, first slot at ``offset``), slots picked
    by a seeded permutation; types 1 and 2 assigned 50/50 by a seeded
    permutation; medium is id 0 / type 0.  Adhesion (types medium, a, b):
    J_mm=0, J_aa=2, J_bb=16, J_ab=11, J_am=J_bm=16; target area 200,
    lambda=1, T=10.  Returns (ids[n_rep, L, L] int32, cell_type, target_area,
    J[3,3], params)."""
    rng = np.random.default_rng(seed)
    n_slots_1d = (L - offset) // slot
    n_slots = n_slots_1d * n_slots_1d
    if n_cells > n_slots:
        raise ValueError("not enough slots for the cells")
    ids = np.zeros((n_rep, L, L), np.int32)
    for r in range(n_rep):
        pick = rng.permutation(n_slots)[:n_cells]
        for c, sidx in enumerate(pick):
            sy, sx = divmod(int(sidx), n_slots_1d)
            y0, x0 = offset + sy * slot, offset + sx * slot
            ids[r, y0:y0 + side, x0:x0 + side] = c + 1
    cell_type = np.zeros(n_cells + 1, np.int8)
    perm = rng.permutation(n_cells)
    cell_type[1 + perm[: n_cells // 2]] = 1
    cell_type[1 + perm[n_cells // 2:]] = 2
    target_area = np.full(n_cells + 1, 200, np.int32)
    target_area[0] = 0
    J = np.array([[0, 16, 16], [16, 2, 11], [16, 11, 16]], np.float32)
    params = dict(lambda_area=1.0, temperature=10.0, seed=4, n_mcs=2000)
    return ids, cell_type, target_area, J, params


def cpm_paper_aggregate(n_rep=16, L=64, side=5, grid=6, seed=1006):
    """The paper's own CPM setting (Results, Table 2): an aggregate of
    grid x grid square cells of side x side sites (36 cells of area 25)
    touching each other, centred in an L x L medium; types light (1) and dark
    (2) half and half by a seeded permutation per replica; target area 25,
    lambda 1, k_B T = 8, adhesion (medium, light, dark) J_mm = 0,
    J_ml = J_md = 16, J_ll = 2, J_dd = 14, J_ld = 11.  Returns (ids[n_rep, L,
    L] int32, cell_type[n_rep][n + 1] int8, target_area, J[3, 3], params)."""
    rng = np.random.default_rng(seed)
    n_cells = grid * grid
    y0 = (L - grid * side) // 2
    ids = np.zeros((n_rep, L, L), np.int32)
    types = []
    for r in range(n_rep):
        for c in range(n_cells):
            gy, gx = divmod(c, grid)
            ids[r, y0 + gy * side:y0 + (gy + 1) * side, y0 + gx * side:y0 + (gx + 1) * side] = c + 1
        ct = np.zeros(n_cells + 1, np.int8)
        perm = rng.permutation(n_cells)
        ct[1 + perm[: n_cells // 2]] = 1
        ct[1 + perm[n_cells // 2:]] = 2
        types.append(ct)
    target_area = np.full(n_cells + 1, side * side, np.int32)
    target_area[0] = 0
    J = np.array([[0, 16, 16], [16, 2, 11], [16, 11, 14]], np.float32)
    params = dict(lambda_area=1.0, temperature=8.0, seed=6)
    return ids, types, target_area, J, params


def surrogate_points(n=100_000, seed=1005):
    """(beta, Jx, Jy, h) uniform on [0.3,0.6] x [0.5,1.5]^2 x [-0.1,0.1]."""
    rng = np.random.default_rng(seed)
    beta = rng.uniform(0.3, 0.6, n)
    Jx = rng.uniform(0.5, 1.5, n)
    Jy = rng.uniform(0.5, 1.5, n)
    h = rng.uniform(-0.1, 0.1, n)
    return np.stack([beta, Jx, Jy, h], axis=1).astype(np.float32)


def random_ising(Ly, Lx, rng):
    """iid +/-1 int8 lattice from a numpy generator."""
    return (2 * rng.integers(0, 2, size=(Ly, Lx)) - 1).astype(np.int8)


def random_potts(Ly, Lx, q, rng):
    return rng.integers(0, q, size=(Ly, Lx)).astype(np.uint8)
