"""Surrogate over Cellular Potts adhesion parameters: the 4-128-128-3 network
of the Ising surrogate, trained on the library's own CPM runs of the paper's
cell-sorting setting (Results, Table 2), steering an inverse problem with
Monte Carlo as arbiter and fallback.

* inputs: (J_light_dark, J_dark_dark, J_cell_medium, k_BT) on a box around
  Table 2 (J_medium_medium = 0 and J_light_light = 2 fixed; every value on a
  1/8 grid, so the fixed-point energies stay exact);
* outputs: the mean von Neumann boundary lengths light-medium, dark-medium
  and light-dark after a fixed number of Monte Carlo steps from the paper's
  aggregate (36 cells of area 25 in 64 x 64, half light, half dark);
* inverse problem: the J_light_dark that gives a target light-dark boundary
  with the other parameters at Table 2 -- the surrogate proposes, one Monte
  Carlo evaluation verifies, Monte Carlo secant steps continue if needed;
  the Monte-Carlo-only solver runs the secant steps from the start.

Every Monte Carlo step and every network pass runs in the library's kernels.
"""
import time

import numpy as np
import torch

import synth

from .sampler import Sampler
from .surrogate import SurrogateMLP

# (J_light_dark, J_dark_dark, J_cell_medium, k_BT)
BOX_LO = np.array([4.0, 2.0, 8.0, 4.0])
BOX_HI = np.array([16.0, 16.0, 20.0, 12.0])
TABLE2 = np.array([11.0, 14.0, 16.0, 8.0])
J_LL = 2.0


def snap(x):
    """Round to the 1/8 grid (exact in the CPM fixed-point scale S = 8)."""
    return np.round(np.asarray(x, np.float64) * 8.0) / 8.0


def adhesion(p):
    jld, jdd, jcm, _ = (float(v) for v in p)
    return np.array([[0.0, jcm, jcm], [jcm, J_LL, jld], [jcm, jld, jdd]], np.float32)


def cpm_boundaries(points, n_rep=4, mcs=500, seed=6, rid0=0, chunk=4096, L=64):
    """Mean boundary lengths (light-medium, dark-medium, light-dark) after
    `mcs` Monte Carlo steps for every parameter point (rows of `points`,
    snapped to the 1/8 grid), each over n_rep replicas of the paper's
    aggregate; replica j of every point uses the j-th aggregate (common
    cell-type draws).  Returns float64 [n, 3] and the per-point standard
    errors [n, 3]."""
    pts = snap(np.atleast_2d(points))
    ids, types, A, _, prm = synth.cpm_paper_aggregate(n_rep=n_rep, L=L)
    out = np.zeros((len(pts), 3))
    se = np.zeros((len(pts), 3))
    per = max(1, chunk // n_rep)
    for c0 in range(0, len(pts), per):
        blk = pts[c0:c0 + per]
        reps = []
        for i, p in enumerate(blk):
            J = adhesion(p)
            for j in range(n_rep):
                reps.append(dict(model=2, Lx=L, Ly=L, q=len(types[j]) - 1,
                                 rid=rid0 + (c0 + i) * n_rep + j, adhesion=J, cell_type=types[j],
                                 target_area=A, lambda_area=prm["lambda_area"],
                                 temperature=float(p[3])))
        smp = Sampler(reps, seed, init=False)
        for r in range(len(reps)):
            smp.set_state(r, ids[r % n_rep])
        smp.sweep(mcs)
        st, _ = smp.measure()
        smp.close()
        b = st[:, [1, 2, 4]].double().cpu().numpy().reshape(len(blk), n_rep, 3)
        out[c0:c0 + len(blk)] = b.mean(axis=1)
        if n_rep > 1:
            se[c0:c0 + len(blk)] = b.std(axis=1, ddof=1) / np.sqrt(n_rep)
    return out, se


def training_points(n, seed=1007):
    """Uniform points of the box, snapped to the 1/8 grid."""
    rng = np.random.default_rng(seed)
    return snap(BOX_LO + rng.random((n, 4)) * (BOX_HI - BOX_LO))


def make_net(seed=0):
    net = SurrogateMLP(seed)
    net.x_lo = torch.tensor(BOX_LO, dtype=torch.float32, device=net.dev)
    net.x_hi = torch.tensor(BOX_HI, dtype=torch.float32, device=net.dev)
    return net


def _mc_b4(jld, n_rep, mcs, seed, rid0):
    p = TABLE2.copy()
    p[0] = jld
    b, se = cpm_boundaries(p[None], n_rep=n_rep, mcs=mcs, seed=seed, rid0=rid0)
    return float(b[0, 2]), float(se[0, 2])


def _secant(target, x0, f0, x1, f1, evaluate, tol, max_iter, lo=4.0, hi=16.0):
    """Secant steps on J_light_dark (clipped to the box, snapped to the 1/8
    grid) until |f - target| <= tol * target; returns (x, f, evaluations)."""
    n = 0
    while abs(f1 - target) > tol * target and n < max_iter:
        if f1 == f0:
            x2 = x1 + (0.5 if f1 > target else -0.5)
        else:
            x2 = x1 - (f1 - target) * (x1 - x0) / (f1 - f0)
        x2 = float(snap(min(max(x2, lo), hi)))
        if x2 == x1:
            x2 = float(snap(min(max(x1 + (0.125 if f1 > target else -0.125), lo), hi)))
        x0, f0 = x1, f1
        x1, f1 = x2, evaluate(x2)
        n += 1
    return x1, f1, n


def mc_only_solve(target, tol=0.03, n_rep=16, mcs=500, seed=8, max_iter=20):
    """Monte Carlo secant steps on J_light_dark from 11 and 12."""
    k = [0]

    def ev(x):
        k[0] += 1
        return _mc_b4(x, n_rep, mcs, seed, 10_000_000 + 1000 * k[0])[0]
    t0 = time.perf_counter()
    x0, x1 = 11.0, 12.0
    f0, f1 = ev(x0), ev(x1)
    x, f, n = _secant(target, x0, f0, x1, f1, ev, tol, max_iter)
    torch.cuda.synchronize()
    return dict(J_light_dark=x, b4=f, evaluations=k[0], seconds=time.perf_counter() - t0,
                converged=abs(f - target) <= tol * target)


def surrogate_solve(net, target, tol=0.03, n_rep=16, mcs=500, seed=8, max_iter=20):
    """The surrogate's J_light_dark (the 1/8 grid point of the box whose
    predicted light-dark boundary is closest to the target, other
    parameters at Table 2), one Monte Carlo verification, then Monte Carlo
    secant steps if the verified error exceeds the tolerance."""
    k = [0]

    def ev(x):
        k[0] += 1
        return _mc_b4(x, n_rep, mcs, seed, 20_000_000 + 1000 * k[0])[0]
    t0 = time.perf_counter()
    grid = np.arange(BOX_LO[0], BOX_HI[0] + 1e-9, 0.125)
    X = np.tile(TABLE2, (len(grid), 1))
    X[:, 0] = grid
    with torch.no_grad():
        pred = net.predict(torch.tensor(X, dtype=torch.float32, device=net.dev))[:, 2]
    pred = pred.cpu().numpy()
    i = int(np.argmin(np.abs(pred - target)))
    x1 = float(grid[i])
    f1 = ev(x1)
    if abs(f1 - target) > tol * target:
        # second point for the secant: the surrogate's local slope
        j = min(i + 1, len(grid) - 1) if i + 1 < len(grid) else i - 1
        x0 = float(grid[j])
        f0 = f1 + float(pred[j] - pred[i])
        x1, f1, _ = _secant(target, x0, f0, x1, f1, ev, tol, max_iter)
    torch.cuda.synchronize()
    return dict(J_light_dark=x1, b4=f1, evaluations=k[0], seconds=time.perf_counter() - t0,
                converged=abs(f1 - target) <= tol * target, surrogate_guess=float(grid[i]))


def experiment(n_points=2048, n_rep=4, mcs=500, epochs=300, targets=(80.0, 95.0, 110.0),
               log=print):
    """Labels, training and the inverse problem for a few targets of the
    light-dark boundary; returns a dict of timings and results."""
    t0 = time.perf_counter()
    X = training_points(n_points)
    Y, _ = cpm_boundaries(X, n_rep=n_rep, mcs=mcs)
    t_lab = time.perf_counter() - t0
    Xv = training_points(256, seed=1008)
    Yv, _ = cpm_boundaries(Xv, n_rep=n_rep, mcs=mcs, rid0=50_000_000)
    t1 = time.perf_counter()
    net = make_net().fit(X, Y, epochs=epochs, batch=256, lr=2e-3, lr_min=1e-4)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t1
    with torch.no_grad():
        pv = net.predict(torch.tensor(Xv, dtype=torch.float32, device=net.dev)).cpu().numpy()
    mae = np.abs(pv - Yv).mean(axis=0)
    log(f"labels {t_lab:.2f} s, training {t_fit:.2f} s, validation MAE {mae.round(2)} "
        f"(label sd {Yv.std(axis=0).round(1)})")
    rows = []
    for tg in targets:
        a = mc_only_solve(tg)
        b = surrogate_solve(net, tg)
        log(f"target {tg}: MC only {a}; surrogate {b}")
        rows.append(dict(target=tg, mc_only=a, surrogate=b))
    return dict(labels_s=t_lab, training_s=t_fit, validation_mae=mae.tolist(),
                label_sd=Yv.std(axis=0).tolist(), inverse=rows)


if __name__ == "__main__":
    experiment()
