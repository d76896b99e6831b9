"""Learned surrogate of equilibrium Ising observables, trained on the
sampler's own data, steering an inverse problem with Monte Carlo as arbiter
and fallback.

Pipeline (all device work in libspinmc kernels; this module marshals):
  1. labels: batched Monte Carlo on LxL Ising replicas at parameter points
     (beta, Jx, Jy, h); <e>, <|m|> and chi from the covariance kernel's exact
     integer moments (spinmc_grad means);
  2. training: 4-128-128-3 MLP (spinmc_mlp_forward / backward / adam, BF16
     matrix cores, FP32 master weights, Adam with the paper's settings);
  3. inverse problem: find (Jx, Jy) with <|m|>(beta, Jx, Jy, h) = target.
     Surrogate-steered: gradient descent on the network's inputs
     (input gradients from spinmc_mlp_backward), then one Monte Carlo
     verification; if the verified error exceeds the tolerance, Monte Carlo
     bracketed Newton steps on the couplings (slopes from the covariance
     estimator) continue from the surrogate's answer.  Monte-Carlo-only: the
     same bracketed Newton iteration from the start.
"""
import ctypes as C
import time

import numpy as np
import torch

from ._lib import check, lib
from .sampler import Sampler

# parameter box of the training points (beta, Jx, Jy, h)
BOX_LO = np.array([0.3, 0.5, 0.5, -0.1])
BOX_HI = np.array([0.6, 1.5, 1.5, 0.1])


def _p(t):
    return C.c_void_p(t.data_ptr())


class SurrogateMLP:
    """The 4-128-128-3 network on the library's MLP kernels."""

    def __init__(self, seed=0, device="cuda"):
        self.dev = torch.device(device)
        L = lib()
        self.np = L.spinmc_mlp_num_params()
        g = np.random.default_rng(seed)
        parts = []
        for shp in ((128, 4), (128,), (128, 128), (128,), (3, 128), (3,)):
            if len(shp) == 2:
                b = np.sqrt(6.0 / shp[1])
                parts.append(g.uniform(-b, b, size=shp).reshape(-1))
            else:
                parts.append(np.zeros(shp))
        self.params = torch.tensor(np.concatenate(parts), dtype=torch.float32, device=self.dev)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step_no = 0
        self.x_lo = torch.tensor(BOX_LO, dtype=torch.float32, device=self.dev)
        self.x_hi = torch.tensor(BOX_HI, dtype=torch.float32, device=self.dev)
        self.y_mu = torch.zeros(3, dtype=torch.float32, device=self.dev)
        self.y_sd = torch.ones(3, dtype=torch.float32, device=self.dev)
        self._ws = {}

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def normalise_x(self, x):
        return (2.0 * (x - self.x_lo) / (self.x_hi - self.x_lo) - 1.0).contiguous()

    def _buffers(self, B):
        if B not in self._ws:
            L = lib()
            self._ws[B] = dict(
                act=torch.empty(L.spinmc_mlp_act_floats(B), dtype=torch.float32, device=self.dev),
                ws=torch.empty(L.spinmc_mlp_workspace_floats(B), dtype=torch.float32,
                               device=self.dev),
                y=torch.empty((B, 3), dtype=torch.float32, device=self.dev),
                dx=torch.empty((B, 4), dtype=torch.float32, device=self.dev),
                loss=torch.empty(1, dtype=torch.float32, device=self.dev))
        return self._ws[B]

    def forward_normalised(self, xn, act=None):
        B = xn.shape[0]
        b = self._buffers(B)
        check(lib().spinmc_mlp_forward(_p(self.params), _p(xn), B, _p(b["y"]),
                                       _p(act) if act is not None else None, self._stream()))
        return b["y"]

    def predict(self, x):
        """Physical outputs (<e>, <|m|>, chi) for physical inputs x [B, 4]."""
        y = self.forward_normalised(self.normalise_x(x))
        return y * self.y_sd + self.y_mu

    def train_step(self, xn, tn, w, lr=1e-3):
        """Forward, backward and Adam in one library call (three launches)."""
        B = xn.shape[0]
        b = self._buffers(B)
        self.step_no += 1
        check(lib().spinmc_mlp_train_step(_p(self.params), _p(xn), _p(tn), _p(w), B,
                                          _p(self.grad), _p(self.m), _p(self.v), self.step_no, lr,
                                          0.9, 0.999, 1e-8, _p(b["loss"]), _p(b["act"]),
                                          _p(b["ws"]), self._stream()))
        return b["loss"]

    def input_grad(self, xn, tn, w):
        """d/dx of sum_j w_j (y_j - t_j)^2 / B at normalised inputs xn."""
        B = xn.shape[0]
        b = self._buffers(B)
        L = lib()
        s = self._stream()
        check(L.spinmc_mlp_forward(_p(self.params), _p(xn), B, _p(b["y"]), _p(b["act"]), s))
        check(L.spinmc_mlp_backward(_p(self.params), _p(xn), _p(b["act"]), _p(tn), _p(w), B,
                                    _p(self.grad), _p(b["dx"]), _p(b["loss"]), _p(b["ws"]), s))
        return b["dx"], b["y"]

    def fit(self, x, y, epochs=60, batch=1024, lr=1e-3, lr_min=None, seed=0, log=None):
        """Train on physical (x, y); labels are standardised per output.  With
        lr_min the learning rate follows a cosine from lr to lr_min over the
        epochs."""
        x = torch.as_tensor(x, dtype=torch.float32, device=self.dev)
        y = torch.as_tensor(y, dtype=torch.float32, device=self.dev)
        self.y_mu = y.mean(dim=0)
        self.y_sd = y.std(dim=0).clamp_min(1e-6)
        xn = self.normalise_x(x)
        yn = ((y - self.y_mu) / self.y_sd).contiguous()
        w = torch.ones(3, dtype=torch.float32, device=self.dev)
        g = torch.Generator(device="cpu").manual_seed(seed)
        n = x.shape[0]
        for ep in range(epochs):
            lr_ep = lr
            if lr_min is not None and epochs > 1:
                lr_ep = lr_min + 0.5 * (lr - lr_min) * (1.0 + np.cos(np.pi * ep / (epochs - 1)))
            perm = torch.randperm(n, generator=g).to(self.dev)
            last = None
            for k in range(0, n - batch + 1, batch):
                idx = perm[k:k + batch]
                last = self.train_step(xn[idx].contiguous(), yn[idx].contiguous(), w, lr_ep)
            if log and (ep % 10 == 9 or ep == epochs - 1):
                log(f"epoch {ep + 1}: batch loss {float(last.item()):.4g}")
        return self


# ----------------------------------------------------------------- labels
def mc_observables(points, L=64, burn=300, measure=700, every=1, seed=5, rid0=0, chunk=16384,
                   log=None):
    """Monte Carlo labels (<e>, <|m|>, chi) for points [N, 4] = (beta, Jx,
    Jy, h), one LxL replica per point, plus the standard error of <|m|> from
    batch means.  Returns (labels [N, 3], se_absm [N]) as numpy arrays."""
    pts = np.asarray(points, np.float64)
    out = np.zeros((len(pts), 3))
    se = np.zeros(len(pts))
    for c0 in range(0, len(pts), chunk):
        part = pts[c0:c0 + chunk]
        reps = [dict(model=0, Lx=L, Ly=L, beta=float(b), Jx=float(jx), Jy=float(jy), h=float(h),
                     rid=rid0 + c0 + i) for i, (b, jx, jy, h) in enumerate(part)]
        smp = Sampler(reps, seed, init=True)
        smp.sweep(burn)
        st = smp.sweep(measure, every)
        means, _, _ = smp.grad(st, 0)
        m = means.cpu().numpy()
        out[c0:c0 + len(part)] = m[:, [0, 1, 3]]
        # standard error of <|m|> from 10 batch means of the recorded |M|/N
        am = st[:, :, 0].abs().double().cpu().numpy() / (L * L)
        nb = 10
        bm = am[: (am.shape[0] // nb) * nb].reshape(nb, -1, am.shape[1]).mean(axis=1)
        se[c0:c0 + len(part)] = bm.std(axis=0, ddof=1) / np.sqrt(nb)
        smp.close()
        if log:
            log(f"labels: {c0 + len(part)} / {len(pts)} points")
    return out, se


def mc_absm_and_grad(beta, Jx, Jy, h, L=64, n_rep=16, burn=300, measure=700, seed=7, rid0=0,
                     se_abs=None, n_max=None):
    """<|m|> over replicas and its gradient wrt (Jx, Jy) by the covariance
    estimator; returns (absm, se, dJx, dJy, replicas used).  Replicas run in
    batches of n_rep; with se_abs, batches are added (up to n_max replicas)
    until the standard error of <|m|> is at most se_abs."""
    n_max = n_max or n_rep
    am, gx, gy = [], [], []
    while True:
        k = len(am)
        reps = [dict(model=0, Lx=L, Ly=L, beta=float(beta), Jx=float(Jx), Jy=float(Jy),
                     h=float(h), rid=rid0 + k + i) for i in range(n_rep)]
        smp = Sampler(reps, seed, init=True)
        smp.sweep(burn)
        st = smp.sweep(measure, 1)
        means, grads, _ = smp.grad(st, 0)
        am += means[:, 1].cpu().tolist()
        g = grads[:, 1, :2].cpu().numpy()
        gx += g[:, 0].tolist()
        gy += g[:, 1].tolist()
        smp.close()
        se = float(np.std(am, ddof=1) / np.sqrt(len(am)))
        if se_abs is None or se <= se_abs or len(am) + n_rep > n_max:
            break
    return float(np.mean(am)), se, float(np.mean(gx)), float(np.mean(gy)), len(am)


# --------------------------------------------------------- inverse problem
def mc_only_solve(target, beta=0.4, h=0.0, start=(1.0, 1.0), tol=0.01, max_iter=40, se_rel=None,
                  n_max=None, j_lo=0.05, j_hi=3.0, max_step=0.5, **mc):
    """Monte Carlo root finding of <|m|>(Jx, Jy) = target along the
    coupling diagonal through the start, J(s) = start + s (1, 1): a
    bracketed, damped Newton iteration on s whose slope is the covariance
    estimator's d<|m|>/dJx + d<|m|>/dJy.  <|m|> rises with both couplings,
    so every evaluation below the target raises the bracket's lower end and
    every one above lowers its upper end (initially the couplings' range
    [j_lo, j_hi]).  A Newton step is capped at max_step and, if it leaves the
    bracket or the slope is not positive, replaced by the secant through the
    bracket's measured ends (or its midpoint while an end is unmeasured).
    Stops when the Monte Carlo <|m|> is within tol (relative) of the target.
    With se_rel every evaluation adds replicas until its standard error is at
    most se_rel * target (at most n_max replicas), so the tolerance is
    resolved."""
    x0, y0 = float(start[0]), float(start[1])
    lo, hi = j_lo - min(x0, y0), j_hi - max(x0, y0)  # bracket on s
    m_lo = m_hi = None
    s_cur = 0.0
    t0 = time.perf_counter()
    hist = []
    se_abs = se_rel * target if se_rel else None
    n_used = 0
    for it in range(max_iter):
        Jx, Jy = x0 + s_cur, y0 + s_cur
        m, se, gx, gy, n = mc_absm_and_grad(beta, Jx, Jy, h, rid0=100_000 * it, se_abs=se_abs,
                                            n_max=n_max, **mc)
        n_used += n
        hist.append((Jx, Jy, m, se, n))
        if abs(m - target) <= tol * target:
            return dict(Jx=Jx, Jy=Jy, absm=m, se=se, iters=it + 1, mc_calls=it + 1,
                        replicas=n_used, seconds=time.perf_counter() - t0, converged=True,
                        history=hist)
        if m < target:
            lo, m_lo = s_cur, m
        else:
            hi, m_hi = s_cur, m
        slope = gx + gy
        s_new = None
        if slope > 0:
            s_new = s_cur + float(np.clip((target - m) / slope, -max_step, max_step))
            if not lo < s_new < hi:
                s_new = None
        if s_new is None:
            if m_lo is not None and m_hi is not None and m_hi > m_lo:
                s_new = lo + (target - m_lo) * (hi - lo) / (m_hi - m_lo)
            else:
                s_new = 0.5 * (lo + hi)
        s_cur = s_new
    return dict(Jx=hist[-1][0], Jy=hist[-1][1], absm=hist[-1][2], se=hist[-1][3], iters=max_iter,
                mc_calls=max_iter, replicas=n_used, seconds=time.perf_counter() - t0,
                converged=False, history=hist)


def surrogate_solve(net, target, beta=0.4, h=0.0, start=(1.0, 1.0), tol=0.01, steps=100, lr=0.01,
                    grid=64, max_iter=40, se_rel=None, n_max=None, **mc):
    """The surrogate's answer, one Monte Carlo check, and the Monte Carlo
    root finding of mc_only_solve from that answer if the check fails.  The answer: the network
    over a grid x grid set of couplings (one forward call) gives the points
    of the target level set, the one nearest to the start is refined by
    gradient descent on the network's inputs (input gradients from the
    backward kernel)."""
    dev = net.dev
    t0 = time.perf_counter()
    g = torch.linspace(-1.0, 1.0, grid, device=dev)
    gx, gy = torch.meshgrid(g, g, indexing="ij")
    x0 = net.normalise_x(torch.tensor([[beta, start[0], start[1], h]], dtype=torch.float32,
                                      device=dev))
    xg = x0.repeat(grid * grid, 1)
    xg[:, 1] = gx.reshape(-1)
    xg[:, 2] = gy.reshape(-1)
    xg = xg.contiguous()
    pred = (net.forward_normalised(xg) * net.y_sd + net.y_mu)[:, 1]
    err = (pred - target).abs()
    ok = err <= torch.clamp(err.min() * 1.5, min=0.002 * target)
    dist = (xg[:, 1] - x0[0, 1]) ** 2 + (xg[:, 2] - x0[0, 2]) ** 2
    dist = torch.where(ok, dist, torch.full_like(dist, float("inf")))
    xn = xg[int(torch.argmin(dist))].reshape(1, 4).contiguous()
    tn = ((torch.tensor([[0.0, target, 0.0]], device=dev) - net.y_mu) / net.y_sd).to(
        torch.float32).contiguous()
    w = torch.tensor([0.0, 1.0, 0.0], dtype=torch.float32, device=dev)
    for _ in range(steps):
        dx, _ = net.input_grad(xn, tn, w)
        step = torch.zeros_like(xn)  # move only the couplings (inputs 1, 2)
        step[:, 1:3] = dx[:, 1:3]
        xn = (xn - lr * step).clamp(-1.0, 1.0).contiguous()
    xp = (xn + 1.0) / 2.0 * (net.x_hi - net.x_lo) + net.x_lo
    Jx, Jy = float(xp[0, 1]), float(xp[0, 2])
    t_sur = time.perf_counter() - t0
    res = mc_only_solve(target, beta, h, start=(Jx, Jy), tol=tol, max_iter=max_iter, se_rel=se_rel,
                        n_max=n_max, **mc)
    res["surrogate_seconds"] = t_sur
    res["surrogate_guess"] = (Jx, Jy)
    res["seconds"] += t_sur
    res["fallback_iters"] = res["iters"] - 1
    return res


# ------------------------------------------------------------ experiment
def experiment(n_points=100_000, L=64, burn=1000, measure=2000, epochs=200, lr=2e-3,
               targets=(0.2, 0.35, 0.5, 0.65, 0.8), beta=0.4, tol=0.01, se_rel=0.0025,
               n_rep=1024, n_max=65536, log=print, seed=1005):
    """The surrogate workload end to end: labels on the sampler, 90/10
    train/validation split, training, and for every target the wall time of
    the surrogate-steered solve against the Monte-Carlo-only solve (both
    Monte-Carlo-verified to `tol`, each evaluation resolved to a standard
    error of se_rel * target with up to n_max replicas)."""
    import synth
    pts = synth.surrogate_points(n_points, seed=seed)
    t0 = time.perf_counter()
    y, se = mc_observables(pts, L=L, burn=burn, measure=measure, log=log)
    torch.cuda.synchronize()
    t_label = time.perf_counter() - t0
    log(f"labels: {n_points} points in {t_label:.1f} s")
    n_tr = int(0.9 * n_points)
    net = SurrogateMLP(seed=0)
    t0 = time.perf_counter()
    net.fit(pts[:n_tr], y[:n_tr], epochs=epochs, lr=lr, lr_min=lr / 100, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    pv = net.predict(torch.tensor(pts[n_tr:], device=net.dev)).cpu().numpy()
    err = np.abs(pv - y[n_tr:])
    val = dict(mae_e=float(err[:, 0].mean()), mae_absm=float(err[:, 1].mean()),
               mae_chi=float(err[:, 2].mean()), label_se_absm=float(np.median(se[n_tr:])))
    log(f"training {t_train:.1f} s; validation MAE {val}")
    runs = []
    mc_kw = dict(n_rep=n_rep, L=L, burn=burn, measure=measure, se_rel=se_rel, n_max=n_max)
    keys = ("Jx", "Jy", "absm", "se", "iters", "replicas", "seconds", "converged")
    for tg in targets:
        mc = mc_only_solve(tg, beta=beta, tol=tol, **mc_kw)
        su = surrogate_solve(net, tg, beta=beta, tol=tol, **mc_kw)
        runs.append(dict(target=tg, mc_only={k: mc[k] for k in keys},
                         surrogate=dict({k: su[k] for k in keys},
                                        surrogate_guess=su["surrogate_guess"],
                                        fallback_iters=su["fallback_iters"])))
        log(f"target {tg}: MC-only {mc['seconds']:.2f} s ({mc['iters']} MC evals, "
            f"{mc['replicas']} replicas, |m| {mc['absm']:.4f} +- {mc['se']:.4f}); surrogate "
            f"{su['seconds']:.2f} s ({su['iters']} MC evals, {su['replicas']} replicas, "
            f"|m| {su['absm']:.4f} +- {su['se']:.4f})")
    tot_mc = sum(r["mc_only"]["seconds"] for r in runs)
    tot_su = sum(r["surrogate"]["seconds"] for r in runs)
    log(f"all targets: MC-only {tot_mc:.2f} s; surrogate {tot_su:.2f} s without and "
        f"{tot_su + t_label + t_train:.2f} s with the one-off labels and training")
    return dict(label_seconds=t_label, train_seconds=t_train, validation=val, solves=runs,
                total_seconds=dict(mc_only=tot_mc, surrogate=tot_su,
                                   surrogate_with_labels_and_training=tot_su + t_label + t_train),
                config=dict(n_points=n_points, L=L, burn=burn, measure=measure, epochs=epochs,
                            lr=lr, beta=beta, tol=tol, se_rel=se_rel, n_rep=n_rep, n_max=n_max))


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--points", type=int, default=100_000)
    ap.add_argument("--burn", type=int, default=1000)
    ap.add_argument("--measure", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--n-rep", type=int, default=1024)
    ap.add_argument("--n-max", type=int, default=65536)
    ap.add_argument("--se-rel", type=float, default=0.0025)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    res = experiment(n_points=a.points, burn=a.burn, measure=a.measure, epochs=a.epochs,
                     n_rep=a.n_rep, n_max=a.n_max, se_rel=a.se_rel,
                     log=lambda m: print(m, flush=True))
    txt = json.dumps(res)
    print(txt)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt)
