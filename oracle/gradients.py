"""Fluctuation (covariance) estimator of observable gradients -- TEST
INFRASTRUCTURE ONLY.

The paper differentiates its chain through a logistic relaxation
(Methods, Algorithm 2).  The gradient of an equilibrium expectation has an
exact identity that needs no relaxation: for a Boltzmann weight
exp(-beta H(s; theta)),

    d<O>/dtheta = <dO/dtheta> - beta Cov(O, dH/dtheta).

For the Ising energy of Eq. (1) with H = -Jx Bx - Jy By - h M:
    dH/dJx = -Bx, dH/dJy = -By, dH/dh = -M.
Observables: O0 = e = H/N (so de/dJx = -Bx/N, de/dJy = -By/N, de/dh = -M/N)
and O1 = |m| = |M|/N (no explicit dependence).

Plain two-pass FP64: means first, then centred products.  ``weights`` lets a
test feed an exact distribution (enumeration) instead of samples.

Pins: exact enumeration of the 4x4 torus and finite differences of exact
expectations (tests/test_oracle_exact.py).
"""
import numpy as np


def _wmean(x, w):
    return np.sum(w * x) / np.sum(w)


def ising_grad(M, Bx, By, Jx, Jy, h, beta, N, weights=None):
    """Samples of one replica -> (means[2], grads[2, 3]) for O = (e, |m|)
    and theta = (Jx, Jy, h)."""
    M = np.asarray(M, np.float64)
    Bx = np.asarray(Bx, np.float64)
    By = np.asarray(By, np.float64)
    w = np.ones_like(M) if weights is None else np.asarray(weights, np.float64)
    e = -(Jx * Bx + Jy * By + h * M) / N
    am = np.abs(M) / N
    X = [Bx, By, M]  # = -dH/dtheta
    dO = [[-Bx / N, -By / N, -M / N], [0.0 * M, 0.0 * M, 0.0 * M]]
    means = np.zeros(2)
    grads = np.zeros((2, 3))
    for i, O in enumerate((e, am)):
        mO = _wmean(O, w)
        means[i] = mO
        for j in range(3):
            mX = _wmean(X[j], w)
            cov = _wmean((O - mO) * (X[j] - mX), w)
            grads[i, j] = _wmean(dO[i][j], w) + beta * cov
    return means, grads


def ising_grad_batch(stats, Jx, Jy, h, beta, N, burn_in, grad_out=None):
    """stats[n_rec, R, 8] -> means[R, 2], grads[R, 2, 3] over samples
    t >= burn_in; with grad_out[R, 2] also the contraction dtheta[R, 3]."""
    s = np.asarray(stats)[burn_in:]
    R = s.shape[1]
    means = np.zeros((R, 2))
    grads = np.zeros((R, 2, 3))
    for r in range(R):
        means[r], grads[r] = ising_grad(s[:, r, 0], s[:, r, 1], s[:, r, 2], float(Jx[r]),
                                        float(Jy[r]), float(h[r]), float(beta[r]), N)
    if grad_out is None:
        return means, grads
    g = np.asarray(grad_out, np.float64)
    return means, grads, np.einsum("ro,rop->rp", g, grads)
