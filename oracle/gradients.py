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


def ising_grad_exact(M, Bx, By, Jx, Jy, h, beta, N):
    """The same estimator in exact rational arithmetic, for parity at FP64
    rounding level.  Integer moments of the samples (Python ints), every
    parameter taken as the exact value of its binary floating-point number
    (``Fraction(float)``), covariances Cov(a, b) = (n S_ab - S_a S_b) / n^2.

    Returns (values, scales), two dicts of ``Fraction`` keyed "e", "absm",
    "m2", "chi" (the replica means, chi = beta N (<m^2> - <|m|>^2)) and
    "grad" (a 2 x 3 nested list, O = (e, |m|), theta = (Jx, Jy, h)).  A
    scale is the sum of the absolute values of the terms that make up its
    value: a floating-point evaluation of the same expression that rounds
    each term and each operation errs by a few units of 2^-53 of it."""
    from fractions import Fraction as F
    M = [int(v) for v in np.asarray(M, np.int64)]
    Bx = [int(v) for v in np.asarray(Bx, np.int64)]
    By = [int(v) for v in np.asarray(By, np.int64)]
    n = len(M)
    aM = [abs(v) for v in M]
    X = [Bx, By, M]
    S = [sum(x) for x in X]
    Sa = sum(aM)

    def cov(a, b):
        return F(n * sum(u * v for u, v in zip(a, b)) - sum(a) * sum(b), n * n)

    Jx, Jy, h, beta = F(float(Jx)), F(float(Jy)), F(float(h)), F(float(beta))
    N = F(int(N))
    J = [Jx, Jy, h]
    vals, scales = {}, {}
    vals["e"] = -(Jx * S[0] + Jy * S[1] + h * S[2]) / (n * N)
    scales["e"] = (abs(Jx * S[0]) + abs(Jy * S[1]) + abs(h * S[2])) / (n * N)
    vals["absm"] = scales["absm"] = F(Sa, n) / N
    vals["m2"] = scales["m2"] = F(sum(v * v for v in M), n) / (N * N)
    vals["chi"] = beta * cov(aM, aM) / N
    scales["chi"] = abs(vals["chi"])
    C = [[cov(X[i], X[j]) for j in range(3)] for i in range(3)]
    g, gs = [[None] * 3, [None] * 3], [[None] * 3, [None] * 3]
    for j in range(3):
        adh = sum(J[i] * C[i][j] for i in range(3))
        g[0][j] = -F(S[j], n) / N - beta * adh / N
        gs[0][j] = abs(F(S[j], n) / N) + beta * sum(abs(J[i] * C[i][j]) for i in range(3)) / N
        g[1][j] = beta * cov(aM, X[j]) / N
        gs[1][j] = abs(g[1][j])
    vals["grad"], scales["grad"] = g, gs
    return vals, scales
