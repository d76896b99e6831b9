"""FP64 observables from integer statistics -- TEST INFRASTRUCTURE ONLY.

Ising, Eq. (1) with H = -Jx Bx - Jy By - h M (every bond once):
    e = H / N,  |m| = |M| / N,  m2 = (M / N)^2,
    chi = beta N (<m2> - <|m|>^2)   (two-pass FP64 means).
Potts, Eq. (2) with H = -J (Nx + Ny) - h S:
    e = H / N,  m_P = (q nmax / N - 1) / (q - 1).
Cellular Potts, Eq. (3): H = (H*S) / S from the int64 fixed-point statistic,
boundary lengths = von Neumann bonds between different ids by type pair
(the cell-sorting boundary measure of the Results section).

Pins: integer statistics are recounted from lattices in the tests; the energy
conventions are pinned through exact enumeration; chi through the exact 4x4
distribution, where beta N <m^2> at h = 0 equals the field derivative
d<m>/dh of the exact magnetisation, and through oracle chains; the CPM energy
against a brute-force Eq. (3) and the boundary slots against a recount
(tests/test_oracle_exact.py, tests/test_oracle_cpm.py).
"""
import numpy as np


def ising(stats, Jx, Jy, h, N):
    """stats[..., 8] int (M, Bx, By, ...) -> dict of FP64 arrays e, absm, m2."""
    s = np.asarray(stats, np.int64)
    M, Bx, By = s[..., 0].astype(np.float64), s[..., 1].astype(np.float64), s[..., 2].astype(np.float64)
    Jx = np.asarray(Jx, np.float64)
    Jy = np.asarray(Jy, np.float64)
    h = np.asarray(h, np.float64)
    H = -(Jx * Bx + Jy * By + h * M)
    return dict(e=H / N, absm=np.abs(M) / N, m2=(M / N) ** 2)


def susceptibility(absm, m2, beta, N, axis=0, weights=None):
    """chi = beta N (<m^2> - <|m|>^2) with plain FP64 means over ``axis``;
    ``weights`` (same shape as the samples) turns the means into weighted
    means, so that a test can feed an exact distribution."""
    absm = np.asarray(absm, np.float64)
    m2 = np.asarray(m2, np.float64)
    if weights is None:
        mean_abs = np.mean(absm, axis=axis)
        mean_m2 = np.mean(m2, axis=axis)
    else:
        w = np.asarray(weights, np.float64)
        mean_abs = np.sum(w * absm, axis=axis) / np.sum(w, axis=axis)
        mean_m2 = np.sum(w * m2, axis=axis) / np.sum(w, axis=axis)
    return np.asarray(beta, np.float64) * N * (mean_m2 - mean_abs ** 2)


def potts(stats, q, J, h, N):
    s = np.asarray(stats, np.int64)
    Nx, Ny, S, nmax = (s[..., i].astype(np.float64) for i in range(4))
    q = np.asarray(q, np.float64)
    H = -(np.asarray(J, np.float64) * (Nx + Ny) + np.asarray(h, np.float64) * S)
    return dict(e=H / N, mP=(q * nmax / N - 1.0) / (q - 1.0))


def cpm(stats, S):
    s = np.asarray(stats, np.int64)
    lo = s[..., 10] & 0xFFFFFFFF
    hi = s[..., 11]
    H = (hi << 32) | lo
    return dict(H=H.astype(np.float64) / S, boundary=s[..., :10].copy())
