"""Exact results used to pin the oracle (test helpers, independent of it).

* brute-force enumeration of small Ising and Potts tori;
* a row transfer matrix for the q-state Potts energy distribution;
* Kaufman's exact partition function of the finite Ising torus
  (B. Kaufman, Phys. Rev. 76, 1232 (1949));
* Onsager's infinite-lattice energy per site and Yang's spontaneous
  magnetisation (C. N. Yang, Phys. Rev. 85, 808 (1952));
* the Potts critical coupling ln(1 + sqrt q).

Conventions (the ferromagnetic reading of Eq. (1) and Eq. (2)):
Ising H = -Jx sum_h s s' - Jy sum_v s s' - h sum s; Potts
H = -J sum delta(s, s') - h sum s; every nearest-neighbour bond once.
"""
import itertools
import math

import mpmath as mp
import numpy as np
from scipy.special import ellipk


# ---------------------------------------------------------------- Ising
def ising_states(Ly, Lx):
    """All 2^(Ly*Lx) states as int8 [n, Ly, Lx] in {-1,+1}."""
    n = Ly * Lx
    idx = np.arange(2 ** n, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(n)[None, :]) & 1
    return (2 * bits - 1).astype(np.int8).reshape(-1, Ly, Lx)


def ising_bond_sums(states):
    s = states.astype(np.int64)
    M = s.sum(axis=(1, 2))
    Bx = (s * np.roll(s, -1, axis=2)).sum(axis=(1, 2))
    By = (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    return M, Bx, By


def tri_bond_sums(states):
    """M and the bond sums of the triangular lattice's three directions:
    (y, x)-(y, x+1), (y, x)-(y+1, x), (y, x)-(y+1, x-1)."""
    s = states.astype(np.int64)
    M = s.sum(axis=(1, 2))
    Bh = (s * np.roll(s, -1, axis=2)).sum(axis=(1, 2))
    Bv = (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    Bd = (s * np.roll(np.roll(s, -1, axis=1), 1, axis=2)).sum(axis=(1, 2))
    return M, Bh, Bv, Bd


def tri_exact(Ly, Lx, J, h, beta):
    """Exact <e> and <|m|> of the triangular-lattice Ising torus by
    enumeration, H = -J (Bh + Bv + Bd) - h M."""
    st = ising_states(Ly, Lx)
    M, Bh, Bv, Bd = tri_bond_sums(st)
    N = Ly * Lx
    E = -(J * (Bh + Bv + Bd) + h * M)
    a = -beta * E
    w = np.exp(a - a.max())
    p = w / w.sum()
    return dict(e=float((p * E).sum() / N), absm=float((p * np.abs(M)).sum() / N))


def ising_exact(Ly, Lx, Jx, Jy, h, beta):
    """Exact <e>, <|m|>, <m^2>, ln Z and Boltzmann weights by enumeration."""
    st = ising_states(Ly, Lx)
    M, Bx, By = ising_bond_sums(st)
    N = Ly * Lx
    E = -(Jx * Bx + Jy * By + h * M)
    a = -beta * E
    amax = a.max()
    w = np.exp(a - amax)
    Z = w.sum()
    p = w / Z
    return dict(e=float((p * E).sum() / N), absm=float((p * np.abs(M)).sum() / N),
                m2=float((p * (M / N) ** 2).sum()), lnZ=float(np.log(Z) + amax), p=p, M=M,
                Bx=Bx, By=By)


def ising_energy(sigma, Jx, Jy, h):
    """Brute-force energy of one Ising lattice (float64)."""
    s = sigma.astype(np.int64)
    Bx = int((s * np.roll(s, -1, axis=1)).sum())
    By = int((s * np.roll(s, -1, axis=0)).sum())
    M = int(s.sum())
    return -(Jx * Bx + Jy * By + h * M), (Bx, By, M)


def kaufman_lnZ(m, n, K):
    """ln Z of the isotropic Ising model (coupling K = beta J, h = 0) on an
    n-row by m-column torus, Kaufman's four-term product formula (evaluated
    at the caller's mpmath precision)."""
    K = mp.mpf(K)
    c2 = mp.cosh(2 * K) * mp.cosh(2 * K) / mp.sinh(2 * K)

    def gamma(l):
        if l == 0:
            return 2 * K + mp.log(mp.tanh(K))
        return mp.acosh(c2 - mp.cos(mp.pi * l / n))

    g_odd = [gamma(2 * r + 1) for r in range(n)]
    g_even = [gamma(2 * r) for r in range(n)]
    Z1 = mp.fprod(2 * mp.cosh(m * g / 2) for g in g_odd)
    Z2 = mp.fprod(2 * mp.sinh(m * g / 2) for g in g_odd)
    Z3 = mp.fprod(2 * mp.cosh(m * g / 2) for g in g_even)
    Z4 = mp.fprod(2 * mp.sinh(m * g / 2) for g in g_even)
    lnZ = mp.log(mp.mpf(1) / 2) + (mp.mpf(m * n) / 2) * mp.log(2 * mp.sinh(2 * K)) + \
        mp.log(Z1 + Z2 + Z3 + Z4)
    return lnZ


def kaufman_energy(L, beta):
    """Exact energy per site u = -(1/N) d lnZ / d beta on an L x L torus, J=1."""
    with mp.workdps(60):
        f = lambda k: kaufman_lnZ(L, L, k)  # noqa: E731
        return float(-mp.diff(f, mp.mpf(beta)) / (L * L))


def onsager_energy(beta):
    """Infinite-lattice energy per site of the isotropic model (J = 1)."""
    K = beta
    k = 2 * math.sinh(2 * K) / math.cosh(2 * K) ** 2
    K1 = ellipk(k * k)
    return -1.0 / math.tanh(2 * K) * (1 + 2 / math.pi * (2 * math.tanh(2 * K) ** 2 - 1) * K1)


def yang_magnetisation(beta):
    s = math.sinh(2 * beta)
    return (1 - s ** -4) ** 0.125 if s > 1 else 0.0


BETA_C_ISING = 0.5 * math.log(1 + math.sqrt(2))


# ---------------------------------------------------------------- Potts
def potts_energy(s, J, h):
    s = s.astype(np.int64)
    Nx = int((s == np.roll(s, -1, axis=1)).sum())
    Ny = int((s == np.roll(s, -1, axis=0)).sum())
    S = int(s.sum())
    return -(J * (Nx + Ny) + h * S), (Nx, Ny, S)


def potts_enumerate(Ly, Lx, q):
    """All q^(Ly*Lx) states (small tori only)."""
    n = Ly * Lx
    return np.array(list(itertools.product(range(q), repeat=n)), np.int8).reshape(-1, Ly, Lx)


def potts_bond_histogram(Ly, Lx, q):
    """g[n] = number of states with n equal nearest-neighbour bonds on an
    Ly x Lx torus, by a row-to-row transfer matrix whose entries are
    monomials x^(equal bonds added by the new row); trace over row 0."""
    rows = np.array(list(itertools.product(range(q), repeat=Lx)), np.int64)
    R = len(rows)
    intra = (rows == np.roll(rows, -1, axis=1)).sum(axis=1)
    inter = (rows[:, None, :] == rows[None, :, :]).sum(axis=2)
    E = inter + intra[None, :]          # bonds added when row b follows row a
    deg = 2 * Ly * Lx + 1
    vec = np.zeros((R, R, deg), np.int64)   # [first row a0, current row, degree]
    vec[np.arange(R), np.arange(R), 0] = 1
    for _ in range(Ly):
        new = np.zeros_like(vec)
        for e in range(int(E.max()) + 1):
            Me = (E == e).astype(np.int64)
            part = np.einsum("zad,ab->zbd", vec, Me)
            new[:, :, e:] += part[:, :, :deg - e]
        vec = new
    return vec[np.arange(R), np.arange(R), :].sum(axis=0)


def potts_exact_energy(g, J, beta, N):
    """<e> = -J <n_eq> / N from the bond histogram g (exact rationals via mp)."""
    with mp.workdps(40):
        w = [mp.mpf(int(c)) * mp.e ** (beta * J * n) for n, c in enumerate(g)]
        Z = mp.fsum(w)
        En = mp.fsum(n * wi for n, wi in enumerate(w)) / Z
        return float(-J * En / N), float(mp.log(Z))


def potts_beta_c(q):
    return math.log(1 + math.sqrt(q))
