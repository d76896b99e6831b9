"""The oracle against exact results: enumeration, Kaufman, Onsager, Yang,
the Potts critical point, detailed balance, and exact gradients.

Equilibrium tests run many independent replicas and compare replica means
with the exact value at 4 standard errors (sigma from the replica spread).
"""
import math

import numpy as np
import pytest

import exact
from oracle import gradients, observables


def _replica_means(x, burn):
    """x[R, n_rec] -> per-replica means after burn-in."""
    return np.asarray(x, np.float64)[:, burn:].mean(axis=1)


def _within(est, want, nsig=4.0, floor=0.0):
    m = est.mean()
    se = est.std(ddof=1) / math.sqrt(len(est))
    assert abs(m - want) <= nsig * se + floor, (m, want, se)


# --------------------------------------------------------------- helpers
def test_enumeration_matches_kaufman():
    for Ly, Lx in [(4, 4), (2, 4), (4, 2), (2, 6), (6, 2), (3, 4)]:
        for beta in (0.2, 0.44, 0.7):
            en = exact.ising_exact(Ly, Lx, 1.0, 1.0, 0.0, beta)["lnZ"]
            ka = float(exact.kaufman_lnZ(Lx, Ly, beta))
            assert abs(en - ka) < 1e-10 * abs(en)


def test_kaufman_large_L_matches_onsager_away_from_criticality():
    for beta in (0.3, 0.6):
        assert abs(exact.kaufman_energy(256, beta) - exact.onsager_energy(beta)) < 1e-10


def test_potts_transfer_matrix_matches_enumeration():
    for Ly, Lx, q in [(3, 3, 3), (2, 4, 3), (4, 2, 2), (2, 2, 4)]:
        g = exact.potts_bond_histogram(Ly, Lx, q)
        st = exact.potts_enumerate(Ly, Lx, q)
        n = (st == np.roll(st, -1, 2)).sum(axis=(1, 2)) + (st == np.roll(st, -1, 1)).sum(axis=(1, 2))
        assert np.array_equal(np.bincount(n, minlength=len(g)), g.astype(np.int64))


def test_potts_q2_is_ising_at_half_coupling():
    """delta(s,s') = (1 + sigma sigma')/2: Potts q=2 at J equals Ising at J/2
    shifted by -J per site (2 bonds per site)."""
    g = exact.potts_bond_histogram(4, 4, 2)
    for beta in (0.3, 0.88, 1.4):
        eP, _ = exact.potts_exact_energy(g, 1.0, beta, 16)
        eI = exact.ising_exact(4, 4, 0.5, 0.5, 0.0, beta)["e"]
        assert abs(eP - (eI - 1.0)) < 1e-12


# --------------------------------------------------------- detailed balance
def test_ising_table_detailed_balance(orc):
    """pi(s) a(s -> -s) = pi(-s) a(-s -> s) class by class, with
    pi(s) ~ exp(beta s u), u = Jx Sx + Jy Sy + h, a = T / 2^32."""
    for Jx, Jy, h, beta in [(1.0, 1.0, 0.0, 0.44), (0.3, 1.7, 0.25, 0.8), (1.0, 0.5, -0.4, 2.0)]:
        Jx, Jy, h = (float(np.float32(v)) for v in (Jx, Jy, h))
        T = orc.ising_table(Jx, Jy, h, beta).astype(np.float64) / 2.0 ** 32
        for a in range(3):
            for b in range(3):
                u = Jx * (2 * a - 2) + Jy * (2 * b - 2) + h
                up, dn = T[9 + 3 * a + b], T[3 * a + b]
                lhs = math.exp(beta * u) * up
                rhs = math.exp(-beta * u) * dn
                # each threshold is ceil(2^32 p): at most 2^-32 above p
                tol = 2.0 ** -32 * (math.exp(beta * u) + math.exp(-beta * u))
                assert abs(lhs - rhs) <= tol
                assert max(up, dn) == 1.0


def test_potts_table_detailed_balance(orc):
    for q, J, h, beta in [(3, 1.0, 0.0, 1.0), (5, 0.7, 0.1, 1.3), (8, 1.0, -0.05, 2.5)]:
        J, h = float(np.float32(J)), float(np.float32(h))
        T = orc.potts_table(q, J, h, beta).astype(np.float64) / 2.0 ** 32
        w = 2 * q - 1
        for dn in range(-4, 5):
            for ds in range(-(q - 1), q):
                if ds == 0:
                    continue
                dE = -(J * dn + h * ds)
                fwd = T[(dn + 4) * w + ds + q - 1]
                rev = T[(-dn + 4) * w - ds + q - 1]
                lhs, rhs = fwd, math.exp(-beta * dE) * rev
                assert abs(lhs - rhs) <= 2.0 ** -32 * (1 + math.exp(-beta * dE))


def test_exact_sweep_kernel_leaves_boltzmann_stationary(orc):
    """Full colour-pass transition matrices on a 2x4 torus built from the
    oracle's thresholds: pi K0 = pi and pi K1 = pi exactly (to rounding of
    the quantised acceptance)."""
    Ly, Lx = 2, 4
    Jx, Jy, h, beta = 0.9, 1.2, 0.15, 0.7
    Jx, Jy, h = (float(np.float32(v)) for v in (Jx, Jy, h))
    T = orc.ising_table(Jx, Jy, h, beta).astype(np.float64) / 2.0 ** 32
    ex = exact.ising_exact(Ly, Lx, Jx, Jy, h, beta)
    st = exact.ising_states(Ly, Lx)
    n = len(st)
    pi = ex["p"]
    code = {tuple(s.reshape(-1)): i for i, s in enumerate(st)}
    for c in (0, 1):
        K = np.zeros((n, n))
        for i, s in enumerate(st):
            sites = [(y, x) for y in range(Ly) for x in range(Lx) if (x + y) % 2 == c]
            probs = []
            for y, x in sites:
                Sx = s[y, (x - 1) % Lx] + s[y, (x + 1) % Lx]
                Sy = s[(y - 1) % Ly, x] + s[(y + 1) % Ly, x]
                probs.append(T[9 * (s[y, x] > 0) + 3 * (Sx // 2 + 1) + (Sy // 2 + 1)])
            for mask in range(1 << len(sites)):
                t = s.copy()
                pr = 1.0
                for j, (y, x) in enumerate(sites):
                    if mask >> j & 1:
                        t[y, x] = -t[y, x]
                        pr *= probs[j]
                    else:
                        pr *= 1 - probs[j]
                K[i, code[tuple(t.reshape(-1))]] += pr
        assert np.allclose(K.sum(axis=1), 1.0, atol=1e-12)
        assert np.max(np.abs(pi @ K - pi)) < 1e-8


# --------------------------------------------------- equilibrium: Ising
@pytest.mark.parametrize("Jx,Jy,h,beta", [(1.0, 1.0, 0.0, 0.44), (0.8, 1.2, 0.1, 0.5)])
def test_ising_chain_matches_4x4_enumeration(orc, Jx, Jy, h, beta):
    Jx, Jy, h = (float(np.float32(v)) for v in (Jx, Jy, h))
    R, n, burn = 64, 3000, 300
    states = [orc.ising_init(4, 4, 11, r) for r in range(R)]
    _, st = orc.ising_run_batch(states, [Jx] * R, [Jy] * R, [h] * R, [beta] * R, 11,
                                np.arange(R), 0, n, 1)
    obs = observables.ising(st, Jx, Jy, h, 16)
    ex = exact.ising_exact(4, 4, Jx, Jy, h, beta)
    for k in ("e", "absm", "m2"):
        _within(_replica_means(obs[k], burn), ex[k])


@pytest.mark.slow
def test_ising_chain_matches_kaufman_32(orc):
    """The 32x32 torus at beta = 0.44 (near criticality)."""
    R, n, burn = 16, 6000, 1000
    states = [orc.ising_init(32, 32, 1, r) for r in range(R)]
    _, st = orc.ising_run_batch(states, [1.0] * R, [1.0] * R, [0.0] * R, [0.44] * R, 1,
                                np.arange(R), 0, n, 1)
    e = observables.ising(st, 1.0, 1.0, 0.0, 1024)["e"]
    _within(_replica_means(e, burn), exact.kaufman_energy(32, 0.44))


@pytest.mark.parametrize("beta", [0.3, 0.6])
def test_ising_chain_matches_onsager_and_yang(orc, beta):
    R, n, burn, L = 8, 600, 100, 48
    states = [orc.ising_init(L, L, 5, r) for r in range(R)]
    _, st = orc.ising_run_batch(states, [1.0] * R, [1.0] * R, [0.0] * R, [beta] * R, 5,
                                np.arange(R), 0, n, 1)
    obs = observables.ising(st, 1.0, 1.0, 0.0, L * L)
    _within(_replica_means(obs["e"], burn), exact.kaufman_energy(L, beta))
    if beta > exact.BETA_C_ISING:
        # finite-size corrections to |m| are exponentially small here
        _within(_replica_means(obs["absm"], burn), exact.yang_magnetisation(beta), floor=2e-4)


# --------------------------------------------------- equilibrium: Potts
@pytest.mark.parametrize("q,beta", [(3, 0.6), (3, 1.0050525), (3, 1.5)])
def test_potts_chain_matches_4x4_transfer_matrix(orc, q, beta):
    R, n, burn = 48, 3000, 300
    g = exact.potts_bond_histogram(4, 4, q)
    want, _ = exact.potts_exact_energy(g, 1.0, beta, 16)
    states = [orc.potts_init(4, 4, q, 21, r) for r in range(R)]
    _, st = orc.potts_run_batch(states, [q] * R, [1.0] * R, [0.0] * R, [beta] * R, 21,
                                np.arange(R), 0, n, 1)
    e = observables.potts(st, q, 1.0, 0.0, 16)["e"]
    _within(_replica_means(e, burn), want)


def test_potts_q2_chain_matches_ising_at_half_coupling(orc):
    R, n, burn, L, beta = 16, 1500, 200, 8, 0.9
    states = [orc.potts_init(L, L, 2, 3, r) for r in range(R)]
    _, st = orc.potts_run_batch(states, [2] * R, [1.0] * R, [0.0] * R, [beta] * R, 3,
                                np.arange(R), 0, n, 1)
    eP = _replica_means(observables.potts(st, 2, 1.0, 0.0, L * L)["e"], burn)
    istates = [orc.ising_init(L, L, 4, r) for r in range(R)]
    _, sti = orc.ising_run_batch(istates, [0.5] * R, [0.5] * R, [0.0] * R, [beta] * R, 4,
                                 np.arange(R), 0, n, 1)
    eI = _replica_means(observables.ising(sti, 0.5, 0.5, 0.0, L * L)["e"], burn) - 1.0
    se = math.hypot(eP.std(ddof=1) / math.sqrt(R), eI.std(ddof=1) / math.sqrt(R))
    assert abs(eP.mean() - eI.mean()) < 4 * se


@pytest.mark.slow
@pytest.mark.parametrize("q", [3, 4, 8])
def test_potts_transition_brackets_critical_point(orc, q):
    """The order-disorder transition sits at beta_c = ln(1 + sqrt q): on a
    32x32 torus the order parameter m_P is small at 0.8 beta_c (random
    start) and close to 1 at 1.2 beta_c (ordered start)."""
    R, n, burn, L = 8, 600, 300, 32
    bc = exact.potts_beta_c(q)
    hot = [orc.potts_init(L, L, q, 8, r) for r in range(R)]
    cold = [np.zeros((L, L), np.uint8) for _ in range(R)]
    for b, states, lo, hi in [(0.8 * bc, hot, 0.0, 0.15), (1.2 * bc, cold, 0.85, 1.0)]:
        _, st = orc.potts_run_batch(states, [q] * R, [1.0] * R, [0.0] * R, [b] * R, 9,
                                    np.arange(R), 0, n, 1)
        mP = _replica_means(observables.potts(st, q, 1.0, 0.0, L * L)["mP"], burn).mean()
        assert lo <= mP <= hi, (b, mP)


# ------------------------------------------------------------ gradients
def _exact_expectations(Jx, Jy, h, beta):
    ex = exact.ising_exact(4, 4, Jx, Jy, h, beta)
    return ex["e"], ex["absm"]


def test_covariance_estimator_equals_exact_derivative():
    """With the exact Boltzmann weights of the 4x4 torus as sample weights,
    the estimator equals the derivative of the exact expectation (central
    differences of enumeration at +-1e-5)."""
    Jx, Jy, h, beta = 0.9, 1.1, 0.07, 0.44
    ex = exact.ising_exact(4, 4, Jx, Jy, h, beta)
    means, grads = gradients.ising_grad(ex["M"], ex["Bx"], ex["By"], Jx, Jy, h, beta, 16,
                                        weights=ex["p"])
    assert abs(means[0] - ex["e"]) < 1e-12 and abs(means[1] - ex["absm"]) < 1e-12
    eps = 1e-5
    base = [Jx, Jy, h]
    for j in range(3):
        up, dn = list(base), list(base)
        up[j] += eps
        dn[j] -= eps
        fu, fd = _exact_expectations(*up, beta), _exact_expectations(*dn, beta)
        for o in range(2):
            fdiff = (fu[o] - fd[o]) / (2 * eps)
            assert abs(grads[o, j] - fdiff) < 1e-7, (o, j, grads[o, j], fdiff)


def test_covariance_estimator_isotropic_values():
    """beta = 0.44, J = 1, h = 0 on 4x4: d<|m|>/dJ (J = Jx = Jy) and d<e>/dJ
    by finite differences of the exact expectation."""
    ex = exact.ising_exact(4, 4, 1.0, 1.0, 0.0, 0.44)
    _, g = gradients.ising_grad(ex["M"], ex["Bx"], ex["By"], 1.0, 1.0, 0.0, 0.44, 16,
                                weights=ex["p"])
    eps = 1e-5
    fu = _exact_expectations(1 + eps, 1 + eps, 0.0, 0.44)
    fd = _exact_expectations(1 - eps, 1 - eps, 0.0, 0.44)
    assert abs((g[1, 0] + g[1, 1]) - (fu[1] - fd[1]) / (2 * eps)) < 1e-7
    assert abs((g[0, 0] + g[0, 1]) - (fu[0] - fd[0]) / (2 * eps)) < 1e-7
    assert abs(g[1, 2]) < 1e-12  # h -> -h symmetry


def test_covariance_estimator_on_oracle_chain_within_3sigma(orc):
    Jx = Jy = float(np.float32(0.8))
    h = float(np.float32(0.05))
    beta, R, n, burn = 0.5, 64, 4000, 400
    states = [orc.ising_init(4, 4, 31, r) for r in range(R)]
    _, st = orc.ising_run_batch(states, [Jx] * R, [Jy] * R, [h] * R, [beta] * R, 31,
                                np.arange(R), 0, n, 1)
    stats = np.transpose(st, (1, 0, 2))
    _, grads = gradients.ising_grad_batch(stats, [Jx] * R, [Jy] * R, [h] * R, [beta] * R, 16,
                                          burn)
    ex = exact.ising_exact(4, 4, Jx, Jy, h, beta)
    _, g_exact = gradients.ising_grad(ex["M"], ex["Bx"], ex["By"], Jx, Jy, h, beta, 16,
                                      weights=ex["p"])
    for o in range(2):
        for j in range(3):
            est = grads[:, o, j]
            se = est.std(ddof=1) / math.sqrt(R)
            assert abs(est.mean() - g_exact[o, j]) <= 4 * se + 1e-3 * abs(g_exact[o, j]), (o, j)


# ---------------------------------------------------------- susceptibility
def _exact_m(Jx, Jy, h, beta):
    ex = exact.ising_exact(4, 4, Jx, Jy, h, beta)
    return float((ex["p"] * ex["M"]).sum() / 16)


@pytest.mark.parametrize("beta", [0.2, 0.44, 0.7])
def test_susceptibility_with_exact_weights(beta):
    """chi = beta N (<m^2> - <|m|>^2) over the exact 4x4 distribution.  At
    h = 0 the first term is the field response of the exact magnetisation,
    beta N <m^2> = d<m>/dh (fluctuation-dissipation, <m> = 0 by symmetry),
    taken here by central differences of the enumeration; the second uses the
    exact <|m|>."""
    ex = exact.ising_exact(4, 4, 1.0, 1.0, 0.0, beta)
    absm = np.abs(ex["M"]) / 16.0
    m2 = (ex["M"] / 16.0) ** 2
    chi = float(observables.susceptibility(absm, m2, beta, 16, weights=ex["p"]))
    eps = 1e-5
    dm_dh = (_exact_m(1.0, 1.0, eps, beta) - _exact_m(1.0, 1.0, -eps, beta)) / (2 * eps)
    want = dm_dh - beta * 16 * ex["absm"] ** 2
    # central differences err by O(eps^2) of the larger term d<m>/dh
    assert abs(chi - want) < 1e-8 * max(1.0, abs(dm_dh)), (chi, want)
    # the plain-sample form equals the weighted one on equally weighted samples
    rng = np.random.default_rng(3)
    idx = rng.choice(len(absm), size=5000, p=ex["p"])
    assert abs(float(observables.susceptibility(absm[idx], m2[idx], beta, 16)) -
               float(observables.susceptibility(absm[idx], m2[idx], beta, 16,
                                                weights=np.ones(5000)))) < 1e-12


def test_susceptibility_on_oracle_chain_within_4sigma(orc):
    """chi of each replica's recorded chain, averaged over replicas, against
    the exact 4x4 value (per-replica chi carries an O(1/n) bias from its own
    mean, far below the tolerance at 3000 samples)."""
    beta, R, n, burn = 0.44, 64, 3000, 300
    states = [orc.ising_init(4, 4, 17, r) for r in range(R)]
    _, st = orc.ising_run_batch(states, [1.0] * R, [1.0] * R, [0.0] * R, [beta] * R, 17,
                                np.arange(R), 0, n, 1)
    obs = observables.ising(st, 1.0, 1.0, 0.0, 16)
    chi = observables.susceptibility(obs["absm"][:, burn:], obs["m2"][:, burn:], beta, 16,
                                     axis=1)
    ex = exact.ising_exact(4, 4, 1.0, 1.0, 0.0, beta)
    want = beta * 16 * (ex["m2"] - ex["absm"] ** 2)
    _within(chi, want)


def test_exact_rational_estimator_equals_two_pass(orc):
    """The rational form of the estimator (used for FP64 parity) equals the
    two-pass FP64 form, which the tests above pin to the derivative of the
    exact expectation, on chain samples to rounding."""
    Jx, Jy, h = (float(np.float32(v)) for v in (0.7, 0.9, 0.05))
    states = [orc.ising_init(4, 4, 5, r) for r in range(4)]
    _, st = orc.ising_run_batch(states, [Jx] * 4, [Jy] * 4, [h] * 4, [0.5] * 4, 5,
                                np.arange(4), 0, 800, 1)
    for r in range(4):
        s = st[r, 100:]
        mo, go = gradients.ising_grad(s[:, 0], s[:, 1], s[:, 2], Jx, Jy, h, 0.5, 16)
        v, sc = gradients.ising_grad_exact(s[:, 0], s[:, 1], s[:, 2], Jx, Jy, h, 0.5, 16)
        assert abs(float(v["e"]) - mo[0]) <= 1e-12 * float(sc["e"])
        assert abs(float(v["absm"]) - mo[1]) <= 1e-12 * float(sc["absm"])
        for o in range(2):
            for j in range(3):
                assert abs(float(v["grad"][o][j]) - go[o, j]) <= 1e-9 * float(sc["grad"][o][j])
