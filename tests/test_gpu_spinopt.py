"""GPU spin-value optimisation: the energy kernel, the quantised step and the
three methods (annealed Monte Carlo, gradient, differentiable Monte Carlo)
against the FP64 oracle, then the comparison on J = 1 and +-J lattices."""
import numpy as np
import pytest

from oracle import dmc as odmc
from oracle import spinopt as oso

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _couplings(rng, R, Ly, Lx, kind):
    if kind == "ferro":
        return np.ones((R, Ly, Lx), np.float32), np.ones((R, Ly, Lx), np.float32)
    if kind == "glass":
        J = rng.choice([-1.0, 1.0], size=(2, R, Ly, Lx)).astype(np.float32)
        return J[0], J[1]
    J = rng.uniform(-1, 1, size=(2, R, Ly, Lx)).astype(np.float32)
    return J[0], J[1]


def _opt(Jx, Jy, h=0.0, seed=1):
    from paper_2304_01772_amd.spinopt import SpinOptimiser
    return SpinOptimiser(torch.tensor(Jx, device="cuda"), torch.tensor(Jy, device="cuda"), h,
                         seed)


# 2 x 2 (smallest torus), several 1024-thread strides (34 x 136) and a ragged one
@pytest.mark.parametrize("R,Ly,Lx", [(3, 6, 8), (2, 34, 136), (1, 2, 2), (2, 10, 6)])
def test_energy_and_gradient_match_oracle(R, Ly, Lx):
    rng = np.random.default_rng(R * 100 + Lx)
    h = float(np.float32(0.15))
    # +-1 spins with +-J: every term is an integer, the results are exact
    s = rng.choice([-1.0, 1.0], size=(R, Ly, Lx)).astype(np.float32)
    Jx, Jy = _couplings(rng, R, Ly, Lx, "glass")
    o = _opt(Jx, Jy, 0.0)
    e, g = o.energy(torch.tensor(s, device="cuda"), grad=True)
    We, Wg = oso.energy(s, Jx, Jy, 0.0)
    assert np.array_equal(e.cpu().numpy(), We.numpy())
    assert np.array_equal(g.cpu().numpy(), Wg.numpy().astype(np.float32))
    # continuous spins and couplings, with a field
    s = rng.uniform(-1, 1, size=(R, Ly, Lx)).astype(np.float32)
    Jx, Jy = _couplings(rng, R, Ly, Lx, "real")
    o = _opt(Jx, Jy, h)
    e, g = o.energy(torch.tensor(s, device="cuda"), grad=True)
    We, Wg = oso.energy(s, Jx, Jy, h)
    np.testing.assert_allclose(e.cpu().numpy(), We.numpy(), rtol=1e-12, atol=1e-12 * Ly * Lx)
    np.testing.assert_allclose(g.cpu().numpy(), Wg.numpy(), rtol=0, atol=1e-5)


def test_discretize_matches_oracle():
    from paper_2304_01772_amd._lib import check, lib
    import ctypes as C
    rng = np.random.default_rng(7)
    n = 70001  # several workgroups and a ragged tail
    base = rng.uniform(-1, 1, n).astype(np.float32)
    g = rng.normal(size=n).astype(np.float32)
    base[:3] = [0.0, -0.0, 1e-30]
    g[:3] = 0.0
    eta = 0.37
    b, gg = torch.tensor(base, device="cuda"), torch.tensor(g, device="cuda")
    out = torch.empty_like(b)
    check(lib().spinmc_dmc_discretize(n, C.c_void_p(b.data_ptr()), C.c_void_p(gg.data_ptr()),
                                      eta, C.c_void_p(out.data_ptr()), None))
    want = oso.discretize_step(base[None], g[None], float(np.float32(eta)))[0].numpy()
    v = base.astype(np.float64) - np.float32(eta) * g.astype(np.float64)
    clear = np.abs(v) > 1e-6  # the FP32 and FP64 differences decide the same sign
    assert np.array_equal(out.cpu().numpy()[clear], want[clear])
    assert out.cpu().numpy()[:3].tolist() == [1.0, 1.0, 1.0]
    check(lib().spinmc_dmc_discretize(n, C.c_void_p(b.data_ptr()), None, 0.0,
                                      C.c_void_p(out.data_ptr()), None))
    assert np.array_equal(out.cpu().numpy(), np.where(base < 0, -1.0, 1.0))


@pytest.mark.parametrize("kind", ["ferro", "glass"])
def test_annealed_mc_and_gradient_runs_equal_the_oracle(kind):
    """Both methods take integer decisions from exactly representable inputs
    (the betas are the FP32 values the kernels use): every step's state and
    energy equal the oracle's."""
    rng = np.random.default_rng(11)
    R, L, steps = 3, 16, 8
    s0 = rng.choice([-1.0, 1.0], size=(R, L, L)).astype(np.float32)
    Jx, Jy = _couplings(rng, R, L, L, kind)
    betas = [float(np.float32(b)) for b in np.linspace(0.3, 2.0, steps)]
    o = _opt(Jx, Jy, 0.0, seed=5)
    for method, kw in (("mc", dict(betas=betas)), ("gradient", dict(eta=1.0))):
        hist, s = o.run(method, torch.tensor(s0, device="cuda"), steps, **kw)
        Wh, Ws = oso.run(method, s0, Jx, Jy, 0.0, steps, seed=5, **kw)
        assert np.array_equal(s.cpu().numpy(), Ws.numpy().astype(np.float32)), method
        np.testing.assert_allclose(hist, Wh, rtol=0, atol=1e-12)


def test_dmc_steps_match_the_oracle_step_by_step():
    """Each GPU step, from the GPU's current state, equals the oracle's step
    from that state wherever the oracle's pre-discretisation value is not
    within 1e-3 of zero (FP32 chain and gradient against FP64)."""
    rng = np.random.default_rng(12)
    R, L, steps, alpha, n_sw, eta = 2, 12, 6, 20.0, 2, 0.05
    s = rng.choice([-1.0, 1.0], size=(R, L, L)).astype(np.float32)
    Jx, Jy = _couplings(rng, R, L, L, "glass")
    betas = [float(np.float32(b)) for b in np.linspace(0.4, 2.0, steps)]
    o = _opt(Jx, Jy, 0.0, seed=9)
    clear_total = 0
    for k in range(steps):
        got = o.dmc_step(torch.tensor(s, device="cuda"), betas[k], alpha, n_sw, eta, k)
        got = got.cpu().numpy()
        # the oracle's value before discretisation
        s0 = torch.tensor(s.astype(np.float64), requires_grad=True)
        sc = odmc.forward(s0, torch.tensor(Jx, dtype=torch.float64),
                          torch.tensor(Jy, dtype=torch.float64), 0.0, betas[k], alpha, 9,
                          list(range(R)), k * n_sw, n_sw)
        H, _ = oso.energy(sc, Jx, Jy, 0.0)
        H.sum().backward()
        v = (sc.detach() - float(np.float32(eta)) * s0.grad).numpy()
        want = np.where(v < 0, -1.0, 1.0)
        clear = np.abs(v) > 1e-3
        clear_total += int(clear.sum())
        assert np.array_equal(got[clear], want[clear]), k
        s = got.astype(np.float32)
    assert clear_total > 0.98 * steps * R * L * L


@pytest.mark.parametrize("kind", ["ferro", "glass"])
def test_comparison_of_the_three_methods(kind):
    """From random +-1 states (energy ~ 0): every method lowers the energy;
    the gradient-only descent stalls in a local minimum above the annealed
    Monte Carlo; the best state DMC visits is at least as low as the
    gradient's."""
    rng = np.random.default_rng(21)
    R, L, steps = 8, 32, 60
    s0 = torch.tensor(rng.choice([-1.0, 1.0], size=(R, L, L)).astype(np.float32), device="cuda")
    Jx, Jy = _couplings(rng, R, L, L, kind)
    o = _opt(Jx, Jy, 0.0, seed=3)
    res = o.compare(s0, steps)
    e_start = res["mc"][0][0].mean()
    assert abs(e_start) < 0.2
    for m in ("mc", "gradient", "dmc"):
        assert res[m][1].mean() < e_start - 0.8, m
    assert res["gradient"][0][-1].mean() > res["mc"][0][-1].mean()
    assert res["dmc"][1].mean() <= res["gradient"][1].mean()
