"""GPU differentiable Monte Carlo (relaxed chain of Algorithm 2): forward and
reverse-mode gradients against the FP64 oracle, the hard limit against the
oracle's Metropolis decisions, and the spin-pattern optimisation."""
import numpy as np
import pytest

from oracle import dmc as odmc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(seed, R, Ly, Lx):
    rng = np.random.default_rng(seed)
    s0 = rng.uniform(-1, 1, size=(R, Ly, Lx)).astype(np.float32)
    Jx = rng.uniform(0.1, 0.9, size=(R, Ly, Lx)).astype(np.float32)
    Jy = rng.uniform(-0.5, 0.9, size=(R, Ly, Lx)).astype(np.float32)
    g = rng.normal(size=(R, Ly, Lx)).astype(np.float32)
    return s0, Jx, Jy, g


@pytest.mark.parametrize("R,Ly,Lx,alpha,beta,n", [
    (3, 6, 8, 4.0, 0.5, 4), (2, 16, 32, 10.0, 0.8, 3), (2, 2, 2, 2.0, 1.0, 5),
    (1, 10, 6, 0.5, 0.3, 6)])
def test_forward_and_backward_match_oracle(R, Ly, Lx, alpha, beta, n):
    from paper_2304_01772_amd.dmc import relaxed_ising
    s0, Jx, Jy, g = _case(R * 1000 + Lx, R, Ly, Lx)
    beta32, alpha32, h32 = float(np.float32(beta)), float(np.float32(alpha)), float(np.float32(0.03))
    seed, t0, rid0 = 0xDEADBEEF12345, 7, 11
    dev = "cuda"
    s0t = torch.tensor(s0, device=dev, requires_grad=True)
    jx = torch.tensor(Jx, device=dev, requires_grad=True)
    jy = torch.tensor(Jy, device=dev, requires_grad=True)
    s = relaxed_ising(s0t, jx, jy, beta32, alpha32, h32, n, seed, t0, rid0)
    (s * torch.tensor(g, device=dev)).sum().backward()
    torch.cuda.synchronize()
    rids = [rid0 + r for r in range(R)]
    want, gs0, gJx, gJy, _ = odmc.forward_backward(s0, Jx, Jy, h32, beta32, alpha32, seed, rids,
                                                   t0, n, g)
    np.testing.assert_allclose(s.detach().cpu().numpy(), want, rtol=0, atol=2e-5)
    for got, ref in ((s0t.grad, gs0), (jx.grad, gJx), (jy.grad, gJy)):
        got = got.cpu().numpy()
        scale = max(1.0, float(np.abs(ref).max()))
        np.testing.assert_allclose(got, ref, rtol=0, atol=2e-4 * scale)


def test_hard_limit_equals_oracle_metropolis_chain():
    """alpha = 1e9 saturates q at 0 or 1 in FP32: the spins stay at +-1 and
    equal the oracle's hard-limit chain site by site."""
    from paper_2304_01772_amd.dmc import relaxed_ising
    rng = np.random.default_rng(3)
    R, L, n = 4, 32, 10
    s0 = rng.choice([-1.0, 1.0], size=(R, L, L)).astype(np.float32)
    J = np.full((R, L, L), 1.0, np.float32)
    s = relaxed_ising(torch.tensor(s0, device="cuda"), torch.tensor(J, device="cuda"),
                      torch.tensor(J, device="cuda"), 0.42, 1e9, 0.0, n, 5, 0, 0)
    got = s.cpu().numpy()
    assert np.all(np.abs(got) == 1.0)
    want = odmc.forward(torch.tensor(s0, dtype=torch.float64), torch.tensor(J, dtype=torch.float64),
                        torch.tensor(J, dtype=torch.float64), 0.0, float(np.float32(0.42)), 1e9,
                        5, list(range(R)), 0, n).numpy()
    assert np.array_equal(got, want)


def test_spin_pattern_optimisation_lowers_the_loss():
    """Adam on the couplings (the paper's spin-pattern optimisation) drives
    the relaxed chain towards a striped target: the first losses follow the
    same optimisation run on the FP64 oracle (torch Adam), the loss falls by
    more than 30 % and the discretised lattice matches most of the target."""
    from paper_2304_01772_amd.dmc import optimise_couplings
    L, lr, beta, alpha, n_sw, seed = 16, 0.05, 1.0, 10.0, 8, 3
    y = torch.arange(L).view(-1, 1).expand(L, L)
    target = torch.where((y // 2) % 2 == 0, 1.0, -1.0).view(1, L, L)
    g = torch.Generator(device="cpu").manual_seed(0)
    s0 = torch.rand((1, L, L), generator=g) * 2 - 1
    J0 = torch.full((1, L, L), 0.5)
    _, _, hist, s_disc = optimise_couplings(target.cuda(), s0.cuda(), J0.cuda(), J0.cuda(),
                                            steps=150, lr=lr, beta=beta, alpha=alpha,
                                            n_sweeps=n_sw, seed=seed)
    # the same run on the oracle for the first steps
    Jx = J0.double().clone().requires_grad_(True)
    Jy = J0.double().clone().requires_grad_(True)
    opt = torch.optim.Adam([Jx, Jy], lr=lr)
    ref = []
    for _ in range(5):
        opt.zero_grad()
        s = odmc.forward(s0.double(), Jx, Jy, 0.0, beta, alpha, seed, [0], 0, n_sw)
        loss = ((s - target.double()) ** 2).mean()
        loss.backward()
        opt.step()
        ref.append(float(loss.detach()))
    np.testing.assert_allclose(hist[:5], ref, rtol=1e-4)
    assert hist[-1] < 0.7 * hist[0], (hist[0], hist[-1])
    assert (s_disc.cpu() == target).float().mean() > 0.75
