"""GPU parity of the multispin-coded Ising chain (32 replicas per uint32,
shared random words) against the oracle: initial words, whole runs and the
per-replica statistics bit-exact, resumed counters, observables."""
import numpy as np
import pytest

from oracle import chain as orc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _grp(Ly, Lx, Jx, Jy, h, beta, rid):
    return dict(model=5, Lx=Lx, Ly=Ly, Jx=Jx, Jy=Jy, h=h, beta=beta, rid=rid)


@pytest.mark.parametrize("shapes", [
    [(2, 8), (6, 16), (8, 8)],
    [(64, 40), (130, 128)],  # several workgroups per group, ragged tails
])
def test_msc_runs_match_oracle(shapes):
    from paper_2304_01772_amd.sampler import Sampler
    params = [(1.0, 1.0, 0.0, 0.4407), (0.7, -0.3, 0.05, 0.9), (1.2, 0.4, -0.1, 0.3)]
    groups = [_grp(Ly, Lx, *params[i % 3], 40 + i) for i, (Ly, Lx) in enumerate(shapes)]
    seed = 0xBEEF_0042
    smp = Sampler(groups, seed, init=True)
    assert smp.R == 32 * len(groups)
    init = [smp.get_state(g) for g in range(len(groups))]
    for g, (Ly, Lx) in enumerate(shapes):
        assert np.array_equal(init[g], orc.msc_init(Lx, Ly, seed, 40 + g)), g
    n = 5
    st = smp.sweep(n, 1).cpu().numpy()
    st2 = smp.sweep(4, 4).cpu().numpy()
    stats, obs = smp.measure()
    stats, obs = stats.cpu().numpy(), obs.cpu().numpy()
    for g, (Ly, Lx) in enumerate(shapes):
        Jx, Jy, h, beta = params[g % 3]
        w1, ost = orc.msc_run(init[g], Jx, Jy, h, beta, seed, 40 + g, 0, n, 1)
        assert np.array_equal(st[:, 32 * g:32 * g + 32], ost), g
        w2, ost2 = orc.msc_run(w1, Jx, Jy, h, beta, seed, 40 + g, n, 4, 4)
        assert np.array_equal(smp.get_state(g), w2), g
        assert np.array_equal(st2[:, 32 * g:32 * g + 32], ost2), g
        want = orc.msc_stats(w2)
        assert np.array_equal(stats[32 * g:32 * g + 32], want)
        N = Ly * Lx
        for b in (0, 17, 31):
            M, Bx, By = want[b, :3]
            e = -(float(np.float32(Jx)) * Bx + float(np.float32(Jy)) * By
                  + float(np.float32(h)) * M) / N
            assert abs(obs[32 * g + b, 0] - e) < 1e-12
    smp.close()


def test_msc_set_state_and_thresholds():
    from paper_2304_01772_amd.sampler import Sampler
    smp = Sampler([_grp(4, 16, 0.9, 0.6, 0.0, 0.5, 3)], 7, init=False)
    assert np.all(smp.get_state(0) == 0)
    T, _ = smp.thresholds(0)
    assert np.array_equal(T, orc.ising_table(np.float32(0.9), np.float32(0.6), 0.0, 0.5))
    rng = np.random.default_rng(0)
    w = rng.integers(0, 2 ** 32, size=(4, 16), dtype=np.uint64).astype(np.uint32)
    smp.set_state(0, w)
    smp.sweep(3)
    want, _ = orc.msc_run(w, 0.9, 0.6, 0.0, 0.5, 7, 3, 0, 3)
    assert np.array_equal(smp.get_state(0), want)
    smp.close()
    with pytest.raises(Exception):
        Sampler([_grp(4, 12, 1.0, 1.0, 0.0, 0.5, 0)], 1)  # Lx not a multiple of 8
