"""GPU parity of the triangular-lattice Ising chain (six neighbours, three
colours) against the oracle: the initial state, the states and recorded
statistics of whole runs bit-exact, and the observables."""
import numpy as np
import pytest

from oracle import chain as orc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rep(Ly, Lx, J, h, beta, rid):
    return dict(model=3, Lx=Lx, Ly=Ly, Jx=J, Jy=J, h=h, beta=beta, rid=rid)


# 3 x 3 (smallest), row counts with k-blocks across rows, several workgroups
# per replica with a ragged tail (93 x 99: 3069 blocks of 4 sites per colour)
@pytest.mark.parametrize("shapes", [
    [(3, 3), (6, 9), (9, 6)],
    [(12, 15), (3, 30)],
    [(93, 99), (30, 33)],
    # every Lx a multiple of 12: the span kernel (one row span per lane)
    [(12, 12), (6, 24), (9, 36)],
    [(99, 96), (33, 60), (3, 12)],
])
def test_tri_runs_match_oracle(shapes):
    from paper_2304_01772_amd.sampler import Sampler
    params = [(0.9, 0.05, 0.3), (-1.0, 0.0, 0.8), (1.0, -0.2, 0.2736)]
    reps = []
    for i, (Ly, Lx) in enumerate(shapes):
        J, h, beta = params[i % len(params)]
        reps.append(_rep(Ly, Lx, J, h, beta, 10 + i))
    seed = 0x5EED_1234_5678
    smp = Sampler(reps, seed, init=True)
    init = [smp.get_state(r) for r in range(len(reps))]
    for r, (Ly, Lx) in enumerate(shapes):
        want = orc.ising_init(Lx, Ly, seed, 10 + r).reshape(Ly, Lx)
        assert np.array_equal(init[r], want), r
    n, every = 7, 1
    st = smp.sweep(n, every).cpu().numpy()
    st2 = smp.sweep(5, 5).cpu().numpy()  # resumes at sweep counter 7
    stats, obs = smp.measure()
    stats, obs = stats.cpu().numpy(), obs.cpu().numpy()
    for r, (Ly, Lx) in enumerate(shapes):
        J, h, beta = params[r % len(params)]
        s1, ost = orc.tri_run(init[r], J, h, beta, seed, 10 + r, 0, n, every)
        assert np.array_equal(st[:, r], ost), r
        s2, ost2 = orc.tri_run(s1, J, h, beta, seed, 10 + r, n, 5, 5)
        assert np.array_equal(smp.get_state(r), s2), r
        assert np.array_equal(st2[:, r], ost2), r
        M, Bh, Bv, Bd = orc.tri_stats(s2)[:4]
        assert np.array_equal(stats[r][:4], [M, Bh, Bv, Bd])
        N = Ly * Lx
        e = -(float(np.float32(J)) * float(Bh + Bv + Bd) + float(np.float32(h)) * float(M)) / N
        assert abs(obs[r, 0] - e) < 1e-12 and abs(obs[r, 1] - abs(M) / N) < 1e-15
    smp.close()


def test_tri_thresholds_and_set_state():
    from paper_2304_01772_amd.sampler import Sampler
    reps = [_rep(6, 6, 0.7, 0.1, 0.45, 0), _rep(9, 12, -0.4, 0.0, 1.3, 1)]
    smp = Sampler(reps, 3, init=False)
    for r, d in enumerate(reps):
        T, _ = smp.thresholds(r)
        assert np.array_equal(T, orc.tri_table(np.float32(d["Jx"]), np.float32(d["h"]),
                                               d["beta"]))
        assert np.all(smp.get_state(r) == -1)  # init = 0: every spin -1
    rng = np.random.default_rng(0)
    s = rng.choice([-1, 1], size=(9, 12)).astype(np.int8)
    smp.set_state(1, s)
    smp.sweep(3)
    want, _ = orc.tri_run(s, np.float32(-0.4), 0.0, 1.3, 3, 1, 0, 3)
    assert np.array_equal(smp.get_state(1), want)
    with pytest.raises(Exception):
        smp.set_state(1, np.zeros((9, 12), np.int8))
    smp.close()


@pytest.mark.parametrize("mode", ["auto", "stream"])
def test_tri_unrecorded_sweeps_resident_and_streamed(mode):
    """Unrecorded sweeps run resident in LDS (every Lx a multiple of 12,
    lattices <= 64 KiB) unless the stream schedule is set; both equal the
    oracle, across two calls (the sweep counter carries over)."""
    from paper_2304_01772_amd.sampler import Sampler
    shapes = [(12, 12), (96, 96), (30, 36), (180, 180)]
    reps = [_rep(Ly, Lx, 1.0, 0.0, 0.2747, 60 + i) for i, (Ly, Lx) in enumerate(shapes)]
    smp = Sampler(reps, 21, init=True)
    if mode == "stream":
        smp.set_schedule(mode="stream")
    init = [smp.get_state(r) for r in range(len(reps))]
    smp.sweep(13)
    smp.sweep(7)
    for r, (Ly, Lx) in enumerate(shapes):
        want, _ = orc.tri_run(init[r], 1.0, 0.0, 0.2747, 21, 60 + r, 0, 20)
        assert np.array_equal(smp.get_state(r), want), (mode, r)
    smp.close()


def test_tri_large_batch_streamed_two_blocks_per_lane():
    """Large streamed passes (here 1368 replicas, 192 x 192 but the first
    180 x 180, a ragged last workgroup; over 2^22 Philox blocks per pass)
    give each lane two blocks; 6 x 1368 workgroups, a multiple of 8, take the
    XCD-grouped order.  Sampled replicas equal the oracle bit for bit."""
    from paper_2304_01772_amd.sampler import Sampler
    n_rep = 1368
    shapes = [(180, 180)] + [(192, 192)] * (n_rep - 1)
    reps = [_rep(Ly, Lx, 1.0, 0.05, 0.2747, 500 + i) for i, (Ly, Lx) in enumerate(shapes)]
    smp = Sampler(reps, 23, init=True)
    smp.set_schedule(mode="stream")
    picks = [0, 1, 683, n_rep - 1]
    init = {r: smp.get_state(r) for r in picks}
    smp.sweep(3)
    for r in picks:
        want, _ = orc.tri_run(init[r], 1.0, 0.05, 0.2747, 23, 500 + r, 0, 3)
        assert np.array_equal(smp.get_state(r), want), r
    smp.close()


def test_tri_streamed_xcd_order_small_grid():
    """Eight replicas of one workgroup each (24 x 24 and 36 x 48): the
    streamed grid of 8 workgroups takes the XCD-grouped order; recorded
    states and statistics equal the oracle's."""
    from paper_2304_01772_amd.sampler import Sampler
    shapes = [(24, 24)] * 4 + [(36, 48)] * 4
    reps = [_rep(Ly, Lx, 0.8, 0.1, 0.5, 300 + i) for i, (Ly, Lx) in enumerate(shapes)]
    smp = Sampler(reps, 31, init=True)
    smp.set_schedule(mode="stream")
    init = [smp.get_state(r) for r in range(len(reps))]
    st = smp.sweep(6, 2).cpu().numpy()
    for r in range(len(reps)):
        want, ost = orc.tri_run(init[r], 0.8, 0.1, 0.5, 31, 300 + r, 0, 6, 2)
        assert np.array_equal(smp.get_state(r), want), r
        assert np.array_equal(st[:, r], ost), r
    smp.close()
