"""GPU parity of the Ising and Potts sweeps against the oracle.

Lattice states and integer statistics must be bit-identical to the oracle
for the same seed, replica ids and sweep counter; FP64 observables agree to
1e-12 relative.  Cases cover both kernel paths (16-byte SWAR chunks when
Lx/2 is a multiple of 16, per-site otherwise), both schedules (resident in
LDS, streamed colour passes with several row-tile heights), ragged tiles,
tiny and degenerate lattices, resume across calls, and mixed batches.
"""
import numpy as np
import pytest

import synth
from oracle import chain as orc
from oracle import observables as oobs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def S():
    from paper_2304_01772_amd.sampler import Sampler
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return Sampler


def _run_oracle(rep, state, seed, t0, n, re):
    if rep["model"] == 0:
        return orc.ising_run(state, rep["Jx"], rep["Jy"], rep["h"], rep["beta"], seed, rep["rid"],
                             t0, n, re)
    return orc.potts_run(state, rep["q"], rep["Jx"], rep["h"], rep["beta"], seed, rep["rid"], t0,
                         n, re)


def _init_oracle(rep, seed):
    if rep["model"] == 0:
        return orc.ising_init(rep["Lx"], rep["Ly"], seed, rep["rid"])
    return orc.potts_init(rep["Lx"], rep["Ly"], rep["q"], seed, rep["rid"])


def _f32(x):
    return float(np.float32(x))


def _check_batch(S, reps, seed, n, re, schedule=None, split=None):
    smp = S(reps, seed, init=True)
    if schedule:
        smp.set_schedule(**schedule)
    states = [_init_oracle(r, seed) for r in reps]
    for i in range(len(reps)):
        assert np.array_equal(smp.get_state(i), states[i]), f"init differs, replica {i}"
    calls = split or [n]
    t0 = 0
    for m in calls:
        st = smp.sweep(m, re)
        torch.cuda.synchronize()
        for i, r in enumerate(reps):
            states[i], ost = _run_oracle(r, states[i], seed, t0, m, re)
            got = smp.get_state(i)
            assert np.array_equal(got, states[i]), f"state differs: replica {i} {r} t0={t0}"
            if re > 0:
                g = st[:, i, :].cpu().numpy()
                assert np.array_equal(g, ost), f"stats differ: replica {i}"
        t0 += m
    assert smp.t == t0
    smp.close()


def test_single_ising_32x32_1000_sweeps(S):
    """32x32 periodic Ising, J=1, h=0, beta=0.44, 1000 sweeps, E/site and
    |M|/site after every sweep: bit-identical chain and FP64 observables."""
    cfg = synth.single_ising()
    rep = dict(model=0, Lx=32, Ly=32, q=2, Jx=1.0, Jy=1.0, h=0.0, beta=cfg["beta"], rid=0)
    smp = S([rep], cfg["seed"], init=True)
    st = smp.sweep(cfg["n_sweeps"], 1)
    torch.cuda.synchronize()
    s0 = orc.ising_init(32, 32, cfg["seed"], 0)
    want, ost = orc.ising_run(s0, 1.0, 1.0, 0.0, cfg["beta"], cfg["seed"], 0, 0, cfg["n_sweeps"], 1)
    assert np.array_equal(smp.get_state(0), want)
    g = st[:, 0, :].cpu().numpy()
    assert np.array_equal(g, ost)
    eo = oobs.ising(ost, 1.0, 1.0, 0.0, 1024)
    eg = oobs.ising(g, 1.0, 1.0, 0.0, 1024)
    np.testing.assert_allclose(eg["e"], eo["e"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(eg["absm"], eo["absm"], rtol=1e-12, atol=0)
    # device FP64 observables of the final state
    stats, obs = smp.measure()
    o = obs.cpu().numpy()[0]
    ref = oobs.ising(orc.ising_stats(want), 1.0, 1.0, 0.0, 1024)
    assert abs(o[0] - ref["e"]) <= 1e-12 * abs(ref["e"])
    assert abs(o[1] - ref["absm"]) <= 1e-12 * max(abs(ref["absm"]), 1e-300)


ISING_SHAPES = [(4, 4), (2, 2), (6, 8), (8, 2), (2, 10), (32, 32), (32, 64), (64, 32), (96, 34),
                (34, 96), (128, 128)]


@pytest.mark.parametrize("mode", ["resident", "stream"])
@pytest.mark.parametrize("shape", ISING_SHAPES)
def test_ising_shapes(S, shape, mode):
    Lx, Ly = shape
    rng = np.random.default_rng(Lx * 1000 + Ly)
    reps = []
    for i in range(3):
        reps.append(dict(model=0, Lx=Lx, Ly=Ly, q=2, Jx=_f32(rng.uniform(0.2, 1.5)),
                         Jy=_f32(rng.uniform(0.2, 1.5)), h=_f32(rng.uniform(-0.3, 0.3)),
                         beta=float(rng.uniform(0.1, 1.2)), rid=int(rng.integers(0, 2 ** 32))))
    _check_batch(S, reps, seed=int(rng.integers(1, 2 ** 63)), n=13, re=3,
                 schedule=dict(mode=mode))


@pytest.mark.parametrize("tile_rows", [2, 6, 16, 0])
@pytest.mark.parametrize("threads", [256, 512])
def test_ising_stream_tiling_invariance(S, tile_rows, threads):
    """Streamed colour passes with several row-tile heights (ragged last
    tile) and workgroup sizes give the oracle's bits."""
    reps = [dict(model=0, Lx=Lx, Ly=Ly, q=2, Jx=1.0, Jy=0.7, h=0.05, beta=0.5, rid=i)
            for i, (Lx, Ly) in enumerate([(32, 30), (64, 64), (160, 22), (32, 2)])]
    _check_batch(S, reps, seed=99, n=9, re=2,
                 schedule=dict(mode="stream", tile_rows=tile_rows, wg_threads=threads))


POTTS_CASES = [(2, (32, 32)), (3, (32, 32)), (4, (64, 32)), (8, (32, 64)), (37, (32, 34)),
               (128, (64, 64)), (3, (4, 4)), (5, (6, 10)), (3, (2, 2))]


@pytest.mark.parametrize("mode", ["resident", "stream"])
@pytest.mark.parametrize("q,shape", POTTS_CASES)
def test_potts(S, q, shape, mode):
    Lx, Ly = shape
    rng = np.random.default_rng(q * 7919 + Lx)
    reps = [dict(model=1, Lx=Lx, Ly=Ly, q=q, Jx=_f32(J), Jy=_f32(J), h=_f32(h),
                 beta=float(b) * np.log1p(np.sqrt(q)), rid=int(rng.integers(0, 2 ** 32)))
            for J, h, b in [(1.0, 0.0, 1.0), (0.8, 0.1, 1.3), (1.2, -0.05, 0.7)]]
    _check_batch(S, reps, seed=int(rng.integers(1, 2 ** 63)), n=11, re=4,
                 schedule=dict(mode=mode))


def test_mixed_batch_resume_and_streaming(S):
    """Ising and Potts replicas in one context, resumed across calls,
    streamed; the chain equals one uninterrupted oracle run."""
    reps = []
    for i, (m, L, q) in enumerate([(0, 64, 2), (1, 32, 3), (0, 32, 2), (1, 64, 8), (1, 96, 4)]):
        reps.append(dict(model=m, Lx=L, Ly=L, q=q, Jx=1.0, Jy=1.0, h=0.0,
                         beta=0.44 if m == 0 else 1.0, rid=10 + i))
    _check_batch(S, reps, seed=5, n=12, re=1, schedule=dict(mode="stream", tile_rows=8),
                 split=[5, 0, 7])


def test_set_state_roundtrip_and_validation(S):
    from paper_2304_01772_amd import SpinmcError
    reps = [dict(model=0, Lx=8, Ly=6, rid=0, beta=0.3), dict(model=1, Lx=32, Ly=4, q=5, rid=1,
                                                              beta=1.0)]
    smp = S(reps, 3, init=False)
    rng = np.random.default_rng(0)
    a = synth.random_ising(6, 8, rng)
    b = synth.random_potts(4, 32, 5, rng)
    smp.set_state(0, a)
    smp.set_state(1, b)
    assert np.array_equal(smp.get_state(0), a)
    assert np.array_equal(smp.get_state(1), b)
    bad = a.copy()
    bad[0, 0] = 0
    with pytest.raises(SpinmcError):
        smp.set_state(0, bad)
    assert np.array_equal(smp.get_state(0), a)
    badp = b.copy()
    badp[1, 1] = 5
    with pytest.raises(SpinmcError):
        smp.set_state(1, badp)
    smp.close()


def test_thresholds_bitwise_equal_to_oracle(S):
    reps = [dict(model=0, Lx=8, Ly=8, Jx=_f32(0.37), Jy=_f32(1.21), h=_f32(-0.07), beta=0.83,
                 rid=0),
            dict(model=1, Lx=8, Ly=8, q=7, Jx=_f32(0.9), Jy=_f32(0.9), h=_f32(0.11), beta=1.7,
                 rid=1)]
    smp = S(reps, 1)
    T0, _ = smp.thresholds(0)
    T1, _ = smp.thresholds(1)
    assert np.array_equal(T0, orc.ising_table(reps[0]["Jx"], reps[0]["Jy"], reps[0]["h"], 0.83))
    assert np.array_equal(T1, orc.potts_table(7, reps[1]["Jx"], reps[1]["h"], 1.7))
    smp.close()


def test_measure_matches_oracle_stats(S):
    rng = np.random.default_rng(4)
    reps = [dict(model=0, Lx=32, Ly=16, Jx=_f32(0.9), Jy=_f32(1.1), h=_f32(0.2), beta=0.4, rid=0),
            dict(model=1, Lx=64, Ly=32, q=6, Jx=1.0, Jy=1.0, h=0.1, beta=1.0, rid=1),
            dict(model=0, Lx=6, Ly=4, Jx=1.0, Jy=1.0, h=0.0, beta=0.4, rid=2)]
    smp = S(reps, 8, init=False)
    st = [synth.random_ising(16, 32, rng), synth.random_potts(32, 64, 6, rng),
          synth.random_ising(4, 6, rng)]
    for i, s in enumerate(st):
        smp.set_state(i, s)
    stats, obs = smp.measure()
    stats = stats.cpu().numpy()
    obs = obs.cpu().numpy()
    assert np.array_equal(stats[0], orc.ising_stats(st[0]))
    assert np.array_equal(stats[1], orc.potts_stats(st[1], 6))
    assert np.array_equal(stats[2], orc.ising_stats(st[2]))
    e0 = oobs.ising(stats[0], _f32(0.9), _f32(1.1), _f32(0.2), 512)
    assert abs(obs[0, 0] - e0["e"]) <= 1e-12 * abs(e0["e"])
    p1 = oobs.potts(stats[1], 6, 1.0, _f32(0.1), 2048)
    assert abs(obs[1, 0] - p1["e"]) <= 1e-12 * abs(p1["e"])
    assert abs(obs[1, 1] - p1["mP"]) <= 1e-12 * max(abs(p1["mP"]), 1e-300)
    smp.close()


def test_invalid_arguments_leave_no_state(S):
    from paper_2304_01772_amd import SpinmcError
    with pytest.raises(SpinmcError):
        S([dict(model=0, Lx=7, Ly=8)], 1)
    with pytest.raises(SpinmcError):
        S([dict(model=1, Lx=8, Ly=8, q=1)], 1)
    with pytest.raises(SpinmcError):
        S([dict(model=0, Lx=8, Ly=8, beta=float("nan"))], 1)
    smp = S([dict(model=0, Lx=8, Ly=8, beta=0.5)], 1)
    before = smp.get_state(0)
    with pytest.raises(SpinmcError):
        smp.sweep(-1)
    with pytest.raises(SpinmcError):
        smp.set_schedule(mode="stream", tile_rows=3)
    assert np.array_equal(smp.get_state(0), before) and smp.t == 0
    smp.close()


def test_hybrid_graphs_and_autotune_keep_the_chain(S):
    """Hybrid schedule (LDS-resident small lattices concurrent with streamed
    large ones) replayed from captured graphs of 50-sweep chunks plus a
    remainder; the autotuner times candidates on a scratch copy and leaves
    the state and sweep counter untouched."""
    reps = [dict(model=0, Lx=512, Ly=512, Jx=1.0, Jy=1.0, h=0.0, beta=0.44, rid=0),
            dict(model=1, Lx=512, Ly=256, q=4, Jx=1.0, Jy=1.0, h=0.0, beta=1.1, rid=1),
            dict(model=0, Lx=64, Ly=64, Jx=1.0, Jy=1.0, h=0.0, beta=0.3, rid=2),
            dict(model=1, Lx=32, Ly=32, q=3, Jx=1.0, Jy=1.0, h=0.0, beta=1.0, rid=3),
            dict(model=0, Lx=6, Ly=10, Jx=1.0, Jy=1.0, h=0.0, beta=0.5, rid=4)]
    seed = 77
    smp = S(reps, seed, init=True)
    smp.set_schedule(mode="hybrid")
    states = [_init_oracle(r, seed) for r in reps]
    t0 = 0
    for n in (60, 7):
        smp.sweep(n)
        torch.cuda.synchronize()
        for i, r in enumerate(reps):
            states[i], _ = _run_oracle(r, states[i], seed, t0, n, 0)
            assert np.array_equal(smp.get_state(i), states[i]), (n, i)
        t0 += n
    chosen, rates = smp.autotune(trial_sweeps=3)
    assert len(rates) >= 2 and all(r > 0 for r in rates)
    assert smp.t == t0
    for i in range(len(reps)):
        assert np.array_equal(smp.get_state(i), states[i])
    smp.sweep(5)
    torch.cuda.synchronize()
    for i, r in enumerate(reps):
        states[i], _ = _run_oracle(r, states[i], seed, t0, 5, 0)
        assert np.array_equal(smp.get_state(i), states[i]), (chosen, i)
    smp.close()


@pytest.mark.parametrize("shape,n", [((32, 32), 2048), ((6, 10), 1101), ((64, 64), 1027)])
def test_resident_packing_many_small_replicas(S, shape, n):
    """Enough replicas of one small shape that the resident kernel packs
    several per workgroup (each with its own thresholds and LDS slot)."""
    Lx, Ly = shape
    rng = np.random.default_rng(n + Lx)
    reps = [dict(model=int(i % 3 == 0), Lx=Lx, Ly=Ly, q=int(rng.integers(2, 9)),
                 Jx=1.0, Jy=1.0, h=0.0, beta=float(rng.uniform(0.2, 1.5)), rid=i) for i in range(n)]
    for r in reps:
        if r["model"] == 0:
            r["Jx"] = r["Jy"] = _f32(rng.uniform(0.5, 1.5))
    seed = 1234
    smp = S(reps, seed, init=True)
    smp.set_schedule(mode="resident")
    st = smp.sweep(12, 4)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    ising = [i for i, r in enumerate(reps) if r["model"] == 0]
    potts = [i for i, r in enumerate(reps) if r["model"] == 1]
    si = [orc.ising_init(Lx, Ly, seed, reps[i]["rid"]) for i in ising]
    out_i, st_i = orc.ising_run_batch(si, [reps[i]["Jx"] for i in ising], [reps[i]["Jy"] for i in ising],
                                      [0.0] * len(ising), [reps[i]["beta"] for i in ising], seed,
                                      np.array([reps[i]["rid"] for i in ising]), 0, 12, 4)
    sp = [orc.potts_init(Lx, Ly, reps[i]["q"], seed, reps[i]["rid"]) for i in potts]
    out_p, st_p = orc.potts_run_batch(sp, [reps[i]["q"] for i in potts], [1.0] * len(potts),
                                      [0.0] * len(potts), [reps[i]["beta"] for i in potts], seed,
                                      np.array([reps[i]["rid"] for i in potts]), 0, 12, 4)
    for k, i in enumerate(ising):
        assert np.array_equal(st[:, i], st_i[k]), i
    for k, i in enumerate(potts):
        assert np.array_equal(st[:, i], st_p[k]), i
    for k, i in list(enumerate(ising))[:50] + list(enumerate(ising))[-50:]:
        assert np.array_equal(smp.get_state(i), out_i[k])
    for k, i in list(enumerate(potts))[:50] + list(enumerate(potts))[-50:]:
        assert np.array_equal(smp.get_state(i), out_p[k])
    smp.close()


@pytest.mark.parametrize("nt", [True, False])
def test_nontemporal_streaming_keeps_the_chain(S, nt):
    """Streamed Ising and Potts passes with the own-plane loads and stores
    nontemporal (forced on) or cached (forced off): the same chain as the
    oracle, with and without recording, resumed across calls."""
    rng = np.random.default_rng(77 + int(nt))
    reps = [dict(model=0, Lx=64, Ly=48, q=2, Jx=_f32(0.9), Jy=_f32(1.1), h=_f32(0.02), beta=0.45,
                 rid=3),
            dict(model=1, Lx=96, Ly=32, q=5, Jx=1.0, Jy=1.0, h=0.0, beta=1.2, rid=9),
            dict(model=1, Lx=32, Ly=64, q=3, Jx=_f32(0.7), Jy=_f32(0.7), h=_f32(0.05), beta=1.0,
                 rid=11)]
    _check_batch(S, reps, seed=int(rng.integers(1, 2 ** 62)), n=9, re=3,
                 schedule=dict(mode="stream", tile_rows=8, nt=nt), split=[6, 3])
    _check_batch(S, reps, seed=int(rng.integers(1, 2 ** 62)), n=7, re=0,
                 schedule=dict(mode="stream", nt=nt), split=[5, 2])


# Persistent streamed passes: whole replicas packed per workgroup and row
# slabs that wait on their neighbours' pass flags, across graph-chunk
# boundaries (50 sweeps), recorded calls in between (one launch per pass),
# thin (2-row), ragged and two-slab replicas, and the hybrid schedule with
# resident groups running beside them.
def _pers_batch(kind):
    rng = np.random.default_rng(5)
    reps = []
    if kind in ("ising", "mixed"):
        for i, (lx, ly) in enumerate([(64, 64), (64, 64), (128, 64), (32, 128), (64, 130), (256, 32),
                                      (512, 512)]):
            reps.append(dict(model=0, Lx=lx, Ly=ly, Jx=_f32(rng.uniform(0.2, 0.6)),
                             Jy=_f32(rng.uniform(0.2, 0.6)), h=_f32(rng.uniform(-0.1, 0.1)),
                             beta=1.0, rid=i))
    if kind in ("potts", "mixed"):
        for i, (lx, ly, q) in enumerate([(64, 64, 3), (96, 48, 8), (32, 70, 5), (128, 128, 4),
                                         (384, 384, 6)]):
            reps.append(dict(model=1, Lx=lx, Ly=ly, q=q, Jx=1.0, Jy=1.0,
                             h=0.0 if i % 2 == 0 else _f32(0.05), beta=float(rng.uniform(0.8, 1.3)),
                             rid=100 + i))
    return reps


@pytest.mark.parametrize("kind,mode,tile_rows", [
    ("ising", "stream", 0), ("ising", "stream", 6), ("ising", "stream", 64),
    ("potts", "stream", 0), ("potts", "stream", 16), ("mixed", "hybrid", 0),
    ("mixed", "stream", 32)])
def test_persistent_schedule_keeps_the_chain(S, kind, mode, tile_rows):
    reps = _pers_batch(kind)
    _check_batch(S, reps, seed=41, n=None, re=0,
                 schedule=dict(mode=mode, tile_rows=tile_rows, persistent=True),
                 split=[120, 7, 53])
    # recorded sweeps (one launch per pass) between persistent chunks
    smp = S(reps, 42, init=True)
    smp.set_schedule(mode=mode, tile_rows=tile_rows, persistent=True)
    states = [_init_oracle(r, 42) for r in reps]
    t0 = 0
    for m, re in ((60, 0), (6, 3), (51, 0)):
        st = smp.sweep(m, re)
        torch.cuda.synchronize()
        for i, r in enumerate(reps):
            states[i], ost = _run_oracle(r, states[i], 42, t0, m, re)
            assert np.array_equal(smp.get_state(i), states[i]), f"replica {i} after {t0 + m}"
            if re:
                assert np.array_equal(st[:, i].cpu().numpy(), ost)
        t0 += m
    smp.close()


def test_persistent_schedule_direct_launches_and_profile(S):
    """Profiled (direct, per-launch timed) persistent chunks in the hybrid
    schedule: chunks of 50 sweeps with a sweep offset inside the call."""
    reps = _pers_batch("mixed")
    smp = S(reps, 43, init=True)
    smp.set_schedule(mode="hybrid", persistent=True)
    smp.profile(True)
    smp.sweep(110)
    torch.cuda.synchronize()
    ms_i, n_i = smp.profile_read("persist_ising")
    ms_p, n_p = smp.profile_read("persist_potts")
    smp.profile(False)
    assert n_i == 3 and n_p == 3 and ms_i > 0 and ms_p > 0
    for i, r in enumerate(reps):
        want, _ = _run_oracle(r, _init_oracle(r, 43), 43, 0, 110, 0)
        assert np.array_equal(smp.get_state(i), want), f"replica {i}"
    smp.close()


@pytest.mark.parametrize("rpb", [1, 2, 4, 8])
def test_forced_resident_packing_keeps_the_chain(S, rpb):
    """Replicas per resident workgroup forced by the schedule (the
    autotuner's rpb candidates), for a group larger and one smaller than the
    packing, recorded and not."""
    rng = np.random.default_rng(rpb)
    reps = [dict(model=0, Lx=64, Ly=32, Jx=_f32(rng.uniform(0.3, 0.6)), Jy=0.5, h=0.0,
                 beta=1.0, rid=i) for i in range(11)]
    reps += [dict(model=1, Lx=32, Ly=32, q=5, Jx=1.0, Jy=1.0, h=0.0, beta=1.2, rid=50 + i)
             for i in range(3)]
    _check_batch(S, reps, seed=7 + rpb, n=None, re=0,
                 schedule=dict(mode="resident", rpb=rpb), split=[30, 4])
    _check_batch(S, reps, seed=8 + rpb, n=6, re=2, schedule=dict(mode="resident", rpb=rpb))


def test_autotune_cache_and_bypass(S):
    """A second context with the same shapes reuses the first one's choice
    without trials; cache=False times the candidates again; the chain is
    unchanged either way."""
    reps = [dict(model=0, Lx=64, Ly=64, Jx=1.0, Jy=1.0, h=0.0, beta=0.4, rid=i) for i in range(5)]
    reps += [dict(model=1, Lx=160, Ly=96, q=3, Jx=1.0, Jy=1.0, h=0.0, beta=1.0, rid=9)]
    a = S(reps, 3, init=True)
    chosen_a, rates_a = a.autotune(trial_sweeps=2)
    assert len(rates_a) > 0
    b = S(reps, 3, init=True)
    chosen_b, rates_b = b.autotune(trial_sweeps=2)
    assert rates_b == [] and chosen_b == chosen_a and b.get_schedule() == chosen_a
    chosen_c, rates_c = b.autotune(trial_sweeps=2, cache=False)
    assert len(rates_c) > 0
    b.sweep(12)
    torch.cuda.synchronize()
    for i, r in enumerate(reps):
        want, _ = _run_oracle(r, _init_oracle(r, 3), 3, 0, 12, 0)
        assert np.array_equal(b.get_state(i), want)
    a.close()
    b.close()


def test_zero_sweeps_and_schedule_boundaries(S):
    """Degenerate calls and the LDS-residency boundary: zero sweeps change
    nothing; a lattice of exactly 128 KiB stays resident and one two rows
    larger is streamed under the hybrid schedule, both on the oracle's chain;
    q above 128 is rejected."""
    from paper_2304_01772_amd import SpinmcError
    reps = [dict(model=0, Lx=512, Ly=256, q=2, Jx=1.0, Jy=1.0, h=0.0, beta=0.42, rid=5),
            dict(model=0, Lx=512, Ly=258, q=2, Jx=1.0, Jy=1.0, h=0.0, beta=0.42, rid=6),
            dict(model=1, Lx=256, Ly=512, q=4, Jx=1.0, Jy=1.0, h=0.0, beta=1.1, rid=7)]
    smp = S(reps, 99, init=True)
    smp.set_schedule(mode="hybrid")
    streamed, resident = smp.schedule_sites(by_model=True)
    assert resident["ising"] == 512 * 256 and streamed["ising"] == 512 * 258
    assert resident["potts"] == 256 * 512 and streamed["potts"] == 0
    before = [smp.get_state(i) for i in range(3)]
    smp.sweep(0)
    st = smp.sweep(0, 1)
    torch.cuda.synchronize()
    assert smp.t == 0 and st.shape[0] == 0
    for i in range(3):
        assert np.array_equal(smp.get_state(i), before[i])
    smp.close()
    _check_batch(S, reps, seed=99, n=4, re=2, schedule=dict(mode="hybrid"), split=[3, 1])
    with pytest.raises(SpinmcError):
        S([dict(model=1, Lx=32, Ly=32, q=129)], 1)


def test_batched_workload_full_size_sampled(S):
    """The benchmark's batched workload at full size (1024 Ising 256^2 + 512
    Potts up to 1024^2) under its tuned schedule, sweeps replayed as graphs
    and recorded: sampled replicas, among them the largest Potts lattices,
    bit-exact with the oracle; every replica's recorded statistics equal a
    recount of its final state."""
    reps = synth.batched_ising_potts()
    seed, n = 2, 7
    smp = S(reps, seed, init=True)
    smp.autotune(trial_sweeps=2)
    smp.sweep(5)                 # graph replays (5-sweep chunk)
    st = smp.sweep(2, 2)         # one recorded sweep pair, direct launches
    torch.cuda.synchronize()
    big = [i for i, r in enumerate(reps) if r["model"] == 1 and r["Lx"] == 1024][:2]
    sample = [0, 517, 1023, 1024, 1535] + big
    for i in sample:
        r = reps[i]
        want, _ = _run_oracle(r, _init_oracle(r, seed), seed, 0, n, 0)
        assert np.array_equal(smp.get_state(i), want), f"replica {i} {r}"
    stats, _ = smp.measure()
    torch.cuda.synchronize()
    assert np.array_equal(st[0].cpu().numpy()[:, :3], stats.cpu().numpy()[:, :3])
    smp.close()


def test_batched_workload_full_length_sampled(S):
    """The benchmark's batched workload as one step runs it: autotuned
    schedule, 10^4 unrecorded sweeps replayed as graphs.  Sampled replicas
    at the full length are bit-exact with the oracle: three Ising 256^2,
    Potts lattices of 64^2, 128^2 and 256^2 (LDS-resident when the tuner
    picks the hybrid schedule) and a Potts 512^2 (always streamed)."""
    reps = synth.batched_ising_potts()
    seed, n = 2, 10_000
    smp = S(reps, seed, init=True)
    smp.autotune(trial_sweeps=20)
    st_sites, res_sites = smp.schedule_sites(by_model=True)
    smp.sweep(n)
    torch.cuda.synchronize()
    first = {}
    for i, r in enumerate(reps):
        if r["model"] == 1:
            first.setdefault(r["Lx"], i)
    sample = [0, 517, 1023, first[64], first[128], first[256], first[512]]
    print(f"full-length batched parity: schedule {smp.get_schedule()}, streamed sites "
          f"{st_sites}, resident sites {res_sites}, sample {sample}", flush=True)
    for i in sample:
        r = reps[i]
        want, _ = _run_oracle(r, _init_oracle(r, seed), seed, 0, n, 0)
        assert np.array_equal(smp.get_state(i), want), f"replica {i} {r}"
    smp.close()


def test_ising_stream_8192_nontemporal_full_size_sampled(S):
    """The HBM-bound probe configuration (8192 Ising replicas of 256^2, 512
    MiB of lattices, streamed with nontemporal own-plane access, 128-row
    tiles): sampled replicas bit-exact with the oracle."""
    reps = synth.batched_ising_potts(n_ising=8192, n_potts=0)
    seed, n = 2, 3
    smp = S(reps, seed, init=True)
    smp.set_schedule(mode="stream", tile_rows=128, wg_threads=256, nt=True)
    smp.sweep(n)
    torch.cuda.synchronize()
    for i in (0, 1, 4095, 4096, 8191):
        r = reps[i]
        want, _ = _run_oracle(r, _init_oracle(r, seed), seed, 0, n, 0)
        assert np.array_equal(smp.get_state(i), want), f"replica {i}"
    smp.close()
