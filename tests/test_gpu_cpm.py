"""GPU parity of the Cellular Potts copy-attempt sweep against the oracle.

Cell-id lattices and integer statistics (boundary bonds by type pair, the
fixed-point energy) must be bit-identical to the oracle's for the same seed,
replica ids and Monte Carlo step counter.
"""
import numpy as np
import pytest

import synth
from oracle import chain as orc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def S():
    from paper_2304_01772_amd.sampler import Sampler
    assert torch.cuda.is_available()
    return Sampler


def _rep(ids, J, ctype, A, lam, T, rid):
    return dict(model=2, Lx=ids.shape[1], Ly=ids.shape[0], q=len(ctype) - 1, rid=rid,
                adhesion=J, cell_type=ctype, target_area=A, lambda_area=lam, temperature=T)


def _random_case(seed, shape, n_cells, n_types=3):
    rng = np.random.default_rng(seed)
    ids = rng.integers(0, n_cells + 1, size=shape).astype(np.int32)
    ctype = np.concatenate([[0], rng.integers(1, n_types, size=n_cells)]).astype(np.int8)
    A = np.concatenate([[0], rng.integers(5, 40, size=n_cells)]).astype(np.int32)
    return ids, ctype, A


JS = {
    "sorting": np.array([[0, 16, 16], [16, 2, 11], [16, 11, 16]], np.float32),
    "halves": np.array([[0, 3.5, 4.5], [3.5, 1.5, 2.0], [4.5, 2.0, 0.5]], np.float32),
}


@pytest.mark.parametrize("shape,n_cells,Jname,lam,T,tile_rows", [
    ((16, 16), 6, "sorting", 1.0, 10.0, 0),
    ((8, 10), 3, "halves", 0.5, 3.0, 2),
    ((24, 32), 12, "sorting", 2.0, 25.0, 4),
    ((2, 4), 2, "halves", 0.0, 1.0, 0),
    ((64, 64), 30, "sorting", 1.0, 10.0, 6),
    # more cells than the LDS cell tables hold: the per-site kernel
    ((128, 128), 17000, "sorting", 1.0, 10.0, 0),
])
@pytest.mark.parametrize("threads", [0, 256])  # one site per lane (1024), one quad per lane
def test_cpm_matches_oracle(S, shape, n_cells, Jname, lam, T, tile_rows, threads):
    J = JS[Jname]
    reps, init = [], []
    for r in range(3):
        ids, ctype, A = _random_case(100 * r + shape[0], shape, n_cells)
        reps.append(_rep(ids, J, ctype, A, lam, T, 7 + r))
        init.append(ids)
    smp = S(reps, 17, init=False)
    smp.set_schedule(mode="stream", tile_rows=tile_rows, wg_threads=threads)
    for i, ids in enumerate(init):
        smp.set_state(i, ids)
    n, re = 6, 2
    st = smp.sweep(n, re)
    torch.cuda.synchronize()
    for i, rp in enumerate(reps):
        want, area, ost = orc.cpm_run(init[i], J, rp["cell_type"], rp["target_area"], lam, T, 17,
                                      rp["rid"], 0, n, re)
        assert np.array_equal(smp.get_state(i), want), f"replica {i}"
        assert np.array_equal(st[:, i].cpu().numpy(), ost), f"stats replica {i}"
    smp.close()


def test_cpm_thresholds_equal_oracle_formula(S):
    ids, ctype, A = _random_case(1, (8, 8), 4)
    smp = S([_rep(ids, JS["halves"], ctype, A, 0.5, 3.0, 0)], 1, init=False)
    T, K0 = smp.thresholds(0)
    # the oracle draws T(k) = ceil(2^32 exp(-k/(S temp))); S = 2 here
    assert orc.cpm_scale(JS["halves"], 0.5) == 2
    import math
    for k, t in enumerate(T, start=1):
        assert t == math.ceil(math.ldexp(math.exp(-k / (2 * 3.0)), 32))
    assert math.ceil(math.ldexp(math.exp(-(len(T) + 1) / 6.0), 32)) == 1
    assert math.ldexp(math.exp(-K0 / 6.0), 32) == 0.0
    assert math.ldexp(math.exp(-(K0 - 1) / 6.0), 32) > 0.0
    smp.close()


def test_cell_sorting_config_full_size(S):
    """8 replicas of 512x512, 1000 square 14x14 cells, two types 50/50, target
    area 200, lambda 1, T = 10, the sorting adhesion matrix: a few Monte Carlo
    steps bit-exact with the oracle, then invariants on a longer run."""
    ids, ctype, A, J, prm = synth.cpm_sorting()
    reps = [_rep(ids[r], J, ctype, A, prm["lambda_area"], prm["temperature"], r)
            for r in range(ids.shape[0])]
    smp = S(reps, prm["seed"], init=False)
    for r in range(len(reps)):
        smp.set_state(r, ids[r])
    n = 3
    st = smp.sweep(n, 1)
    torch.cuda.synchronize()
    for r in (0, 5):
        want, _, ost = orc.cpm_run(ids[r], J, ctype, A, prm["lambda_area"], prm["temperature"],
                                   prm["seed"], r, 0, n, 1)
        assert np.array_equal(smp.get_state(r), want)
        assert np.array_equal(st[:, r].cpu().numpy(), ost)
    smp.sweep(50)
    stats, obs = smp.measure()
    stats = stats.cpu().numpy()
    for r in (1, 7):
        got = smp.get_state(r)
        assert set(np.unique(got)) <= set(np.unique(ids[r]))
        assert np.array_equal(stats[r], orc.cpm_stats(got, J, ctype, A, prm["lambda_area"]))
    smp.close()


def test_cell_sorting_config_full_length(S):
    """The cell-sorting workload at its full length, 2000 Monte Carlo steps:
    the first 1000 unrecorded (cached graph replays, as the benchmark runs
    them), the next 1000 recorded every 100 steps (direct launches).  Two
    replicas' states and recorded statistics bit-exact with the oracle (the
    two oracle chains run on two host threads)."""
    from concurrent.futures import ThreadPoolExecutor
    ids, ctype, A, J, prm = synth.cpm_sorting()
    reps = [_rep(ids[r], J, ctype, A, prm["lambda_area"], prm["temperature"], r)
            for r in range(ids.shape[0])]
    smp = S(reps, prm["seed"], init=False)
    for r in range(len(reps)):
        smp.set_state(r, ids[r])
    half = prm["n_mcs"] // 2
    smp.sweep(half)
    st = smp.sweep(half, 100)
    torch.cuda.synchronize()
    sample = (2, 6)

    def oracle(r):
        lam, T, seed = prm["lambda_area"], prm["temperature"], prm["seed"]
        mid, _, _ = orc.cpm_run(ids[r], J, ctype, A, lam, T, seed, r, 0, half)
        return orc.cpm_run(mid, J, ctype, A, lam, T, seed, r, half, half, 100)

    with ThreadPoolExecutor(len(sample)) as ex:
        outs = list(ex.map(oracle, sample))
    for r, (want, _, ost) in zip(sample, outs):
        assert np.array_equal(smp.get_state(r), want), f"replica {r}"
        assert np.array_equal(st[:, r].cpu().numpy(), ost), f"stats replica {r}"
    smp.close()


@pytest.mark.parametrize("shape,tile_rows,n_rep", [((64, 64), 16, 3), ((128, 96), 0, 2),
                                                   ((32, 64), 2, 2), ((48, 40), 0, 4)])
def test_tiled_persistent_passes_match_oracle(S, shape, tile_rows, n_rep):
    """Tiled persistent CPM passes (one workgroup per tile, ids in LDS,
    border exchange at a per-replica barrier after every pass): states
    bit-exact with the oracle across a 500-step chunk boundary, with
    recorded steps (per-pass launches) in between; thin (2-row) tiles,
    32- and 8-column tiles."""
    J = JS["sorting"]
    cases = [_random_case(900 + 17 * r + shape[0], shape, 9) for r in range(n_rep)]
    reps = [_rep(ids, J, ct, A, 1.0, 10.0, 60 + r) for r, (ids, ct, A) in enumerate(cases)]
    smp = S(reps, 23, init=False)
    smp.set_schedule(mode="stream", tile_rows=tile_rows, persistent=True)
    for r, (ids, _, _) in enumerate(cases):
        smp.set_state(r, ids)
    cur = [ids for ids, _, _ in cases]
    t0 = 0
    smp.profile(True)
    for n, re in ((505, 0), (4, 2), (9, 0)):
        st = smp.sweep(n, re)
        torch.cuda.synchronize()
        for r, (_, ct, A) in enumerate(cases):
            cur[r], _, ost = orc.cpm_run(cur[r], J, ct, A, 1.0, 10.0, 23, 60 + r, t0, n, re)
            assert np.array_equal(smp.get_state(r), cur[r]), (r, t0)
            if re:
                assert np.array_equal(st[:, r].cpu().numpy(), ost)
        t0 += n
    ms, n_l = smp.profile_read("cpm_tiled")
    assert n_l == 3 and ms > 0  # 500 + 5 steps, then 9
    smp.close()


def test_cell_sorting_full_length_tiled_persistent(S):
    """The cell-sorting workload at 2000 Monte Carlo steps on the tiled
    persistent passes (64 x 64 tiles, 64 per replica): two replicas' states
    bit-exact with the oracle, and the launches were the tiled kernel."""
    from concurrent.futures import ThreadPoolExecutor
    ids, ctype, A, J, prm = synth.cpm_sorting()
    reps = [_rep(ids[r], J, ctype, A, prm["lambda_area"], prm["temperature"], r)
            for r in range(ids.shape[0])]
    smp = S(reps, prm["seed"], init=False)
    smp.set_schedule(mode="stream", persistent=True)
    for r in range(len(reps)):
        smp.set_state(r, ids[r])
    smp.profile(True)
    smp.sweep(prm["n_mcs"])
    torch.cuda.synchronize()
    ms, n_l = smp.profile_read("cpm_tiled")
    smp.profile(False)
    assert n_l == 4 and ms > 0
    sample = (1, 6)

    def oracle(r):
        return orc.cpm_run(ids[r], J, ctype, A, prm["lambda_area"], prm["temperature"],
                           prm["seed"], r, 0, prm["n_mcs"])

    with ThreadPoolExecutor(len(sample)) as ex:
        outs = list(ex.map(oracle, sample))
    for r, (want, _, _) in zip(sample, outs):
        assert np.array_equal(smp.get_state(r), want), f"replica {r}"
    smp.close()


def test_paper_cell_sorting_setting(S):
    """The paper's own CPM setting (36 cells of area 25 in a touching 6 x 6
    aggregate, Table 2 adhesion, k_B T = 8, A = 25, lambda = 1) on 16
    replicas of 64 x 64: 2000 Monte Carlo steps bit-exact with the oracle
    for two replicas (state and recorded statistics), and the sorting the
    paper reports: the light cells lose all contact with the medium and the
    light-dark boundary shrinks (statistics: b1 light-medium, b2
    dark-medium, b4 light-dark)."""
    ids, types, A, J, prm = synth.cpm_paper_aggregate()
    reps = [_rep(ids[r], J, types[r], A, prm["lambda_area"], prm["temperature"], r)
            for r in range(ids.shape[0])]
    smp = S(reps, prm["seed"], init=False)
    for r in range(len(reps)):
        smp.set_state(r, ids[r])
    start, _ = smp.measure()
    start = start.cpu().numpy()
    n, every = 2000, 500
    st = smp.sweep(n, every).cpu().numpy()
    for r in (0, 9):
        want, _, ost = orc.cpm_run(ids[r], J, types[r], A, prm["lambda_area"], prm["temperature"],
                                   prm["seed"], r, 0, n, every)
        assert np.array_equal(smp.get_state(r), want)
        assert np.array_equal(st[:, r], ost)
    end = st[-1]
    assert start[:, 1].mean() > 30 and end[:, 1].mean() < 0.1 * start[:, 1].mean()
    assert end[:, 4].mean() < 0.75 * start[:, 4].mean()
    assert end[:, 2].mean() > start[:, 2].mean()  # the dark cells now face the medium
    smp.close()


def _rep5(ids, J, ctype, A, lam, T, rid):
    d = _rep(ids, J, ctype, A, lam, T, rid)
    d["cpm_range"] = 2
    return d


# the 5x5 neighbourhood: 3x3 sublattice, one site per lane; several tiles
# (tile_rows rounds down to whole periods of 6 rows) and widths that are not
# multiples of 8
@pytest.mark.parametrize("shape,n_cells,Jname,lam,T,tile_rows", [
    ((6, 6), 3, "sorting", 1.0, 10.0, 0),
    ((12, 18), 8, "halves", 0.5, 3.0, 6),
    ((36, 48), 20, "sorting", 2.0, 25.0, 8),
    ((66, 60), 40, "sorting", 1.0, 10.0, 0),
])
def test_cpm5_matches_oracle(S, shape, n_cells, Jname, lam, T, tile_rows):
    J = JS[Jname]
    reps, cases = [], []
    for rid in range(3):
        ids, ctype, A = _random_case(100 * rid + n_cells, shape, n_cells)
        cases.append((ids, ctype, A))
        reps.append(_rep5(ids, J, ctype, A, lam, T, rid))
    smp = S(reps, 77, init=False)
    if tile_rows:
        smp.set_schedule(mode="stream", tile_rows=tile_rows)
    for r, (ids, _, _) in enumerate(cases):
        smp.set_state(r, ids)
    n = 4
    st = smp.sweep(n, 1).cpu().numpy()
    for r, (ids, ctype, A) in enumerate(cases):
        want, area, ost = orc.cpm_run(ids, J, ctype, A, lam, T, 77, r, 0, n, 1, nrange=2)
        assert np.array_equal(smp.get_state(r), want), r
        assert np.array_equal(st[:, r], ost), r
    stats, _ = smp.measure()
    for r in range(3):
        got = smp.get_state(r)
        assert np.array_equal(stats.cpu().numpy()[r],
                              orc.cpm_stats(got, J, cases[r][1], cases[r][2], lam, nrange=2))
    smp.close()


def test_paper_setting_with_the_second_shell(S):
    """The paper's aggregate in a 66 x 66 medium with the 5x5 neighbourhood:
    300 Monte Carlo steps bit-exact with the oracle for two replicas.  With
    Table 2's adhesion summed over 24 neighbours the boundary cost outweighs
    the lambda = 1 area term at k_B T = 8 and the cells dissolve into the
    medium (the oracle shows the same), which supports reading the paper's
    setting with the 3x3 neighbourhood."""
    ids, types, A, J, prm = synth.cpm_paper_aggregate(n_rep=8, L=66)
    reps = [_rep5(ids[r], J, types[r], A, prm["lambda_area"], prm["temperature"], r)
            for r in range(ids.shape[0])]
    smp = S(reps, prm["seed"], init=False)
    for r in range(len(reps)):
        smp.set_state(r, ids[r])
    start, _ = smp.measure()
    start = start.cpu().numpy()
    n = 300
    st = smp.sweep(n, 100).cpu().numpy()
    for r in (0, 5):
        want, _, ost = orc.cpm_run(ids[r], J, types[r], A, prm["lambda_area"],
                                   prm["temperature"], prm["seed"], r, 0, n, 100, nrange=2)
        assert np.array_equal(smp.get_state(r), want)
        assert np.array_equal(st[:, r], ost)
    assert start[:, 1].mean() > 30
    for r in range(len(reps)):
        assert len(np.unique(smp.get_state(r))) < 37  # cells have vanished
    smp.close()


def test_measure_right_after_set_state_counts_the_areas(S):
    """set_state defers the area count: a measurement straight after setting
    every replica's state (no sweep in between) still sees the new areas in
    its energy, and a second batch of set_state calls replaces them."""
    J = JS["sorting"]
    cases = [_random_case(500 + r, (16, 24), 9) for r in range(3)]
    reps = [_rep(ids, J, ct, A, 1.5, 10.0, r) for r, (ids, ct, A) in enumerate(cases)]
    smp = S(reps, 3, init=False)
    for _ in range(2):
        cases = [(np.roll(ids, 1, axis=1), ct, A) for ids, ct, A in cases]
        for r, (ids, _, _) in enumerate(cases):
            smp.set_state(r, ids)
        stats, _ = smp.measure()
        stats = stats.cpu().numpy()
        for r, (ids, ct, A) in enumerate(cases):
            assert np.array_equal(stats[r], orc.cpm_stats(ids, J, ct, A, 1.5))
    smp.close()


@pytest.mark.parametrize("cpm_range", [1, 2])
def test_unrecorded_steps_replay_graphs(S, cpm_range):
    """Unrecorded Monte Carlo steps of the streamed schedule replay captured
    graphs of whole chunks (here 55 = 50 + 5 steps, then 3 more after a
    change of tile rows, which drops the graphs): the states equal the
    oracle's."""
    J = JS["sorting"]
    shape = (24, 24) if cpm_range == 1 else (24, 30)
    cases = [_random_case(800 + r, shape, 10) for r in range(2)]
    reps = [dict(_rep(ids, J, ct, A, 1.0, 12.0, r), cpm_range=cpm_range)
            for r, (ids, ct, A) in enumerate(cases)]
    smp = S(reps, 5, init=False)
    smp.set_schedule(mode="stream")  # small range-1 lattices would run resident
    for r, (ids, _, _) in enumerate(cases):
        smp.set_state(r, ids)
    smp.sweep(55)
    smp.set_schedule(mode="stream", tile_rows=6)
    smp.sweep(3)
    for r, (ids, ct, A) in enumerate(cases):
        want, _, _ = orc.cpm_run(ids, J, ct, A, 1.0, 12.0, 5, r, 0, 58, nrange=cpm_range)
        assert np.array_equal(smp.get_state(r), want), r
    smp.close()


@pytest.mark.parametrize("cpm_range", [1, 2])
def test_unrecorded_steps_resident(S, cpm_range):
    """Unrecorded steps of lattices whose ids and tables fit 64 KiB of LDS run
    in one workgroup per replica: mixed shapes and cell counts, two calls
    (the step counter carries over) and a chunk boundary (500 steps); states
    and then measured statistics equal the oracle's."""
    J = JS["sorting"]
    if cpm_range == 1:
        shapes = [((16, 24), 7), ((64, 64), 30), ((8, 8), 2), ((40, 32), 25)]
    else:
        shapes = [((18, 24), 7), ((66, 66), 30), ((6, 6), 2), ((36, 48), 25)]
    cases = [_random_case(900 + r, sh, nc) for r, (sh, nc) in enumerate(shapes)]
    reps = [dict(_rep(ids, J, ct, A, 1.0, 10.0, 40 + r), cpm_range=cpm_range)
            for r, (ids, ct, A) in enumerate(cases)]
    smp = S(reps, 9, init=False)
    for r, (ids, _, _) in enumerate(cases):
        smp.set_state(r, ids)
    smp.sweep(520)
    smp.sweep(7)
    stats, _ = smp.measure()
    stats = stats.cpu().numpy()
    for r, (ids, ct, A) in enumerate(cases):
        want, area, _ = orc.cpm_run(ids, J, ct, A, 1.0, 10.0, 9, 40 + r, 0, 527,
                                    nrange=cpm_range)
        assert np.array_equal(smp.get_state(r), want), r
        assert np.array_equal(stats[r], orc.cpm_stats(want, J, ct, A, 1.0, nrange=cpm_range)), r
    smp.close()


@pytest.mark.parametrize("threads", [0, 512, 256])
def test_streamed_passes_over_ragged_tiles_match_oracle(S, threads):
    """The 3x3 streamed pass, recorded, over several tiles of 8 rows with a
    ragged last one (22 rows), in both forms (one site per lane in
    workgroups of 1024 or 512, one quad per lane in 256): states and
    statistics equal the oracle's."""
    J = JS["sorting"]
    cases = [_random_case(950 + r, (22, 40), 9) for r in range(2)]
    reps = [_rep(ids, J, ct, A, 1.0, 10.0, 60 + r) for r, (ids, ct, A) in enumerate(cases)]
    smp = S(reps, 13, init=False)
    smp.set_schedule(mode="stream", tile_rows=8, wg_threads=threads)
    for r, (ids, _, _) in enumerate(cases):
        smp.set_state(r, ids)
    st = smp.sweep(6, 3).cpu().numpy()
    for r, (ids, ct, A) in enumerate(cases):
        want, _, ost = orc.cpm_run(ids, J, ct, A, 1.0, 10.0, 13, 60 + r, 0, 6, 3)
        assert np.array_equal(smp.get_state(r), want), r
        assert np.array_equal(st[:, r], ost), r
    smp.close()


def test_autotune_keeps_the_chain(S):
    """The autotuner's trials (resident, and streamed passes over several
    tile heights) restore the state and the step counter; the chosen
    schedule continues the oracle's chain."""
    J = JS["sorting"]
    cases = [_random_case(970 + r, (32, 48), 11) for r in range(3)]
    reps = [_rep(ids, J, ct, A, 1.0, 10.0, 80 + r) for r, (ids, ct, A) in enumerate(cases)]
    smp = S(reps, 15, init=False)
    for r, (ids, _, _) in enumerate(cases):
        smp.set_state(r, ids)
    smp.sweep(4)
    chosen, rates = smp.autotune(trial_sweeps=5)
    # resident, five streamed tile heights of the quad form, five of the
    # one-site-per-lane form (1024 and 512 lanes), two tiled persistent
    assert len(rates) == 13 and all(x > 0 for x in rates)
    smp.sweep(5)
    for r, (ids, ct, A) in enumerate(cases):
        want, _, _ = orc.cpm_run(ids, J, ct, A, 1.0, 10.0, 15, 80 + r, 0, 9)
        assert np.array_equal(smp.get_state(r), want), (r, chosen)
    smp.close()
