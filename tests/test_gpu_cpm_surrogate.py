"""The surrogate over CPM adhesion parameters, reduced: its labels equal
the oracle's chains for the same replicas, the network learns them, and the
surrogate-steered inverse problem reaches a Monte-Carlo-verified answer."""
import numpy as np
import pytest

import synth
from oracle import chain as orc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_labels_equal_the_oracle_chains():
    from paper_2304_01772_amd import cpm_surrogate as cs
    pts = cs.snap([[9.3, 12.1, 15.0, 7.0], [14.0, 3.0, 10.0, 11.0]])
    n_rep, mcs, seed, rid0 = 2, 20, 6, 100
    b, _ = cs.cpm_boundaries(pts, n_rep=n_rep, mcs=mcs, seed=seed, rid0=rid0)
    ids, types, A, _, prm = synth.cpm_paper_aggregate(n_rep=n_rep, L=64)
    for i, p in enumerate(pts):
        want = []
        for j in range(n_rep):
            out, _, _ = orc.cpm_run(ids[j], cs.adhesion(p), types[j], A, prm["lambda_area"],
                                    float(p[3]), seed, rid0 + i * n_rep + j, 0, mcs)
            st = orc.cpm_stats(out, cs.adhesion(p), types[j], A, prm["lambda_area"])
            want.append([st[1], st[2], st[4]])
        assert np.array_equal(b[i], np.mean(want, axis=0))


def test_reduced_pipeline():
    from paper_2304_01772_amd import cpm_surrogate as cs
    X = cs.training_points(512)
    Y, _ = cs.cpm_boundaries(X, n_rep=2, mcs=200)
    Xv = cs.training_points(128, seed=99)
    Yv, _ = cs.cpm_boundaries(Xv, n_rep=2, mcs=200, rid0=9_000_000)
    net = cs.make_net().fit(X, Y, epochs=150, batch=128, lr=2e-3, lr_min=1e-4)
    with torch.no_grad():
        pv = net.predict(torch.tensor(Xv, dtype=torch.float32, device=net.dev)).cpu().numpy()
    mae = np.abs(pv - Yv).mean(axis=0)
    assert np.all(mae < 0.5 * Yv.std(axis=0)), (mae, Yv.std(axis=0))
    res = cs.surrogate_solve(net, 150.0, tol=0.05, mcs=200)
    assert res["converged"], res
    assert 4.0 <= res["J_light_dark"] <= 16.0
