"""The learned surrogate end to end at a reduced size: labels from the
sampler, training on the MLP kernels, and the inverse problem solved with
Monte Carlo verification, against the Monte-Carlo-only solve."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_surrogate_pipeline_reduced():
    from paper_2304_01772_amd import surrogate as sg
    pts = synth.surrogate_points(4096, seed=1005)
    y, se = sg.mc_observables(pts, L=32, burn=150, measure=250)
    assert np.all(np.isfinite(y)) and np.all(y[:, 1] >= 0) and np.all(y[:, 1] <= 1)
    net = sg.SurrogateMLP(seed=0)
    net.fit(pts[:3686], y[:3686], epochs=80, batch=256)
    pv = net.predict(torch.tensor(pts[3686:], device=net.dev)).cpu().numpy()
    mae = np.abs(pv[:, 1] - y[3686:, 1]).mean()
    # the network must beat the best constant predictor by a wide margin
    base = np.abs(y[3686:, 1] - np.median(y[:3686, 1])).mean()
    assert mae < 0.25 * base, (mae, base)
    # inverse problem: target <|m|> = 0.8 at beta = 0.4 on 32x32 lattices,
    # every Monte Carlo evaluation resolved to a standard error of 0.5 %
    kw = dict(L=32, n_rep=64, burn=200, measure=400, se_rel=0.005, n_max=1024)
    mc = sg.mc_only_solve(0.8, beta=0.4, tol=0.02, max_iter=25, **kw)
    su = sg.surrogate_solve(net, 0.8, beta=0.4, tol=0.02, max_iter=25, **kw)
    assert mc["converged"] and su["converged"]
    assert abs(su["absm"] - 0.8) <= 0.02 * 0.8
    # what the network gains: its answer, checked by Monte Carlo, is far
    # closer to the target than the common starting point
    err_start = abs(mc["history"][0][2] - 0.8)
    err_guess = abs(su["history"][0][2] - 0.8)
    assert err_guess < 0.25 * err_start, (err_guess, err_start)
