"""GPU parity of the surrogate-MLP kernels (BF16 matrix cores, FP32
accumulation) with the FP64 oracle that rounds at the same points.

Tolerance (derived from the arithmetic): a BF16 rounding decision taken from
an FP32 sum can differ from the one taken from the FP64 sum by one BF16 step
(2^-8 relative), and FP32 accumulation adds ~K 2^-24.  Each result is
therefore compared with 2^-7 times its magnitude bound (the same products
taken over absolute values), and the median deviation must stay below
1e-4 of the bound, which a dropped term or transposed operand would exceed.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    from paper_2304_01772_amd import _lib
    assert torch.cuda.is_available()
    return _lib.lib()


def _p(t):
    return C.c_void_p(t.data_ptr())


def _close(got, want, bound):
    got, want, bound = (np.asarray(a, np.float64).reshape(-1) for a in (got, want, bound))
    dev = np.abs(got - want)
    assert np.all(dev <= 2.0 ** -7 * bound + 1e-7), np.max(dev / (bound + 1e-30))
    assert np.median(dev / (bound + 1e-30)) < 1e-4


def _run(L, P, x, t, w):
    dev = torch.device("cuda")
    B = x.shape[0]
    Pt = torch.tensor(P, dtype=torch.float32, device=dev)
    xt = torch.tensor(x, dtype=torch.float32, device=dev)
    tt = torch.tensor(t, dtype=torch.float32, device=dev)
    wt = torch.tensor(w, dtype=torch.float32, device=dev)
    y = torch.empty((B, 3), dtype=torch.float32, device=dev)
    act = torch.empty(L.spinmc_mlp_act_floats(B), dtype=torch.float32, device=dev)
    g = torch.empty(mlp.NP, dtype=torch.float32, device=dev)
    dx = torch.empty((B, 4), dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ws = torch.empty(L.spinmc_mlp_workspace_floats(B), dtype=torch.float32, device=dev)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.spinmc_mlp_forward(_p(Pt), _p(xt), B, _p(y), _p(act), s) == 0
    assert L.spinmc_mlp_backward(_p(Pt), _p(xt), _p(act), _p(tt), _p(wt), B, _p(g), _p(dx),
                                 _p(loss), _p(ws), s) == 0
    torch.cuda.synchronize()
    return y.cpu().numpy(), g.cpu().numpy(), dx.cpu().numpy(), float(loss.item())


@pytest.mark.parametrize("B", [1, 37, 64, 100, 1025])
def test_forward_backward_match_oracle(L, B):
    rng = np.random.default_rng(B)
    P = mlp.init_params(rng)
    P[-3:] = rng.normal(size=3).astype(np.float32) * 0.1
    # nonzero hidden biases
    P[512:640] = rng.normal(size=128).astype(np.float32) * 0.1
    x = rng.normal(size=(B, 4)).astype(np.float32)
    t = rng.normal(size=(B, 3)).astype(np.float32)
    w = np.array([1.0, 0.5, 2.0], np.float32)
    y, g, dx, loss = _run(L, P, x, t, w)
    yo, _ = mlp.forward(P, x)
    go, dxo, losso = mlp.backward(P, x, t, w)
    by, bg, bdx = mlp.magnitude_bounds(P, x, t, w)
    _close(y, yo, by)
    _close(g, go, bg)
    _close(dx, dxo, bdx)
    assert abs(loss - losso) <= 2.0 ** -6 * losso + 1e-6


def test_backward_is_deterministic(L):
    rng = np.random.default_rng(9)
    P = mlp.init_params(rng)
    x = rng.normal(size=(300, 4)).astype(np.float32)
    t = rng.normal(size=(300, 3)).astype(np.float32)
    w = np.ones(3, np.float32)
    a = _run(L, P, x, t, w)
    b = _run(L, P, x, t, w)
    for u, v in zip(a[:3], b[:3]):
        assert np.array_equal(u, v)


def test_adam_matches_oracle(L):
    rng = np.random.default_rng(4)
    dev = torch.device("cuda")
    p = rng.normal(size=mlp.NP).astype(np.float32)
    pt = torch.tensor(p, device=dev)
    mt = torch.zeros(mlp.NP, device=dev)
    vt = torch.zeros(mlp.NP, device=dev)
    po, mo, vo = p.astype(np.float64), np.zeros(mlp.NP), np.zeros(mlp.NP)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for step in range(1, 6):
        g = rng.normal(size=mlp.NP).astype(np.float32)
        gt = torch.tensor(g, device=dev)
        assert L.spinmc_mlp_adam(_p(pt), _p(gt), _p(mt), _p(vt), step, 1e-3, 0.9, 0.999, 1e-8, s) == 0
        po, mo, vo = mlp.adam(po, g, mo, vo, step)
    torch.cuda.synchronize()
    np.testing.assert_allclose(pt.cpu().numpy(), po, rtol=1e-5, atol=1e-6)


def test_train_step_equals_the_separate_calls(L):
    """spinmc_mlp_train_step (forward, backward, reduction fused with Adam)
    leaves parameters, moments, gradient and loss bit-identical to the
    separate forward / backward / adam calls, over three steps, and each
    gradient matches the oracle's."""
    rng = np.random.default_rng(21)
    dev = torch.device("cuda")
    B = 200
    P = mlp.init_params(rng)
    x = torch.tensor(rng.normal(size=(B, 4)).astype(np.float32), device=dev)
    t = torch.tensor(rng.normal(size=(B, 3)).astype(np.float32), device=dev)
    w = torch.tensor([1.0, 0.5, 2.0], dtype=torch.float32, device=dev)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    state = {}
    for name in ("sep", "fused"):
        state[name] = dict(p=torch.tensor(P, device=dev), m=torch.zeros(mlp.NP, device=dev),
                           v=torch.zeros(mlp.NP, device=dev),
                           g=torch.empty(mlp.NP, device=dev), loss=torch.empty(1, device=dev),
                           act=torch.empty(L.spinmc_mlp_act_floats(B), device=dev),
                           ws=torch.empty(L.spinmc_mlp_workspace_floats(B), device=dev))
    y = torch.empty((B, 3), device=dev)
    for step in range(1, 4):
        a = state["sep"]
        p_before = a["p"].cpu().numpy().copy()
        assert L.spinmc_mlp_forward(_p(a["p"]), _p(x), B, _p(y), _p(a["act"]), s) == 0
        assert L.spinmc_mlp_backward(_p(a["p"]), _p(x), _p(a["act"]), _p(t), _p(w), B, _p(a["g"]),
                                     None, _p(a["loss"]), _p(a["ws"]), s) == 0
        assert L.spinmc_mlp_adam(_p(a["p"]), _p(a["g"]), _p(a["m"]), _p(a["v"]), step, 1e-3, 0.9,
                                 0.999, 1e-8, s) == 0
        b = state["fused"]
        assert L.spinmc_mlp_train_step(_p(b["p"]), _p(x), _p(t), _p(w), B, _p(b["g"]), _p(b["m"]),
                                       _p(b["v"]), step, 1e-3, 0.9, 0.999, 1e-8, _p(b["loss"]),
                                       _p(b["act"]), _p(b["ws"]), s) == 0
        torch.cuda.synchronize()
        for k in ("p", "m", "v", "g", "loss"):
            assert torch.equal(a[k], b[k]), (step, k)
        go, _, _ = mlp.backward(p_before, x.cpu().numpy(), t.cpu().numpy(), w.cpu().numpy())
        _, bg, _ = mlp.magnitude_bounds(p_before, x.cpu().numpy(), t.cpu().numpy(),
                                        w.cpu().numpy())
        _close(b["g"].cpu().numpy(), go, bg)
