"""Argument guards that need a context (hence a device): the pass counter of
every model must fit the 32-bit Philox counter word, and the covariance
estimator's int64 moment sums must not overflow.  Every call here is refused
before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    from paper_2304_01772_amd import _lib
    assert torch.cuda.is_available()
    return _lib.lib()


def _cpm(rng):
    J = np.array([[0, 16], [16, 2]], np.float32)
    return dict(model=2, Lx=12, Ly=12, q=1, rid=0, adhesion=J, cell_type=np.array([0, 1], np.int8),
                target_area=np.array([0, 20], np.int32), lambda_area=1.0, temperature=4.0,
                cpm_range=rng)


@pytest.mark.parametrize("rep,n_col", [
    (dict(model=0, Lx=8, Ly=8, beta=0.4), 2),
    (dict(model=3, Lx=9, Ly=9, beta=0.3), 3),
    (dict(model=4, Lx=8, Ly=8, Lz=2, beta=0.2), 2),
    ("cpm1", 4),
    ("cpm2", 9),
])
def test_pass_counter_guard(L, rep, n_col):
    """n sweeps with n * n_col > 2^32 are refused (the pass p = n_col t + c
    would wrap and repeat earlier random words); the counter stays at 0."""
    from paper_2304_01772_amd.sampler import Sampler
    if rep == "cpm1":
        rep = _cpm(1)
    elif rep == "cpm2":
        rep = _cpm(2)
    smp = Sampler([rep], seed=1, init=rep["model"] != 2)
    if rep["model"] == 2:
        ids = np.zeros((12, 12), np.int32)
        ids[:4, :5] = 1
        smp.set_state(0, ids)
    n = 2 ** 32 // n_col + 1
    if n < 2 ** 31:
        rc = L.spinmc_sweep(smp.ctx, n, 0, None)
        assert rc == -1, L.spinmc_last_error()
        assert b"pass counter" in L.spinmc_last_error()
    assert smp.t == 0
    smp.sweep(2)  # the context still works
    torch.cuda.synchronize()
    assert smp.t == 2
    smp.close()


def test_grad_refuses_moment_overflow(L):
    """A 16384^2 lattice (2^28 sites): 127 samples keep n N^2 below 2^63,
    128 reach it (the int64 sums could overflow) and are refused."""
    from paper_2304_01772_amd.sampler import Sampler
    smp = Sampler([dict(model=0, Lx=16384, Ly=16384, beta=0.4)], seed=1, init=False)
    stats = torch.zeros((128, 1, smp.width), dtype=torch.int32, device="cuda")
    with pytest.raises(Exception) as ei:
        smp.grad(stats, 0)
    assert "overflow" in str(ei.value)
    means, grads, _ = smp.grad(stats[:127], 0)
    torch.cuda.synchronize()
    assert torch.isfinite(grads).all()
    smp.close()
