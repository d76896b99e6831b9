"""spinmc_grad_noalloc (chunk sums in the library's static per-device array)
against spinmc_grad, called through the C ABI: bit-identical outputs on two
calls in a row, the second with a smaller record, and the size limit."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _f32(v):
    return float(np.float32(v))


def _call(entry, smp, stats, n_rec, burn, gout):
    from paper_2304_01772_amd._lib import lib
    R = smp.R
    means = torch.full((R, 4), float("nan"), dtype=torch.float64, device="cuda")
    grads = torch.full((R, 2, 3), float("nan"), dtype=torch.float64, device="cuda")
    dth = torch.full((R, 3), float("nan"), dtype=torch.float64, device="cuda")
    rc = getattr(lib(), entry)(smp.ctx, C.c_void_p(stats.data_ptr()), int(n_rec), int(burn),
                               C.c_void_p(gout.data_ptr()), C.c_void_p(means.data_ptr()),
                               C.c_void_p(grads.data_ptr()), C.c_void_p(dth.data_ptr()))
    return rc, means, grads, dth


def test_grad_noalloc_matches_grad_on_two_calls():
    from paper_2304_01772_amd.sampler import Sampler
    assert torch.cuda.is_available()
    rng = np.random.default_rng(7)
    R = 70  # two stage-1 workgroups of 64 replicas, the second ragged
    reps = [dict(model=0, Lx=L, Ly=L, Jx=_f32(rng.uniform(0.3, 0.6)),
                 Jy=_f32(rng.uniform(0.3, 0.6)), h=_f32(rng.uniform(-0.05, 0.05)), beta=1.0, rid=i)
            for i, L in enumerate([8, 16, 32, 64, 16] * 14)]
    smp = Sampler(reps, 5, init=True)
    stats = smp.sweep(2500, 1).contiguous()
    gout = torch.tensor(rng.normal(size=(R, 2)), dtype=torch.float64, device="cuda")
    # first call: 2300 samples (36 chunks, the last ragged); second: 250
    # samples (spinmc_grad takes its one-workgroup form there, the
    # allocation-free call its chunked form: the integer sums agree)
    for n_rec, burn in ((2500, 200), (300, 50)):
        want = _call("spinmc_grad", smp, stats, n_rec, burn, gout)
        got = _call("spinmc_grad_noalloc", smp, stats, n_rec, burn, gout)
        torch.cuda.synchronize()
        assert want[0] == 0 and got[0] == 0
        for a, b in zip(want[1:], got[1:]):
            assert torch.isfinite(b).all()
            assert torch.equal(a, b)
    smp.close()


def test_grad_noalloc_rejects_records_beyond_its_array():
    from paper_2304_01772_amd._lib import lib
    from paper_2304_01772_amd.sampler import Sampler
    R = 64
    smp = Sampler([dict(model=0, Lx=4, Ly=4, Jx=0.5, Jy=0.5, h=0.0, beta=1.0, rid=i)
                   for i in range(R)], 1, init=True)
    # 64 replicas x 40,384 samples = 631 chunks x 13 x 64 int64 > 4 MiB
    n_rec = 40384
    stats = torch.zeros((n_rec, R, smp.width), dtype=torch.int32, device="cuda")
    gout = torch.zeros((R, 2), dtype=torch.float64, device="cuda")
    rc, *_ = _call("spinmc_grad_noalloc", smp, stats, n_rec, 0, gout)
    assert rc == -1
    assert b"static scratch" in lib().spinmc_last_error()
    # one chunk less fits, and equals spinmc_grad
    n_rec = 40320
    want = _call("spinmc_grad", smp, stats, n_rec, 0, gout)
    got = _call("spinmc_grad_noalloc", smp, stats, n_rec, 0, gout)
    torch.cuda.synchronize()
    assert want[0] == 0 and got[0] == 0
    for a, b in zip(want[1:], got[1:]):
        assert torch.equal(a, b)
    smp.close()
