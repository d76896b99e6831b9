"""The C ABI without a GPU: the library loads, exports every function that
include/spinmc.h declares, validates arguments before touching a device, and
reports a missing device cleanly."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spinmc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spinmc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2304_01772_amd import _lib
    return _lib.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["spinmc_create", "spinmc_sweep", "spinmc_measure", "spinmc_grad",
                 "spinmc_destroy", "spinmc_get_state", "spinmc_set_state", "spinmc_autotune",
                 "spinmc_mlp_forward", "spinmc_mlp_backward", "spinmc_mlp_adam"]:
        assert must in names


def test_every_declared_symbol_is_exported(L):
    from paper_2304_01772_amd import _lib
    nm = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                        text=True, check=True).stdout
    exported = set(l.split()[-1] for l in nm.splitlines() if l.strip())
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    # and the Python binding knows all of them
    assert set(declared_functions()) <= set(_lib.SIGNATURES)


def _desc(**kw):
    from paper_2304_01772_amd import _lib
    d = (_lib.ReplicaDesc * 1)()
    d[0].model, d[0].Lx, d[0].Ly, d[0].q = 0, 8, 8, 2
    d[0].Jx = d[0].Jy = 1.0
    d[0].beta = 0.5
    for k, v in kw.items():
        setattr(d[0], k, v)
    return d


@pytest.mark.parametrize("kw,code", [
    (dict(Lx=7), -1), (dict(Ly=0), -1), (dict(model=6), -1), (dict(beta=-1.0), -1),
    (dict(beta=float("nan")), -1), (dict(model=1, q=1), -1), (dict(model=1, q=300), -1),
    (dict(model=1, q=200), -2), (dict(model=1, q=3, Jy=0.5), -2), (dict(h=float("inf")), -1),
    # triangular lattice: multiples of 3, one coupling
    (dict(model=3), -1), (dict(model=3, Lx=9, Ly=10), -1), (dict(model=3, Lx=9, Ly=9, Jy=0.5), -1),
    (dict(model=3, Lx=9, Ly=9, beta=-1.0), -1),
    # chain / cubic: Lx even, Ly and Lz 1 or even
    (dict(model=4, Lx=7), -1), (dict(model=4, Ly=3), -1), (dict(model=4, Lz=3), -1),
    (dict(model=4, Lz=-2), -1), (dict(model=4, Jy=0.5), -1),
    # multispin coding: Lx a multiple of 8, Ly even
    (dict(model=5, Lx=12), -1), (dict(model=5, Ly=7), -1), (dict(model=5, beta=-2.0), -1),
])
def test_validation_precedes_device(L, kw, code):
    ctx = C.c_void_p()
    rc = L.spinmc_create(_desc(**kw), 1, 1, 1, None, C.byref(ctx))
    assert rc == code, L.spinmc_last_error()
    assert not ctx.value
    assert L.spinmc_last_error()


def test_null_and_count_checks(L):
    ctx = C.c_void_p()
    assert L.spinmc_create(None, 1, 1, 1, None, C.byref(ctx)) == -1
    assert L.spinmc_create(_desc(), 0, 1, 1, None, C.byref(ctx)) == -1
    assert L.spinmc_create(_desc(), 1, 1, 7, None, C.byref(ctx)) == -1
    assert L.spinmc_sweep(None, 1, 0, None) == -1
    assert L.spinmc_destroy(None) == 0


def test_no_device_is_reported(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    ctx = C.c_void_p()
    assert L.spinmc_create(_desc(), 1, 1, 1, None, C.byref(ctx)) == -4
    assert b"device" in L.spinmc_last_error()


def test_mlp_parameter_count(L):
    assert L.spinmc_mlp_num_params() == 4 * 128 + 128 + 128 * 128 + 128 + 3 * 128 + 3


def _dmc(**kw):
    from paper_2304_01772_amd import _lib
    p = _lib.DmcParams()
    p.R, p.Lx, p.Ly, p.n_sweeps = 2, 8, 6, 3
    p.beta, p.alpha, p.h = 0.5, 4.0, 0.0
    p.seed, p.t0, p.rid0 = 1, 0, 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_dmc_sizes_and_validation_without_a_device(L):
    """Buffer sizes of the differentiable-MC calls, and their argument checks
    (rejected before anything touches a device)."""
    p = _dmc()
    assert L.spinmc_dmc_save_floats(C.byref(p)) == 2 * 3 * 2 * 6 * 4
    assert L.spinmc_dmc_work_floats(C.byref(p)) == 2 * 2 * 6 * 4
    for bad in (dict(Lx=7), dict(Ly=0), dict(R=0), dict(n_sweeps=-1), dict(alpha=-1.0),
                dict(beta=float("nan")), dict(h=float("inf")), dict(rid0=2 ** 32 - 1),
                # pass counters p = 2t + c of every sweep must fit 32 bits
                dict(t0=2 ** 31 - 2), dict(t0=2 ** 40)):
        q = _dmc(**bad)
        assert L.spinmc_dmc_save_floats(C.byref(q)) < 0, bad
        assert L.spinmc_dmc_forward(C.byref(q), 1, 1, 1, 1, None) == -1, bad
    # null buffers
    assert L.spinmc_dmc_forward(C.byref(p), None, 1, 1, 1, None) == -1
    assert L.spinmc_dmc_forward(C.byref(p), 1, 1, 1, None, None) == -1
    assert L.spinmc_dmc_backward(C.byref(p), 1, 1, 1, 1, 1, 1, 1, None, None) == -1
    assert L.spinmc_adam(1, 1, 1, 1, 0, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert L.spinmc_adam(1, 1, 1, 1, 10, 0, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    # spin-value optimisation pieces
    assert L.spinmc_dmc_energy(C.byref(_dmc(Lx=7)), 1, 1, 1, 1, None, None) == -1
    assert L.spinmc_dmc_energy(C.byref(p), 1, 1, 1, None, None, None) == -1
    assert L.spinmc_dmc_discretize(-1, 1, None, 1.0, 1, None) == -1
    assert L.spinmc_dmc_discretize(2 ** 31 + 1, 1, None, 1.0, 1, None) == -1
    assert L.spinmc_dmc_discretize(4, 1, None, float("nan"), 1, None) == -1
    assert L.spinmc_dmc_discretize(4, None, None, 1.0, 1, None) == -1
    assert L.spinmc_dmc_discretize(0, None, None, 1.0, None, None) == 0


def test_cpm_neighbourhood_validation_without_a_device(L):
    """cpm_range outside {0, 1, 2}, the 5x5 neighbourhood on widths that are
    not multiples of 6, and mixed ranges in one context are rejected before
    any device call."""
    import numpy as np
    from paper_2304_01772_amd import _lib
    J = np.zeros((2, 2), np.float32)
    ct = np.array([0, 1], np.int8)
    A = np.array([0, 4], np.int32)

    def descs(*specs):
        d = (_lib.ReplicaDesc * len(specs))()
        for i, (Lx, Ly, rng) in enumerate(specs):
            d[i].model, d[i].Lx, d[i].Ly, d[i].q, d[i].rid = 2, Lx, Ly, 1, i
            d[i].n_types = 2
            d[i].adhesion = J.ctypes.data_as(C.POINTER(C.c_float))
            d[i].cell_type = ct.ctypes.data_as(C.POINTER(C.c_int8))
            d[i].target_area = A.ctypes.data_as(C.POINTER(C.c_int32))
            d[i].lambda_area, d[i].temperature, d[i].cpm_range = 1.0, 2.0, rng
        return d
    ctx = C.c_void_p()
    for specs in [((12, 12, 3),), ((12, 12, -1),), ((8, 12, 2),), ((12, 16, 2),),
                  ((12, 12, 2), (12, 12, 1))]:
        assert L.spinmc_create(descs(*specs), len(specs), 1, 0, None, C.byref(ctx)) == -1, specs
        assert not ctx.value
