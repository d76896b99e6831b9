"""ctypes loader for ``libspinmc.so`` (argument marshalling only).

The library is built in-tree by ``paper_2304_01772_amd/build.py``.  There is
no fallback: if the shared object is missing, ``lib()`` raises.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspinmc.so")

OK, E_INVALID, E_UNSUPPORTED, E_NOMEM, E_DEVICE, E_NOT_REPRESENTABLE, E_STATE = 0, -1, -2, -3, -4, -5, -6
ISING, POTTS, CPM, ISING_TRI, ISING_HC, ISING_MSC = 0, 1, 2, 3, 4, 5


class SpinmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"spinmc error {code}: {msg}")
        self.code = code


class ReplicaDesc(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("Lx", C.c_int32), ("Ly", C.c_int32), ("q", C.c_int32),
        ("Jx", C.c_float), ("Jy", C.c_float), ("h", C.c_float),
        ("beta", C.c_double), ("rid", C.c_uint32),
        ("n_types", C.c_int32), ("adhesion", C.POINTER(C.c_float)),
        ("cell_type", C.POINTER(C.c_int8)), ("target_area", C.POINTER(C.c_int32)),
        ("lambda_area", C.c_float), ("temperature", C.c_double), ("cpm_range", C.c_int32),
        ("Lz", C.c_int32),
    ]


class Schedule(C.Structure):
    _fields_ = [("mode", C.c_int32), ("tile_rows", C.c_int32), ("wg_threads", C.c_int32),
                ("flags", C.c_int32), ("rpb", C.c_int32)]


class DmcParams(C.Structure):
    _fields_ = [("R", C.c_int32), ("Lx", C.c_int32), ("Ly", C.c_int32), ("n_sweeps", C.c_int32),
                ("beta", C.c_float), ("alpha", C.c_float), ("h", C.c_float),
                ("reserved", C.c_float), ("seed", C.c_uint64), ("t0", C.c_uint64),
                ("rid0", C.c_uint32), ("reserved2", C.c_uint32)]


# name -> (restype, argtypes); the exported C ABI of include/spinmc.h
SIGNATURES = {
    "spinmc_create": (C.c_int, [C.POINTER(ReplicaDesc), C.c_int32, C.c_uint64, C.c_int32,
                                C.c_void_p, C.POINTER(C.c_void_p)]),
    "spinmc_destroy": (C.c_int, [C.c_void_p]),
    "spinmc_set_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t]),
    "spinmc_get_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t]),
    "spinmc_sweep": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "spinmc_measure": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "spinmc_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p]),
    "spinmc_grad_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p]),
    "spinmc_sweep_counter": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64)]),
    "spinmc_stats_width": (C.c_int, [C.c_void_p]),
    "spinmc_num_replicas": (C.c_int, [C.c_void_p]),
    "spinmc_thresholds": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_uint64), C.c_int32,
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "spinmc_set_schedule": (C.c_int, [C.c_void_p, C.POINTER(Schedule)]),
    "spinmc_get_schedule": (C.c_int, [C.c_void_p, C.POINTER(Schedule)]),
    "spinmc_schedule_sites": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "spinmc_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Schedule),
                                  C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32)]),
    "spinmc_last_error": (C.c_char_p, []),
    "spinmc_profile": (C.c_int, [C.c_void_p, C.c_int32]),
    "spinmc_profile_read": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                      C.POINTER(C.c_int64)]),
    "spinmc_mlp_num_params": (C.c_int, []),
    "spinmc_mlp_act_floats": (C.c_int, [C.c_int32]),
    "spinmc_mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "spinmc_mlp_workspace_floats": (C.c_int, [C.c_int32]),
    "spinmc_mlp_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p]),
    "spinmc_mlp_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                                        C.c_float, C.c_float, C.c_float, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p]),
    "spinmc_mlp_adam": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                  C.c_float, C.c_float, C.c_float, C.c_float, C.c_void_p]),
    "spinmc_adam": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                              C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float,
                              C.c_void_p]),
    "spinmc_dmc_save_floats": (C.c_int64, [C.POINTER(DmcParams)]),
    "spinmc_dmc_work_floats": (C.c_int64, [C.POINTER(DmcParams)]),
    "spinmc_dmc_forward": (C.c_int, [C.POINTER(DmcParams), C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "spinmc_dmc_backward": (C.c_int, [C.POINTER(DmcParams), C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p]),
    "spinmc_dmc_energy": (C.c_int, [C.POINTER(DmcParams), C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p]),
    "spinmc_dmc_discretize": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_float,
                                        C.c_void_p, C.c_void_p]),
}

_LIB = None


def lib():
    """Load the in-tree HIP library; raise if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python paper_2304_01772_amd/build.py` "
                          "(or __graft_entry__.build()) first")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def check(rc):
    if rc != OK:
        msg = lib().spinmc_last_error()
        raise SpinmcError(rc, msg.decode() if msg else "")
    return rc
