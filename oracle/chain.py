"""ctypes binding of the oracle's C chain (``spinmc_oracle.c``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

All lattices are natural row-major ``[Ly, Lx]`` numpy arrays:
Ising ``int8`` spins in {-1, +1}; Potts ``uint8`` labels in [0, q); CPM
``int32`` cell ids in [0, n_cells].  Statistics rows have 8 int32 entries
(Ising: M, Bx, By; Potts: Nx, Ny, S, nmax) or 16 (CPM: 10 boundary-bond
counts by type pair, H*S as int64 in entries 10/11).

Pins (tests/test_oracle_*.py): Philox known-answer vectors and the rocRAND
implementation; thresholds against brute-force energy differences; chains
against exact enumeration (4x4 Ising, 4x4 q=3 Potts) and exact detailed
balance; CPM invariants and its lambda=0 two-id reduction.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    """Load (building first if needed) ``oracle/liborc.so``."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(_HERE, "liborc.so")
    if not os.path.exists(path):
        from . import build as _b
        _b.build(force=True)
    L = C.CDLL(path)
    L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.orc_philox4x32_10.restype = None
    L.orc_ising_table.argtypes = [C.c_float, C.c_float, C.c_float, C.c_double, _u64p]
    L.orc_ising_table.restype = C.c_int
    L.orc_potts_table.argtypes = [C.c_int, C.c_float, C.c_float, C.c_double, _u64p]
    L.orc_potts_table.restype = C.c_int
    L.orc_ising_init.argtypes = [C.c_int, C.c_int, C.c_uint64, C.c_uint32, _i8p]
    L.orc_ising_init.restype = None
    L.orc_potts_init.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_uint32, _u8p]
    L.orc_potts_init.restype = None
    L.orc_ising_stats.argtypes = [C.c_int, C.c_int, _i8p, _i32p]
    L.orc_ising_stats.restype = None
    L.orc_potts_stats.argtypes = [C.c_int, C.c_int, C.c_int, _u8p, _i32p]
    L.orc_potts_stats.restype = None
    L.orc_ising_run.argtypes = [C.c_int, C.c_int, C.c_float, C.c_float, C.c_float, C.c_double,
                                C.c_uint64, C.c_uint32, C.c_uint64, C.c_int, C.c_int, _i8p,
                                C.c_void_p]
    L.orc_ising_run.restype = C.c_int
    L.orc_potts_run.argtypes = [C.c_int, C.c_int, C.c_int, C.c_float, C.c_float, C.c_double,
                                C.c_uint64, C.c_uint32, C.c_uint64, C.c_int, C.c_int, _u8p,
                                C.c_void_p]
    L.orc_potts_run.restype = C.c_int
    L.orc_cpm_scale.argtypes = [C.c_int, _f32p, C.c_float, C.POINTER(C.c_int32)]
    L.orc_cpm_scale.restype = C.c_int
    L.orc_cpm_stats.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _f32p, _i8p, _i32p,
                                C.c_float, _i32p, _i32p]
    L.orc_cpm_stats.restype = None
    L.orc_cpm_run.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _f32p, _i8p, _i32p, C.c_float,
                              C.c_double, C.c_uint64, C.c_uint32, C.c_uint64, C.c_int, C.c_int,
                              _i32p, _i32p, C.c_void_p]
    L.orc_cpm_run.restype = C.c_int
    L.orc_tri_table.argtypes = [C.c_float, C.c_float, C.c_double, _u64p]
    L.orc_tri_table.restype = C.c_int
    L.orc_tri_stats.argtypes = [C.c_int, C.c_int, _i8p, _i32p]
    L.orc_tri_stats.restype = None
    L.orc_tri_run.argtypes = [C.c_int, C.c_int, C.c_float, C.c_float, C.c_double, C.c_uint64,
                              C.c_uint32, C.c_uint64, C.c_int, C.c_int, _i8p, C.c_void_p]
    L.orc_tri_run.restype = C.c_int
    L.orc_hc_stats.argtypes = [C.c_int, C.c_int, C.c_int, _i8p, _i32p]
    L.orc_hc_stats.restype = None
    L.orc_hc_run.argtypes = [C.c_int, C.c_int, C.c_int, C.c_float, C.c_float, C.c_double,
                             C.c_uint64, C.c_uint32, C.c_uint64, C.c_int, C.c_int, _i8p,
                             C.c_void_p]
    L.orc_hc_run.restype = C.c_int
    L.orc_msc_init.argtypes = [C.c_int, C.c_int, C.c_uint64, C.c_uint32, _u32p]
    L.orc_msc_init.restype = None
    L.orc_msc_stats.argtypes = [C.c_int, C.c_int, _u32p, _i32p]
    L.orc_msc_stats.restype = None
    L.orc_msc_run.argtypes = [C.c_int, C.c_int, C.c_float, C.c_float, C.c_float, C.c_double,
                              C.c_uint64, C.c_uint32, C.c_uint64, C.c_int, C.c_int, _u32p,
                              C.c_void_p]
    L.orc_msc_run.restype = C.c_int
    L.orc_cpm_stats_r.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _f32p, _i8p, _i32p,
                                  C.c_float, _i32p, C.c_int, _i32p]
    L.orc_cpm_stats_r.restype = None
    L.orc_cpm_run_r.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _f32p, _i8p, _i32p,
                                C.c_float, C.c_double, C.c_uint64, C.c_uint32, C.c_uint64,
                                C.c_int, C.c_int, C.c_int, _i32p, _i32p, C.c_void_p]
    L.orc_cpm_run_r.restype = C.c_int
    L.orc_ising_run_batch.argtypes = [C.c_int, _i32p, _i32p, _f32p, _f32p, _f32p, _f64p,
                                      C.c_uint64, _u32p, C.c_uint64, C.c_int, C.c_int, _i8p,
                                      _i64p, C.c_void_p]
    L.orc_ising_run_batch.restype = C.c_int
    L.orc_potts_run_batch.argtypes = [C.c_int, _i32p, _i32p, _i32p, _f32p, _f32p, _f64p,
                                      C.c_uint64, _u32p, C.c_uint64, C.c_int, C.c_int, _u8p,
                                      _i64p, C.c_void_p]
    L.orc_potts_run_batch.restype = C.c_int
    L.orc_philox_grid.argtypes = [C.c_int, C.c_uint32, _u32p, C.c_int, C.c_uint32, C.c_uint32,
                                  C.c_uint32, _u32p]
    L.orc_philox_grid.restype = None
    L.orc_num_threads.argtypes = []
    L.orc_num_threads.restype = C.c_int
    L.orc_set_num_threads.argtypes = [C.c_int]
    L.orc_set_num_threads.restype = None
    _LIB = L
    return L


def _check(rc, what):
    if rc < 0:
        raise ValueError(f"oracle {what} rejected its arguments (code {rc})")
    return rc


# --------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    """Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(c, k, out)
    return out


def philox_grid(n_blocks, c1, rids, c3, seed):
    """Philox4x32-10 words for counters (b, c1, rid, c3), b < n_blocks, one
    row per replica id: uint32 array [len(rids), n_blocks, 4]."""
    rids = np.ascontiguousarray(rids, dtype=np.uint32)
    out = np.zeros((len(rids), n_blocks, 4), np.uint32)
    lib().orc_philox_grid(int(n_blocks), int(c1) & 0xFFFFFFFF, rids, len(rids), int(c3),
                          int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF, out)
    return out


def ising_table(Jx, Jy, h, beta):
    """18 Metropolis thresholds (uint64, in [0, 2^32]) indexed 9[s>0]+3(Sx/2+1)+(Sy/2+1)."""
    T = np.zeros(18, np.uint64)
    _check(lib().orc_ising_table(Jx, Jy, h, beta, T), "ising_table")
    return T


def potts_table(q, J, h, beta):
    """9*(2q-1) thresholds indexed (dn+4)(2q-1) + (s'-s+q-1)."""
    T = np.zeros(9 * (2 * q - 1), np.uint64)
    _check(lib().orc_potts_table(q, J, h, beta, T), "potts_table")
    return T


def ising_init(Lx, Ly, seed, rid):
    s = np.zeros((Ly, Lx), np.int8)
    lib().orc_ising_init(Lx, Ly, seed, rid, s)
    return s


def potts_init(Lx, Ly, q, seed, rid):
    s = np.zeros((Ly, Lx), np.uint8)
    lib().orc_potts_init(Lx, Ly, q, seed, rid, s)
    return s


def ising_stats(sigma):
    sigma = np.ascontiguousarray(sigma, np.int8)
    out = np.zeros(8, np.int32)
    lib().orc_ising_stats(sigma.shape[1], sigma.shape[0], sigma, out)
    return out


def potts_stats(s, q):
    s = np.ascontiguousarray(s, np.uint8)
    out = np.zeros(8, np.int32)
    lib().orc_potts_stats(s.shape[1], s.shape[0], q, s, out)
    return out


def ising_run(sigma, Jx, Jy, h, beta, seed, rid, t0, n_sweeps, record_every=0):
    """Run n sweeps in place on a copy; returns (state, stats[n_rec, 8])."""
    s = np.ascontiguousarray(sigma, np.int8).copy()
    n_rec = n_sweeps // record_every if record_every > 0 else 0
    stats = np.zeros((max(n_rec, 1), 8), np.int32)
    rc = lib().orc_ising_run(s.shape[1], s.shape[0], Jx, Jy, h, beta, seed, rid, t0, n_sweeps,
                             record_every, s, stats.ctypes.data)
    _check(rc, "ising_run")
    return s, stats[:n_rec]


def potts_run(s, q, J, h, beta, seed, rid, t0, n_sweeps, record_every=0):
    s = np.ascontiguousarray(s, np.uint8).copy()
    n_rec = n_sweeps // record_every if record_every > 0 else 0
    stats = np.zeros((max(n_rec, 1), 8), np.int32)
    rc = lib().orc_potts_run(s.shape[1], s.shape[0], q, J, h, beta, seed, rid, t0, n_sweeps,
                             record_every, s, stats.ctypes.data)
    _check(rc, "potts_run")
    return s, stats[:n_rec]


def tri_table(J, h, beta):
    """Thresholds of the triangular-lattice Ising flip, idx = 7 [s > 0] +
    (S6 + 6) / 2."""
    T = np.zeros(14, np.uint64)
    _check(lib().orc_tri_table(J, h, beta, T), "tri_table")
    return T


def tri_stats(sigma):
    """[M, Bh, Bv, Bd, 0...] of a triangular-lattice state (int8 [Ly, Lx])."""
    sigma = np.ascontiguousarray(sigma, np.int8)
    out = np.zeros(8, np.int32)
    lib().orc_tri_stats(sigma.shape[1], sigma.shape[0], sigma, out)
    return out


def tri_run(sigma, J, h, beta, seed, rid, t0, n_sweeps, record_every=0):
    """Triangular-lattice Ising chain on a copy: (state, stats[n_rec, 8])."""
    s = np.ascontiguousarray(sigma, np.int8).copy()
    n_rec = n_sweeps // record_every if record_every > 0 else 0
    stats = np.zeros((max(n_rec, 1), 8), np.int32)
    rc = lib().orc_tri_run(s.shape[1], s.shape[0], J, h, beta, seed, rid, t0, n_sweeps,
                           record_every, s, stats.ctypes.data)
    _check(rc, "tri_run")
    return s, stats[:n_rec]


def hc_init(Lx, Ly, Lz, seed, rid):
    """Initial state of an Lz x Ly x Lx lattice: the Ising init stream over
    the natural index n = (z Ly + y) Lx + x."""
    return ising_init(Lx, Ly * Lz, seed, rid).reshape(Lz, Ly, Lx)


def hc_stats(sigma):
    """[M, Bx, By, Bz, 0...] of an int8 [Lz, Ly, Lx] state."""
    sigma = np.ascontiguousarray(sigma, np.int8)
    out = np.zeros(8, np.int32)
    lib().orc_hc_stats(sigma.shape[2], sigma.shape[1], sigma.shape[0], sigma.reshape(-1), out)
    return out


def hc_run(sigma, J, h, beta, seed, rid, t0, n_sweeps, record_every=0):
    """Chain / square / cubic Ising chain on a copy of an int8 [Lz, Ly, Lx]
    state: (state, stats[n_rec, 8])."""
    s = np.ascontiguousarray(sigma, np.int8).copy()
    n_rec = n_sweeps // record_every if record_every > 0 else 0
    stats = np.zeros((max(n_rec, 1), 8), np.int32)
    rc = lib().orc_hc_run(s.shape[2], s.shape[1], s.shape[0], J, h, beta, seed, rid, t0,
                          n_sweeps, record_every, s.reshape(-1), stats.ctypes.data)
    _check(rc, "hc_run")
    return s, stats[:n_rec]


def msc_init(Lx, Ly, seed, rid):
    """Multispin-coded initial words [Ly, Lx] (uint32, bit b = replica b)."""
    w = np.zeros(Lx * Ly, np.uint32)
    lib().orc_msc_init(Lx, Ly, seed, rid, w)
    return w.reshape(Ly, Lx)


def msc_stats(words):
    """[32, 8] statistics [M, Bx, By, 0...] of the 32 packed replicas."""
    words = np.ascontiguousarray(words, np.uint32)
    out = np.zeros((32, 8), np.int32)
    lib().orc_msc_stats(words.shape[1], words.shape[0], words.reshape(-1), out.reshape(-1))
    return out


def msc_run(words, Jx, Jy, h, beta, seed, rid, t0, n_sweeps, record_every=0):
    """Multispin-coded chain on a copy: (words, stats[n_rec, 32, 8])."""
    w = np.ascontiguousarray(words, np.uint32).copy()
    n_rec = n_sweeps // record_every if record_every > 0 else 0
    stats = np.zeros((max(n_rec, 1), 32, 8), np.int32)
    rc = lib().orc_msc_run(w.shape[1], w.shape[0], Jx, Jy, h, beta, seed, rid, t0, n_sweeps,
                           record_every, w.reshape(-1), stats.ctypes.data)
    _check(rc, "msc_run")
    return w, stats[:n_rec]


def msc_unpack(words):
    """int8 spins [32, Ly, Lx] of packed words."""
    w = np.asarray(words, np.uint32)
    return np.stack([np.where((w >> np.uint32(b)) & np.uint32(1), 1, -1).astype(np.int8)
                     for b in range(32)])


def cpm_scale(J, lam):
    J = np.ascontiguousarray(J, np.float32)
    S = C.c_int32(0)
    rc = lib().orc_cpm_scale(J.shape[0], J.reshape(-1), lam, C.byref(S))
    _check(rc, "cpm_scale")
    return int(S.value)


def cpm_stats(ids, J, cell_type, target_area, lam, nrange=1):
    """nrange: neighbourhood range of the adhesion energy (1: Moore 3x3,
    2: 5x5)."""
    ids = np.ascontiguousarray(ids, np.int32)
    J = np.ascontiguousarray(J, np.float32)
    out = np.zeros(16, np.int32)
    lib().orc_cpm_stats_r(ids.shape[1], ids.shape[0], len(cell_type) - 1, J.shape[0],
                          J.reshape(-1), np.ascontiguousarray(cell_type, np.int8),
                          np.ascontiguousarray(target_area, np.int32), lam, ids, int(nrange),
                          out)
    return out


def cpm_run(ids, J, cell_type, target_area, lam, temperature, seed, rid, t0, n_mcs,
            record_every=0, nrange=1):
    """Returns (ids, area[n_cells+1], stats[n_rec, 16]).  nrange: 1 (Moore
    3x3, 4 colours) or 2 (5x5, 9 colours; Lx and Ly multiples of 6)."""
    ids = np.ascontiguousarray(ids, np.int32).copy()
    J = np.ascontiguousarray(J, np.float32)
    n_cells = len(cell_type) - 1
    area = np.zeros(n_cells + 1, np.int32)
    n_rec = n_mcs // record_every if record_every > 0 else 0
    stats = np.zeros((max(n_rec, 1), 16), np.int32)
    rc = lib().orc_cpm_run_r(ids.shape[1], ids.shape[0], n_cells, J.shape[0], J.reshape(-1),
                             np.ascontiguousarray(cell_type, np.int8),
                             np.ascontiguousarray(target_area, np.int32), lam, temperature,
                             seed, rid, t0, n_mcs, record_every, int(nrange), ids, area,
                             stats.ctypes.data)
    _check(rc, "cpm_run")
    return ids, area, stats[:n_rec]


def ising_run_batch(states, Jx, Jy, h, beta, seed, rids, t0, n_sweeps, record_every=0):
    """Independent Ising chains, OpenMP over replicas.  ``states``: list of
    [Ly, Lx] int8 arrays.  Returns (states, stats[R, n_rec, 8])."""
    R = len(states)
    Ly = np.array([s.shape[0] for s in states], np.int32)
    Lx = np.array([s.shape[1] for s in states], np.int32)
    sizes = (Lx.astype(np.int64) * Ly)
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    flat = np.concatenate([np.ascontiguousarray(s, np.int8).reshape(-1) for s in states])
    n_rec = n_sweeps // record_every if record_every > 0 else 0
    stats = np.zeros((R, max(n_rec, 1), 8), np.int32)
    rc = lib().orc_ising_run_batch(R, Lx, Ly, np.asarray(Jx, np.float32),
                                   np.asarray(Jy, np.float32), np.asarray(h, np.float32),
                                   np.asarray(beta, np.float64), seed,
                                   np.asarray(rids, np.uint32), t0, n_sweeps, record_every,
                                   flat, off, stats.ctypes.data)
    _check(rc, "ising_run_batch")
    out = [flat[o:o + n].reshape(y, x) for o, n, y, x in zip(off, sizes, Ly, Lx)]
    return out, stats[:, :n_rec]


def potts_run_batch(states, q, J, h, beta, seed, rids, t0, n_sweeps, record_every=0):
    R = len(states)
    Ly = np.array([s.shape[0] for s in states], np.int32)
    Lx = np.array([s.shape[1] for s in states], np.int32)
    sizes = (Lx.astype(np.int64) * Ly)
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    flat = np.concatenate([np.ascontiguousarray(s, np.uint8).reshape(-1) for s in states])
    n_rec = n_sweeps // record_every if record_every > 0 else 0
    stats = np.zeros((R, max(n_rec, 1), 8), np.int32)
    rc = lib().orc_potts_run_batch(R, Lx, Ly, np.asarray(q, np.int32), np.asarray(J, np.float32),
                                   np.asarray(h, np.float32), np.asarray(beta, np.float64), seed,
                                   np.asarray(rids, np.uint32), t0, n_sweeps, record_every,
                                   flat, off, stats.ctypes.data)
    _check(rc, "potts_run_batch")
    out = [flat[o:o + n].reshape(y, x) for o, n, y, x in zip(off, sizes, Ly, Lx)]
    return out, stats[:, :n_rec]


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(n):
    """OpenMP threads of later oracle calls (1: every chain on one thread)."""
    lib().orc_set_num_threads(int(n))
