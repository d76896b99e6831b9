"""Thin Python binding of libspinmc: argument marshalling only.

PyTorch provides the device buffers (statistics, observables, gradients) and
the HIP stream; every step of the sweep runs in the library's kernels.
"""
import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import (CPM, ISING, ISING_HC, ISING_MSC, ISING_TRI, POTTS, ReplicaDesc, Schedule,
                   check, lib)

__all__ = ["Sampler", "ISING", "POTTS", "CPM", "MODES"]

MODES = {"auto": 0, "resident": 1, "stream": 2, "hybrid": 3}
NT_ON, NT_OFF, PERSIST = 1, 2, 4  # spinmc_schedule.flags


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream, C.c_void_p(stream.cuda_stream)


class Sampler:
    """A batch of independent replicas (Methods, batched tensors) behind one
    libspinmc context.

    ``replicas``: sequence of dicts with keys model (0 Ising, 1 Potts, 2 CPM,
    3 triangular-lattice Ising, 4 chain / square / cubic Ising with an extra
    key Lz, 5 a multispin-coded group of 32 square-lattice Ising replicas,
    whose state is one uint32 word per site), Lx, Ly and the model's
    parameters (q, Jx,
    Jy, h, beta, rid; CPM: n_cells as q, n_types,
    adhesion, cell_type, target_area, lambda_area, temperature and optionally
    cpm_range, 1 for the Moore 3x3 neighbourhood or 2 for 5x5).
    """

    def __init__(self, replicas, seed, init=True, stream=None, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("spinmc needs a GPU (HIP device); none is visible")
        self.device = torch.device(device)
        self.stream, sh = _stream_handle(stream)
        n = len(replicas)
        descs = (ReplicaDesc * n)()
        self._keep = []
        self.replicas = [dict(r) for r in replicas]
        for i, r in enumerate(replicas):
            d = descs[i]
            d.model = int(r.get("model", ISING))
            d.Lx, d.Ly = int(r["Lx"]), int(r["Ly"])
            d.q = int(r.get("q", 2))
            d.Jx = float(r.get("Jx", 1.0))
            d.Jy = float(r.get("Jy", r.get("Jx", 1.0)))
            d.h = float(r.get("h", 0.0))
            d.beta = float(r.get("beta", 0.0))
            d.rid = int(r.get("rid", i))
            d.Lz = int(r.get("Lz", 1))
            if d.model == CPM:
                adh = np.ascontiguousarray(r["adhesion"], np.float32)
                ct = np.ascontiguousarray(r["cell_type"], np.int8)
                ta = np.ascontiguousarray(r["target_area"], np.int32)
                self._keep += [adh, ct, ta]
                d.n_types = int(adh.shape[0])
                d.adhesion = adh.ctypes.data_as(C.POINTER(C.c_float))
                d.cell_type = ct.ctypes.data_as(C.POINTER(C.c_int8))
                d.target_area = ta.ctypes.data_as(C.POINTER(C.c_int32))
                d.lambda_area = float(r["lambda_area"])
                d.temperature = float(r["temperature"])
                d.cpm_range = int(r.get("cpm_range", 1))
        ctx = C.c_void_p()
        check(lib().spinmc_create(descs, n, int(seed), 1 if init else 0, sh, C.byref(ctx)))
        self._keep = []
        self.ctx = ctx
        self.R = lib().spinmc_num_replicas(ctx)  # 32 per multispin-coded group
        self.width = lib().spinmc_stats_width(ctx)

    # -------------------------------------------------------------- basics
    def close(self):
        if getattr(self, "ctx", None):
            lib().spinmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self):
        v = C.c_uint64()
        check(lib().spinmc_sweep_counter(self.ctx, C.byref(v)))
        return int(v.value)

    def _elem(self, r):
        m = self.replicas[r].get("model", ISING)
        return {ISING: np.int8, ISING_TRI: np.int8, ISING_HC: np.int8, POTTS: np.uint8,
                CPM: np.int32, ISING_MSC: np.uint32}[m]

    def _shape(self, r):
        rep = self.replicas[r]
        if rep.get("model", ISING) == ISING_HC:
            return (max(int(rep.get("Lz", 1)), 1), rep["Ly"], rep["Lx"])
        return (rep["Ly"], rep["Lx"])

    def get_state(self, r):
        out = np.empty(self._shape(r), self._elem(r))
        check(lib().spinmc_get_state(self.ctx, r, out.ctypes.data, out.nbytes))
        return out

    def set_state(self, r, arr):
        arr = np.ascontiguousarray(arr, self._elem(r))
        check(lib().spinmc_set_state(self.ctx, r, arr.ctypes.data, arr.nbytes))

    def thresholds(self, r):
        n = C.c_int32()
        aux = C.c_int64()
        check(lib().spinmc_thresholds(self.ctx, r, None, 0, C.byref(n), C.byref(aux)))
        T = np.zeros(max(n.value, 1), np.uint64)
        check(lib().spinmc_thresholds(self.ctx, r, T.ctypes.data_as(C.POINTER(C.c_uint64)),
                                      len(T), C.byref(n), C.byref(aux)))
        return T[: n.value], int(aux.value)

    # ------------------------------------------------------------- sweeps
    def _same_device(self, t):
        want = self.device
        if t.device.type != want.type:
            return False
        if want.index is not None:
            return t.device.index == want.index
        return want.type != "cuda" or t.device.index == torch.cuda.current_device()

    def _check_stats(self, stats, rows, what):
        """The library writes or reads stats rows through a raw pointer: the
        tensor must be int32, contiguous, on this sampler's device, shaped
        [>= rows, R, width]."""
        if not isinstance(stats, torch.Tensor):
            raise ValueError(f"{what}: stats must be a torch.Tensor")
        if stats.dtype != torch.int32:
            raise ValueError(f"{what}: stats must be int32, got {stats.dtype}")
        if not self._same_device(stats):
            raise ValueError(f"{what}: stats is on {stats.device}, the sampler on {self.device}")
        if not stats.is_contiguous():
            raise ValueError(f"{what}: stats must be contiguous")
        if stats.dim() != 3 or tuple(stats.shape[1:]) != (self.R, self.width) or \
                stats.shape[0] < rows:
            raise ValueError(f"{what}: stats of shape {tuple(stats.shape)}, need "
                             f"[>= {rows}, {self.R}, {self.width}]")

    def sweep(self, n, record_every=0, stats=None):
        """Run n sweeps; returns the int32 statistics tensor
        [n // record_every, R, width] on the device (or None)."""
        if record_every > 0:
            n_rec = n // record_every
            if stats is None:
                stats = torch.empty((max(n_rec, 1), self.R, self.width), dtype=torch.int32,
                                    device=self.device)
            self._check_stats(stats, n_rec, "sweep")
            ptr = C.c_void_p(stats.data_ptr())
        else:
            ptr = None
        check(lib().spinmc_sweep(self.ctx, int(n), int(record_every), ptr))
        return stats[: n // record_every] if record_every > 0 else None

    def measure(self):
        stats = torch.empty((self.R, self.width), dtype=torch.int32, device=self.device)
        obs = torch.empty((self.R, 4), dtype=torch.float64, device=self.device)
        check(lib().spinmc_measure(self.ctx, C.c_void_p(stats.data_ptr()),
                                   C.c_void_p(obs.data_ptr())))
        return stats, obs

    def grad(self, stats, burn_in, grad_out=None):
        """Covariance-estimator gradients from recorded statistics.
        Returns (means [R,4] = (<e>, <|m|>, <m^2>, chi), grads [R,2,3],
        dtheta [R,3] or None)."""
        return self._grad("spinmc_grad", stats, burn_in, grad_out)

    def grad_noalloc(self, stats, burn_in, grad_out=None):
        """As grad, through spinmc_grad_noalloc (chunk sums in the library's
        static per-device array; the library allocates nothing, the outputs
        are still new tensors here)."""
        return self._grad("spinmc_grad_noalloc", stats, burn_in, grad_out)

    def _grad(self, entry, stats, burn_in, grad_out):
        if isinstance(stats, torch.Tensor) and stats.dim() == 3:
            stats = stats.contiguous()
        self._check_stats(stats, 1, "grad")
        n_rec = stats.shape[0]
        means = torch.empty((self.R, 4), dtype=torch.float64, device=self.device)
        grads = torch.empty((self.R, 2, 3), dtype=torch.float64, device=self.device)
        dth = None
        gptr = None
        if grad_out is not None:
            grad_out = grad_out.to(device=self.device, dtype=torch.float64).contiguous()
            dth = torch.empty((self.R, 3), dtype=torch.float64, device=self.device)
            gptr = C.c_void_p(grad_out.data_ptr())
        check(getattr(lib(), entry)(self.ctx, C.c_void_p(stats.data_ptr()), int(n_rec),
                                    int(burn_in), gptr, C.c_void_p(means.data_ptr()),
                                    C.c_void_p(grads.data_ptr()),
                                    C.c_void_p(dth.data_ptr()) if dth is not None else None))
        return means, grads, dth

    # ------------------------------------------------------------- timing
    KERNELS = {"stream_ising": 0, "resident": 1, "cpm_pass": 3, "stream_potts": 4, "tri_pass": 5,
               "hc_pass": 6, "msc_pass": 7, "persist_ising": 8, "persist_potts": 9,
               "cpm_tiled": 10}

    def profile(self, enable=True):
        check(lib().spinmc_profile(self.ctx, 1 if enable else 0))

    def profile_read(self, kind):
        ms = C.c_double()
        n = C.c_int64()
        check(lib().spinmc_profile_read(self.ctx, self.KERNELS.get(kind, kind), C.byref(ms),
                                        C.byref(n)))
        return float(ms.value), int(n.value)

    # ---------------------------------------------------------- schedules
    def set_schedule(self, mode="auto", tile_rows=0, wg_threads=0, nt=None, persistent=False,
                     rpb=0, flags=None):
        """nt: None (size rule), True or False (nontemporal own-plane access
        of the streamed passes forced on / off); persistent: unrecorded
        sweeps run the streamed replicas in one persistent launch per chunk
        (tile_rows = slab height, 0 = sized by the chip's occupancy); rpb:
        replicas per resident workgroup (0 = packing rule).  flags, if
        given, replaces nt and persistent (the raw schedule flags)."""
        if flags is None:
            flags = 0 if nt is None else (NT_ON if nt else NT_OFF)
            if persistent:
                flags |= PERSIST
        s = Schedule(MODES[mode] if isinstance(mode, str) else int(mode), int(tile_rows),
                     int(wg_threads), int(flags), int(rpb))
        check(lib().spinmc_set_schedule(self.ctx, C.byref(s)))

    def get_schedule(self):
        s = Schedule()
        check(lib().spinmc_get_schedule(self.ctx, C.byref(s)))
        return dict(mode=s.mode, tile_rows=s.tile_rows, wg_threads=s.wg_threads, flags=s.flags,
                    rpb=s.rpb)

    def schedule_sites(self, by_model=False):
        """(streamed, resident) sites per sweep under the current schedule;
        with by_model, two dicts keyed "ising", "potts", "cpm"."""
        a, b = (C.c_int64 * 3)(), (C.c_int64 * 3)()
        check(lib().spinmc_schedule_sites(self.ctx, a, b))
        if by_model:
            names = ("ising", "potts", "cpm")
            return ({n: int(a[i]) for i, n in enumerate(names)},
                    {n: int(b[i]) for i, n in enumerate(names)})
        return int(sum(a)), int(sum(b))

    def autotune(self, trial_sweeps=20, mode=None, cache=True):
        """Time candidate schedules (optionally of one mode) and keep the
        fastest; returns (schedule dict, candidate rates in attempts/ns).
        With cache, a choice already made in this process (or in the file
        named by SPINMC_AUTOTUNE_CACHE) for the same device and shapes is
        reused without trials (the rates list is then empty)."""
        m = MODES[mode] if isinstance(mode, str) else int(mode or 0)
        if not cache:
            if m > 0:
                raise ValueError("autotune: cache=False tries every mode")
            m = -1
        s = Schedule(m, 0, 0, 0, 0)
        rates = (C.c_double * 64)()
        n = C.c_int32()
        check(lib().spinmc_autotune(self.ctx, int(trial_sweeps), C.byref(s), rates, 64,
                                    C.byref(n)))
        return dict(mode=s.mode, tile_rows=s.tile_rows, wg_threads=s.wg_threads, flags=s.flags,
                    rpb=s.rpb), [rates[i] for i in range(n.value)]
