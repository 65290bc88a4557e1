"""Python binding of ``libmcheis.so`` (the C ABI in ``include/mcheis.h``).

Argument marshalling only: every step of the sweep runs in the library's HIP
kernels.  PyTorch supplies device memory (spin planes, scratch) and the HIP
stream.  If the built library is missing, importing this module raises.

Model: Eq. (1) of arXiv:2106.11286 (anisotropic classical Heisenberg
Hamiltonian); dynamics: single-spin Metropolis by sublattice colour; the
magnetisation follows Eq. (2).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcheis.so")

SC, BCC, FCC = 0, 1, 2
F32, F64 = 0, 1
INIT_RANDOM, INIT_ALIGNED, INIT_USER = 0, 1, 2
MEASURE = 1
PERSISTENT = 2
TUNED_LAUNCH = 4
BLOCK_CONFLICTS = 4
BLOCK_RESET = 8
STATUS = {0: "MC_OK", -1: "MC_E_ARG", -2: "MC_E_UNSUPPORTED", -3: "MC_E_BUFFER",
          -4: "MC_E_DEVICE", -5: "MC_E_STATE"}
KINDS = {"sc": SC, "bcc": BCC, "fcc": FCC}


class MCError(RuntimeError):
    def __init__(self, func, status, message):
        super().__init__(f"{func}: {STATUS.get(status, status)}: {message}")
        self.status = status


class ReplicaDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
                ("Lz", ctypes.c_int32), ("periodic_mask", ctypes.c_uint32),
                ("replica_id", ctypes.c_uint32), ("sphere_radius", ctypes.c_double),
                ("J", ctypes.c_double), ("K", ctypes.c_double), ("e", ctypes.c_double * 3),
                ("T", ctypes.c_double)]


class SpinBuffers(ctypes.Structure):
    _fields_ = [("sx", ctypes.c_void_p), ("sy", ctypes.c_void_p), ("sz", ctypes.c_void_p),
                ("capacity_sites", ctypes.c_uint64)]


class Obs(ctypes.Structure):
    _fields_ = [("sweep", ctypes.c_uint64), ("n_sites", ctypes.c_uint64),
                ("n_accepted", ctypes.c_uint64), ("M", ctypes.c_double * 3),
                ("absM", ctypes.c_double), ("E", ctypes.c_double), ("E_exch", ctypes.c_double),
                ("E_anis", ctypes.c_double)]


class Schedule(ctypes.Structure):
    _fields_ = [("n_T", ctypes.c_int32), ("T", ctypes.POINTER(ctypes.c_double)),
                ("n_equil", ctypes.c_uint32), ("n_meas", ctypes.c_uint32),
                ("measure_every", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64)] + [(k, ctypes.c_double) for k in (
        "abs_m", "abs_m_err", "m2", "m2_err", "m4", "m4_err", "e", "e_err", "U4", "C", "chi",
        "acceptance", "U4_err")]


# Every exported symbol with its argument types (checked against the header in
# the CPU test suite).
_SIGNATURES = {
    "mc_required_sites": (ctypes.c_int, [ctypes.POINTER(ReplicaDesc), ctypes.POINTER(ctypes.c_uint64)]),
    "mc_occupied_sites": (ctypes.c_int, [ctypes.POINTER(ReplicaDesc), ctypes.POINTER(ctypes.c_uint64)]),
    "mc_required_scratch": (ctypes.c_int, [ctypes.POINTER(ReplicaDesc), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_uint64)]),
    "mc_init_lattice": (ctypes.c_int, [ctypes.POINTER(ReplicaDesc), ctypes.c_int32, ctypes.c_int,
                                       ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(SpinBuffers),
                                       ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "mc_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32]),
    "mc_sweep_timed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "mc_observables": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Obs), ctypes.c_int32]),
    "mc_measure_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Obs), ctypes.c_int32]),
    "mc_run_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Schedule), ctypes.POINTER(Obs),
                                       ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]),
    "mc_set_temperatures": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                           ctypes.c_int32]),
    "mc_debug_pass": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p)]),
    "mc_layout_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "mc_set_tile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32]),
    "mc_set_second_buffers": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SpinBuffers)]),
    "mc_get_state_buffers": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.POINTER(SpinBuffers)]),
    "mc_get_tile": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint64)]),
    "mc_get_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "mc_set_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "mc_num_colours": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "mc_series_stats": (ctypes.c_int, [ctypes.POINTER(Obs), ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_double, ctypes.POINTER(Stats)]),
    "mc_set_watchdog": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    "mc_set_persistent_mode": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "mc_block_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32,
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "mc_block_steps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                      ctypes.c_uint64]),
    "mc_block_counts": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_uint64)]),
    "mc_exchange_init": (ctypes.c_int, [ctypes.c_void_p]),
    "mc_exchange_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_uint32]),
    "mc_exchange_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "mc_get_persistent_queues": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "mc_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_char_p,
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "mc_measure_buffers": (ctypes.c_int, [ctypes.POINTER(ReplicaDesc), ctypes.c_int,
                                          ctypes.POINTER(SpinBuffers), ctypes.c_void_p,
                                          ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]),
    "mc_measure_buffers_static": (ctypes.c_int, [ctypes.POINTER(ReplicaDesc), ctypes.c_int,
                                                 ctypes.POINTER(SpinBuffers), ctypes.c_void_p,
                                                 ctypes.c_void_p]),
    "mc_get_tuned_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "mc_tune_device_key": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_char_p, ctypes.c_uint64]),
    "mc_synchronize": (ctypes.c_int, [ctypes.c_void_p]),
    "mc_destroy": (None, [ctypes.c_void_p]),
    "mc_last_error": (ctypes.c_char_p, []),
    "mc_version": (ctypes.c_char_p, []),
    "mc_stream_probe": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_double)]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2106_11286_amd.build` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def _check(name, status):
    if status != 0:
        raise MCError(name, status, LIB.mc_last_error().decode())


def last_error() -> str:
    return LIB.mc_last_error().decode()


def version() -> str:
    return LIB.mc_version().decode()


def tune_device_key(arch: str, n_cu: int, n_xcd: int) -> str:
    """``mc_tune_device_key``: the device part of the autotuner's cache key."""
    buf = ctypes.create_string_buffer(256)
    _check("mc_tune_device_key", LIB.mc_tune_device_key(arch.encode(), int(n_cu), int(n_xcd), buf,
                                                        len(buf)))
    return buf.value.decode()


def stream_probe(x, y, z, grid: int = 2048, reps: int = 10, stream=None) -> float:
    """``mc_stream_probe``: mean ms per launch of a colour pass's HBM access
    pattern (no arithmetic) over three device tensors of 2*P elements (float32
    or float64; overwritten)."""
    import torch

    for t in (x, y, z):
        if not (t.is_cuda and t.is_contiguous() and t.dtype == x.dtype and t.numel() == x.numel()):
            raise ValueError("x, y, z must be contiguous CUDA tensors of one dtype and size")
    prec = {torch.float32: F32, torch.float64: F64}[x.dtype]
    st = (stream or torch.cuda.current_stream(x.device)).cuda_stream
    ms = ctypes.c_double()
    _check("mc_stream_probe", LIB.mc_stream_probe(prec, x.data_ptr(), y.data_ptr(), z.data_ptr(),
                                                  x.numel() // 2, int(grid), int(reps),
                                                  ctypes.c_void_p(st), ctypes.byref(ms)))
    return ms.value


@dataclass
class Replica:
    """One lattice replica (see ``mc_replica_desc``)."""
    kind: str = "sc"
    L: Sequence[int] = (16, 16, 16)
    periodic_mask: int = 7
    sphere_radius: float = 0.0
    J: float = 1.0
    K: float = 0.0
    e: Sequence[float] = (0.0, 0.0, 1.0)
    T: float = 1.0
    replica_id: int = 0

    def desc(self) -> ReplicaDesc:
        d = ReplicaDesc()
        d.kind = KINDS[self.kind] if isinstance(self.kind, str) else int(self.kind)
        L = list(self.L) if not isinstance(self.L, int) else [self.L] * 3
        d.Lx, d.Ly, d.Lz = int(L[0]), int(L[1]), int(L[2])
        d.periodic_mask = int(self.periodic_mask)
        d.replica_id = int(self.replica_id)
        d.sphere_radius = float(self.sphere_radius)
        d.J, d.K, d.T = float(self.J), float(self.K), float(self.T)
        for i in range(3):
            d.e[i] = float(self.e[i])
        return d


def required_sites(rep: Replica) -> int:
    n = ctypes.c_uint64()
    d = rep.desc()
    _check("mc_required_sites", LIB.mc_required_sites(ctypes.byref(d), ctypes.byref(n)))
    return int(n.value)


MEASURE_WORKSPACE_BYTES = 65536  # MC_MEASURE_WORKSPACE_BYTES


def _record_dict(r) -> dict:
    return {"M": np.array(r[0:3]), "E_exch": float(r[3]), "E_anis": float(r[4]),
            "E": float(r[3] + r[4]), "n_sites": int(r[5])}


def measure_buffers(rep: Replica, precision: str, sx, sy, sz, workspace=None) -> dict:
    """``mc_measure_buffers``: from-scratch observables of spins held in three
    device tensors (library layout) on the current stream; synchronises and
    returns {M (sums), E_exch, E_anis, E, n_sites}."""
    prec = {"f32": F32, "f64": F64}[precision]
    d = rep.desc()
    b = SpinBuffers(sx.data_ptr(), sy.data_ptr(), sz.data_ptr(), int(sx.numel()))
    if workspace is None:
        workspace = torch.empty(MEASURE_WORKSPACE_BYTES, dtype=torch.uint8, device=sx.device)
    rec = torch.zeros(8, dtype=torch.float64, device=sx.device)
    stream = torch.cuda.current_stream(sx.device).cuda_stream
    _check("mc_measure_buffers", LIB.mc_measure_buffers(
        ctypes.byref(d), prec, ctypes.byref(b), workspace.data_ptr(), workspace.numel(),
        rec.data_ptr(), stream))
    return _record_dict(rec.cpu().tolist())


def measure_buffers_static(rep: Replica, precision: str, sx, sy, sz, record=None) -> dict:
    """``mc_measure_buffers_static``: as ``measure_buffers`` with the library's
    static scratch (no workspace).  ``record`` (8 doubles on the device) may
    be passed in; synchronises and returns the same dict."""
    prec = {"f32": F32, "f64": F64}[precision]
    d = rep.desc()
    b = SpinBuffers(sx.data_ptr(), sy.data_ptr(), sz.data_ptr(), int(sx.numel()))
    rec = torch.zeros(8, dtype=torch.float64, device=sx.device) if record is None else record
    stream = torch.cuda.current_stream(sx.device).cuda_stream
    _check("mc_measure_buffers_static", LIB.mc_measure_buffers_static(
        ctypes.byref(d), prec, ctypes.byref(b), rec.data_ptr(), stream))
    return _record_dict(rec.cpu().tolist())


def occupied_sites(rep: Replica) -> int:
    n = ctypes.c_uint64()
    d = rep.desc()
    _check("mc_occupied_sites", LIB.mc_occupied_sites(ctypes.byref(d), ctypes.byref(n)))
    return int(n.value)


def required_scratch(reps: Sequence[Replica]) -> int:
    arr = (ReplicaDesc * len(reps))(*[r.desc() for r in reps])
    n = ctypes.c_uint64()
    _check("mc_required_scratch", LIB.mc_required_scratch(arr, len(reps), ctypes.byref(n)))
    return int(n.value)


def obs_to_dict(o: Obs) -> dict:
    return {"sweep": int(o.sweep), "n_sites": int(o.n_sites), "n_accepted": int(o.n_accepted),
            "M": np.array(o.M[:]), "absM": o.absM, "E": o.E, "E_exch": o.E_exch,
            "E_anis": o.E_anis}


def obs_array_to_numpy(arr, n) -> np.ndarray:
    """(n, 10) float64: sweep, n_accepted, Mx, My, Mz, |M|, E, E_exch, E_anis, n_sites."""
    out = np.empty((n, 10))
    for i in range(n):
        o = arr[i]
        out[i] = (o.sweep, o.n_accepted, o.M[0], o.M[1], o.M[2], o.absM, o.E, o.E_exch,
                  o.E_anis, o.n_sites)
    return out


class Simulation:
    """A handle over one or more replicas of one lattice kind (``mc_init_lattice``).

    Spin planes and scratch are torch tensors on ``device``; all work runs on
    ``stream`` (a dedicated ``torch.cuda.Stream`` by default, so schedules can
    be replayed as HIP graphs)."""

    def __init__(self, replicas: Sequence[Replica], precision: str = "f32", seed: int = 0,
                 init: str = "random", device: str = "cuda:0", stream=None,
                 user_spins: Optional[List] = None, scratch: Optional[torch.Tensor] = None):
        if not torch.cuda.is_available():
            raise MCError("mc_init_lattice", -4, "no GPU visible to torch")
        self.replicas = list(replicas)
        self.n_reps = len(self.replicas)
        self.prec = F64 if precision in ("f64", "fp64", F64) else F32
        self.dtype = torch.float64 if self.prec == F64 else torch.float32
        self.device = torch.device(device)
        self.seed = int(seed)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.sites = [required_sites(r) for r in self.replicas]
        self.n_occ = [occupied_sites(r) for r in self.replicas]
        self.spins = [[torch.zeros(n, dtype=self.dtype, device=self.device) for _ in range(3)]
                      for n in self.sites]
        # the default tile's work list, or 4 MiB, whichever is larger: room
        # for the autotuner's smaller tiles on small lattices
        nbytes = max(required_scratch(self.replicas), 4 << 20)
        if scratch is None:
            scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.scratch = scratch
        self._descs = (ReplicaDesc * self.n_reps)(*[r.desc() for r in self.replicas])
        bufs = (SpinBuffers * self.n_reps)()
        for i, (pl, n) in enumerate(zip(self.spins, self.sites)):
            bufs[i].sx, bufs[i].sy, bufs[i].sz = pl[0].data_ptr(), pl[1].data_ptr(), pl[2].data_ptr()
            bufs[i].capacity_sites = n
        mode = {"random": INIT_RANDOM, "aligned": INIT_ALIGNED, "user": INIT_USER}[init]
        torch.cuda.synchronize(self.device)
        h = ctypes.c_void_p()
        _check("mc_init_lattice",
               LIB.mc_init_lattice(self._descs, self.n_reps, self.prec,
                                   ctypes.c_uint64(self.seed & (2**64 - 1)), mode, bufs,
                                   ctypes.c_void_p(self.scratch.data_ptr()),
                                   self.scratch.numel(), ctypes.c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(h)))
        self._h = h
        if user_spins is not None:
            for r, xyz in enumerate(user_spins):
                self.from_natural(r, xyz)

    # -- lifetime --------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            LIB.mc_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None:
            raise MCError("handle", -5, "simulation was closed")
        return self._h

    # -- the four entry points --------------------------------------------
    def sweep(self, n: int = 1, measure: bool = False, persistent: bool = False,
              tuned: bool = False):
        """``mc_sweep``: enqueue n sweeps (asynchronous); ``persistent`` runs them
        as one persistent launch, ``tuned`` in the launch mode the autotuner
        chose with ``tune_launch``."""
        flags = ((MEASURE if measure else 0) | (PERSISTENT if persistent else 0) |
                 (TUNED_LAUNCH if tuned else 0))
        _check("mc_sweep", LIB.mc_sweep(self.handle, int(n), flags))

    def tuned_launch(self) -> str:
        """``mc_get_tuned_launch``: "persistent" or "per-pass"."""
        v = ctypes.c_int32()
        _check("mc_get_tuned_launch", LIB.mc_get_tuned_launch(self.handle, ctypes.byref(v)))
        return "persistent" if v.value else "per-pass"

    def synchronize_checked(self):
        """``mc_synchronize``: wait and report deferred errors."""
        _check("mc_synchronize", LIB.mc_synchronize(self.handle))

    def set_watchdog(self, spins: int):
        _check("mc_set_watchdog", LIB.mc_set_watchdog(self.handle, int(spins)))

    def block_steps(self, n: int, step0: int, n_steps: int, conflicts: bool = True,
                    reset: bool = False):
        """``mc_block_steps``: n_steps synchronous steps of the paper's block
        scheme (blocks of n sites) from step index step0; the workspace is
        kept on the object (its counters are zeroed when it is created or
        with reset)."""
        need = ctypes.c_uint64()
        _check("mc_block_workspace", LIB.mc_block_workspace(self.handle, int(n), ctypes.byref(need)))
        ws = getattr(self, "_block_ws", None)
        if ws is None or ws.numel() < need.value:
            self._block_ws = torch.empty(int(need.value), dtype=torch.uint8, device=self.device)
            reset = True
        flags = (BLOCK_CONFLICTS if conflicts else 0) | (BLOCK_RESET if reset else 0)
        _check("mc_block_steps", LIB.mc_block_steps(self.handle, int(n), int(step0), int(n_steps),
                                                    flags, self._block_ws.data_ptr(),
                                                    self._block_ws.numel()))

    def block_counts(self):
        """``mc_block_counts``: (attempts, accepted, conflicts) since the last
        call, then zeroed."""
        c = (ctypes.c_uint64 * 3)()
        _check("mc_block_counts", LIB.mc_block_counts(self.handle, self._block_ws.data_ptr(), c))
        return int(c[0]), int(c[1]), int(c[2])

    def exchange_init(self):
        """``mc_exchange_init``: start replica exchange over the current
        temperatures (identical lattices)."""
        _check("mc_exchange_init", LIB.mc_exchange_init(self.handle))

    def exchange_sweep(self, n_rounds: int, sweeps_per_round: int, persistent: bool = False):
        """``mc_exchange_sweep``: rounds of sweeps, each followed by one
        exchange step between neighbouring temperatures."""
        _check("mc_exchange_sweep", LIB.mc_exchange_sweep(self.handle, int(n_rounds),
                                                          int(sweeps_per_round),
                                                          PERSISTENT if persistent else 0))

    def exchange_state(self):
        """``mc_exchange_state``: dict(replica_at_slot, T_slot, attempted,
        accepted, rounds); attempted/accepted per slot pair (k, k+1)."""
        n = self.n_reps
        ra = (ctypes.c_int32 * n)()
        T = (ctypes.c_double * n)()
        att = (ctypes.c_uint64 * max(n - 1, 1))()
        acc = (ctypes.c_uint64 * max(n - 1, 1))()
        rounds = ctypes.c_uint64()
        _check("mc_exchange_state", LIB.mc_exchange_state(self.handle, ra, T, att, acc,
                                                          ctypes.byref(rounds)))
        return {"replica_at_slot": list(ra), "T_slot": list(T), "attempted": list(att)[:n - 1],
                "accepted": list(acc)[:n - 1], "rounds": int(rounds.value)}

    PERSIST_MODES = {"auto": 0, "global": 1, "xcd": 2}

    def set_persistent_mode(self, mode: str):
        """``mc_set_persistent_mode``: work queues of persistent launches,
        "auto", "global" (one queue) or "xcd" (one queue per XCD)."""
        _check("mc_set_persistent_mode",
               LIB.mc_set_persistent_mode(self.handle, self.PERSIST_MODES[mode]))

    def persistent_queues(self) -> int:
        """Queues a persistent launch uses now (1 or 8)."""
        n = ctypes.c_int32()
        _check("mc_get_persistent_queues", LIB.mc_get_persistent_queues(self.handle, ctypes.byref(n)))
        return int(n.value)

    def sweep_timed(self, n: int, measure: bool = False):
        """``mc_sweep_timed``: (mean ms per colour-pass launch, total ms)."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check("mc_sweep_timed", LIB.mc_sweep_timed(self.handle, int(n), MEASURE if measure else 0,
                                                    ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def observables(self) -> List[dict]:
        """``mc_observables``: records of the last measured sweep."""
        out = (Obs * self.n_reps)()
        _check("mc_observables", LIB.mc_observables(self.handle, out, self.n_reps))
        return [obs_to_dict(o) for o in out]

    def measure_state(self) -> List[dict]:
        out = (Obs * self.n_reps)()
        _check("mc_measure_state", LIB.mc_measure_state(self.handle, out, self.n_reps))
        return [obs_to_dict(o) for o in out]

    def run_schedule(self, T, n_equil: int, n_meas: int, measure_every: int = 1,
                     persistent: bool = False, tuned: bool = False) -> np.ndarray:
        """``mc_run_schedule``: T is (n_T,) or (n_T, n_reps).  Returns an array
        (n_T, n_rec, n_reps, 10) of records (see ``obs_array_to_numpy``)."""
        T = np.asarray(T, dtype=np.float64)
        if T.ndim == 1:
            T = np.repeat(T[:, None], self.n_reps, axis=1)
        T = np.ascontiguousarray(T)
        n_T = T.shape[0]
        n_rec = n_meas // measure_every
        cap = n_T * n_rec * self.n_reps
        series = (Obs * max(cap, 1))()
        s = Schedule()
        s.n_T = n_T
        s.T = T.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s.n_equil, s.n_meas, s.measure_every = int(n_equil), int(n_meas), int(measure_every)
        s.flags = PERSISTENT if persistent else (TUNED_LAUNCH if tuned else 0)
        nw = ctypes.c_uint64()
        _check("mc_run_schedule", LIB.mc_run_schedule(self.handle, ctypes.byref(s), series, cap,
                                                      ctypes.byref(nw)))
        self.last_series = series
        return obs_array_to_numpy(series, int(nw.value)).reshape(n_T, n_rec, self.n_reps, 10)

    # -- helpers -----------------------------------------------------------
    def set_temperatures(self, T):
        arr = (ctypes.c_double * self.n_reps)(*[float(v) for v in np.broadcast_to(T, (self.n_reps,))])
        _check("mc_set_temperatures", LIB.mc_set_temperatures(self.handle, arr, self.n_reps))

    def num_colours(self) -> int:
        n = ctypes.c_int32()
        _check("mc_num_colours", LIB.mc_num_colours(self.handle, ctypes.byref(n)))
        return int(n.value)

    def get_sweep(self) -> int:
        t = ctypes.c_uint64()
        _check("mc_get_sweep", LIB.mc_get_sweep(self.handle, ctypes.byref(t)))
        return int(t.value)

    def set_sweep(self, t: int):
        _check("mc_set_sweep", LIB.mc_set_sweep(self.handle, int(t)))

    def set_tile(self, tx: int, ty: int, zc: int, kernel: int = 0):
        """``mc_set_tile``: kernel 0 = tile (tx x ty threads), 1 = sc row strip
        (tx threads along the row, ty rows per thread), 2 = sc band, 3 = whole
        sweeps in LDS (tx threads per replica), 4 = sc pair strip (two columns
        per thread), 5 = sc band of pairs, 6 = bcc/fcc strip, 7 = bcc/fcc band of
        cell pairs, 8 = sc tiles of ty whole rows staged through LDS (tx = 256),
        9 = sc fused sweep over tiles of ty whole rows (tx = 256; needs
        ``enable_fused``); zc planes per tile."""
        _check("mc_set_tile", LIB.mc_set_tile(self.handle, int(kernel), int(tx), int(ty), int(zc)))

    def enable_fused(self):
        """Allocate every replica's second spin buffer set and hand it to the
        library (``mc_set_second_buffers``), so the fused sweep kernel (9) can
        be chosen; it writes each sweep's new state into the other set.
        Calling it again does nothing."""
        if getattr(self, "alt_spins", None) is not None:
            return
        alt = [[torch.zeros(n, dtype=self.dtype, device=self.device) for _ in range(3)]
               for n in self.sites]
        bufs = (SpinBuffers * self.n_reps)()
        for i, (pl, n) in enumerate(zip(alt, self.sites)):
            bufs[i].sx, bufs[i].sy, bufs[i].sz = pl[0].data_ptr(), pl[1].data_ptr(), pl[2].data_ptr()
            bufs[i].capacity_sites = n
        _check("mc_set_second_buffers", LIB.mc_set_second_buffers(self.handle, bufs))
        self.alt_spins = alt

    def state_spins(self, r: int = 0):
        """The three component tensors that hold replica r's current state
        (``mc_get_state_buffers``: the initial set, or the second one after an
        odd number of fused sweeps)."""
        b = SpinBuffers()
        _check("mc_get_state_buffers", LIB.mc_get_state_buffers(self.handle, int(r), ctypes.byref(b)))
        for pl in [self.spins[r]] + ([self.alt_spins[r]] if getattr(self, "alt_spins", None) else []):
            if pl[0].data_ptr() == b.sx:
                return pl
        raise MCError("mc_get_state_buffers", -5, "state buffers unknown to this binding")

    def autotune(self, trial_sweeps: int = 5, measure: bool = True, persistent: bool = False,
                 cache_path: Optional[str] = None, tune_launch: bool = False):
        """``mc_autotune``: pick the fastest kernel / tile shape (the trial
        sweeps advance the chain); with ``tune_launch`` also the launch mode
        (per-pass graphs or persistent) used by ``sweep(tuned=True)``.
        Returns (kernel, tx, ty, zc)."""
        flags = ((MEASURE if measure else 0) | (PERSISTENT if persistent else 0) |
                 (TUNED_LAUNCH if tune_launch else 0))
        k, a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        path = cache_path.encode() if cache_path else None
        _check("mc_autotune", LIB.mc_autotune(self.handle, int(trial_sweeps), flags, path,
                                              ctypes.byref(k), ctypes.byref(a), ctypes.byref(b),
                                              ctypes.byref(c)))
        return int(k.value), int(a.value), int(b.value), int(c.value)

    def get_tile(self):
        """(kernel, tx, ty, zc, n_work_items)."""
        k, a, b, c, n = (ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(),
                         ctypes.c_uint64())
        _check("mc_get_tile", LIB.mc_get_tile(self.handle, ctypes.byref(k), ctypes.byref(a),
                                              ctypes.byref(b), ctypes.byref(c), ctypes.byref(n)))
        return int(k.value), int(a.value), int(b.value), int(c.value), int(n.value)

    def debug_pass(self, colour: int):
        """``mc_debug_pass``: one colour pass at the current counter; returns
        per-replica (dH, accepted) tensors in the spin layout."""
        dh = [torch.full((n,), float("nan"), dtype=self.dtype, device=self.device)
              for n in self.sites]
        acc = [torch.full((n,), 255, dtype=torch.uint8, device=self.device) for n in self.sites]
        torch.cuda.synchronize(self.device)
        pd = (ctypes.c_void_p * self.n_reps)(*[t.data_ptr() for t in dh])
        pa = (ctypes.c_void_p * self.n_reps)(*[t.data_ptr() for t in acc])
        _check("mc_debug_pass", LIB.mc_debug_pass(self.handle, int(colour), pd, pa))
        return dh, acc

    def to_natural(self, replica: int = 0):
        """Spins of one replica in natural order (x, y, z component tensors)."""
        n = self.sites[replica]
        out = [torch.empty(n, dtype=self.dtype, device=self.device) for _ in range(3)]
        torch.cuda.synchronize(self.device)
        _check("mc_layout_copy", LIB.mc_layout_copy(self.handle, replica, 1, *[t.data_ptr() for t in out]))
        return out

    def from_natural(self, replica: int, xyz):
        """Set one replica's spins from natural-order components (arrays or tensors)."""
        n = self.sites[replica]
        src = [torch.as_tensor(np.asarray(a) if not torch.is_tensor(a) else a, dtype=self.dtype)
               .to(self.device).contiguous() for a in xyz]
        for t in src:
            if t.numel() != n:
                raise ValueError(f"expected {n} sites, got {t.numel()}")
        torch.cuda.synchronize(self.device)
        _check("mc_layout_copy", LIB.mc_layout_copy(self.handle, replica, 0, *[t.data_ptr() for t in src]))

    def synchronize(self):
        self.stream.synchronize()


def init_lattice(replicas, **kw) -> Simulation:
    """``mc_init_lattice``: create a Simulation (see ``Simulation``)."""
    return Simulation(replicas, **kw)


def series_stats(records: np.ndarray, n_sites: int, T: float) -> dict:
    """``mc_series_stats`` over an (n, 10) record array of one replica."""
    n = records.shape[0]
    arr = (Obs * n)()
    for i, r in enumerate(records):
        arr[i].sweep = int(r[0])
        arr[i].n_accepted = int(r[1])
        for a in range(3):
            arr[i].M[a] = r[2 + a]
        arr[i].absM, arr[i].E, arr[i].E_exch, arr[i].E_anis = r[5], r[6], r[7], r[8]
        arr[i].n_sites = int(n_sites)
    st = Stats()
    _check("mc_series_stats", LIB.mc_series_stats(arr, n, 1, float(T), ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in Stats._fields_}
