"""Python driver for the FP64 CPU oracle (``mc_oracle.c``).

TEST INFRASTRUCTURE ONLY: the correctness reference for the GPU library.  Only
``tests/``, the smoke check and the CPU-baseline leg of the benchmark may import
this module.  It shares no code with the GPU package and imports nothing from it.

The model is Eq. (1) of Charilaou, arXiv:2106.11286 (anisotropic classical
Heisenberg Hamiltonian, nearest-neighbour bonds counted once); the update is the
single-spin Metropolis rule of the paper's Monte Carlo paragraph; the
magnetisation is Eq. (2).  Spin arrays are natural (canonical) order:
``s = ((z*Ly + y)*Lx + x)*n_basis + b``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mc_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "libmc_oracle.so")

SC, BCC, FCC = 0, 1, 2
INIT_RANDOM, INIT_ALIGNED = 0, 1

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math, no FMA contraction)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-D_GNU_SOURCE", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [("J", ctypes.c_double), ("K", ctypes.c_double), ("e", ctypes.c_double * 3),
                ("T", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("replica_id", ctypes.c_uint32)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            L = ctypes.CDLL(_LIB_PATH)
            vp, i64, u32, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int
            dp = ctypes.POINTER(ctypes.c_double)
            L.orc_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
            L.orc_philox4x32_10.restype = None
            L.orc_uniform.argtypes = [u32]
            L.orc_uniform.restype = ctypes.c_double
            L.orc_sphere_point.argtypes = [ctypes.c_double, ctypes.c_double, dp]
            L.orc_sphere_point.restype = None
            L.orc_lattice_new.argtypes = [i32, i32, i32, i32, u32, ctypes.c_double]
            L.orc_lattice_new.restype = vp
            L.orc_lattice_free.argtypes = [vp]
            L.orc_lattice_free.restype = None
            for name in ("orc_lattice_n_box", "orc_lattice_n_occ", "orc_lattice_n_bonds"):
                getattr(L, name).argtypes = [vp]
                getattr(L, name).restype = i64
            for name in ("orc_lattice_n_colours", "orc_lattice_same_colour_bonds",
                         "orc_lattice_zmax"):
                getattr(L, name).argtypes = [vp]
                getattr(L, name).restype = i32
            L.orc_lattice_tables.argtypes = [vp, vp, vp, vp, vp]
            L.orc_lattice_tables.restype = None
            L.orc_site_index.argtypes = [vp, i32, i32, i32, i32]
            L.orc_site_index.restype = i64
            P = ctypes.POINTER(_Params)
            L.orc_init.argtypes = [vp, P, i32, vp, vp, vp]
            L.orc_init.restype = None
            L.orc_delta_h.argtypes = [dp, dp, dp, ctypes.c_double, dp]
            L.orc_delta_h.restype = ctypes.c_double
            L.orc_pass.argtypes = [vp, P, i32, u32, vp, vp, vp, vp, vp, vp]
            L.orc_pass.restype = i64
            L.orc_sweep.argtypes = [vp, P, u32, vp, vp, vp]
            L.orc_sweep.restype = i64
            L.orc_observables.argtypes = [vp, P, vp, vp, vp, dp]
            L.orc_observables.restype = None
            L.orc_geometry_new.argtypes = [i32, i32, i32, i32, u32, ctypes.c_double]
            L.orc_geometry_new.restype = vp
            L.orc_site_attempt.argtypes = [vp, P, u32, vp, vp, vp, i64, dp]
            L.orc_site_attempt.restype = i32
            L.orc_run.argtypes = [vp, P, u32, u32, vp, vp, vp, vp]
            L.orc_run.restype = None
            L.orc_num_threads.argtypes = []
            L.orc_num_threads.restype = i32
            L.orc_set_num_threads.argtypes = [i32]
            L.orc_set_num_threads.restype = None
            _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def philox(ctr, key):
    """Philox4x32-10 block: counter (4 x u32), key (2 x u32) -> 4 x u32."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform(word: int) -> float:
    return float(lib().orc_uniform(int(word) & 0xFFFFFFFF))


def sphere_point(u0: float, u1: float):
    o = (ctypes.c_double * 3)()
    lib().orc_sphere_point(u0, u1, o)
    return np.array(o[:], dtype=np.float64)


def delta_h(h, S, Sn, K, e):
    """Energy change of one spin move (Eq. (1)); e must be a unit vector."""
    arr = [(ctypes.c_double * 3)(*map(float, v)) for v in (h, S, Sn, e)]
    return float(lib().orc_delta_h(arr[0], arr[1], arr[2], float(K), arr[3]))


class Params:
    """Model and stream parameters: J, K, easy axis e, temperature T (J/k_B,
    T=0 greedy, T=inf infinite temperature), Philox seed and replica id."""

    def __init__(self, J=1.0, K=0.0, e=(0.0, 0.0, 1.0), T=1.0, seed=0, replica_id=0):
        self.J, self.K, self.e, self.T = float(J), float(K), tuple(map(float, e)), float(T)
        self.seed, self.replica_id = int(seed), int(replica_id)

    def c(self):
        p = _Params()
        p.J, p.K, p.T = self.J, self.K, self.T
        for i in range(3):
            p.e[i] = self.e[i]
        p.seed = self.seed & 0xFFFFFFFFFFFFFFFF
        p.replica_id = self.replica_id & 0xFFFFFFFF
        return p

    @property
    def e_unit(self):
        e = np.array(self.e, dtype=np.float64)
        return e / np.sqrt(np.dot(e, e))


class Lattice:
    """Explicit lattice (sc / bcc / fcc conventional cells, optional centred
    sphere of occupied sites, periodic or open faces per axis)."""

    def __init__(self, kind, Lx, Ly=None, Lz=None, periodic_mask=7, sphere_radius=0.0):
        Ly = Lx if Ly is None else Ly
        Lz = Lx if Lz is None else Lz
        self.kind, self.Lx, self.Ly, self.Lz = int(kind), int(Lx), int(Ly), int(Lz)
        self.periodic_mask, self.sphere_radius = int(periodic_mask), float(sphere_radius)
        h = lib().orc_lattice_new(self.kind, self.Lx, self.Ly, self.Lz, self.periodic_mask,
                                  self.sphere_radius)
        if not h:
            raise ValueError("oracle: invalid lattice")
        self._h = ctypes.c_void_p(h)
        L = lib()
        self.n_box = int(L.orc_lattice_n_box(self._h))
        self.n_occ = int(L.orc_lattice_n_occ(self._h))
        self.n_bonds = int(L.orc_lattice_n_bonds(self._h))
        self.n_colours = int(L.orc_lattice_n_colours(self._h))
        self.same_colour_bonds = bool(L.orc_lattice_same_colour_bonds(self._h))
        self.zmax = int(L.orc_lattice_zmax(self._h))
        self.n_basis = {SC: 1, BCC: 2, FCC: 4}[self.kind]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_lattice_free(h)
            self._h = None

    def tables(self):
        """(occupied[n_box], colour[n_box], n_neighbours[n_box], nbr[n_box, zmax])."""
        occ = np.empty(self.n_box, np.uint8)
        col = np.empty(self.n_box, np.uint8)
        nnb = np.empty(self.n_box, np.int8)
        nbr = np.empty((self.n_box, self.zmax), np.int32)
        lib().orc_lattice_tables(self._h, _ptr(occ), _ptr(col), _ptr(nnb), _ptr(nbr))
        return occ.astype(bool), col, nnb, nbr

    def site_index(self, x, y, z, b=0):
        return int(lib().orc_site_index(self._h, x, y, z, b))

    def new_spins(self):
        return [np.zeros(self.n_box, np.float64) for _ in range(3)]


class Geometry:
    """Lattice geometry without tables, for single-site evaluation of lattices
    too large to tabulate (neighbours found by brute force per site)."""

    def __init__(self, kind, Lx, Ly=None, Lz=None, periodic_mask=7, sphere_radius=0.0):
        Ly = Lx if Ly is None else Ly
        Lz = Lx if Lz is None else Lz
        h = lib().orc_geometry_new(int(kind), int(Lx), int(Ly), int(Lz), int(periodic_mask),
                                   float(sphere_radius))
        if not h:
            raise ValueError("oracle: invalid geometry")
        self._h = ctypes.c_void_p(h)
        self.n_box = int(Lx) * int(Ly) * int(Lz) * {SC: 1, BCC: 2, FCC: 4}[int(kind)]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_lattice_free(h)
            self._h = None

    def site_attempt(self, p: Params, t: int, spins, s: int):
        """One site's attempt at sweep t from natural-order FP64 spins:
        dict(dH, accepted, margin, S_after, h); None if s is unoccupied."""
        out = (ctypes.c_double * 9)()
        pc = p.c()
        rc = lib().orc_site_attempt(self._h, ctypes.byref(pc), int(t), *[_ptr(a) for a in spins],
                                    int(s), out)
        if rc != 0:
            return None
        return {"dH": out[0], "accepted": bool(out[1]), "margin": out[2],
                "S_after": np.array(out[3:6]), "h": np.array(out[6:9])}


def init(lat: Lattice, p: Params, mode=INIT_RANDOM):
    """Initial state (random on the sphere from Philox tag 1, or along e)."""
    s = lat.new_spins()
    pc = p.c()
    lib().orc_init(lat._h, ctypes.byref(pc), int(mode), *[_ptr(a) for a in s])
    return s


def run_pass(lat: Lattice, p: Params, colour: int, t: int, spins, outputs=False):
    """One colour pass at sweep counter t, in place.  Returns n_accepted, or
    (n_accepted, dH, accepted, margin) with per-site arrays (NaN / 0 off-colour)."""
    pc = p.c()
    if outputs:
        dh = np.full(lat.n_box, np.nan)
        acc = np.zeros(lat.n_box, np.uint8)
        mg = np.full(lat.n_box, np.nan)
        n = lib().orc_pass(lat._h, ctypes.byref(pc), int(colour), int(t),
                           *[_ptr(a) for a in spins], _ptr(dh), _ptr(acc), _ptr(mg))
        return int(n), dh, acc.astype(bool), mg
    n = lib().orc_pass(lat._h, ctypes.byref(pc), int(colour), int(t),
                       *[_ptr(a) for a in spins], None, None, None)
    return int(n)


def sweep(lat: Lattice, p: Params, t: int, spins):
    pc = p.c()
    return int(lib().orc_sweep(lat._h, ctypes.byref(pc), int(t), *[_ptr(a) for a in spins]))


def observables(lat: Lattice, p: Params, spins):
    """From-scratch observables: dict with M (sum vector), m (= M / N, Eq. (2)),
    E_exch, E_anis, E (all extensive, FP64)."""
    o = (ctypes.c_double * 5)()
    pc = p.c()
    lib().orc_observables(lat._h, ctypes.byref(pc), *[_ptr(a) for a in spins], o)
    M = np.array(o[0:3])
    return {"M": M, "m": M / lat.n_occ, "E_exch": o[3], "E_anis": o[4], "E": o[3] + o[4]}


def run(lat: Lattice, p: Params, t0: int, n_sweeps: int, spins, record=True):
    """n sweeps from counter t0, in place.  With record, returns an (n, 6)
    array of per-sweep {Mx, My, Mz (sums), E_exch, E_anis, n_accepted}."""
    pc = p.c()
    rec = np.zeros((n_sweeps, 6)) if record else None
    lib().orc_run(lat._h, ctypes.byref(pc), int(t0), int(n_sweeps), *[_ptr(a) for a in spins],
                  _ptr(rec))
    return rec


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))
