"""Seeded synthetic workloads (lattices, parameters, temperature ladders and
random spin states).  Serves both the GPU library and the CPU oracle in tests
and benchmarks; contains none of the method's arithmetic.

The lattices follow the paper's setup (simple cubic, periodic, J = 1, small
uniaxial K, unit spins; arXiv:2106.11286, simulation-setup paragraph and
Figs. 2-3) at the sizes of the benchmark configurations, plus an FCC
nanoparticle with open surface for the claim of the abstract and conclusion
that the method fits any crystal lattice.
"""
from __future__ import annotations

import numpy as np

# Each workload: dict of replica fields (kind, L, periodic_mask, sphere_radius,
# J, K, e, T, replica_id) plus run parameters.
C1_SC16_TRAJECTORY = dict(
    name="sc-L16-fp64-trajectory", kind="sc", L=(16, 16, 16), periodic_mask=7,
    J=1.0, K=0.1, e=(0.0, 0.0, 1.0), T=1.2, seed=0, sweeps=1000, precision="f64")

C2_SC256_TSWEEP = dict(
    name="sc-L256-temperature-sweep", kind="sc", L=(256, 256, 256), periodic_mask=7,
    J=1.0, K=0.05, e=(0.0, 0.0, 1.0), T_ladder=tuple(np.round(np.linspace(0.4, 2.0, 17), 10)),
    n_equil=2000, n_meas=2000, seed=1)

C3_BATCHED = dict(
    name="sc-batched-64-replicas", kind="sc", n_reps=64, L_choices=(32, 48, 64, 96),
    periodic_mask=7, J=1.0, K=0.1, e=(0.0, 0.0, 1.0), T_range=(0.8, 2.0), sweeps=5000, seed=2)

C4_FCC_PARTICLE = dict(
    name="fcc-nanoparticle-128cells-R60", kind="fcc", L=(128, 128, 128), periodic_mask=0,
    sphere_radius=60.0, J=1.0, K=0.05, e=(1.0, 1.0, 1.0), T=0.9, seed=3,
    n_equil=2000, n_meas=2000)

C5_SC464_ROOFLINE = dict(
    name="sc-L464-1e8-spins", kind="sc", L=(464, 464, 464), periodic_mask=7,
    J=1.0, K=0.02, e=(0.0, 0.0, 1.0), T=1.4, seed=4, sweeps=1000)

# bcc at the benchmark's scale: 2 x 368^3 = 99,672,064 spins, periodic, in the
# ordered phase at moderate acceptance (the claim that the method fits any
# crystal lattice, at the paper's 10^8-spin size)
BCC_368_1E8 = dict(
    name="bcc-L368-1e8-spins", kind="bcc", L=(368, 368, 368), periodic_mask=7,
    J=1.0, K=0.02, e=(0.0, 0.0, 1.0), T=1.9, seed=6, sweeps=200)

# fcc at the same scale: 4 x 292^3 = 99,588,352 spins, periodic
FCC_292_1E8 = dict(
    name="fcc-L292-1e8-spins", kind="fcc", L=(292, 292, 292), periodic_mask=7,
    J=1.0, K=0.02, e=(0.0, 0.0, 1.0), T=2.8, seed=9, sweeps=100)

# replica exchange across the critical region: 32 copies of one sc 64^3
# lattice at temperatures evenly spaced over 1.41 .. 1.48 (about 0.0023 apart)
EXCHANGE_SC64 = dict(
    name="sc-L64-exchange-32-replicas", kind="sc", L=(64, 64, 64), periodic_mask=7,
    J=1.0, K=0.01, e=(0.0, 0.0, 1.0), T_range=(1.41, 1.48), n_reps=32, seed=7,
    rounds=500, sweeps_per_round=4)

# the paper's block scheme against the colour sweep on its Fig. 1 system:
# sc 128^3, T = 0.9 T_C (T_C = 1.445 as printed), blocks of 8 sites
BLOCK_SC128 = dict(
    name="sc-L128-block-scheme-vs-colour-sweep", kind="sc", L=(128, 128, 128), periodic_mask=7,
    J=1.0, K=0.01, e=(0.0, 0.0, 1.0), T=1.3, seed=8, n_block=8, n_equil=1000, n_meas=2000)

REPLICA_KEYS = ("kind", "L", "periodic_mask", "sphere_radius", "J", "K", "e", "T", "replica_id")


def replica_fields(w: dict, **over) -> dict:
    """The replica fields of a workload dict (with overrides)."""
    d = {k: w[k] for k in REPLICA_KEYS if k in w}
    d.update(over)
    return d


def c3_replicas(w: dict = C3_BATCHED):
    """Replica fields of the batched workload: sizes drawn from L_choices with
    a seeded numpy generator, temperatures evenly spaced over T_range."""
    rng = np.random.default_rng(w["seed"])
    Ls = rng.choice(np.array(w["L_choices"]), size=w["n_reps"])
    T = np.linspace(w["T_range"][0], w["T_range"][1], w["n_reps"])
    out = []
    for r in range(w["n_reps"]):
        L = int(Ls[r])
        out.append(dict(kind=w["kind"], L=(L, L, L), periodic_mask=w["periodic_mask"],
                        J=w["J"], K=w["K"], e=w["e"], T=float(T[r]), replica_id=r))
    return out


def random_unit_vectors(n: int, seed: int, dtype=np.float64):
    """n unit vectors (x, y, z component arrays) from a seeded normal draw,
    normalised; values are exactly representable in ``dtype``."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    v = v.astype(dtype).astype(np.float64)
    return v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy()
