"""The paper's block scheme (implementation paragraph), the oracle of its
synchronous form.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/``, the
smoke check and the CPU-baseline leg of the benchmark may import it.

The paper linearises the spins into arrays and gives each of N_b GPU blocks n
consecutive entries; at every step each block picks one of its spins at random
and makes one Metropolis attempt there (propose a new orientation uniformly on
the sphere, accept if dH <= 0 or P <= exp(-dH/T)), the field coming from the
neighbours' values in global memory, which other blocks update at the same
time.  With few spins per block this concurrency breaks the Markov chain, as
the implementation paragraph itself notes.  Which value of a concurrently updated
neighbour an attempt sees depends on hardware timing; the form written here
makes it definite and extreme: every attempt of a step sees the state from
before the step, and all accepted moves are written together.

Definitions (the choices the paper leaves open):

* The linear index is the canonical site index s = ((z Ly + y) Lx + x) n_basis
  + b; block k holds s in [k n, min(N, (k + 1) n)) and has m_k entries.
* Step j (counted from 0 over the whole run) draws, for block k, the
  Philox4x32-10 block with counter (k, replica_id, j, 3) and key (seed low,
  seed high) -- tag 3, beside the colour sweep's 0 and 1; word 3 picks the
  site s = k n + floor(w3 m_k / 2^32); words 0 and 1 give the proposal and
  word 2 the acceptance uniform, exactly as in a colour-pass attempt.
* One Monte Carlo step per spin is n steps (N attempts), the paper's unit.
* An attempt at an unoccupied site changes nothing.
* A conflict is an attempt at a site that has an attempted nearest neighbour
  in the same step (the pairs whose concurrency the paper warns about).
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O

TAG_BLOCK = 3


def chosen_sites(n_box: int, n: int, rid: int, step: int, seed: int):
    """[(site, philox words)] of every block at one step."""
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    out = []
    for k in range((n_box + n - 1) // n):
        m = min(n, n_box - k * n)
        w = O.philox([k, rid, step, TAG_BLOCK], key)
        out.append((k * n + ((w[3] * m) >> 32), w))
    return out


def block_step(lat: O.Lattice, p: O.Params, spins, n: int, step: int, tables=None):
    """One synchronous step of the block scheme, in place on natural-order
    FP64 spins.  Returns (attempts, accepted, conflicts)."""
    occ, _, nnb, nbr = tables if tables is not None else lat.tables()
    e = p.e_unit
    chosen = chosen_sites(lat.n_box, n, p.replica_id, step, p.seed)
    picked = np.zeros(lat.n_box, bool)
    for s, _ in chosen:
        picked[s] = True
    beta = 1.0 / p.T if p.T > 0.0 else 0.0
    moves = []
    attempts = accepted = conflicts = 0
    for s, w in chosen:
        if not occ[s]:
            continue
        attempts += 1
        nb = nbr[s, :nnb[s]]
        if np.any(picked[nb]):
            conflicts += 1
        h = p.J * np.array([spins[a][nb].sum() for a in range(3)])
        S = np.array([spins[a][s] for a in range(3)])
        Sn = O.sphere_point(O.uniform(w[0]), O.uniform(w[1]))
        dH = O.delta_h(h, S, Sn, p.K, e)
        P = O.uniform(w[2])
        acc = dH <= 0.0 or (p.T > 0.0 and P <= math.exp(-beta * dH))
        if acc:
            accepted += 1
            moves.append((s, Sn / np.sqrt(np.dot(Sn, Sn))))
    for s, v in moves:
        for a in range(3):
            spins[a][s] = v[a]
    return attempts, accepted, conflicts


def run(lat: O.Lattice, p: O.Params, spins, n: int, step0: int, n_steps: int):
    """n_steps steps from step0; returns the per-step (attempts, accepted,
    conflicts) as an (n_steps, 3) array."""
    tables = lat.tables()
    return np.array([block_step(lat, p, spins, n, step0 + j, tables) for j in range(n_steps)],
                    dtype=np.int64)
