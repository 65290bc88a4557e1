"""Replica exchange (parallel tempering) over identical lattices: the oracle of
the swap step.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/``, the
smoke check and the CPU-baseline leg of the benchmark may import it.

The paper runs one temperature per simulation; exchanging configurations
between simulations at neighbouring temperatures is the standard replica
exchange method (Swendsen and Wang 1986; Hukushima and Nemoto 1996), added
here for batches of replicas.  Its rule, written out:

* The ladder holds the temperatures T_0 <= T_1 <= ... <= T_{n-1} of the
  replicas when tempering starts; slot k has beta_k = 1/T_k.  ``rep_at[k]``
  is the replica that currently runs at slot k.
* Round r (r = 0, 1, ...) attempts the disjoint pairs (k, k+1) with
  k = r mod 2, r mod 2 + 2, ... (k + 1 < n).  For replicas i = rep_at[k],
  j = rep_at[k+1] with total energies E_i, E_j (Eq. (1) of the paper, the
  state after the round's sweeps) the exchange is accepted with probability
  min(1, exp(Delta)), Delta = (beta_k - beta_{k+1}) (E_i - E_j): accepted iff
  Delta >= 0 or u < exp(Delta).  This ratio makes the product over slots of
  the Boltzmann weights exp(-beta_k E_{rep_at[k]}) stationary.
* u is the first word of the Philox4x32-10 block with counter
  (k, 0, t, 2) and key (seed low, seed high), t = sweeps done so far, mapped
  to (w >> 9 + 1/2) 2^-23 as every uniform of the method (counter tag 2 keeps
  these draws apart from the Metropolis (tag 0) and initial-state (tag 1)
  streams).
* An accepted exchange swaps rep_at[k] and rep_at[k+1]: each replica keeps
  its spins and takes the other temperature.
"""
from __future__ import annotations

import math

from . import oracle as O

TAG_EXCHANGE = 2


def ladder(T):
    """Slots of the replicas' temperatures: (rep_at, T_slot), ascending T,
    ties in replica order."""
    order = sorted(range(len(T)), key=lambda r: (float(T[r]), r))
    return list(order), [float(T[r]) for r in order]


def exchange_uniform(k: int, t: int, seed: int) -> float:
    w = O.philox([k, 0, t, TAG_EXCHANGE], [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])
    return O.uniform(w[0])


def swap_round(E, T_slot, rep_at, round_index: int, t: int, seed: int):
    """One round of exchange attempts, in place on ``rep_at``.  E[r] is the
    total energy of replica r.  Returns [(k, accepted), ...]."""
    n = len(rep_at)
    out = []
    for k in range(round_index % 2, n - 1, 2):
        i, j = rep_at[k], rep_at[k + 1]
        delta = (1.0 / T_slot[k] - 1.0 / T_slot[k + 1]) * (E[i] - E[j])
        acc = delta >= 0.0 or exchange_uniform(k, t, seed) < math.exp(delta)
        if acc:
            rep_at[k], rep_at[k + 1] = j, i
        out.append((k, acc))
    return out
