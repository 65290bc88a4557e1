"""Replica exchange between neighbouring temperatures on the GPU, against the
oracle's exchange rule (oracle/tempering.py) and between launch modes."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import tempering as PT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2106_11286_amd import mcheis

    return mcheis


def natural(sim, r=0):
    return [t.double().cpu().numpy() for t in sim.to_natural(r)]


def _reps(M, Ts, L=(4, 4, 4), kind="sc", K=0.1):
    return [M.Replica(kind=kind, L=L, J=1.0, K=K, e=(0.0, 0.0, 1.0), T=T, replica_id=r)
            for r, T in enumerate(Ts)]


def test_exchange_fp64_follows_oracle(M):
    """FP64, five replicas of one periodic sc 4^3 lattice at unsorted
    temperatures, 24 rounds of 3 sweeps: after every round the slot of every
    replica equals the oracle's chain (oracle sweeps at each replica's slot
    temperature, its energies and its exchange rule); at the end the exchange
    counts match and the spins agree to 1e-12."""
    Ts = [1.9, 1.0, 1.45, 1.2, 1.7]
    seed = 77
    reps = _reps(M, Ts)
    sim = M.Simulation(reps, precision="f64", seed=seed)
    sim.exchange_init()
    lat = O.Lattice(O.SC, 4, 4, 4)
    spins = [O.init(lat, O.Params(J=1.0, K=0.1, T=T, seed=seed, replica_id=r))
             for r, T in enumerate(Ts)]
    rep_at, T_slot = PT.ladder(Ts)
    att, acc = [0] * 4, [0] * 4
    t = 0
    for rnd in range(24):
        sim.exchange_sweep(1, 3)
        slot_of = {r: k for k, r in enumerate(rep_at)}
        E = []
        for r in range(5):
            p = O.Params(J=1.0, K=0.1, T=T_slot[slot_of[r]], seed=seed, replica_id=r)
            rec = O.run(lat, p, t, 3, spins[r])
            E.append(rec[-1, 3] + rec[-1, 4])
        t += 3
        for k, a in PT.swap_round(E, T_slot, rep_at, rnd, t, seed):
            att[k] += 1
            acc[k] += int(a)
        st = sim.exchange_state()
        assert st["replica_at_slot"] == rep_at, (rnd, st, rep_at)
    print("accepted per pair", acc, "of", att)
    assert st["attempted"] == att and st["accepted"] == acc and st["rounds"] == 24
    assert st["T_slot"] == T_slot
    assert sum(acc) >= 2
    for r in range(5):
        for a, b in zip(natural(sim, r), spins[r]):
            assert np.max(np.abs(a - b)) <= 1e-12, r


def test_exchange_persistent_equals_per_pass_and_survives_retile(M):
    """FP32, 16 replicas of one sc 16^3 lattice (per-XCD persistent queues):
    exchange rounds through persistent launches equal those through per-pass
    launches bitwise (slots, counts, spins); a tile change between rounds
    keeps the exchange table and the chain."""
    import torch

    Ts = list(np.linspace(1.2, 1.7, 16))
    reps = _reps(M, Ts, L=(16, 16, 16))
    sims = [M.Simulation(reps, precision="f32", seed=5,
                         scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
            for _ in range(3)]
    for s in sims:
        s.set_tile(256, 2, 4, kernel=2)
        s.exchange_init()
    sims[0].exchange_sweep(10, 2)
    sims[1].exchange_sweep(10, 2, persistent=True)
    sims[2].exchange_sweep(4, 2)
    sims[2].set_tile(32, 8, 4, kernel=0)
    sims[2].exchange_sweep(6, 2)
    states = [s.exchange_state() for s in sims]
    print(states[0])
    for st in states[1:]:
        assert st == states[0]
    assert sum(states[0]["accepted"]) >= 1
    for r in range(16):
        ref = natural(sims[0], r)
        for s in sims[1:]:
            for a, b in zip(natural(s, r), ref):
                assert np.array_equal(a, b), r


def test_exchange_errors(M):
    """Exchange needs identical lattices, 0 < T < inf and an init; explicit
    temperatures end it."""
    mixed = M.Simulation([M.Replica(kind="sc", L=(4, 4, 4), T=1.0),
                          M.Replica(kind="sc", L=(6, 4, 4), T=1.2, replica_id=1)],
                         precision="f32")
    with pytest.raises(M.MCError) as ei:
        mixed.exchange_init()
    assert ei.value.status == -1
    cold = M.Simulation(_reps(M, [0.0, 1.0]), precision="f32")
    with pytest.raises(M.MCError) as ei:
        cold.exchange_init()
    assert ei.value.status == -1
    sim = M.Simulation(_reps(M, [1.0, 1.3, 1.6]), precision="f32")
    with pytest.raises(M.MCError) as ei:
        sim.exchange_sweep(1, 1)
    assert ei.value.status == -5
    sim.exchange_init()
    sim.exchange_sweep(3, 2)
    st = sim.exchange_state()
    assert st["rounds"] == 3 and sum(st["attempted"]) == 3  # pairs (0,1), (1,2), (0,1)
    sim.set_temperatures([1.0, 1.1, 1.2])
    with pytest.raises(M.MCError) as ei:
        sim.exchange_sweep(1, 1)
    assert ei.value.status == -5
