"""The paper's block scheme (synchronous form) on the GPU against the oracle
(oracle/block_scheme.py)."""
import ctypes

import numpy as np
import pytest

from oracle import block_scheme as BS
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2106_11286_amd import mcheis

    return mcheis


def natural(sim, r=0):
    return [t.double().cpu().numpy() for t in sim.to_natural(r)]


REPS = [dict(L=(8, 8, 6), periodic_mask=7, sphere_radius=0.0, T=1.2),
        dict(L=(8, 6, 4), periodic_mask=5, sphere_radius=0.0, T=0.9),
        dict(L=(10, 10, 10), periodic_mask=0, sphere_radius=4.2, T=1.5)]


def _run_both(M, prec, n, steps, seed=13):
    reps = [M.Replica(kind="sc", J=1.0, K=0.2, e=(0.0, 0.6, 0.8), replica_id=r, **f)
            for r, f in enumerate(REPS)]
    sim = M.Simulation(reps, precision=prec, seed=seed)
    sim.block_steps(n, 5, steps, conflicts=True, reset=True)
    counts = sim.block_counts()
    ref = []
    tot = np.zeros(3, np.int64)
    for r, f in enumerate(REPS):
        lat = O.Lattice(O.SC, *f["L"], periodic_mask=f["periodic_mask"],
                        sphere_radius=f["sphere_radius"])
        p = O.Params(J=1.0, K=0.2, e=(0.0, 0.6, 0.8), T=f["T"], seed=seed, replica_id=r)
        s = O.init(lat, p)
        tot += BS.run(lat, p, s, n, 5, steps).sum(0)
        ref.append(s)
    return sim, counts, ref, tot


@pytest.mark.parametrize("n", [8, 5])
def test_block_fp64_matches_oracle(M, n):
    """FP64, three sc replicas (periodic, partly open, an open-surface sphere),
    blocks of 8 and of 5 sites (a shorter last block), 24 steps: spins agree
    with the oracle to 1e-12 and the attempt, acceptance and conflict counts
    are equal."""
    sim, counts, ref, tot = _run_both(M, "f64", n, 24)
    print("GPU counts", counts, "oracle", tot.tolist())
    assert list(counts) == tot.tolist()
    assert counts[2] > 0
    for r in range(len(REPS)):
        for a, b in zip(natural(sim, r), ref[r]):
            assert np.max(np.abs(a - b)) <= 1e-12, r


def test_block_fp32_counts(M):
    """FP32: attempts and conflicts depend only on the random choices and
    equal the oracle's; acceptances agree up to near-ties."""
    sim, counts, ref, tot = _run_both(M, "f32", 8, 16)
    assert counts[0] == tot[0] and counts[2] == tot[2]
    assert abs(counts[1] - tot[1]) <= 3


def test_block_errors(M):
    import torch

    bcc = M.Simulation([M.Replica(kind="bcc", L=(4, 4, 4))], precision="f32")
    with pytest.raises(M.MCError) as ei:
        bcc.block_steps(8, 0, 1)
    assert ei.value.status in (-2,)
    sim = M.Simulation([M.Replica(kind="sc", L=(8, 8, 8))], precision="f32")
    need = ctypes.c_uint64()
    assert M.LIB.mc_block_workspace(sim.handle, 0, ctypes.byref(need)) == -1
    assert M.LIB.mc_block_workspace(sim.handle, 8, ctypes.byref(need)) == 0
    small = torch.empty(int(need.value) - 256, dtype=torch.uint8, device="cuda")
    assert M.LIB.mc_block_steps(sim.handle, 8, 0, 1, 0, small.data_ptr(), small.numel()) == -3
