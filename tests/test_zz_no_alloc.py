"""The allocation-free measurement entry point (mc_measure_buffers_static)
against the workspace one (mc_measure_buffers), through the C ABI: two calls
in a row, the second on a smaller lattice, give bit for bit the records of
the workspace entry point on the same buffers."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2106_11286_amd import mcheis

    return mcheis


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_static_measurement_equals_workspace_measurement(M, prec):
    import torch

    cases = [
        # larger first (more workgroups), then a smaller lattice of another kind
        M.Replica(kind="sc", L=(96, 80, 64), J=1.0, K=0.1, e=(0.0, 0.0, 1.0), T=1.2),
        M.Replica(kind="fcc", L=(10, 9, 8), periodic_mask=0, sphere_radius=3.7, J=1.1, K=0.2,
                  e=(1.0, 1.0, 1.0), T=0.9),
    ]
    assert M.required_sites(cases[1]) < M.required_sites(cases[0])
    ws = torch.empty(M.MEASURE_WORKSPACE_BYTES, dtype=torch.uint8, device="cuda")
    for rep in cases:
        sim = M.Simulation([rep], precision=prec, seed=29)
        sim.sweep(2)
        sim.synchronize()
        a = M.measure_buffers(rep, prec, *sim.spins[0], workspace=ws)
        rec = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
        b = M.measure_buffers_static(rep, prec, *sim.spins[0], record=rec)
        assert b["n_sites"] == a["n_sites"] == M.occupied_sites(rep)
        assert np.array_equal(a["M"], b["M"])
        assert a["E_exch"] == b["E_exch"] and a["E_anis"] == b["E_anis"]
        sim.close()
