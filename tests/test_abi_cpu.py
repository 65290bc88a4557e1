"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/mcheis.h, rejects invalid descriptors before touching a
device, and its host-side series statistics agree with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcheis.h")


@pytest.fixture(scope="module")
def M():
    from paper_2106_11286_amd import mcheis

    return mcheis


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mc_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported(M):
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(M.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    # the binding declares a signature for every exported function
    assert set(names) == set(M._SIGNATURES), set(names) ^ set(M._SIGNATURES)


def test_descriptor_validation(M):
    R = M.Replica
    assert M.required_sites(R(kind="sc", L=(464, 464, 464))) == 464**3
    assert M.required_sites(R(kind="fcc", L=(128, 128, 128))) == 4 * 128**3
    assert M.occupied_sites(R(kind="fcc", L=(128, 128, 128), periodic_mask=0,
                              sphere_radius=60)) == 3618393
    assert M.occupied_sites(R(kind="sc", L=(2, 1, 1), periodic_mask=0)) == 2
    cases = [
        (R(kind="sc", L=(15, 16, 16)), -2),               # odd Lx: no colour packing
        (R(kind="sc", L=(16, 15, 16)), -2),               # odd periodic length
        (R(kind="sc", L=(16, 0, 16)), -1),
        (R(T=-0.5), -1),
        (R(T=float("nan")), -1),
        (R(e=(0.0, 0.0, 0.0)), -1),
        (R(kind=7), -1),
        (R(kind="sc", L=(2048, 2048, 1024)), -2),        # over 2^31 sites
    ]
    for rep, status in cases:
        with pytest.raises(M.MCError) as ei:
            M.required_sites(rep)
        assert ei.value.status == status, (rep, ei.value)
        assert M.last_error()
    # odd lengths are fine on open axes and for bcc / fcc
    M.required_sites(R(kind="sc", L=(16, 15, 7), periodic_mask=1))
    M.required_sites(R(kind="bcc", L=(5, 5, 5)))
    M.required_sites(R(kind="fcc", L=(5, 7, 3)))
    with pytest.raises(M.MCError):
        M.required_scratch([R(kind="sc"), R(kind="fcc")])  # one kind per handle
    assert M.required_scratch([R(kind="sc", L=(464, 464, 464))]) > 0


def test_series_stats_against_oracle(M):
    from oracle import stats as OS

    rng = np.random.default_rng(5)
    n, N, T = 4096, 1000, 1.3
    # AR(1) magnetisation and energy series
    m = np.zeros((n, 3))
    E = np.zeros(n)
    for i in range(1, n):
        m[i] = 0.9 * m[i - 1] + rng.normal(scale=0.05, size=3)
        E[i] = 0.8 * E[i - 1] + rng.normal(scale=3.0)
    E -= 1500.0
    rec = np.zeros((n, 10))
    rec[:, 0] = np.arange(1, n + 1)
    rec[:, 1] = 400
    rec[:, 2:5] = m
    rec[:, 5] = np.linalg.norm(m, axis=1)
    rec[:, 6] = E
    rec[:, 7] = E
    st = M.series_stats(rec, N, T)
    ref = OS.series_summary(np.column_stack([m * N, E, np.zeros(n)]), N, T)
    for k in ("abs_m", "m2", "m4", "e", "U4"):
        assert st[k] == pytest.approx(ref[k], rel=1e-10), k
    for k in ("abs_m_err", "m2_err", "m4_err", "e_err", "U4_err"):
        assert st[k] == pytest.approx(ref[k], rel=1e-10), k
    assert st["C"] == pytest.approx(ref["C"], rel=1e-10)
    assert st["chi"] == pytest.approx(ref["chi"], rel=1e-10)
    assert st["acceptance"] == pytest.approx(0.4)
    # blocked error of an AR(1) mean: sigma/(1-phi)/sqrt(n) within 25 %
    sd_e = 3.0 / np.sqrt(1 - 0.8**2)
    want = sd_e * np.sqrt((1 + 0.8) / (1 - 0.8)) / np.sqrt(n) / N
    assert st["e_err"] == pytest.approx(want, rel=0.25)


def test_simulation_without_gpu_fails_loudly(M):
    import torch

    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(M.MCError):
        M.Simulation([M.Replica(L=(8, 8, 8))])


def test_tune_device_key_separates_devices(M):
    """The autotuner's cache key changes with the architecture, the compute
    unit count and the XCD count (a partition mode changes the last two), so
    a cached tile never carries over between such devices."""
    a = M.tune_device_key("gfx950:sramecc+:xnack-", 256, 8)
    assert a == "gfx950:sramecc+:xnack--cu256-xcd8"
    others = {M.tune_device_key("gfx950:sramecc+:xnack-", 32, 1),
              M.tune_device_key("gfx950:sramecc+:xnack-", 64, 2),
              M.tune_device_key("gfx942:sramecc+:xnack-", 256, 8),
              M.tune_device_key("gfx950:sramecc+:xnack-", 256, 4)}
    assert a not in others and len(others) == 4
    assert " " not in M.tune_device_key("gfx 950/x", 1, 1)
    with pytest.raises(M.MCError) as ei:
        M.tune_device_key("gfx950", -1, 8)
    assert ei.value.status == -1
