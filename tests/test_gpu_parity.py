"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Bars:
  * FP64 path: same chain as the oracle; per-sweep magnetisation within 1e-12,
    energy within 1e-10 relative, identical accepted-move counts (a decision
    flip needs |beta dH + ln P| below rounding, odds ~1e-15 per attempt).
  * FP32 path, one colour pass from an identical FP32-representable state:
    |dH32 - dH64| <= 1e-5 max(|dH64|, J); decisions equal unless
    |beta dH64 + ln P| < 1e-4; accepted spins within 2e-6.
  * Spins are bitwise independent of tile shape, batching and resume.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2106_11286_amd import workloads as W

pytestmark = pytest.mark.gpu

KIND = {"sc": O.SC, "bcc": O.BCC, "fcc": O.FCC}


@pytest.fixture(scope="module")
def M():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2106_11286_amd import mcheis

    return mcheis


def oracle_lattice(rep):
    L = rep.L if not isinstance(rep.L, int) else (rep.L,) * 3
    return O.Lattice(KIND[rep.kind], *L, periodic_mask=rep.periodic_mask,
                     sphere_radius=rep.sphere_radius)


def oracle_params(rep, seed):
    return O.Params(J=rep.J, K=rep.K, e=rep.e, T=rep.T, seed=seed, replica_id=rep.replica_id)


def natural(sim, r=0):
    return [t.double().cpu().numpy() for t in sim.to_natural(r)]


def packed_index(rep):
    """Library layout index of every canonical site (the ABI's layout rule)."""
    L = rep.L if not isinstance(rep.L, int) else (rep.L,) * 3
    Lx, Ly, Lz = L
    nb = {"sc": 1, "bcc": 2, "fcc": 4}[rep.kind]
    s = np.arange(Lx * Ly * Lz * nb)
    if rep.kind == "sc":
        x = s % Lx
        y = (s // Lx) % Ly
        z = s // (Lx * Ly)
        c = (x + y + z) & 1
        return c * (Lx * Ly * Lz // 2) + s // 2
    b = s % nb
    cell = s // nb
    return b * (Lx * Ly * Lz) + cell


SMALL_CASES = [
    # ragged multi-tile sc, periodic
    W.replica_fields(W.C1_SC16_TRAJECTORY, L=(40, 38, 34), K=0.1, T=1.2),
    # sc open in y and z with odd lengths
    dict(kind="sc", L=(10, 7, 5), periodic_mask=1, J=0.9, K=0.3, e=(1.0, 0.5, -0.2), T=0.9),
    # bcc periodic
    dict(kind="bcc", L=(10, 9, 8), periodic_mask=7, J=1.0, K=0.2, e=(0.0, 1.0, 1.0), T=1.7),
    # fcc nanoparticle, open surface
    dict(kind="fcc", L=(14, 14, 14), periodic_mask=0, sphere_radius=5.3, J=1.0, K=0.05,
         e=(1.0, 1.0, 1.0), T=0.9),
    # fcc periodic, ragged
    dict(kind="fcc", L=(9, 7, 6), periodic_mask=7, J=1.1, K=0.4, e=(0.0, 0.0, 1.0), T=2.5),
    # sc long rows (row-strip kernel), periodic, ragged rows per thread
    dict(kind="sc", L=(150, 14, 12), periodic_mask=7, J=1.0, K=0.05, e=(0.0, 0.0, 1.0), T=1.4),
    # sc long rows, open in y and z with odd lengths
    dict(kind="sc", L=(130, 9, 7), periodic_mask=1, J=0.8, K=0.2, e=(0.3, 0.0, 1.0), T=1.1),
    # sc cut to a sphere (open surface): the tile and LDS kernels skip the
    # unoccupied sites
    dict(kind="sc", L=(14, 12, 10), periodic_mask=0, sphere_radius=4.6, J=1.0, K=0.1,
         e=(0.2, 0.3, 1.0), T=1.1),
]


@pytest.mark.parametrize("case", range(len(SMALL_CASES)))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_random_init_matches_oracle(M, case, prec):
    rep = M.Replica(**SMALL_CASES[case], replica_id=3)
    sim = M.Simulation([rep], precision=prec, seed=77)
    g = natural(sim)
    lat = oracle_lattice(rep)
    o = O.init(lat, oracle_params(rep, 77))
    tol = 1e-14 if prec == "f64" else 2e-7
    for a, b in zip(g, o):
        assert np.max(np.abs(a - b)) <= tol
    occ = lat.tables()[0]
    assert np.all(g[0][~occ] == 0) and np.all(g[2][~occ] == 0)


def test_c1_trajectory_fp64(M):
    """sc L=16, K=0.1, T=1.2, seed 0, 1000 sweeps: per-sweep m and E equal the
    oracle's; accepted counts identical."""
    w = W.C1_SC16_TRAJECTORY
    rep = M.Replica(**W.replica_fields(w))
    sim = M.Simulation([rep], precision="f64", seed=w["seed"])
    lat = oracle_lattice(rep)
    p = oracle_params(rep, w["seed"])
    s = O.init(lat, p)
    for a, b in zip(natural(sim), s):
        assert np.max(np.abs(a - b)) <= 1e-14
    n = w["sweeps"]
    rec = sim.run_schedule([rep.T], n_equil=0, n_meas=n)[0, :, 0, :]
    ref = O.run(lat, p, 0, n, s)
    N = lat.n_occ
    assert np.array_equal(rec[:, 0], np.arange(1, n + 1))
    assert np.array_equal(rec[:, 1], ref[:, 5])
    assert np.max(np.abs(rec[:, 2:5] - ref[:, 0:3] / N)) <= 1e-12
    E_ref = ref[:, 3] + ref[:, 4]
    assert np.max(np.abs(rec[:, 6] - E_ref) / np.abs(E_ref)) <= 1e-10
    assert np.max(np.abs(rec[:, 7] - ref[:, 3]) / np.abs(E_ref)) <= 1e-10
    for a, b in zip(natural(sim), s):
        assert np.max(np.abs(a - b)) <= 1e-12


@pytest.mark.parametrize("case", range(len(SMALL_CASES)))
def test_fp64_trajectory_all_lattices(M, case):
    rep = M.Replica(**SMALL_CASES[case], replica_id=1)
    sim = M.Simulation([rep], precision="f64", seed=5)
    lat = oracle_lattice(rep)
    p = oracle_params(rep, 5)
    s = O.init(lat, p)
    ref = O.run(lat, p, 0, 25, s)
    recs = []
    for t in range(25):
        sim.sweep(1, measure=True)
        recs.append(sim.observables()[0])
    N = lat.n_occ
    for t, o in enumerate(recs):
        assert o["sweep"] == t + 1 and o["n_sites"] == N
        assert o["n_accepted"] == ref[t, 5]
        assert np.max(np.abs(o["M"] - ref[t, 0:3] / N)) <= 1e-12
        E = ref[t, 3] + ref[t, 4]
        assert abs(o["E"] - E) <= 1e-10 * max(1.0, abs(E))
        assert abs(o["E_anis"] - ref[t, 4]) <= 1e-10 * max(1.0, abs(E))
    for a, b in zip(natural(sim), s):
        assert np.max(np.abs(a - b)) <= 1e-12
    st = sim.measure_state()[0]
    ob = O.observables(lat, p, s)
    assert abs(st["E"] - ob["E"]) <= 1e-10 * max(1.0, abs(ob["E"]))


def _single_pass_check(M, rep, seed, sweeps, prec="f32"):
    sim = M.Simulation([rep], precision=prec, seed=seed)
    lat = oracle_lattice(rep)
    p = oracle_params(rep, seed)
    occ, col, _, _ = lat.tables()
    pidx = packed_index(rep)
    beta = 0.0 if math.isinf(rep.T) else (1.0 / rep.T if rep.T > 0 else None)
    n_checked = n_margin = 0
    for t in range(sweeps):
        sim.set_sweep(t)
        for c in range(lat.n_colours):
            state = natural(sim)
            ref = [a.copy() for a in state]
            n, dh64, acc64, mg = O.run_pass(lat, p, c, t, ref, outputs=True)
            dh, acc = sim.debug_pass(c)
            dh = dh[0].double().cpu().numpy()[pidx]
            acc = acc[0].cpu().numpy()[pidx]
            sel = occ & (col == c)
            assert np.all(acc[sel] <= 1)
            tol = 1e-5 * np.maximum(np.abs(dh64[sel]), abs(rep.J))
            assert np.all(np.abs(dh[sel] - dh64[sel]) <= tol)
            margin_ok = np.abs(mg[sel]) < 1e-4
            same = acc[sel].astype(bool) == acc64[sel]
            assert np.all(same | margin_ok)
            n_checked += int(sel.sum())
            n_margin += int((~same).sum())
            after = natural(sim)
            a_sel = sel & acc64.astype(bool) & (acc.astype(bool) == acc64)
            for a, b in zip(after, ref):
                assert np.max(np.abs(a[a_sel] - b[a_sel]), initial=0.0) <= 2e-6
            # rejected moves, other colours and unoccupied sites keep their bits
            keep = ~sel | ((acc == 0) & ~acc64.astype(bool))
            assert np.all(acc[~sel] == 255)
            for a, b in zip(after, state):
                assert np.array_equal(a[keep], b[keep])
            # continue both from the oracle's state rounded to the working precision
            sim.from_natural(0, [np.float32(a) if prec == "f32" else a for a in ref])
    return n_checked, n_margin


@pytest.mark.parametrize("case", range(len(SMALL_CASES)))
def test_fp32_single_pass_parity(M, case):
    rep = M.Replica(**SMALL_CASES[case], replica_id=2)
    n, nm = _single_pass_check(M, rep, seed=11, sweeps=3)
    assert n > 0 and nm <= max(2, n // 10000)


def test_fp32_single_pass_edge_temperatures(M):
    for T in (0.0, float("inf"), 0.05):
        rep = M.Replica(kind="sc", L=(12, 10, 8), J=1.0, K=0.2, T=T)
        _single_pass_check(M, rep, seed=3, sweeps=2)


TILES = [None, (0, 8, 8, 3), (0, 64, 4, 34), (0, 16, 2, 1), (1, 64, 1, 5), (1, 64, 4, 34),
         (1, 128, 8, 3), (1, 256, 2, 7), (1, 192, 4, 1), (2, 256, 2, 7), (2, 64, 4, 3),
         (2, 128, 2, 1), (2, 192, 4, 34)]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_tile_shape_and_batching_are_bitwise(M, prec):
    """Spins after several sweeps are bitwise identical for every kernel and
    tile shape, batched with other replicas or alone."""
    import torch

    base = dict(kind="sc", periodic_mask=7, J=1.0, K=0.1, e=(0.0, 0.0, 1.0))
    reps = [M.Replica(L=(24, 24, 24), T=1.0, replica_id=0, **base),
            M.Replica(L=(40, 38, 34), T=1.5, replica_id=1, **base),
            M.Replica(L=(150, 14, 12), T=0.7, replica_id=2, **base),
            M.Replica(L=(130, 9, 7), T=1.2, replica_id=3, kind="sc", periodic_mask=1, J=1.0,
                      K=0.3, e=(1.0, 0.0, 0.0))]
    batched = M.Simulation(reps, precision=prec, seed=9)
    batched.sweep(6, measure=True)
    obs_b = batched.observables()
    for r, rep in enumerate(reps):
        for tile in TILES:
            scratch = torch.empty(16 << 20, dtype=torch.uint8, device="cuda")
            one = M.Simulation([rep], precision=prec, seed=9, scratch=scratch)
            if tile:
                one.set_tile(tile[1], tile[2], tile[3], kernel=tile[0])
            one.sweep(6, measure=True)
            for a, b in zip(natural(one), natural(batched, r)):
                assert np.array_equal(a, b), (r, tile)
            o = one.observables()[0]
            assert o["n_accepted"] == obs_b[r]["n_accepted"]
            assert abs(o["E"] - obs_b[r]["E"]) <= 1e-9 * abs(o["E"])


MEASURE_CASES = [("sc", (64, 40, 30), None), ("sc", (64, 40, 30), (0, 16, 16, 1)),
                 ("sc", (64, 40, 30), (1, 64, 1, 1)), ("sc", (64, 40, 30), (1, 64, 4, 2)),
                 ("sc", (64, 40, 30), (2, 256, 4, 1)), ("sc", (150, 14, 12), (1, 128, 2, 3)),
                 ("bcc", (9, 8, 7), None), ("fcc", (7, 6, 5), None),
                 ("bcc", (9, 8, 7), (0, 8, 8, 2)), ("fcc", (7, 6, 5), (0, 8, 8, 1)),
                 ("sc", (16, 12, 10), (3, 256, 1, 1)), ("sc", (64, 40, 30), (4, 64, 2, 3)),
                 ("sc", (64, 40, 30), (4, 64, 4, 7)), ("sc", (64, 40, 30), (5, 256, 2, 3)),
                 ("sc", (64, 40, 30), (5, 128, 4, 2)), ("fcc", (70, 6, 5), (6, 64, 4, 2)),
                 ("bcc", (9, 8, 7), (6, 64, 2, 3))]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", range(len(MEASURE_CASES)))
def test_measuring_does_not_change_the_chain(M, case, prec):
    """Sweeps with the fused observable reduction leave bitwise the same spins
    as sweeps without it, eager, graph-replayed and persistent alike."""
    import torch

    kind, L, tile = MEASURE_CASES[case]
    if prec == "f64" and tile and tile[0] == 5 and tile[2] == 4:
        pytest.skip("FP64 band-pair tiles take 2-row bands only (refusal tested with the pair "
                    "kernel)")
    rep = M.Replica(kind=kind, L=L, K=0.1, T=1.3, e=(0.0, 0.6, 0.8))
    sims = []
    # the persistent kernel has no instantiation for strips of 1 or 8 rows or
    # for pair tiles
    no_persistent = tile and ((tile[0] == 4 and tile[2] == 4) or (tile[0] == 5 and tile[2] == 4) or
                              (tile[0] == 1 and tile[2] in (1, 8)))
    modes = ("plain", "measured") if no_persistent else ("plain", "measured", "persistent")
    for mode in modes:
        s = M.Simulation([rep], precision=prec, seed=8,
                         scratch=torch.empty(32 << 20, dtype=torch.uint8, device="cuda"))
        if tile:
            s.set_tile(tile[1], tile[2], tile[3], kernel=tile[0])
        if mode == "plain":
            s.sweep(3)
            s.sweep(2)
        else:
            s.sweep(3, measure=True, persistent=mode == "persistent")
            s.sweep(2, measure=True, persistent=mode == "persistent")
        sims.append(natural(s))
    for other in sims[1:]:
        for a, b in zip(sims[0], other):
            assert np.array_equal(a, b)
    if len(modes) == 2:
        with pytest.raises(M.MCError) as ei:
            s.sweep(1, persistent=True)
        assert ei.value.status == -2


PAIR_TILES = [(4, 64, 1, 5), (4, 128, 2, 3), (4, 64, 4, 34), (4, 256, 2, 7), (4, 192, 1, 1),
              (4, 64, 2, 1), (5, 256, 2, 5), (5, 128, 4, 3), (5, 64, 2, 34), (5, 256, 4, 1),
              (5, 192, 2, 2)]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_pair_kernel_is_bitwise(M, prec):
    """Two packed columns per thread (8/16-byte accesses; strip and band
    layouts): spins equal the
    default kernel's bitwise on rows of an even number of packed columns,
    including rows spread over several tiles, ragged rows and open faces."""
    import torch

    base = dict(kind="sc", J=1.0, K=0.1, e=(0.0, 0.6, 0.8))
    reps = [M.Replica(L=(24, 24, 24), T=1.0, replica_id=0, periodic_mask=7, **base),
            M.Replica(L=(40, 38, 34), T=1.5, replica_id=1, periodic_mask=7, **base),
            M.Replica(L=(148, 14, 12), T=0.7, replica_id=2, periodic_mask=7, **base),
            M.Replica(L=(132, 9, 7), T=1.2, replica_id=3, periodic_mask=1, **base),
            M.Replica(L=(520, 4, 6), T=1.3, replica_id=4, periodic_mask=6, **base)]
    ref = M.Simulation(reps, precision=prec, seed=9,
                       scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
    ref.set_tile(16, 16, 2, kernel=0)
    ref.sweep(6, measure=True)
    obs_r = ref.observables()
    for tile in PAIR_TILES:
        scratch = torch.empty(16 << 20, dtype=torch.uint8, device="cuda")
        one = M.Simulation(reps, precision=prec, seed=9, scratch=scratch)
        if prec == "f64" and tile[0] == 5 and tile[2] == 4:
            # FP64 band-pair tiles take 2-row bands only
            with pytest.raises(M.MCError) as ei:
                one.set_tile(tile[1], tile[2], tile[3], kernel=tile[0])
            assert ei.value.status == -2
            one.close()
            continue
        one.set_tile(tile[1], tile[2], tile[3], kernel=tile[0])
        one.sweep(2)
        one.sweep(4, measure=True)
        o = one.observables()
        for r in range(len(reps)):
            for a, b in zip(natural(one, r), natural(ref, r)):
                assert np.array_equal(a, b), (r, tile)
            assert o[r]["n_accepted"] == obs_r[r]["n_accepted"]
            assert abs(o[r]["E"] - obs_r[r]["E"]) <= 1e-9 * abs(o[r]["E"])
    odd = M.Simulation([M.Replica(kind="sc", L=(150, 14, 12))], precision=prec)
    for k in (4, 5):
        with pytest.raises(M.MCError) as ei:
            odd.set_tile(64, 2, 3, kernel=k)
        assert ei.value.status == -2


BSTRIP_TILES = [(6, 64, 1, 3), (6, 64, 4, 5), (6, 128, 2, 1), (6, 256, 1, 7), (6, 64, 2, 34)]


@pytest.mark.parametrize("kind", ["bcc", "fcc"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_basis_strip_kernel_is_bitwise(M, kind, prec):
    """bcc/fcc strip kernel (lanes along x, planes in registers, lane shifts):
    spins equal the tile kernel's bitwise, on rows spanning several waves,
    ragged rows and planes, open faces and the sphere."""
    import torch

    base = dict(kind=kind, J=1.0, K=0.15, e=(0.3, 0.5, 0.8))
    reps = [M.Replica(L=(70, 9, 7), periodic_mask=7, T=1.1, replica_id=0, **base),
            M.Replica(L=(130, 6, 5), periodic_mask=5, T=0.8, replica_id=1, **base),
            M.Replica(L=(12, 10, 8), periodic_mask=0, sphere_radius=4.5, T=1.4, replica_id=2, **base),
            M.Replica(L=(64, 7, 9), periodic_mask=2, T=1.7, replica_id=3, **base)]
    ref = M.Simulation(reps, precision=prec, seed=17,
                       scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
    ref.set_tile(16, 16, 2, kernel=0)
    ref.sweep(5, measure=True)
    obs_r = ref.observables()
    for tile in BSTRIP_TILES:
        one = M.Simulation(reps, precision=prec, seed=17,
                           scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
        one.set_tile(tile[1], tile[2], tile[3], kernel=tile[0])
        one.sweep(2)
        one.sweep(3, measure=True)
        o = one.observables()
        for r in range(len(reps)):
            for a, b in zip(natural(one, r), natural(ref, r)):
                assert np.array_equal(a, b), (r, tile)
            assert o[r]["n_accepted"] == obs_r[r]["n_accepted"], (r, tile)
            assert abs(o[r]["E"] - obs_r[r]["E"]) <= 1e-9 * abs(o[r]["E"])
    sc = M.Simulation([M.Replica(kind="sc", L=(16, 16, 16))], precision=prec)
    with pytest.raises(M.MCError):
        sc.set_tile(64, 1, 1, kernel=6)


BPAIR_TILES = [(7, 64, 1, 3), (7, 64, 2, 5), (7, 128, 2, 1), (7, 256, 1, 7), (7, 64, 2, 34)]


@pytest.mark.parametrize("kind", ["bcc", "fcc"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_basis_pair_kernel_is_bitwise(M, kind, prec):
    """bcc/fcc pair kernel (two cells per lane, bands of rows dealt over the
    lanes, lane shifts and edge words): spins equal the tile kernel's bitwise
    and acceptance counts match, on rows spanning several waves and bands
    running across waves, ragged bands and planes, open faces and the sphere;
    also through persistent launches and the debug pass."""
    import torch

    base = dict(kind=kind, J=1.0, K=0.15, e=(0.3, 0.5, 0.8))
    reps = [M.Replica(L=(70, 9, 7), periodic_mask=7, T=1.1, replica_id=0, **base),
            M.Replica(L=(130, 5, 5), periodic_mask=5, T=0.8, replica_id=1, **base),
            M.Replica(L=(12, 10, 8), periodic_mask=0, sphere_radius=4.5, T=1.4, replica_id=2, **base),
            M.Replica(L=(6, 7, 9), periodic_mask=2, T=1.7, replica_id=3, **base),
            M.Replica(L=(64, 7, 9), periodic_mask=3, T=1.3, replica_id=4, **base)]
    mk = lambda: M.Simulation(reps, precision=prec, seed=17,
                              scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
    ref = mk()
    ref.set_tile(16, 16, 2, kernel=0)
    ref.sweep(5, measure=True)
    obs_r = ref.observables()
    for tile in BPAIR_TILES:
        for pers in (False, True):
            one = mk()
            one.set_tile(tile[1], tile[2], tile[3], kernel=tile[0])
            one.sweep(2, persistent=pers)
            one.sweep(3, measure=True, persistent=pers)
            o = one.observables()
            for r in range(len(reps)):
                for a, b in zip(natural(one, r), natural(ref, r)):
                    assert np.array_equal(a, b), (r, tile, pers)
                assert o[r]["n_accepted"] == obs_r[r]["n_accepted"], (r, tile, pers)
                assert abs(o[r]["E"] - obs_r[r]["E"]) <= 1e-9 * abs(o[r]["E"])
            one.close()
    # the debug pass: per-site dH and decisions equal the tile kernel's
    a, b = mk(), mk()
    a.set_tile(128, 2, 3, kernel=7)
    b.set_tile(16, 16, 2, kernel=0)
    a.sweep(2)
    b.sweep(2)
    n_colours = 2 if kind == "bcc" else 4
    for c in range(n_colours):
        da, aa = a.debug_pass(c)
        db, ab = b.debug_pass(c)
        for r in range(len(reps)):
            assert torch.equal(aa[r], ab[r]), (c, r)
            sel = ab[r] != 255
            assert torch.equal(da[r][sel], db[r][sel]), (c, r)
    odd = M.Simulation([M.Replica(kind=kind, L=(7, 6, 6))], precision=prec)
    with pytest.raises(M.MCError) as ei:
        odd.set_tile(64, 1, 1, kernel=7)
    assert ei.value.status == -2
    sc = M.Simulation([M.Replica(kind="sc", L=(16, 16, 16))], precision=prec)
    with pytest.raises(M.MCError):
        sc.set_tile(64, 1, 1, kernel=7)


LDS_CASES = [("sc", (16, 16, 16), 7, 0.0, "f64"), ("sc", (16, 16, 16), 7, 0.0, "f32"),
             ("sc", (12, 10, 8), 5, 0.0, "f32"), ("bcc", (8, 8, 8), 7, 0.0, "f64"),
             ("bcc", (7, 9, 5), 3, 0.0, "f32"), ("fcc", (6, 6, 6), 0, 2.6, "f32"),
             ("fcc", (7, 6, 5), 7, 0.0, "f64")]


@pytest.mark.parametrize("case", range(len(LDS_CASES)))
def test_lds_kernel_matches_pass_kernels(M, case):
    """Lattices whose state fits one workgroup's LDS run whole sweeps there by
    default; spins equal the pass kernels' bitwise, records agree."""
    kind, L, mask, R, prec = LDS_CASES[case]
    rep = M.Replica(kind=kind, L=L, periodic_mask=mask, sphere_radius=R, K=0.2, T=1.1,
                    e=(0.3, 0.0, 0.95), replica_id=3)
    a = M.Simulation([rep, M.Replica(kind=kind, L=L, periodic_mask=mask, sphere_radius=R,
                                     K=0.05, T=2.0, replica_id=4)], precision=prec, seed=21)
    b = M.Simulation([rep, M.Replica(kind=kind, L=L, periodic_mask=mask, sphere_radius=R,
                                     K=0.05, T=2.0, replica_id=4)], precision=prec, seed=21)
    assert a.get_tile()[0] == 3
    b.set_tile(16, 16, 1, kernel=0)
    ra = a.run_schedule([[1.1, 2.0], [0.9, 1.5]], n_equil=3, n_meas=6)
    rb = b.run_schedule([[1.1, 2.0], [0.9, 1.5]], n_equil=3, n_meas=6)
    assert np.array_equal(ra[..., 0:2], rb[..., 0:2])  # sweep, accepted
    assert np.max(np.abs(ra[..., 2:5] - rb[..., 2:5])) <= 1e-12
    assert np.max(np.abs(ra[..., 6] - rb[..., 6]) / np.abs(rb[..., 6])) <= 1e-10
    a.sweep(5, persistent=True)
    b.sweep(5)
    a.set_tile(64, 1, 1, kernel=3)
    a.sweep(2, measure=True)
    b.sweep(2, measure=True)
    for r in range(2):
        for x, y in zip(natural(a, r), natural(b, r)):
            assert np.array_equal(x, y)
        oa, ob = a.observables()[r], b.observables()[r]
        assert oa["n_accepted"] == ob["n_accepted"] and oa["sweep"] == ob["sweep"]
    # single passes still run (on the pass kernel)
    st = a.measure_state()
    assert st[0]["n_sites"] == a.n_occ[0]


def test_lds_kernel_limits(M):
    big = M.Simulation([M.Replica(kind="sc", L=(64, 64, 64))], precision="f32")
    assert big.get_tile()[0] != 3
    with pytest.raises(M.MCError) as ei:
        big.set_tile(256, 1, 1, kernel=3)
    assert ei.value.status == -2
    small = M.Simulation([M.Replica(kind="sc", L=(8, 8, 8))], precision="f32")
    assert small.get_tile()[0] == 3
    for bad in (32, 100, 2048):
        with pytest.raises(M.MCError) as ei:
            small.set_tile(bad, 1, 1, kernel=3)
        assert ei.value.status == -1
    pm, tot = small.sweep_timed(4, measure=True)
    assert tot > 0 and pm > 0
    o = small.observables()[0]
    assert o["sweep"] == 4


def test_strip_kernel_rejects_other_lattices(M):
    sim = M.Simulation([M.Replica(kind="fcc", L=(6, 6, 6))])
    with pytest.raises(M.MCError):
        sim.set_tile(64, 4, 2, kernel=1)
    with pytest.raises(M.MCError):
        sim.set_tile(64, 2, 2, kernel=2)
    sim = M.Simulation([M.Replica(kind="sc", L=(16, 16, 16))])
    for bad in ((96, 4, 2), (64, 3, 2), (64, 4, 0), (512, 1, 1)):
        with pytest.raises(M.MCError):
            sim.set_tile(*bad, kernel=1)
    for bad in ((256, 1, 2), (256, 3, 2), (256, 8, 2), (100, 2, 2)):
        with pytest.raises(M.MCError):
            sim.set_tile(*bad, kernel=2)
    with pytest.raises(M.MCError):
        sim.set_tile(8, 8, 1, kernel=3)


def test_checkpoint_resume_is_bitwise(M):
    rep = M.Replica(kind="fcc", L=(10, 10, 10), periodic_mask=7, K=0.1, T=1.3)
    a = M.Simulation([rep], precision="f32", seed=21)
    a.sweep(10)
    b = M.Simulation([rep], precision="f32", seed=21)
    b.sweep(4)
    ck = natural(b)
    t = b.get_sweep()
    assert t == 4
    c = M.Simulation([rep], precision="f32", seed=21, init="user", user_spins=[ck])
    c.set_sweep(t)
    c.sweep(6)
    for x, y in zip(natural(a), natural(c)):
        assert np.array_equal(x, y)


def test_graph_replay_matches_eager(M):
    """run_schedule replays captured graphs; the chain and the records equal
    eager sweeps, replay after replay, with other stream work in between."""
    import torch

    rep = M.Replica(kind="sc", L=(32, 32, 32), K=0.1, T=1.3)
    g = M.Simulation([rep], precision="f32", seed=4)
    e = M.Simulation([rep], precision="f32", seed=4, stream=torch.cuda.default_stream())
    rec_g = []
    for rnd in range(3):
        rec_g.append(g.run_schedule([1.3], n_equil=70, n_meas=130)[0, :, 0, :])
        torch.ones(1000, device="cuda").sum().item()  # unrelated eager work between replays
    rec_e = []
    for rnd in range(3):
        e.sweep(70)
        for i in range(130):
            e.sweep(1, measure=True)
            o = e.observables()[0]
            rec_e.append([o["sweep"], o["n_accepted"], o["E"]])
    rec_e = np.array(rec_e).reshape(3, 130, 3)
    for rnd in range(3):
        assert np.array_equal(rec_g[rnd][:, 0], rec_e[rnd][:, 0])
        assert np.array_equal(rec_g[rnd][:, 1], rec_e[rnd][:, 1])
        assert np.allclose(rec_g[rnd][:, 6], rec_e[rnd][:, 2], rtol=1e-12, atol=0)
    for x, y in zip(natural(g), natural(e)):
        assert np.array_equal(x, y)


def test_zero_and_infinite_temperature(M):
    rep = M.Replica(kind="bcc", L=(8, 8, 8), K=0.3, T=0.0)
    sim = M.Simulation([rep], precision="f32", seed=1)
    prev = sim.measure_state()[0]["E"]
    for t in range(10):
        sim.sweep(1, measure=True)
        o = sim.observables()[0]
        assert o["E"] <= prev + 1e-9 * abs(prev)
        prev = o["E"]
    sim.set_temperatures([float("inf")])
    sim.sweep(3, measure=True)
    o = sim.observables()[0]
    assert o["n_accepted"] == o["n_sites"]


def test_aligned_state_energy(M):
    w = W.C4_FCC_PARTICLE
    rep = M.Replica(**W.replica_fields(w))
    sim = M.Simulation([rep], precision="f64", seed=0, init="aligned")
    o = sim.measure_state()[0]
    assert o["n_sites"] == 3618393
    assert o["E"] == pytest.approx(-21518640 * w["J"] - w["K"] * 3618393, rel=1e-12)
    assert np.allclose(o["M"], np.ones(3) / np.sqrt(3), atol=1e-12)


def test_abi_errors(M):
    import torch

    with pytest.raises(M.MCError) as ei:
        M.Simulation([M.Replica(kind="sc", L=(16, 15, 16))])
    assert ei.value.status == -2
    with pytest.raises(M.MCError) as ei:
        M.Simulation([M.Replica(T=-1.0)])
    assert ei.value.status == -1
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(M.MCError) as ei:
        M.Simulation([M.Replica(L=(8, 8, 8))], scratch=small)
    assert ei.value.status == -3
    exact = M.required_scratch([M.Replica(L=(8, 8, 8))])
    sim = M.Simulation([M.Replica(L=(8, 8, 8))],
                       scratch=torch.empty(exact, dtype=torch.uint8, device="cuda"))
    with pytest.raises(M.MCError) as ei:
        sim.observables()
    assert ei.value.status == -5
    with pytest.raises(M.MCError) as ei:
        sim.set_tile(32, 16, 1)
    assert ei.value.status == -1
    with pytest.raises(M.MCError) as ei:
        sim.set_tile(1, 1, 1)  # work list larger than the handle's scratch
    assert ei.value.status == -3


def _sampled_pass(M, sim, rep, geo, p, t, colour, rng, n_sample=4096):
    """One debug pass of a big lattice; check sampled sites of the pass colour
    one by one against the oracle's single-site evaluation."""
    before = natural(sim)
    dh, acc = sim.debug_pass(colour)
    after = natural(sim)
    Lx, Ly, Lz = rep.L
    s = rng.integers(0, Lx * Ly * Lz, size=4 * n_sample)
    x, y, z = s % Lx, (s // Lx) % Ly, s // (Lx * Ly)
    s = s[((x + y + z) & 1) == colour][:n_sample]
    idx = (colour * (Lx * Ly * Lz // 2) + s // 2)
    dh = dh[0][torch_index(idx)].double().cpu().numpy()
    acc = acc[0][torch_index(idx)].cpu().numpy()
    n_flip = 0
    for k, site in enumerate(s):
        r = geo.site_attempt(p, t, before, int(site))
        assert abs(dh[k] - r["dH"]) <= 1e-5 * max(abs(r["dH"]), abs(rep.J)), (site, dh[k], r)
        if bool(acc[k]) != r["accepted"]:
            assert abs(r["margin"]) < 1e-4, (site, r)
            n_flip += 1
            continue
        got = np.array([after[0][site], after[1][site], after[2][site]])
        assert np.max(np.abs(got - r["S_after"])) <= 2e-6
    return before, after, dh, acc, n_flip


def torch_index(idx):
    import torch

    return torch.as_tensor(idx, dtype=torch.int64, device="cuda")


def test_full_size_sc464_sampled(M):
    """The benchmark lattice (sc L=464, 99,897,344 spins, FP32, the autotuned
    tile the benchmark times): after the tuning sweeps and 100 more, both colour
    passes of the next sweep checked at 4096 sampled
    sites each against the oracle's single-site evaluation from the same
    state, plus energy bookkeeping of the whole pass and fused-vs-recomputed
    observables."""
    import torch

    w = W.C5_SC464_ROOFLINE
    rep = M.Replica(**W.replica_fields(w))
    sim = M.Simulation([rep], precision="f32", seed=w["seed"],
                       scratch=torch.empty(64 << 20, dtype=torch.uint8, device="cuda"))
    assert sim.get_tile()[0] == 4  # default: the pair kernel
    # the launch configuration the benchmark times: the autotuner's choice
    tile = sim.autotune(trial_sweeps=6, measure=True)
    print("autotuned tile", tile)
    t0 = sim.get_sweep()
    sim.sweep(99)
    sim.sweep(1, measure=True)
    fused = sim.observables()[0]
    full = sim.measure_state()[0]
    assert fused["n_sites"] == 464**3
    assert abs(fused["E"] - full["E"]) <= 1e-9 * abs(full["E"])
    assert np.max(np.abs(fused["M"] - full["M"])) <= 1e-12
    geo = O.Geometry(O.SC, *rep.L, periodic_mask=rep.periodic_mask)
    p = oracle_params(rep, w["seed"])
    rng = np.random.default_rng(464)
    t = sim.get_sweep()
    assert t == t0 + 100
    n_flip = 0
    for colour in (0, 1):
        before, after, dh, acc, nf = _sampled_pass(M, sim, rep, geo, p, t, colour, rng)
        n_flip += nf
        del before, after
    assert n_flip <= 2


def test_full_size_pass_bookkeeping(M):
    """Energy bookkeeping over every site of both passes at full size."""
    import torch

    w = W.C5_SC464_ROOFLINE
    rep = M.Replica(**W.replica_fields(w))
    sim = M.Simulation([rep], precision="f32", seed=w["seed"])
    sim.sweep(20)
    for colour in (0, 1):
        e0 = sim.measure_state()[0]["E"]
        dh, acc = sim.debug_pass(colour)
        e1 = sim.measure_state()[0]["E"]
        sel = acc[0] == 1
        total = dh[0][sel].double().sum().item()
        assert abs((e1 - e0) - total) <= 1e-6 * 464**3, (e1 - e0, total)
        assert int((acc[0] > 1).sum().item()) == 464**3 // 2  # other colour untouched (255)


def test_full_size_fcc_particle_sampled(M):
    """The FCC nanoparticle (128^3 cells, R = 60, open surface): one sweep's
    four passes at sampled sites against the oracle, after 20 sweeps."""
    w = W.C4_FCC_PARTICLE
    rep = M.Replica(**W.replica_fields(w))
    sim = M.Simulation([rep], precision="f32", seed=w["seed"])
    sim.sweep(20)
    geo = O.Geometry(O.FCC, *rep.L, periodic_mask=rep.periodic_mask,
                     sphere_radius=rep.sphere_radius)
    p = oracle_params(rep, w["seed"])
    rng = np.random.default_rng(128)
    t = sim.get_sweep()
    Lx, Ly, Lz = rep.L
    for colour in range(4):
        before = natural(sim)
        dh, acc = sim.debug_pass(colour)
        after = natural(sim)
        cells = rng.integers(0, Lx * Ly * Lz, size=20000)
        s = cells * 4 + colour
        checked = 0
        for cell, site in zip(cells, s):
            r = geo.site_attempt(p, t, before, int(site))
            k = colour * (Lx * Ly * Lz) + int(cell)
            if r is None:
                assert int(acc[0][k].item()) == 255  # unoccupied: never visited
                continue
            d = float(dh[0][k].item())
            assert abs(d - r["dH"]) <= 1e-5 * max(abs(r["dH"]), 1.0)
            if bool(acc[0][k].item()) == r["accepted"]:
                got = np.array([after[0][site], after[1][site], after[2][site]])
                assert np.max(np.abs(got - r["S_after"])) <= 2e-6
            else:
                assert abs(r["margin"]) < 1e-4
            checked += 1
            if checked >= 1500:
                break
        assert checked >= 1500


def test_full_size_fcc_sampled(M):
    """fcc at the benchmark's scale (4 x 292^3 = 99,588,352 spins, FP32, the
    autotuned tile): after the tuning sweeps and 5 more, all four colour
    passes of the next sweep at 1000 sampled sites each against the oracle,
    and the fused observables against a recomputation."""
    import torch

    w = W.FCC_292_1E8
    rep = M.Replica(**W.replica_fields(w))
    sim = M.Simulation([rep], precision="f32", seed=w["seed"],
                       scratch=torch.empty(64 << 20, dtype=torch.uint8, device="cuda"))
    tile = sim.autotune(trial_sweeps=2, measure=True)
    print("autotuned tile", tile)
    sim.sweep(4)
    sim.sweep(1, measure=True)
    fused = sim.observables()[0]
    full = sim.measure_state()[0]
    assert fused["n_sites"] == 4 * 292**3
    assert abs(fused["E"] - full["E"]) <= 1e-9 * abs(full["E"])
    assert np.max(np.abs(fused["M"] - full["M"])) <= 1e-12
    geo = O.Geometry(O.FCC, *rep.L, periodic_mask=rep.periodic_mask)
    p = oracle_params(rep, w["seed"])
    rng = np.random.default_rng(292)
    t = sim.get_sweep()
    cells_n = 292**3
    n_flip = 0
    for colour in range(4):
        before = natural(sim)
        dh, acc = sim.debug_pass(colour)
        after = natural(sim)
        cells = rng.integers(0, cells_n, size=1000)
        k = torch_index(colour * cells_n + cells)
        dhs = dh[0][k].double().cpu().numpy()
        accs = acc[0][k].cpu().numpy()
        del dh, acc
        for j, cell in enumerate(cells):
            site = int(cell) * 4 + colour
            r = geo.site_attempt(p, t, before, site)
            assert abs(dhs[j] - r["dH"]) <= 1e-5 * max(abs(r["dH"]), 1.0), (site, dhs[j], r)
            if bool(accs[j]) != r["accepted"]:
                assert abs(r["margin"]) < 1e-4, (site, r)
                n_flip += 1
                continue
            got = np.array([after[0][site], after[1][site], after[2][site]])
            assert np.max(np.abs(got - r["S_after"])) <= 2e-6
        del before, after
    assert n_flip <= 2


def test_full_size_bcc_sampled(M):
    """bcc at the benchmark's scale (2 x 368^3 = 99,672,064 spins, FP32, the
    autotuned tile): after the tuning sweeps and 10 more, both colour passes of
    the next sweep at 1500 sampled sites each against the oracle's single-site
    evaluation, and the fused observables against a recomputation."""
    import torch

    w = W.BCC_368_1E8
    rep = M.Replica(**W.replica_fields(w))
    sim = M.Simulation([rep], precision="f32", seed=w["seed"],
                       scratch=torch.empty(64 << 20, dtype=torch.uint8, device="cuda"))
    tile = sim.autotune(trial_sweeps=2, measure=True)
    print("autotuned tile", tile)
    sim.sweep(9)
    sim.sweep(1, measure=True)
    fused = sim.observables()[0]
    full = sim.measure_state()[0]
    assert fused["n_sites"] == 2 * 368**3
    assert abs(fused["E"] - full["E"]) <= 1e-9 * abs(full["E"])
    assert np.max(np.abs(fused["M"] - full["M"])) <= 1e-12
    geo = O.Geometry(O.BCC, *rep.L, periodic_mask=rep.periodic_mask)
    p = oracle_params(rep, w["seed"])
    rng = np.random.default_rng(368)
    t = sim.get_sweep()
    cells_n = 368**3
    n_flip = 0
    for colour in (0, 1):
        before = natural(sim)
        dh, acc = sim.debug_pass(colour)
        after = natural(sim)
        cells = rng.integers(0, cells_n, size=1500)
        k = torch_index(colour * cells_n + cells)
        dhs = dh[0][k].double().cpu().numpy()
        accs = acc[0][k].cpu().numpy()
        del dh, acc
        for j, cell in enumerate(cells):
            site = int(cell) * 2 + colour
            r = geo.site_attempt(p, t, before, site)
            assert abs(dhs[j] - r["dH"]) <= 1e-5 * max(abs(r["dH"]), 1.0), (site, dhs[j], r)
            if bool(accs[j]) != r["accepted"]:
                assert abs(r["margin"]) < 1e-4, (site, r)
                n_flip += 1
                continue
            got = np.array([after[0][site], after[1][site], after[2][site]])
            assert np.max(np.abs(got - r["S_after"])) <= 2e-6
        del before, after
    assert n_flip <= 2


# --------------------------------------------------------------------------
# Persistent batched launches (many replicas, uneven sizes, one launch)
# --------------------------------------------------------------------------
def _batch(M, kind="sc"):
    if kind == "sc":
        Ls = [(16, 16, 16), (24, 24, 24), (32, 32, 32), (48, 48, 48), (20, 18, 22)]
    else:
        Ls = [(6, 6, 6), (9, 7, 8), (10, 10, 10)]
    return [M.Replica(kind=kind, L=L, J=1.0, K=0.1, e=(0.0, 0.0, 1.0), T=0.8 + 0.3 * r,
                      replica_id=r) for r, L in enumerate(Ls)]


@pytest.mark.parametrize("kind,prec", [("sc", "f32"), ("sc", "f64"), ("fcc", "f32"),
                                       ("fcc", "f64")])
def test_persistent_matches_eager(M, kind, prec):
    reps = _batch(M, kind)
    a = M.Simulation(reps, precision=prec, seed=12)
    b = M.Simulation(reps, precision=prec, seed=12)
    if kind == "fcc":  # small enough for the LDS kernel: pin the pass kernel
        for s in (a, b):
            s.set_tile(16, 16, 1, kernel=0)
    for rnd in range(3):
        a.sweep(4, measure=True, persistent=True)
        b.sweep(4, measure=True)
        oa, ob = a.observables(), b.observables()
        for x, y in zip(oa, ob):
            assert x["sweep"] == y["sweep"] and x["n_accepted"] == y["n_accepted"]
            assert abs(x["E"] - y["E"]) <= 1e-12 * abs(y["E"])
            assert np.max(np.abs(x["M"] - y["M"])) <= 1e-14
    for r in range(len(reps)):
        for x, y in zip(natural(a, r), natural(b, r)):
            assert np.array_equal(x, y)


def test_persistent_schedule_and_oracle(M):
    """A persistent, graph-replayed schedule over uneven replicas equals the
    oracle's FP64 chain replica by replica."""
    reps = _batch(M)[:3]
    sim = M.Simulation(reps, precision="f64", seed=31)
    T = np.array([[0.9, 1.2, 1.5], [1.1, 1.3, 2.0]])
    rec = sim.run_schedule(T, n_equil=5, n_meas=9, persistent=True)
    for r, rep in enumerate(reps):
        lat = oracle_lattice(rep)
        s = O.init(lat, oracle_params(rep, 31))
        t = 0
        for step in range(2):
            p = oracle_params(M.Replica(**{**rep.__dict__, "T": T[step, r]}), 31)
            O.run(lat, p, t, 5, s, record=False)
            ref = O.run(lat, p, t + 5, 9, s)
            t += 14
            got = rec[step, :, r, :]
            assert np.array_equal(got[:, 1], ref[:, 5])
            assert np.max(np.abs(got[:, 2:5] - ref[:, 0:3] / lat.n_occ)) <= 1e-12
        for x, y in zip(natural(sim, r), s):
            assert np.max(np.abs(x - y)) <= 1e-12


def test_persistent_watchdog_exits_cleanly(M):
    """A zero wait budget makes the persistent launch give up at its first
    unmet dependency: every workgroup exits, the next synchronising call
    reports MC_E_DEVICE, and the handle keeps working afterwards."""
    reps = _batch(M)[:2]
    sim = M.Simulation(reps, precision="f32", seed=5)
    sim.set_watchdog(0)
    sim.sweep(40, persistent=True)
    with pytest.raises(M.MCError) as ei:
        sim.synchronize_checked()
    assert ei.value.status == -4 and "persistent" in str(ei.value)
    sim.set_watchdog(1 << 24)
    sim.sweep(3, measure=True, persistent=True)
    o = sim.observables()
    assert all(x["n_sites"] > 0 for x in o)


def _xcd_batch(M, kind, n=16):
    """n replicas of four sizes and temperatures from 0.8 to 2.0."""
    if kind == "sc":
        Ls = [(40, 40, 40), (32, 32, 32), (24, 24, 24), (16, 16, 16)]
    else:
        Ls = [(10, 10, 10), (8, 9, 7), (7, 7, 7), (5, 6, 5)]
    return [M.Replica(kind=kind, L=Ls[r % 4], J=1.0, K=0.1, e=(0.0, 0.0, 1.0),
                      T=0.8 + 1.2 * r / max(n - 1, 1), replica_id=r) for r in range(n)]


def _queues(M, sim, mode):
    try:
        sim.set_persistent_mode(mode)
    except M.MCError as e:
        if mode == "xcd" and e.status == -2:
            pytest.skip("device does not deal workgroups to eight XCDs in turn")
        raise
    return sim.persistent_queues()


@pytest.mark.parametrize("kind,prec,tile,n", [
    ("sc", "f32", None, 16), ("sc", "f32", (5, 256, 2, 7), 16), ("sc", "f32", (0, 32, 8, 4), 16),
    ("sc", "f64", (1, 64, 4, 3), 16), ("sc", "f32", None, 5),
    ("bcc", "f32", (0, 16, 16, 1), 16), ("fcc", "f64", (0, 16, 16, 1), 16)])
def test_xcd_queues_match_eager(M, kind, prec, tile, n):
    """Persistent launches with one queue per XCD and with one queue give the
    default launches' chain: spins bitwise equal after three measured calls of
    5 sweeps, the same acceptance counts and energies; the two queue modes
    also give bitwise equal records.  Five replicas leave three queues empty."""
    import torch

    reps = _xcd_batch(M, kind, n)
    sims = [M.Simulation(reps, precision=prec, seed=41,
                         scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
            for _ in range(3)]
    if tile is not None:
        for s in sims:
            s.set_tile(tile[1], tile[2], tile[3], kernel=tile[0])
    assert _queues(M, sims[0], "xcd") == 8
    assert _queues(M, sims[1], "global") == 1
    eager = sims[2]
    for rnd in range(3):
        for s in sims[:2]:
            s.sweep(5, measure=True, persistent=True)
        eager.sweep(5, measure=True)
        oe = eager.observables()
        for s in sims[:2]:
            for x, y in zip(s.observables(), oe):
                assert x["sweep"] == y["sweep"] and x["n_accepted"] == y["n_accepted"]
                assert abs(x["E"] - y["E"]) <= 1e-12 * abs(y["E"])
                assert np.max(np.abs(x["M"] - y["M"])) <= 1e-14
    for r in range(n):
        ref = natural(eager, r)
        for s in sims[:2]:
            for x, y in zip(natural(s, r), ref):
                assert np.array_equal(x, y), r
    T = np.linspace(0.9, 1.9, n)
    rx = sims[0].run_schedule(T, n_equil=3, n_meas=6, persistent=True)
    rg = sims[1].run_schedule(T, n_equil=3, n_meas=6, persistent=True)
    assert np.array_equal(rx, rg)
    for s in sims:
        s.close()


def test_xcd_queue_auto_and_retile(M):
    """Auto mode takes per-XCD queues for 16 balanced replicas and one queue
    for 2; a tile change re-deals the replicas and keeps the chain."""
    reps = _xcd_batch(M, "sc", 16)
    a = M.Simulation(reps, precision="f32", seed=43)
    b = M.Simulation(reps, precision="f32", seed=43)
    q = _queues(M, a, "auto")
    if q != 8:
        pytest.skip("device does not deal workgroups to eight XCDs in turn")
    assert M.Simulation(reps[:2], precision="f32", seed=43).persistent_queues() == 1
    # eight replicas, one of them far larger than the rest: the best deal
    # leaves one queue with most of the work, so auto mode keeps one queue
    skew = [M.Replica(kind="sc", L=(64, 64, 64) if r == 0 else (8, 8, 8), T=1.0, replica_id=r)
            for r in range(8)]
    assert M.Simulation(skew, precision="f32", seed=43).persistent_queues() == 1
    a.sweep(3, persistent=True)
    a.set_tile(32, 8, 4, kernel=0)
    assert a.persistent_queues() == 8
    a.sweep(4, measure=True, persistent=True)
    b.sweep(7, measure=True)
    for r in range(len(reps)):
        for x, y in zip(natural(a, r), natural(b, r)):
            assert np.array_equal(x, y), r


def test_persistent_watchdog_is_sticky(M):
    """A launch that gave up is reported even when another persistent launch
    followed it before the synchronising call."""
    reps = _batch(M)[:2]
    sim = M.Simulation(reps, precision="f32", seed=5)
    sim.set_watchdog(0)
    sim.sweep(40, persistent=True)
    sim.set_watchdog(1 << 24)
    sim.sweep(2, persistent=True)
    with pytest.raises(M.MCError) as ei:
        sim.synchronize_checked()
    assert ei.value.status == -4 and "persistent" in str(ei.value)
    sim.sweep(2, persistent=True)
    sim.synchronize_checked()


def test_autotune_keeps_chain_and_caches(M, tmp_path):
    """The autotuner's trials are ordinary sweeps: after it, the state equals a
    plain run of the same number of sweeps; a second call hits the cache."""
    rep = M.Replica(kind="sc", L=(64, 40, 30), K=0.1, T=1.3)
    import torch

    scratch = torch.empty(32 << 20, dtype=torch.uint8, device="cuda")
    a = M.Simulation([rep], precision="f32", seed=8, scratch=scratch)
    cache = str(tmp_path / "tune.txt")
    tile = a.autotune(trial_sweeps=2, measure=True, cache_path=cache)
    t = a.get_sweep()
    assert t >= 3 and tile == a.get_tile()[:4]
    b = M.Simulation([rep], precision="f32", seed=8)
    b.sweep(t)
    for x, y in zip(natural(a), natural(b)):
        assert np.array_equal(x, y)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1
    c = M.Simulation([rep], precision="f32", seed=8, scratch=torch.empty(32 << 20, dtype=torch.uint8, device="cuda"))
    assert c.autotune(trial_sweeps=2, measure=True, cache_path=cache) == tile
    assert c.get_sweep() == 0  # cache hit: no trial sweeps
    assert len(open(cache).read().splitlines()) == 1


def test_stream_probe_pattern_and_errors(M):
    """The memory-pattern probe reads both halves and writes the first in
    place: after one untimed and two timed launches, first = first + 3 second."""
    import torch

    P = 1000
    base = [torch.arange(2 * P, dtype=torch.float32, device="cuda") * (a + 1) for a in range(3)]
    xs = [b.clone() for b in base]
    ms = M.stream_probe(*xs, grid=3, reps=2)
    assert ms > 0
    for b, x in zip(base, xs):
        want = b[:P] + 3 * b[P:]
        assert torch.equal(x[:P], want) and torch.equal(x[P:], b[P:])
    odd = [torch.zeros(2 * 7, dtype=torch.float32, device="cuda") for _ in range(3)]
    with pytest.raises(M.MCError) as ei:
        M.stream_probe(*odd)
    assert ei.value.status == -1


@pytest.mark.parametrize("persistent", [False, True])
def test_schedule_measure_every(M, persistent):
    """measure_every = 3 records every third sweep of the measurement phase;
    each record equals the record of the same sweep in an every-sweep run."""
    reps = [M.Replica(kind="sc", L=(40, 20, 12), K=0.1, T=1.0, replica_id=0),
            M.Replica(kind="sc", L=(40, 20, 12), K=0.1, T=1.0, replica_id=1)]
    T = [[1.2, 1.6], [0.9, 1.1]]
    a = M.Simulation(reps, precision="f32", seed=31)
    b = M.Simulation(reps, precision="f32", seed=31)
    ra = a.run_schedule(T, n_equil=4, n_meas=12, measure_every=3, persistent=persistent)
    rb = b.run_schedule(T, n_equil=4, n_meas=12, measure_every=1, persistent=persistent)
    assert ra.shape == (2, 4, 2, 10) and rb.shape == (2, 12, 2, 10)
    for i in range(2):
        want = rb[i, 2::3]
        # sweeps completed at records: 16 per temperature, 4 of them equilibration
        sweeps = 16 * i + 4 + 3 * np.arange(1, 5)
        assert np.array_equal(ra[i, :, :, 0], np.repeat(sweeps[:, None], 2, axis=1))
        assert np.array_equal(ra[i], want)
    for r in range(2):
        for x, y in zip(natural(a, r), natural(b, r)):
            assert np.array_equal(x, y)


def test_sc_sphere_kernels(M):
    """A simple-cubic lattice cut to a sphere runs on the tile kernel (and the
    LDS kernel for small lattices), which never updates an unoccupied site;
    the other simple-cubic kernels are refused.  The tile kernel's FP64 chain
    equals the oracle's, and the unoccupied sites stay zero."""
    rep = M.Replica(kind="sc", L=(40, 38, 34), periodic_mask=0, sphere_radius=15.2, J=1.0,
                    K=0.1, e=(0.0, 0.0, 1.0), T=1.3)
    sim = M.Simulation([rep], precision="f64", seed=19)
    assert sim.get_tile()[0] == 0
    for kernel, tx, ty in ((1, 64, 2), (2, 256, 2), (4, 64, 2), (5, 256, 2)):
        with pytest.raises(M.MCError) as ei:
            sim.set_tile(tx, ty, 4, kernel=kernel)
        assert ei.value.status == -2
    sim.set_tile(16, 8, 5, kernel=0)
    lat = oracle_lattice(rep)
    p = oracle_params(rep, 19)
    s = O.init(lat, p)
    ref = O.run(lat, p, 0, 12, s)
    for t in range(12):
        sim.sweep(1, measure=True)
        o = sim.observables()[0]
        assert o["n_accepted"] == ref[t, 5]
        assert np.max(np.abs(o["M"] - ref[t, 0:3] / lat.n_occ)) <= 1e-12
    occ = lat.tables()[0]
    for a, b in zip(natural(sim), s):
        assert np.max(np.abs(a - b)) <= 1e-12
        assert np.all(a[~occ] == 0.0)


@pytest.mark.parametrize("case", range(len(SMALL_CASES)))
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_measure_buffers_matches_oracle(M, case, prec):
    """mc_measure_buffers (no handle; caller workspace) on a simulation's own
    spin buffers after a few sweeps: magnetisation sums and both energy terms
    equal the oracle's from-scratch observables of the same state (every
    product in FP64, so only the summation order differs), and equal
    mc_measure_state's."""
    rep = M.Replica(**SMALL_CASES[case], replica_id=4)
    sim = M.Simulation([rep], precision=prec, seed=23)
    sim.sweep(3)
    sim.synchronize()
    got = M.measure_buffers(rep, prec, *sim.spins[0])
    lat = oracle_lattice(rep)
    ob = O.observables(lat, oracle_params(rep, 23), natural(sim))
    assert got["n_sites"] == lat.n_occ
    assert np.max(np.abs(got["M"] - ob["M"])) <= 1e-12 * lat.n_occ
    for k in ("E_exch", "E_anis"):
        assert abs(got[k] - ob[k]) <= 1e-12 * max(1.0, abs(ob["E"])), (k, got[k], ob[k])
    st = sim.measure_state()[0]
    assert abs(st["E"] - got["E"]) <= 1e-12 * max(1.0, abs(ob["E"]))


def test_measure_buffers_errors(M):
    import torch

    rep = M.Replica(kind="sc", L=(8, 8, 8))
    t = [torch.zeros(512, dtype=torch.float32, device="cuda") for _ in range(3)]
    with pytest.raises(M.MCError) as ei:
        M.measure_buffers(rep, "f32", *t, workspace=torch.empty(1024, dtype=torch.uint8,
                                                                device="cuda"))
    assert ei.value.status == -3
    short = [x[:100] for x in t]
    with pytest.raises(M.MCError) as ei:
        M.measure_buffers(rep, "f32", *short)
    assert ei.value.status == -3
    with pytest.raises(M.MCError) as ei:
        M.measure_buffers(M.Replica(kind="sc", L=(8, 7, 8)), "f32", *t)
    assert ei.value.status == -2


LBAND_TILES = [(8, 256, 1, 3), (8, 256, 2, 5), (8, 256, 4, 2), (8, 256, 7, 34), (8, 256, 3, 1)]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_lds_band_kernel_is_bitwise(M, prec):
    """Rows staged through LDS by asynchronous copies (kernel 8): spins and
    accepted counts equal the tile kernel's bitwise, over periodic and open
    faces, ragged row tiles and several plane chunks; rows that are not a
    multiple of 16 bytes are refused."""
    import torch

    base = dict(kind="sc", J=1.0, K=0.1, e=(0.0, 0.6, 0.8))
    reps = [M.Replica(L=(24, 24, 24), T=1.0, replica_id=0, periodic_mask=7, **base),
            M.Replica(L=(40, 38, 34), T=1.5, replica_id=1, periodic_mask=7, **base),
            M.Replica(L=(48, 14, 12), T=0.7, replica_id=2, periodic_mask=7, **base),
            M.Replica(L=(32, 9, 7), T=1.2, replica_id=3, periodic_mask=1, **base),
            M.Replica(L=(64, 4, 6), T=1.3, replica_id=4, periodic_mask=6, **base)]
    ref = M.Simulation(reps, precision=prec, seed=13,
                       scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
    ref.set_tile(16, 16, 2, kernel=0)
    ref.sweep(3)
    ref.sweep(3, measure=True)
    obs_r = ref.observables()
    for tile in LBAND_TILES:
        one = M.Simulation(reps, precision=prec, seed=13,
                           scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
        one.set_tile(tile[1], tile[2], tile[3], kernel=tile[0])
        one.sweep(3)
        one.sweep(3, measure=True)
        o = one.observables()
        for r in range(len(reps)):
            for a, b in zip(natural(one, r), natural(ref, r)):
                assert np.array_equal(a, b), (r, tile)
            assert o[r]["n_accepted"] == obs_r[r]["n_accepted"], (r, tile)
            assert abs(o[r]["E"] - obs_r[r]["E"]) <= 1e-9 * abs(o[r]["E"])
        one.close()
    # debug pass of the same kernel: per-site dH and decisions as the tile kernel's
    a = M.Simulation(reps[:2], precision=prec, seed=14,
                     scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
    b = M.Simulation(reps[:2], precision=prec, seed=14,
                     scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
    a.set_tile(16, 16, 2, kernel=0)
    b.set_tile(256, 2, 3, kernel=8)
    for c in (0, 1):
        da, aa = a.debug_pass(c)
        db, ab = b.debug_pass(c)
        for r in range(2):
            assert torch.equal(aa[r], ab[r])
            assert torch.equal(torch.nan_to_num(da[r], nan=7.0), torch.nan_to_num(db[r], nan=7.0))
    odd = M.Simulation([M.Replica(kind="sc", L=(18, 8, 8))], precision=prec)
    with pytest.raises(M.MCError) as ei:
        odd.set_tile(256, 2, 3, kernel=8)
    assert ei.value.status == -2


def test_tuned_launch_keeps_the_chain(M, tmp_path):
    """The autotuner choosing the launch mode with the tile (MC_TUNED_LAUNCH):
    sweeps in the chosen mode, and a schedule with the flag, give bitwise the
    spins of plain per-pass sweeps; the choice is cached with the tile."""
    import torch

    reps = [M.Replica(kind="sc", L=(L, L, L), K=0.1, T=0.9 + 0.2 * r, replica_id=r)
            for r, L in enumerate((16, 24, 32, 24, 16, 32, 24, 16, 20))]
    cache = str(tmp_path / "tune.txt")
    a = M.Simulation(reps, precision="f32", seed=31,
                     scratch=torch.empty(32 << 20, dtype=torch.uint8, device="cuda"))
    tile = a.autotune(trial_sweeps=2, measure=True, tune_launch=True, cache_path=cache)
    mode = a.tuned_launch()
    assert mode in ("persistent", "per-pass")
    t = a.get_sweep()
    a.sweep(5, measure=True, tuned=True)
    a.run_schedule([[rep.T for rep in reps]], n_equil=0, n_meas=3, tuned=True)
    b = M.Simulation(reps, precision="f32", seed=31,
                     scratch=torch.empty(32 << 20, dtype=torch.uint8, device="cuda"))
    b.set_tile(tile[1], tile[2], tile[3], kernel=tile[0])
    b.sweep(t + 8)
    for r in range(len(reps)):
        for x, y in zip(natural(a, r), natural(b, r)):
            assert np.array_equal(x, y), r
    c = M.Simulation(reps, precision="f32", seed=31,
                     scratch=torch.empty(32 << 20, dtype=torch.uint8, device="cuda"))
    assert c.autotune(trial_sweeps=2, measure=True, tune_launch=True, cache_path=cache) == tile
    assert c.tuned_launch() == mode
    c.set_tile(tile[1], tile[2], tile[3], kernel=tile[0])
    assert c.tuned_launch() == "per-pass"
    with pytest.raises(M.MCError) as ei:
        M._check("mc_sweep", M.LIB.mc_sweep(a.handle, 1, M.PERSISTENT | M.TUNED_LAUNCH))
    assert ei.value.status == -1


# (kernel, threads, rows, planes): one to three (row, pair) positions per lane
FUSED_TILES = {"f32": [(9, 256, 1, 1), (9, 256, 2, 3), (9, 256, 3, 5), (9, 256, 4, 64),
                       (9, 512, 6, 4), (9, 1024, 5, 7), (9, 256, 20, 3), (9, 256, 40, 2)],
               "f64": [(9, 256, 1, 1), (9, 256, 2, 3), (9, 512, 3, 5), (9, 256, 4, 64)]}


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fused_sweep_is_bitwise(M, prec):
    """The fused sweep (kernel 9: both colours in one launch, next state into
    the second buffer set, halo colour-0 spins recomputed per tile) gives
    bitwise the spins of the two-pass chain and the same accepted counts, on
    periodic, open and mixed faces, ragged row tiles and z chunks, odd and
    even sweep counts; the state moves between the two buffer sets and every
    other entry point follows it."""
    import torch

    base = dict(kind="sc", J=1.0, K=0.1, e=(0.0, 0.6, 0.8))
    reps = [M.Replica(L=(24, 24, 24), T=1.0, replica_id=0, periodic_mask=7, **base),
            M.Replica(L=(40, 38, 34), T=1.5, replica_id=1, periodic_mask=7, **base),
            M.Replica(L=(48, 14, 12), T=0.7, replica_id=2, periodic_mask=7, **base),
            M.Replica(L=(32, 9, 7), T=1.2, replica_id=3, periodic_mask=1, **base),
            M.Replica(L=(64, 4, 6), T=1.3, replica_id=4, periodic_mask=6, **base),
            M.Replica(L=(12, 2, 2), T=0.9, replica_id=5, periodic_mask=7, **base)]
    ref = M.Simulation(reps, precision=prec, seed=13,
                       scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
    ref.set_tile(16, 16, 2, kernel=0)
    ref.sweep(3)
    ref.sweep(3, measure=True)
    obs_r = ref.observables()
    for tile in FUSED_TILES[prec]:
        one = M.Simulation(reps, precision=prec, seed=13,
                           scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
        with pytest.raises(M.MCError) as ei:  # no second buffer set yet
            one.set_tile(tile[1], tile[2], tile[3], kernel=tile[0])
        assert ei.value.status == -5
        one.enable_fused()
        one.set_tile(tile[1], tile[2], tile[3], kernel=tile[0])
        first = [p[0].data_ptr() for p in one.spins]
        one.sweep(3)
        # odd count: the state is in the second set now
        assert [one.state_spins(r)[0].data_ptr() for r in range(len(reps))] == \
            [p[0].data_ptr() for p in one.alt_spins]
        one.sweep(3, measure=True)
        assert [one.state_spins(r)[0].data_ptr() for r in range(len(reps))] == first
        o = one.observables()
        for r in range(len(reps)):
            for a, b in zip(natural(one, r), natural(ref, r)):
                assert np.array_equal(a, b), (r, tile)
            assert o[r]["n_accepted"] == obs_r[r]["n_accepted"], (r, tile)
            assert abs(o[r]["E"] - obs_r[r]["E"]) <= 1e-9 * abs(o[r]["E"]), (r, tile)
            n_sites = int(np.prod(reps[r].L))  # FP64 sums in another order
            assert np.max(np.abs(np.array(o[r]["M"]) - np.array(obs_r[r]["M"]))) <= 1e-9 * n_sites
        one.close()
    # leave the fused kernel with the state in the second set, continue on
    # another kernel, then come back: still the same chain
    a = M.Simulation(reps, precision=prec, seed=21,
                     scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
    b = M.Simulation(reps, precision=prec, seed=21,
                     scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
    b.set_tile(16, 16, 2, kernel=0)
    a.enable_fused()
    a.set_tile(256, 2, 4, kernel=9)
    a.sweep(1)
    a.set_tile(16, 16, 2, kernel=0)
    a.sweep(2)
    a.set_tile(256, 3, 2, kernel=9)
    a.sweep(2, measure=True)
    b.sweep(5, measure=True)
    oa, ob = a.observables(), b.observables()
    for r in range(len(reps)):
        for x, y in zip(natural(a, r), natural(b, r)):
            assert np.array_equal(x, y), r
        assert oa[r]["n_accepted"] == ob[r]["n_accepted"]
    # a schedule on the fused kernel (graph-replayed chunks) equals one on kernel 0
    ra = a.run_schedule([[rep.T for rep in reps]], n_equil=3, n_meas=4)
    rb = b.run_schedule([[rep.T for rep in reps]], n_equil=3, n_meas=4)
    assert np.allclose(ra, rb, rtol=1e-9, atol=1e-6)
    for r in range(len(reps)):
        for x, y in zip(natural(a, r), natural(b, r)):
            assert np.array_equal(x, y), r
    # no single-pass debug on the fused kernel; persistent sweeps refused
    with pytest.raises(M.MCError) as ei:
        a.debug_pass(0)
    assert ei.value.status == -2
    with pytest.raises(M.MCError):
        a.sweep(1, persistent=True)
    # odd packed rows are refused
    odd = M.Simulation([M.Replica(kind="sc", L=(18, 8, 8))], precision=prec)
    odd.enable_fused()
    with pytest.raises(M.MCError) as ei:
        odd.set_tile(256, 2, 3, kernel=9)
    assert ei.value.status == -2
    # shapes beyond the positions a lane can hold are refused
    with pytest.raises(M.MCError) as ei:
        a.set_tile(1024, 64, 2, kernel=9)
    assert ei.value.status == -2
    if prec == "f32":
        with pytest.raises(M.MCError) as ei:  # four positions per lane of 256
            a.set_tile(256, 60, 2, kernel=9)
        assert ei.value.status == -2
    if prec == "f64":
        with pytest.raises(M.MCError) as ei:
            a.set_tile(256, 20, 3, kernel=9)
        assert ei.value.status == -2


def test_autotune_with_fused_candidates(M):
    """With second buffer sets the autotuner times the fused sweep's tiles
    too; whatever it keeps, the chain (odd trial counts leave the state in
    either set) equals plain sweeps on kernel 0."""
    import torch

    reps = [M.Replica(kind="sc", L=(L, L, L), K=0.1, T=1.1 + 0.1 * r, replica_id=r)
            for r, L in enumerate((16, 24, 32))]
    a = M.Simulation(reps, precision="f32", seed=5,
                     scratch=torch.empty(32 << 20, dtype=torch.uint8, device="cuda"))
    a.enable_fused()
    tile = a.autotune(trial_sweeps=1, measure=True)
    a.sweep(3, measure=True)
    t = a.get_sweep()
    b = M.Simulation(reps, precision="f32", seed=5,
                     scratch=torch.empty(32 << 20, dtype=torch.uint8, device="cuda"))
    b.set_tile(16, 16, 2, kernel=0)
    b.sweep(t)
    for r in range(len(reps)):
        for x, y in zip(natural(a, r), natural(b, r)):
            assert np.array_equal(x, y), (r, tile)


def test_lds_allowance_shared_by_handles(M):
    """The dynamic-LDS allowance of a kernel is shared by every handle: a
    second handle with a smaller need must not take away what the first
    handle's launches use (fused sweep kernel and whole-sweep LDS kernel)."""
    import torch

    big = [M.Replica(kind="sc", L=(64, 24, 16), K=0.1, T=1.2)]
    small = [M.Replica(kind="sc", L=(16, 8, 8), K=0.1, T=1.2)]
    a = M.Simulation(big, precision="f64", seed=3,
                     scratch=torch.empty(8 << 20, dtype=torch.uint8, device="cuda"))
    a.enable_fused()
    a.set_tile(512, 10, 4, kernel=9)      # 6 * 12 * 32 * 8 = 18 KiB of LDS
    b = M.Simulation(small, precision="f64", seed=3)
    b.enable_fused()
    b.set_tile(256, 1, 4, kernel=9)       # less
    a.sweep(2)
    b.sweep(2)
    ref = M.Simulation(big, precision="f64", seed=3)
    ref.set_tile(16, 16, 2, kernel=0)
    ref.sweep(2)
    for x, y in zip(natural(a), natural(ref)):
        assert np.array_equal(x, y)
    # whole-sweep LDS kernel: a larger lattice first, then a smaller one
    c = M.Simulation([M.Replica(kind="sc", L=(16, 16, 16), K=0.1, T=1.2)], precision="f64", seed=4)
    d = M.Simulation([M.Replica(kind="sc", L=(8, 8, 8), K=0.1, T=1.2)], precision="f64", seed=4)
    assert c.get_tile()[0] == 3 and d.get_tile()[0] == 3
    c.sweep(3)
    d.sweep(3)
    c.sweep(1)
    e = M.Simulation([M.Replica(kind="sc", L=(16, 16, 16), K=0.1, T=1.2)], precision="f64", seed=4)
    e.set_tile(16, 16, 2, kernel=0)
    e.sweep(4)
    for x, y in zip(natural(c), natural(e)):
        assert np.array_equal(x, y)


def test_fused_state_in_second_set_follows_every_entry_point(M):
    """With the state in the second buffer set (after an odd number of fused
    sweeps), writing spins from natural order, the from-scratch measurement,
    checkpoint/resume of the sweep counter and a later kernel change act on
    that set: the chain equals one run on kernel 0 throughout."""
    import torch

    reps = [M.Replica(kind="sc", L=(24, 16, 12), K=0.1, T=1.3, replica_id=0),
            M.Replica(kind="sc", L=(16, 16, 16), K=0.1, T=0.9, replica_id=1)]
    a = M.Simulation(reps, precision="f32", seed=8,
                     scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
    b = M.Simulation(reps, precision="f32", seed=8,
                     scratch=torch.empty(16 << 20, dtype=torch.uint8, device="cuda"))
    a.enable_fused()
    a.set_tile(256, 2, 3, kernel=9)
    b.set_tile(16, 16, 2, kernel=0)
    a.sweep(3)
    b.sweep(3)
    assert a.state_spins(0)[0].data_ptr() == a.alt_spins[0][0].data_ptr()
    rng = np.random.default_rng(2)
    for r, rep in enumerate(reps):
        n = int(np.prod(rep.L))
        v = rng.normal(size=(3, n))
        v /= np.linalg.norm(v, axis=0)
        a.from_natural(r, [v[0].astype(np.float32), v[1].astype(np.float32), v[2].astype(np.float32)])
        b.from_natural(r, [v[0].astype(np.float32), v[1].astype(np.float32), v[2].astype(np.float32)])
    ma, mb = a.measure_state(), b.measure_state()
    for r in range(len(reps)):
        assert ma[r]["E"] == mb[r]["E"] and np.array_equal(ma[r]["M"], mb[r]["M"])
    t = a.get_sweep()
    a.set_sweep(t + 5)
    b.set_sweep(t + 5)
    a.sweep(1, measure=True)
    b.sweep(1, measure=True)
    a.set_tile(128, 2, 4, kernel=4)
    a.sweep(2)
    b.sweep(2)
    for r in range(len(reps)):
        for x, y in zip(natural(a, r), natural(b, r)):
            assert np.array_equal(x, y), r
