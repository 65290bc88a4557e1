"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics, never against the oracle itself.

Model: Eq. (1) of arXiv:2106.11286; update: the single-spin Metropolis rule of
its Monte Carlo paragraph; magnetisation: Eq. (2).  Each test names the
mistake class it guards against.
"""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as O
from oracle import stats as OS
from oracle import tempering as PT
from oracle import block_scheme as BS

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# Philox4x32-10 against an independent implementation (rocRAND's engine)
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference program")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "philox_rocrand_ref.cpp")])
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    """Guards: wrong multiplier, Weyl constant, word order, key schedule."""
    rng = np.random.default_rng(12345)
    cases = []
    for i in range(400):
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        c[1] &= 0x3FFFFFFF  # the reference maps c1 through a 64-bit offset*4
        k = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        cases.append([int(v) for v in c] + [int(v) for v in k])
    cases += [[0, 0, 0, 0, 0, 0], [5, 7, 11, 0, 0, 1], [123, 1, 999, 1, 0xFFFFFFFF, 0xFFFFFFFF]]
    inp = "\n".join(" ".join(str(v) for v in cs) for cs in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [list(map(int, line.split())) for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for cs, r in zip(cases, ref):
        assert O.philox(cs[:4], cs[4:]) == r, cs


def test_philox_word_statistics():
    """Guards: degenerate outputs (e.g. a round that drops a word)."""
    words = np.array([O.philox([i, 3, 17, 0], [99, 0]) for i in range(20000)], dtype=np.uint64)
    # bit balance per output word and bit: mean 1/2 with sd 1/(2 sqrt(n))
    n = words.shape[0]
    bits = ((words[:, :, None] >> np.arange(32, dtype=np.uint64)) & 1).astype(np.float64)
    frac = bits.mean(axis=0)
    assert np.all(np.abs(frac - 0.5) < 6 * 0.5 / np.sqrt(n))
    # chi-square of the top 4 bits of each word, 16 bins
    for w in range(4):
        counts = np.bincount((words[:, w] >> 28).astype(np.int64), minlength=16)
        chi2 = ((counts - n / 16) ** 2 / (n / 16)).sum()
        assert chi2 < 50.0  # 15 dof: P(chi2 > 50) ~ 1e-5
    # consecutive counters are uncorrelated
    u = (words[:, 0] >> 9).astype(np.float64) / 2**23
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 6 / np.sqrt(n)


def test_uniform_map_exact_in_binary32():
    """u = (k + 1/2) 2^-23 lies in (0, 1) and is exactly representable in FP32,
    so the FP32 and FP64 paths see the same P and the same z = 2u - 1."""
    for w in (0, 1, 511, 512, 2**31, 2**32 - 1, 0x12345678):
        u = O.uniform(w)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u
        z = 2.0 * u - 1.0
        assert float(np.float32(z)) == z
    assert O.uniform(0) == 2.0**-24
    assert O.uniform(2**32 - 1) == 1.0 - 2.0**-24


# --------------------------------------------------------------------------
# Sphere map (proposal / random start)
# --------------------------------------------------------------------------
def test_sphere_map_moments_and_norm():
    """Uniform on S^2: <S> = 0, <S_a S_b> = delta_ab/3, <z^4> = 1/5, |S| = 1.
    Guards: wrong z map (e.g. z = u), missing sqrt, 2 pi factor."""
    lat = O.Lattice(O.SC, 64)
    s = O.init(lat, O.Params(seed=3), O.INIT_RANDOM)
    S = np.stack(s, axis=1)
    n = S.shape[0]
    norms = np.sqrt((S * S).sum(axis=1))
    assert np.max(np.abs(norms - 1.0)) < 1e-12
    assert np.all(np.abs(S.mean(axis=0)) < 5 * np.sqrt(1 / 3 / n))
    C = S.T @ S / n
    assert np.all(np.abs(C - np.eye(3) / 3) < 5 * np.sqrt(4 / 45 / n) + 1e-12)
    z4 = np.mean(S[:, 2] ** 4)
    assert abs(z4 - 0.2) < 5 * np.sqrt((1 / 9 - 1 / 25) / n)
    # azimuth uniform: fraction in each quadrant 1/4
    q = (np.arctan2(S[:, 1], S[:, 0]) // (np.pi / 2)).astype(int) % 4
    frac = np.bincount(q, minlength=4) / n
    assert np.all(np.abs(frac - 0.25) < 5 * np.sqrt(0.25 * 0.75 / n))


# --------------------------------------------------------------------------
# Geometry and colouring
# --------------------------------------------------------------------------
def _positions_half(kind, Lx, Ly, Lz):
    basis = {O.SC: [(0, 0, 0)], O.BCC: [(0, 0, 0), (1, 1, 1)],
             O.FCC: [(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]}[kind]
    nb = len(basis)
    z, y, x, b = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), np.arange(nb),
                             indexing="ij")
    B = np.array(basis)
    pos = np.stack([2 * x + B[b, 0], 2 * y + B[b, 1], 2 * z + B[b, 2]], axis=-1)
    return pos.reshape(-1, 3)


@pytest.mark.parametrize("kind,L,z", [(O.SC, 4, 6), (O.BCC, 3, 8), (O.FCC, 3, 12)])
def test_neighbours_match_distance_matrix(kind, L, z):
    """Neighbour sets equal the nearest-neighbour shell of a minimum-image
    distance matrix.  Guards: wrong basis vector, wrong offset, wrong index."""
    lat = O.Lattice(kind, L)
    occ, col, nnb, nbr = lat.tables()
    pos = _positions_half(kind, L, L, L)
    assert pos.shape[0] == lat.n_box
    d = pos[:, None, :] - pos[None, :, :]
    box = 2 * L
    d = (d + box // 2) % box - box // 2
    d2 = (d * d).sum(-1)
    np.fill_diagonal(d2, 10**9)
    dmin = d2.min()
    assert dmin == {O.SC: 4, O.BCC: 3, O.FCC: 2}[kind]
    for s in range(lat.n_box):
        want = sorted(np.nonzero(d2[s] == dmin)[0].tolist())
        got = sorted(nbr[s, : nnb[s]].tolist())
        assert got == want
        assert nnb[s] == z
    assert lat.n_bonds == z * lat.n_box // 2
    assert not lat.same_colour_bonds


def test_colouring_and_bond_counts():
    """Periodic bond counts zN/2 (sc L=16: 12288; L=464 by formula), open sc
    3 L^2 (L-1), colour classes of equal size, and the 2-colouring failing
    for odd periodic sc."""
    lat = O.Lattice(O.SC, 16)
    occ, col, nnb, nbr = lat.tables()
    assert lat.n_bonds == 12288 and lat.n_colours == 2
    assert np.bincount(col).tolist() == [2048, 2048]
    # every bond joins different colours
    for s in range(lat.n_box):
        assert np.all(col[nbr[s, : nnb[s]]] != col[s])
    lat = O.Lattice(O.SC, 6, periodic_mask=0)
    assert lat.n_bonds == 3 * 36 * 5
    assert O.Lattice(O.SC, 5).same_colour_bonds
    assert not O.Lattice(O.SC, 5, periodic_mask=0).same_colour_bonds
    assert not O.Lattice(O.BCC, 5).same_colour_bonds
    assert not O.Lattice(O.FCC, 5).same_colour_bonds
    # mixed: periodic in x only
    lat = O.Lattice(O.SC, 4, 6, 3, periodic_mask=1)
    assert lat.n_bonds == 4 * 6 * 3 + (4 * 5 * 3) + (4 * 6 * 2)


def _fcc_sphere_counts_numpy(L, R):
    pos = _positions_half(O.FCC, L, L, L) - L  # half-units relative to the centre
    q = (pos * pos).sum(axis=1)
    occ = q <= 4 * R * R
    occ_set = set(map(tuple, pos[occ].tolist()))
    shells = [(a, b, 0) for a in (-1, 1) for b in (-1, 1)]
    shells += [(a, 0, b) for a in (-1, 1) for b in (-1, 1)]
    shells += [(0, a, b) for a in (-1, 1) for b in (-1, 1)]
    assert len(shells) == 12
    half_bonds = 0
    for p in pos[occ]:
        for d in shells:
            if (p[0] + d[0], p[1] + d[1], p[2] + d[2]) in occ_set:
                half_bonds += 1
    return int(occ.sum()), half_bonds // 2


def test_fcc_sphere_counts_small():
    """Open FCC nanoparticle: site and bond counts equal an independent count
    over positions (12 nearest-neighbour vectors in half-cell units)."""
    for L, R in ((12, 4.5), (10, 3.0), (9, 3.7)):
        lat = O.Lattice(O.FCC, L, periodic_mask=0, sphere_radius=R)
        n, nb = _fcc_sphere_counts_numpy(L, R)
        assert lat.n_occ == n and lat.n_bonds == nb
        assert not lat.same_colour_bonds


@pytest.mark.slow
def test_fcc_sphere_counts_c4():
    """The 128^3-cell FCC particle of radius 60 cells: 3,618,393 sites and
    21,518,640 bonds by a vectorised count independent of the oracle loops."""
    L, R = 128, 60
    lat = O.Lattice(O.FCC, L, periodic_mask=0, sphere_radius=R)
    g = np.arange(L)
    basis = [(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
    occ = np.zeros((4, L, L, L), dtype=bool)  # [b, z, y, x]
    for b, (bx, by, bz) in enumerate(basis):
        qx = (2 * g + bx - L)[None, None, :]
        qy = (2 * g + by - L)[None, :, None]
        qz = (2 * g + bz - L)[:, None, None]
        occ[b] = qx * qx + qy * qy + qz * qz <= 4 * R * R
    assert int(occ.sum()) == lat.n_occ == 3618393
    # bonds: pairs of occupied sites at half-offsets (+-1,+-1,0)-type between bases
    B = np.array(basis)
    half = 0
    for b1 in range(4):
        for b2 in range(4):
            if b1 == b2:
                continue
            dv = B[b2] - B[b1]
            # cell offsets along axes where the basis difference is nonzero
            axes_off = [(0,) if dv[a] == 0 else (0, -int(np.sign(dv[a]))) for a in range(3)]
            for ox in axes_off[0]:
                for oy in axes_off[1]:
                    for oz in axes_off[2]:
                        sh = np.roll(occ[b2], shift=(-oz, -oy, -ox), axis=(0, 1, 2))
                        # open faces: no wrap (the particle is far from the faces)
                        half += int((occ[b1] & sh).sum())
    assert half // 2 == lat.n_bonds == 21518640


# --------------------------------------------------------------------------
# Energy change and bookkeeping
# --------------------------------------------------------------------------
def test_delta_h_equals_energy_difference():
    """dH of one site equals E(after) - E(before) from the bond list.
    Guards: sign of exchange or anisotropy, missing factor 2 in bonds, axis."""
    rng = np.random.default_rng(1)
    for kind, L in ((O.SC, 6), (O.BCC, 3), (O.FCC, 3)):
        lat = O.Lattice(kind, L)
        p = O.Params(J=0.7, K=0.35, e=(1.0, -2.0, 0.5), T=1.0, seed=5)
        s = O.init(lat, p)
        occ, col, nnb, nbr = lat.tables()
        for trial in range(20):
            i = int(rng.integers(lat.n_box))
            S = np.array([s[0][i], s[1][i], s[2][i]])
            v = rng.normal(size=3)
            Sn = v / np.linalg.norm(v)
            h = p.J * np.array([s[a][nbr[i, : nnb[i]]].sum() for a in range(3)])
            dh = O.delta_h(h, S, Sn, p.K, p.e_unit)
            e0 = O.observables(lat, p, s)["E"]
            for a in range(3):
                s[a][i] = Sn[a]
            e1 = O.observables(lat, p, s)["E"]
            assert abs((e1 - e0) - dh) < 1e-11 * max(1.0, abs(e0))


@pytest.mark.parametrize("kind,L", [(O.SC, 8), (O.BCC, 4), (O.FCC, 4)])
def test_pass_energy_bookkeeping(kind, L):
    """Per colour pass: E_after - E_before = sum of accepted dH.  Holds only if
    no bond joins two sites of one colour and dH is right."""
    lat = O.Lattice(kind, L)
    p = O.Params(J=0.8, K=0.2, e=(0.3, 0.4, 0.5), T=1.3, seed=11)
    s = O.init(lat, p)
    for t in range(3):
        for c in range(lat.n_colours):
            e0 = O.observables(lat, p, s)["E"]
            n, dh, acc, mg = O.run_pass(lat, p, c, t, s, outputs=True)
            e1 = O.observables(lat, p, s)["E"]
            assert n == int(acc.sum()) and n > 0
            assert abs((e1 - e0) - dh[acc].sum()) < 1e-10 * lat.n_occ
            # decisions follow the rule: accept iff dH <= 0 or beta dH + ln P <= 0
            sel = ~np.isnan(dh)
            rule = (dh[sel] <= 0) | (mg[sel] <= 0)
            assert np.array_equal(rule, acc[sel])


# --------------------------------------------------------------------------
# Closed forms and limits
# --------------------------------------------------------------------------
def test_aligned_state_energy_and_fixed_point():
    """Aligned state: E = -J N_bonds - K N (periodic: -J z N/2 - K N, which is
    -12697.6 for sc L=16, K=0.1); m = e; at T = 0 it never changes."""
    lat = O.Lattice(O.SC, 16)
    p = O.Params(J=1.0, K=0.1, e=(0, 0, 1), T=0.0, seed=0)
    s = O.init(lat, p, O.INIT_ALIGNED)
    ob = O.observables(lat, p, s)
    assert ob["E"] == pytest.approx(-12697.6, abs=1e-9)
    assert np.allclose(ob["m"], [0, 0, 1], atol=1e-15)
    s0 = [a.copy() for a in s]
    rec = O.run(lat, p, 0, 5, s)
    assert np.all(rec[:, 5] == 0)
    for a, b in zip(s, s0):
        assert np.array_equal(a, b)
    # FCC particle with an oblique axis
    lat = O.Lattice(O.FCC, 10, periodic_mask=0, sphere_radius=3.7)
    p = O.Params(J=1.3, K=0.05, e=(1, 1, 1), T=0.0)
    s = O.init(lat, p, O.INIT_ALIGNED)
    ob = O.observables(lat, p, s)
    assert ob["E"] == pytest.approx(-1.3 * lat.n_bonds - 0.05 * lat.n_occ, rel=1e-13)
    assert np.allclose(ob["m"], np.ones(3) / np.sqrt(3), atol=1e-14)


def test_infinite_temperature_moments():
    """beta = 0: every move accepted, states i.i.d. uniform per sweep, so
    <m^2> = 1/N, <m^4> = (5N-2)/(3N^3), <E> = -K N/3,
    Var E = J^2 N_bonds/3 + 4 K^2 N/45."""
    lat = O.Lattice(O.SC, 6)
    J, K = 1.0, 0.6
    p = O.Params(J=J, K=K, e=(0, 1, 0), T=float("inf"), seed=21)
    s = O.init(lat, p)
    n_sw = 4000
    rec = O.run(lat, p, 0, n_sw, s)
    N = lat.n_occ
    assert np.all(rec[:, 5] == N)
    m2 = (rec[:, 0:3] ** 2).sum(1) / N**2
    E = rec[:, 3] + rec[:, 4]

    def check(x, mean, tol_sd=5.0):
        assert abs(x.mean() - mean) < tol_sd * x.std(ddof=1) / np.sqrt(len(x)), (x.mean(), mean)

    check(m2, 1.0 / N)
    check(m2 * m2, (5 * N - 2) / (3 * N**3))
    check(E, -K * N / 3)
    var_exact = J * J * lat.n_bonds / 3 + 4 * K * K * N / 45
    assert abs(E.var(ddof=1) / var_exact - 1) < 5 * np.sqrt(2 / n_sw) * 1.5


def test_zero_temperature_is_greedy():
    """T = 0: only dH <= 0 is accepted, so E never increases over a pass."""
    lat = O.Lattice(O.FCC, 4)
    p = O.Params(J=1.0, K=0.3, e=(0, 0, 1), T=0.0, seed=2)
    s = O.init(lat, p)
    e_prev = O.observables(lat, p, s)["E"]
    for t in range(20):
        for c in range(lat.n_colours):
            O.run_pass(lat, p, c, t, s)
            e = O.observables(lat, p, s)["E"]
            assert e <= e_prev + 1e-12
            e_prev = e


def test_low_temperature_equipartition():
    """Near T = 0 from the aligned start: two transverse modes per spin give
    dE/dT -> 1 per spin (classical equipartition) and m -> 1."""
    lat = O.Lattice(O.SC, 8)
    res = {}
    for T in (0.04, 0.08):
        p = O.Params(J=1.0, K=0.05, e=(0, 0, 1), T=T, seed=31)
        s = O.init(lat, p, O.INIT_ALIGNED)
        O.run(lat, p, 0, 1500, s, record=False)
        rec = O.run(lat, p, 1500, 4000, s)
        e = (rec[:, 3] + rec[:, 4]) / lat.n_occ
        m = np.sqrt((rec[:, 0:3] ** 2).sum(1)) / lat.n_occ
        res[T] = (e.mean(), OS.blocking_error(e), m.mean())
        assert m.mean() > 1 - 2 * T
    e0 = -(3.0 + 0.05)
    for T, (e, err, m) in res.items():
        assert abs((e - e0) / T - 1.0) < 0.1, (T, e, e0)
    slope = (res[0.08][0] - res[0.04][0]) / 0.04
    assert abs(slope - 1.0) < 0.15, slope


def _langevin(x):
    return 1.0 / np.tanh(x) - 1.0 / x


def test_two_spin_langevin_and_histogram():
    """One bond (2x1x1 open sc), K = 0: <S1.S2> = coth(bJ) - 1/(bJ) and the
    density of x = S1.S2 is proportional to exp(bJx) on [-1, 1]."""
    lat = O.Lattice(O.SC, 2, 1, 1, periodic_mask=0)
    assert lat.n_bonds == 1
    J, T = 1.0, 0.7
    p = O.Params(J=J, K=0.0, T=T, seed=41)
    s = O.init(lat, p)
    rec = O.run(lat, p, 0, 200000, s)
    x = -(rec[:, 3]) / J
    want = _langevin(J / T)
    err = OS.blocking_error(x)
    assert abs(x.mean() - want) < 4.5 * err, (x.mean(), want, err)
    edges = np.linspace(-1, 1, 11)
    counts, _ = np.histogram(x, bins=edges)
    b = J / T
    pexp = (np.exp(b * edges[1:]) - np.exp(b * edges[:-1])) / (np.exp(b) - np.exp(-b))
    frac = counts / counts.sum()
    # correlated samples: allow 6 sd of an effective sample of n/5
    sd = np.sqrt(pexp * (1 - pexp) / (len(x) / 5))
    assert np.all(np.abs(frac - pexp) < 6 * sd + 1e-4), (frac, pexp)


def _block_spread(fn, cols, n_blocks=40):
    """Standard error of a statistic of a series from the spread of its value
    over contiguous blocks (blocks much longer than the correlation time)."""
    idx = np.array_split(np.arange(len(cols[0])), n_blocks)
    v = np.array([fn(*[c[i] for c in cols]) for i in idx])
    return float(v.std(ddof=1) / np.sqrt(n_blocks))


def test_two_spin_specific_heat_and_susceptibility():
    """Fluctuation formulas of the series summary (specific heat
    C = (<E^2> - <E>^2)/(N T^2), susceptibility chi = N (<m^2> - <|m|>^2)/T,
    k_B = 1) on one bond (2x1x1 open sc, K = 0), where x = S1.S2 has density
    proportional to exp(bJx) on [-1, 1]: E = -J x, m^2 = (1 + x)/2 and
    |m| = sqrt((1 + x)/2), so every moment is a 1-D quadrature.  T = 0.5 and
    N = 2 make a dropped N or T^2, or <m>^2 in place of <|m|>^2, miss by far
    more than the error bar."""
    lat = O.Lattice(O.SC, 2, 1, 1, periodic_mask=0)
    J, T = 1.0, 0.5
    N = lat.n_occ
    assert N == 2 and lat.n_bonds == 1
    p = O.Params(J=J, K=0.0, T=T, seed=59)
    s = O.init(lat, p)
    rec = O.run(lat, p, 0, 400000, s)
    got = OS.series_summary(rec[:, 0:5], N, T)

    b = J / T
    def mom(f):
        num = integrate.quad(lambda x: f(x) * np.exp(b * (x - 1.0)), -1, 1, epsabs=1e-13)[0]
        den = integrate.quad(lambda x: np.exp(b * (x - 1.0)), -1, 1, epsabs=1e-13)[0]
        return num / den
    x1, x2 = mom(lambda x: x), mom(lambda x: x * x)
    am = mom(lambda x: np.sqrt((1.0 + x) / 2.0))
    C_want = J * J * (x2 - x1 * x1) / (N * T * T)
    chi_want = N * ((1.0 + x1) / 2.0 - am * am) / T
    assert x1 == pytest.approx(_langevin(b), abs=1e-12)  # the quadrature itself

    E = rec[:, 3] + rec[:, 4]
    m = rec[:, 0:3] / N
    m2 = (m * m).sum(1)
    C_err = _block_spread(lambda e: e.var() / (N * T * T), [E])
    chi_err = _block_spread(lambda q: N * (q.mean() - np.sqrt(q).mean() ** 2) / T, [m2])
    assert abs(got["C"] - C_want) < 5 * C_err, (got["C"], C_want, C_err)
    assert abs(got["chi"] - chi_want) < 5 * chi_err, (got["chi"], chi_want, chi_err)
    # the pin separates the plausible mistakes by many error bars
    assert C_want * (N - 1) > 20 * C_err          # N dropped: C x N
    assert C_want * (1 / T**2 - 1) > 20 * C_err  # T^2 dropped
    mvec2 = float((m.mean(0) ** 2).sum())        # <m>^2 for <|m|>^2
    assert N * (am * am - mvec2) / T > 20 * chi_err


def _two_spin_energy_quadrature(beta, J, K):
    def w(dphi, z2, z1, moment):
        c = z1 * z2 + np.sqrt(max(0.0, 1 - z1 * z1)) * np.sqrt(max(0.0, 1 - z2 * z2)) * np.cos(dphi)
        E = -J * c - K * z1 * z1 - K * z2 * z2
        return np.exp(-beta * E) * (E if moment else 1.0)

    kw = dict(epsabs=1e-11, epsrel=1e-11)
    Z = integrate.tplquad(w, -1, 1, -1, 1, 0, 2 * np.pi, args=(False,), **kw)[0]
    E1 = integrate.tplquad(w, -1, 1, -1, 1, 0, 2 * np.pi, args=(True,), **kw)[0]
    return E1 / Z


def test_two_spin_anisotropic_quadrature():
    """One bond with K != 0, e = z: <E> from 3-D quadrature over (z1, z2, dphi)
    of the Boltzmann weight of Eq. (1)."""
    J, K, beta = 1.0, 0.4, 1.3
    want = _two_spin_energy_quadrature(beta, J, K)
    assert want == pytest.approx(-0.70402, abs=5e-5)
    lat = O.Lattice(O.SC, 2, 1, 1, periodic_mask=0)
    p = O.Params(J=J, K=K, e=(0, 0, 1), T=1.0 / beta, seed=43)
    s = O.init(lat, p)
    rec = O.run(lat, p, 0, 200000, s)
    E = rec[:, 3] + rec[:, 4]
    err = OS.blocking_error(E)
    assert abs(E.mean() - want) < 4.5 * err, (E.mean(), want, err)


def test_single_spin_anisotropy():
    """One spin, no bonds: <(S.e)^2> = int x^2 e^{bKx^2} / int e^{bKx^2} on
    [-1, 1], for an oblique axis (guards the projection on e)."""
    lat = O.Lattice(O.SC, 1, 1, 1, periodic_mask=0)
    K, T = 1.5, 0.8
    e = (1.0, 2.0, -2.0)
    p = O.Params(J=1.0, K=K, e=e, T=T, seed=47)
    s = O.init(lat, p)
    rec = O.run(lat, p, 0, 200000, s)
    pe2 = -rec[:, 4] / K
    b = 1.0 / T
    num = integrate.quad(lambda x: x * x * np.exp(b * K * x * x), -1, 1)[0]
    den = integrate.quad(lambda x: np.exp(b * K * x * x), -1, 1)[0]
    err = OS.blocking_error(pe2)
    assert abs(pe2.mean() - num / den) < 4.5 * err


def test_open_chain_energy():
    """Open chain L x 1 x 1, K = 0: bonds are independent, so
    <E> = -(L-1) J (coth(bJ) - 1/(bJ))."""
    L, J, T = 8, 1.0, 0.9
    lat = O.Lattice(O.SC, L, 1, 1, periodic_mask=0)
    assert lat.n_bonds == L - 1
    p = O.Params(J=J, K=0.0, T=T, seed=53)
    s = O.init(lat, p)
    rec = O.run(lat, p, 0, 60000, s)
    E = rec[10000:, 3]
    want = -(L - 1) * J * _langevin(J / T)
    err = OS.blocking_error(E)
    assert abs(E.mean() - want) < 4.5 * err, (E.mean(), want, err)


def _binder(rec, n):
    m2 = (rec[:, 0:3] ** 2).sum(1) / n**2
    return 1.0 - np.mean(m2 * m2) / (3 * np.mean(m2) ** 2)


def _binder_err(rec, n, nblk=20):
    m2 = (rec[:, 0:3] ** 2).sum(1) / n**2
    blk = np.array_split(np.arange(len(m2)), nblk)
    jk = []
    for i in range(nblk):
        keep = np.concatenate([b for j, b in enumerate(blk) if j != i])
        x = m2[keep]
        jk.append(1.0 - np.mean(x * x) / (3 * np.mean(x) ** 2))
    jk = np.array(jk)
    return float(np.sqrt((nblk - 1) / nblk * ((jk - jk.mean()) ** 2).sum()))


def test_binder_jackknife_error_matches_ensemble_spread():
    """The jackknife error of U4 from one correlated series agrees with the
    spread of U4 over many independent series of the same process (AR(1)
    vector magnetisation, autocorrelation time ~10 records)."""
    from oracle import stats as OS

    rng = np.random.default_rng(11)
    n_series, n, phi = 300, 2048, 0.9
    m = np.zeros((n_series, n, 3))
    m[:, 0] = rng.normal(scale=0.05 / np.sqrt(1 - phi * phi), size=(n_series, 3)) + [0.3, 0, 0]
    for i in range(1, n):
        m[:, i] = 0.3 * np.array([1 - phi, 0, 0]) + phi * m[:, i - 1] + \
            rng.normal(scale=0.05, size=(n_series, 3))
    m2 = np.einsum("sij,sij->si", m, m)
    m4 = m2 * m2
    u4 = 1.0 - m4.mean(axis=1) / (3.0 * m2.mean(axis=1) ** 2)
    truth = u4.std(ddof=1)
    est = np.array([OS.binder_jackknife_error(m2[k], m4[k]) for k in range(n_series)])
    assert est.mean() == pytest.approx(truth, rel=0.15)
    # the deletion blocks matter: a per-record jackknife ignores the
    # correlation and underestimates by ~sqrt(2 tau)
    naive = OS.binder_jackknife_error(m2[0], m4[0], n_blocks=n)
    assert naive < 0.6 * est[0]


@pytest.mark.slow
def test_binder_crossing_brackets_paper_tc():
    """Simple cubic, K = 0.01 (the paper's setup): the Binder cumulants of
    L = 8 and L = 16 cross between T = 1.41 and T = 1.48, bracketing the
    printed T_C/J = 1.445 (tests/golden/paper_printed.json)."""
    gold = json.load(open(os.path.join(HERE, "golden", "paper_printed.json")))
    tc = gold["Tc_over_J"]
    K = gold["setup"]["K"]
    lo, hi = 1.41, 1.48
    assert lo < tc < hi
    diff = {}
    for T in (lo, hi):
        u = {}
        for L in (8, 16):
            lat = O.Lattice(O.SC, L)
            p = O.Params(J=1.0, K=K, T=T, seed=1000 + L)
            s = O.init(lat, p, O.INIT_ALIGNED)
            O.run(lat, p, 0, 1500, s, record=False)
            rec = O.run(lat, p, 1500, 16000, s)
            u[L] = (_binder(rec, lat.n_occ), _binder_err(rec, lat.n_occ))
        d = u[16][0] - u[8][0]
        diff[T] = (d, np.hypot(u[16][1], u[8][1]))
    # ordered side: larger L has larger U4; disordered side: smaller
    assert diff[lo][0] > 2 * diff[lo][1], diff
    assert diff[hi][0] < -2 * diff[hi][1], diff


# --------------------------------------------------------------------------
# Determinism: thread count and checkpoint/resume
# --------------------------------------------------------------------------
def test_thread_count_and_resume_are_bitwise():
    lat = O.Lattice(O.FCC, 5)
    p = O.Params(J=1.0, K=0.1, e=(1, 1, 1), T=1.1, seed=77, replica_id=3)
    nt = O.num_threads()
    try:
        O.set_num_threads(1)
        a = O.init(lat, p)
        ra = O.run(lat, p, 0, 12, a)
        O.set_num_threads(max(2, nt))
        b = O.init(lat, p)
        rb1 = O.run(lat, p, 0, 5, b)
        ck = [x.copy() for x in b]
        rb2 = O.run(lat, p, 5, 7, ck)
    finally:
        O.set_num_threads(nt)
    for x, y in zip(a, ck):
        assert np.array_equal(x, y)
    assert np.array_equal(ra[:5, 5], rb1[:, 5]) and np.array_equal(ra[5:, 5], rb2[:, 5])
    assert np.array_equal(ra[:, :5], np.concatenate([rb1, rb2])[:, :5])


def test_replica_id_and_seed_change_streams():
    lat = O.Lattice(O.SC, 4)
    a = O.init(lat, O.Params(seed=1, replica_id=0))
    b = O.init(lat, O.Params(seed=1, replica_id=1))
    c = O.init(lat, O.Params(seed=2, replica_id=0))
    assert not np.array_equal(a[0], b[0]) and not np.array_equal(a[0], c[0])


def test_single_site_attempt_equals_pass():
    """The table-free single-site evaluation reproduces the tabulated pass
    exactly (same neighbours, same stream) on every lattice kind."""
    for kind, L, pm, R in ((O.SC, (6, 4, 5), 3, 0.0), (O.BCC, (4, 4, 4), 7, 0.0),
                           (O.FCC, (6, 6, 6), 0, 2.4)):
        lat = O.Lattice(kind, *L, periodic_mask=pm, sphere_radius=R)
        geo = O.Geometry(kind, *L, periodic_mask=pm, sphere_radius=R)
        p = O.Params(J=0.9, K=0.3, e=(1, 0, 1), T=1.1, seed=9, replica_id=2)
        s = O.init(lat, p)
        occ, col, nnb, nbr = lat.tables()
        for c in range(lat.n_colours):
            before = [a.copy() for a in s]
            n, dh, acc, mg = O.run_pass(lat, p, c, 4, s, outputs=True)
            for site in np.nonzero(occ & (col == c))[0]:
                r = geo.site_attempt(p, 4, before, int(site))
                assert r["dH"] == dh[site] and r["accepted"] == acc[site]
                assert r["margin"] == mg[site]
                assert np.array_equal(r["S_after"], [s[0][site], s[1][site], s[2][site]])
            for site in np.nonzero(~occ)[0][:5]:
                assert geo.site_attempt(p, 4, before, int(site)) is None


# --------------------------------------------------------------------------
# Replica exchange between neighbouring temperatures (oracle/tempering.py)
# --------------------------------------------------------------------------
def test_exchange_pairs_alternate_and_equal_energies_swap():
    """Guards: wrong pair parity, the ladder order, an attempt with Delta = 0
    rejected."""
    rep_at, Ts = PT.ladder([1.6, 1.0, 1.4, 1.2, 1.8])
    assert rep_at == [1, 3, 2, 0, 4] and Ts == [1.0, 1.2, 1.4, 1.6, 1.8]
    out = PT.swap_round([3.0] * 5, Ts, rep_at, 0, 5, 1)
    assert out == [(0, True), (2, True)]
    assert rep_at == [3, 1, 0, 2, 4]
    out = PT.swap_round([3.0] * 5, Ts, rep_at, 1, 6, 1)
    assert out == [(1, True), (3, True)]
    assert rep_at == [3, 0, 1, 4, 2]


def test_exchange_acceptance_is_exp_delta():
    """Guards: an inverted comparison, the sign of Delta, beta taken as T,
    a biased uniform.  Slot 0 at T = 1, slot 1 at T = 2; the replica at slot 0
    has E = -2, the other -1: Delta = (1 - 1/2)(-2 + 1) = -1/2, so the
    exchange is accepted with probability exp(-1/2); the reverse energies
    always exchange."""
    n = 20000
    acc = sum(PT.swap_round([-2.0, -1.0], [1.0, 2.0], [0, 1], 0, t, 99)[0][1] for t in range(n))
    p = np.exp(-0.5)
    assert abs(acc / n - p) <= 4.0 * np.sqrt(p * (1 - p) / n), acc / n
    assert all(PT.swap_round([-1.0, -2.0], [1.0, 2.0], [0, 1], 0, t, 99)[0][1] for t in range(200))


def test_exchange_keeps_each_slot_boltzmann():
    """Guards: any error in the exchange rule that breaks detailed balance.
    Three two-level systems (E in {0, 1}) at T = 0.5, 1, 4, each redrawn from
    its slot's Boltzmann distribution (exact heat bath, numpy) before every
    exchange round: after the exchanges the replica at slot k must still have
    P(E = 1) = 1 / (1 + exp(1/T_k)).  A wrong sign of Delta moves the excited
    systems to the cold slots by ~0.1 in probability, 30 standard errors."""
    rng = np.random.default_rng(5)
    rep_at, Ts = PT.ladder([4.0, 0.5, 1.0])
    E = [0.0, 0.0, 0.0]
    n = 30000
    ones = np.zeros(3)
    for r in range(n):
        for k in range(3):
            E[rep_at[k]] = 1.0 if rng.random() < 1.0 / (1.0 + np.exp(1.0 / Ts[k])) else 0.0
        PT.swap_round(E, Ts, rep_at, r, r, 3)
        for k in range(3):
            ones[k] += E[rep_at[k]]
    for k in range(3):
        p = 1.0 / (1.0 + np.exp(1.0 / Ts[k]))
        assert abs(ones[k] / n - p) <= 5.0 * np.sqrt(p * (1 - p) / n), (k, ones[k] / n, p)


# --------------------------------------------------------------------------
# The paper's block scheme, synchronous form (oracle/block_scheme.py)
# --------------------------------------------------------------------------
def test_block_choice_is_uniform_within_each_block():
    """Guards: a site outside its block, a biased offset, a wrong size of the
    last (partial) block.  N = 100, n = 8: 12 full blocks and one of 4."""
    counts = np.zeros(100)
    for step in range(400):
        for s, _ in BS.chosen_sites(100, 8, 2, step, 9):
            counts[s] += 1
    for k in range(13):
        c = counts[k * 8:min(100, k * 8 + 8)]
        assert c.sum() == 400
        e = 400 / len(c)
        assert np.sum((c - e) ** 2 / e) < 30.0, (k, c)  # chi-square, <= 7 dof


def test_block_step_is_synchronous_and_counts_conflicts():
    """Guards: moves applied in place (an attempt seeing a neighbour's new
    value), a wrong conflict count.  Every attempt of a step is recomputed by
    hand from the state before the step; conflicts are recounted from
    coordinates."""
    lat = O.Lattice(O.SC, 6, 6, 4)
    p = O.Params(J=1.0, K=0.2, e=(0.0, 0.6, 0.8), T=1.1, seed=4)
    spins = O.init(lat, p)
    before = [a.copy() for a in spins]
    att, acc, conf = BS.block_step(lat, p, spins, 4, 17)
    chosen = BS.chosen_sites(lat.n_box, 4, 0, 17, 4)
    picked = {s for s, _ in chosen}

    def coords(s):
        return s % 6, (s // 6) % 6, s // 36

    def nbrs(s):
        x, y, z = coords(s)
        return [((x + dx) % 6) + 6 * ((y + dy) % 6) + 36 * ((z + dz) % 4)
                for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))]

    n_conf = n_acc = 0
    for s, w in chosen:
        nb = nbrs(s)
        n_conf += any(q in picked for q in nb)
        h = np.array([sum(before[a][q] for q in nb) for a in range(3)])
        S = np.array([before[a][s] for a in range(3)])
        Sn = O.sphere_point(O.uniform(w[0]), O.uniform(w[1]))
        dH = O.delta_h(h, S, Sn, p.K, p.e_unit)
        ok = dH <= 0 or O.uniform(w[2]) <= np.exp(-dH / p.T)
        n_acc += ok
        want = Sn / np.linalg.norm(Sn) if ok else S
        assert np.allclose([spins[a][s] for a in range(3)], want, atol=1e-15), s
    assert att == 36 and acc == n_acc and conf == n_conf and conf > 0
    untouched = np.ones(lat.n_box, bool)
    untouched[list(picked)] = False
    for a in range(3):
        assert np.array_equal(spins[a][untouched], before[a][untouched])


def test_one_block_is_exact_metropolis():
    """Guards: a wrong attempt (field, proposal or acceptance) in the block
    step.  With one block (n = N) a step is one single-site Metropolis
    attempt at a random site, no concurrency: its equilibrium <e> and <|m|>
    on sc 4^3 must agree with the colour sweep's (the C oracle) within the
    blocked errors."""
    lat = O.Lattice(O.SC, 4, 4, 4)
    T = 1.6
    p = O.Params(J=1.0, K=0.1, T=T, seed=21)
    spins = O.init(lat, p, O.INIT_ALIGNED)
    tables = lat.tables()
    n_mcs, N = 1500, lat.n_box
    e_b, m_b = [], []
    for t in range(n_mcs):
        for j in range(N):
            _, _, conf = BS.block_step(lat, p, spins, N, t * N + j, tables)
            assert conf == 0
        if t >= 300:
            o = O.observables(lat, p, spins)
            e_b.append(o["E"] / N)
            m_b.append(np.linalg.norm(o["m"]))
    q = O.Params(J=1.0, K=0.1, T=T, seed=22)
    s2 = O.init(lat, q, O.INIT_ALIGNED)
    O.run(lat, q, 0, 2000, s2, record=False)
    rec = O.run(lat, q, 2000, 40000, s2)
    e_c = (rec[:, 3] + rec[:, 4]) / N
    m_c = np.linalg.norm(rec[:, 0:3], axis=1) / N
    for a, b in ((np.array(e_b), e_c), (np.array(m_b), m_c)):
        ea, eb = OS.blocking_error(a), OS.blocking_error(b)
        z = (a.mean() - b.mean()) / np.hypot(ea, eb)
        assert abs(z) <= 4.0, (a.mean(), b.mean(), z)
