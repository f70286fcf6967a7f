"""Pins of the XY oracle (Wolff's embedded clusters in the SW multi-cluster
form) against things other than itself (no GPU needed).

* its random streams (direction, bond uniforms, reflection bits, initial
  angles) against rocRAND's Philox engine, and whole sweeps rebuilt from those
  draws: bonds only between spins on the same side of the line perpendicular
  to the direction, labels = scipy's connected components, each cluster either
  untouched or reflected (the projection on the direction changes sign, the
  perpendicular one does not);
* the chain against exact statistical mechanics: the continuous model on the
  2 x 2 torus (a four-spin ring, Bessel sums), the Ising model (directions on
  multiples of pi/2, cold start) and the 4-state clock model (multiples of
  pi/4) against Kaufman's torus result, and the 16-state clock model on 3 x 3
  against a row transfer matrix;
* the fixed-point observables and the FP64 derived values against closed
  forms (uniform and twisted configurations, rotation invariance).
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import exact_xy as ex
import oracle

TURN = 2.0 ** 32


def _rad(a):
    """Angles of uint32 turn fractions, in radians, in FP64 (numpy)."""
    return np.asarray(a, dtype=np.float64) * (2 * np.pi / TURN)


def _binned_mean(x, nbins=50):
    x = np.asarray(x, dtype=np.float64)
    n = len(x) // nbins * nbins
    b = x[:n].reshape(nbins, -1).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / math.sqrt(nbins))


def _cc_min_labels(bx, by):
    L = bx.shape[0]
    idx = np.arange(L * L).reshape(L, L)
    rows = np.concatenate([idx[bx.astype(bool)], idx[by.astype(bool)]])
    cols = np.concatenate([np.roll(idx, -1, axis=1)[bx.astype(bool)], np.roll(idx, -1, axis=0)[by.astype(bool)]])
    g = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(L * L, L * L))
    _, comp = connected_components(g, directed=False)
    mins = np.full(comp.max() + 1, L * L, dtype=np.int64)
    np.minimum.at(mins, comp, np.arange(L * L))
    return mins[comp].reshape(L, L)


# ------------------------------------------------------------ random streams

def test_xy_streams_match_rocrand(rocrand_philox):
    rng = np.random.Generator(np.random.PCG64(31))
    seeds = [1, 2**32 + 7, int(rng.integers(0, 2**63))]
    for seed in seeds:
        k0, k1 = seed & 0xFFFFFFFF, seed >> 32
        sweeps = [0, 1, 77, 2**32 - 1] + rng.integers(0, 2**32, 20).tolist()
        w = rocrand_philox([[0, 0, t, 3, k0, k1] for t in sweeps])
        for bits in (1, 2, 3, 5, 17, 31, 32):
            keep = 0xFFFFFFFF if bits == 32 else (0xFFFFFFFF ^ (0xFFFFFFFF >> bits))
            assert [oracle.xy_direction(seed, t, bits) for t in sweeps] == [int(v) & keep for v in w[:, 0]]
        sites = [0, 1, 2**32 - 1, 2**32, 2**40 + 3] + rng.integers(0, 2**32, 40).tolist()
        w = rocrand_philox([[i & 0xFFFFFFFF, i >> 32, 0, 6, k0, k1] for i in sites])
        assert [oracle.xy_initangle(seed, i) for i in sites] == [int(v) for v in w[:, 0]]
        t = int(rng.integers(0, 2**32))
        w = rocrand_philox([[i & 0xFFFFFFFF, i >> 32, t, 4, k0, k1] for i in sites])
        for d in (0, 1):
            hi, lo = w[:, 2 * d].astype(object), w[:, 2 * d + 1].astype(object)
            want = [float(((int(h) << 21) | (int(l) >> 11))) / 2.0**53 for h, l in zip(hi, lo)]
            assert [oracle.xy_uniform(seed, t, i, d) for i in sites] == want
        w = rocrand_philox([[i & 0xFFFFFFFF, i >> 32, t, 5, k0, k1] for i in sites])
        assert [oracle.xy_flipbit(seed, t, i) for i in sites] == [int(v) >> 31 for v in w[:, 0]]


def test_xy_random_start_uses_init_draws(rocrand_philox):
    L, seed = 9, 2**33 + 1
    w = rocrand_philox([[i, 0, 0, 6, seed & 0xFFFFFFFF, seed >> 32] for i in range(L * L)])
    assert np.array_equal(oracle.xy_init_angles(L, seed, True).reshape(-1), w[:, 0].astype(np.uint32))
    assert not oracle.xy_init_angles(L, seed, False).any()


def test_xy_reflection():
    rng = np.random.Generator(np.random.PCG64(5))
    a = rng.integers(0, 2**32, 2000, dtype=np.uint64)
    phi = rng.integers(0, 2**32, 2000, dtype=np.uint64)
    r = np.array([oracle.xy_reflect(int(x), int(p)) for x, p in zip(a, phi)], dtype=np.uint64)
    rr = np.array([oracle.xy_reflect(int(x), int(p)) for x, p in zip(r, phi)], dtype=np.uint64)
    assert np.array_equal(rr, a)                                   # an involution
    t, tr, f = _rad(a), _rad(r), _rad(phi)
    # across the line perpendicular to r = (cos phi, sin phi): the component
    # along r changes sign, the perpendicular one is kept
    assert np.allclose(np.cos(tr - f), -np.cos(t - f), atol=1e-9)
    assert np.allclose(np.sin(tr - f), np.sin(t - f), atol=1e-9)
    # the projection the oracle uses is the cosine of the angle to phi
    c = np.array([oracle.xy_projection(int(x), int(p)) for x, p in zip(a, phi)])
    assert np.allclose(c, np.cos(t - f), atol=1e-12)


def test_xy_sincos_quarter_turns_exact_and_accurate():
    for k, want in enumerate([(0.0, 1.0), (1.0, 0.0), (0.0, -1.0), (-1.0, 0.0)]):
        assert oracle.xy_sincos(k << 30) == want
    rng = np.random.Generator(np.random.PCG64(9))
    special = [1, 2**29 - 1, 2**29, 2**29 + 1, 2**30 - 1, 2**30 + 1, 0xDFFFFFFF, 0xE0000000, 0xFFFFFFFF]
    for a in special + rng.integers(0, 2**32, 3000).tolist():
        s, c = oracle.xy_sincos(int(a))
        with mpmath.workdps(40):
            t = 2 * mpmath.pi * mpmath.mpf(int(a)) / 2**32
            S, C = mpmath.sin(t), mpmath.cos(t)
        # each within one unit in the last place of 1 (|sin|, |cos| <= 1)
        assert abs(s - float(S)) <= 2**-52 and abs(c - float(C)) <= 2**-52, a


def test_xy_perpendicular_spins_never_bond():
    """A spin exactly a quarter turn from the direction has zero projection:
    even at K = inf it joins no cluster (and its reflection is itself)."""
    L = 8
    a = np.zeros((L, L), np.uint32)
    a[:, ::2] = 2**30
    lat = oracle.XYOracleLattice(L, float("inf"), 21, dir_bits=2, angles=a)
    for _ in range(8):
        before = lat.a.copy()
        out = lat.sweep()
        c = np.array([oracle.xy_projection(int(v), out["phi"]) for v in before.reshape(-1)]).reshape(L, L)
        for key, axis in (("bx", 1), ("by", 0)):
            cj = np.roll(c, -1, axis=axis)
            assert not (out[key].astype(bool) & ((c == 0) | (cj == 0))).any()
            assert np.array_equal(out[key].astype(bool), c * cj > 0)      # K = inf: every other pair
        assert np.array_equal(lat.a[c == 0], before[c == 0])


# ------------------------------------------------------------- whole sweeps

@pytest.mark.parametrize("L,K,seed,bits", [(13, 0.8, 3, 32), (16, 1.5, 2**32 + 9, 32), (8, 1.0, 4, 5)])
def test_xy_sweep_follows_rocrand_draws(rocrand_philox, L, K, seed, bits):
    lat = oracle.XYOracleLattice(L, K, seed, random_start=True, dir_bits=bits)
    k0, k1 = seed & 0xFFFFFFFF, seed >> 32
    for t in range(4):
        a = lat.a.copy()
        out = lat.sweep()
        phi = int(rocrand_philox([[0, 0, t, 3, k0, k1]])[0, 0])
        phi &= 0xFFFFFFFF if bits == 32 else (0xFFFFFFFF ^ (0xFFFFFFFF >> bits))
        assert out["phi"] == phi
        c = np.cos(_rad(a) - _rad(phi))
        w = rocrand_philox([[i, 0, t, 4, k0, k1] for i in range(L * L)])
        u = [(((w[:, 2 * d].astype(object) << 21) | (w[:, 2 * d + 1].astype(object) >> 11)).astype(np.float64)
              / 2.0**53).reshape(L, L) for d in (0, 1)]
        for d, (key, axis) in enumerate((("bx", 1), ("by", 0))):
            cj = np.roll(c, -1, axis=axis)
            want = (c * cj > 0) & (u[d] < -np.expm1(-(2 * K * c) * cj))
            assert np.array_equal(out[key].astype(bool), want), f"{key}, sweep {t}"
            assert not (out[key].astype(bool) & (c * cj <= 0)).any()
        roots = _cc_min_labels(out["bx"], out["by"])
        assert np.array_equal(out["labels"], roots)
        bit = rocrand_philox([[int(r), 0, t, 5, k0, k1] for r in range(L * L)])[:, 0] >> 31
        flip = bit[roots.reshape(-1)].reshape(L, L).astype(bool)
        assert np.array_equal(lat.a[~flip], a[~flip])
        tn = _rad(lat.a)
        assert np.allclose(np.cos(tn - _rad(phi))[flip], -c[flip], atol=1e-9)
        assert np.allclose(np.sin(tn - _rad(phi))[flip], np.sin(_rad(a) - _rad(phi))[flip], atol=1e-9)
        assert out["obs"][0] == out["bx"].sum() + out["by"].sum()


def test_xy_zero_coupling_singletons():
    lat = oracle.XYOracleLattice(12, 0.0, 6)
    for _ in range(3):
        out = lat.sweep()
        assert not out["bx"].any() and not out["by"].any()
        assert np.array_equal(out["labels"].reshape(-1), np.arange(144))


def test_xy_infinite_coupling_cold_start_one_cluster():
    lat = oracle.XYOracleLattice(10, float("inf"), 8, random_start=False)
    for _ in range(6):
        out = lat.sweep()
        assert out["bx"].all() and out["by"].all()
        assert len(np.unique(lat.a)) == 1
        assert out["obs"][0] == 200


# --------------------------------------------------- exact statistical pins

@pytest.mark.parametrize("K", [0.5, 1.0])
def test_xy_L2_continuous_against_bessel_ring(K):
    lat = oracle.XYOracleLattice(2, K, 11)
    lat.run(1000)
    obs = lat.run(300_000).astype(np.float64) * oracle.XY_UNIT
    e, se_e = _binned_mean(obs[:, 1] + obs[:, 2])
    m2, se_m = _binned_mean(obs[:, 5] ** 2 + obs[:, 6] ** 2)
    assert abs(e - ex.xy_L2_bond_cos_sum(K)) < 4.5 * se_e
    assert abs(m2 - ex.xy_L2_m2(K)) < 4.5 * se_m
    assert se_e < 0.005 * 8 and se_m < 0.005 * 16              # the test has teeth
    # on the 2 x 2 torus the two +x bonds of a pair give sin d + sin(-d)
    assert not obs[:, 3].any() and not obs[:, 4].any()


@pytest.mark.parametrize("L,K", [(16, 0.44), (8, 0.3)])
def test_xy_ising_directions_against_kaufman(L, K):
    """Directions on multiples of pi/2 and a cold start keep the angles on
    {0, pi}: the chain is SW for the Ising model at coupling K."""
    lat = oracle.XYOracleLattice(L, K, 12, random_start=False, dir_bits=2)
    lat.run(400)
    obs = lat.run(40_000)
    a = lat.a
    assert set(np.unique(a).tolist()) <= {0, 2**31}
    m, se = _binned_mean((obs[:, 1] + obs[:, 2]).astype(np.float64) * oracle.XY_UNIT)
    assert abs(m - ex.ising_mean_bond_sum(L, K)) < 4.5 * se
    assert se < 0.01 * L * L


@pytest.mark.parametrize("L,K", [(8, 1.0), (6, 0.7)])
def test_xy_four_state_clock_against_kaufman(L, K):
    lat = oracle.XYOracleLattice(L, K, 13, random_start=False, dir_bits=3)
    lat.run(400)
    obs = lat.run(40_000)
    assert set(np.unique(lat.a).tolist()) <= {0, 2**30, 2**31, 3 * 2**30}
    m, se = _binned_mean((obs[:, 1] + obs[:, 2]).astype(np.float64) * oracle.XY_UNIT)
    assert abs(m - ex.ising_mean_bond_sum(L, K / 2)) < 4.5 * se
    assert se < 0.01 * L * L


def test_xy_sixteen_state_clock_against_transfer_matrix():
    L, K = 3, 1.0
    lat = oracle.XYOracleLattice(L, K, 14, random_start=False, dir_bits=5)
    lat.run(1000)
    obs = lat.run(200_000)
    assert not (lat.a % 2**28).any()
    m, se = _binned_mean((obs[:, 1] + obs[:, 2]).astype(np.float64) * oracle.XY_UNIT)
    exact = ex.clock_mean_cos_sum(L, 16, K)
    assert abs(m - exact) < 4.5 * se
    assert se < 0.005 * exact


def test_exact_routes_agree():
    # the exact results cross-checked before they pin the oracle
    for K in (0.3, 1.2):
        for r in (1, 2):
            assert abs(ex.ring_correlation(4, 2 * K, r) - ex.clock_ring_correlation(4, 2 * K, r, 64)) < 1e-12
        assert abs(ex.clock_mean_cos_sum(3, 4, K) - ex.ising_mean_bond_sum(3, K / 2)) < 1e-9
        assert abs(ex.clock_mean_cos_sum(3, 2, K) - ex.ising_mean_bond_sum(3, K)) < 1e-9
    # small coupling: <cos> per bond -> I1(k)/I0(k) ~ k/2 on any lattice
    assert abs(ex.ring_correlation(4, 0.02, 1) - 0.01) < 1e-5


# ------------------------------------------------------------- observables

def test_xy_observables_closed_forms():
    L = 16
    N = L * L
    u = oracle.xy_observe(np.zeros((L, L), np.uint32))
    assert u.tolist() == [0, N * 2**30, N * 2**30, 0, 0, N * 2**30, 0]
    q = oracle.xy_observe(np.full((L, L), 2**30, np.uint32))          # all along +y
    assert q.tolist() == [0, N * 2**30, N * 2**30, 0, 0, 0, N * 2**30]
    # a twist by one turn along x: every +x difference is -1/16 turn
    tw = (np.arange(L, dtype=np.uint64)[None, :] * 2**28 * np.ones((L, 1), np.uint64)).astype(np.uint32)
    o = oracle.xy_observe(tw)
    assert o[1] == N * round(math.cos(2 * math.pi / 16) * 2**30)
    assert o[3] == -N * round(math.sin(2 * math.pi / 16) * 2**30)
    assert o[2] == N * 2**30 and o[4] == 0
    assert abs(o[5]) <= N and abs(o[6]) <= N                            # sum of a full turn of unit vectors
    # rotating every spin by the same angle leaves the pair sums bit-identical
    rng = np.random.Generator(np.random.PCG64(2))
    a = rng.integers(0, 2**32, (L, L), dtype=np.uint64).astype(np.uint32)
    b = (a.astype(np.uint64) + 123456789).astype(np.uint32)
    oa, ob = oracle.xy_observe(a), oracle.xy_observe(b)
    assert np.array_equal(oa[1:5], ob[1:5])
    # against plain FP64 sums: each term is rounded to 2^-30
    t = _rad(a)
    assert abs(oa[1] * oracle.XY_UNIT - np.cos(t - np.roll(t, -1, 1)).sum()) < N * 2**-30
    assert abs(oa[4] * oracle.XY_UNIT - np.sin(t - np.roll(t, -1, 0)).sum()) < N * 2**-30
    assert abs(oa[6] * oracle.XY_UNIT - np.sin(t).sum()) < N * 2**-30


def test_xy_derived_closed_forms():
    L, K = 16, 0.9
    N = L * L
    tw = (np.arange(L, dtype=np.uint64)[None, :] * 2**28 * np.ones((L, 1), np.uint64)).astype(np.uint32)
    d = oracle.xy_derived(tw, K)
    c, s = math.cos(2 * math.pi / 16), math.sin(2 * math.pi / 16)
    assert d["e"] == pytest.approx(-(c + 1.0), rel=1e-12)
    assert d["m2"] == pytest.approx(0.0, abs=1e-20)
    assert d["Y"] == pytest.approx((N * (c + 1) / 2 - K * (N * s) ** 2 / 2) / N, rel=1e-12)
    u = oracle.xy_derived(np.full((L, L), 5 * 2**27, np.uint32), K)
    assert u["e"] == pytest.approx(-2.0, rel=1e-15) and u["m2"] == pytest.approx(1.0, rel=1e-15)
    assert u["Y"] == pytest.approx(1.0, rel=1e-15)
