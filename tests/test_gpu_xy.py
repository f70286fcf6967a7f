"""GPU parity of the XY sweep (Wolff's embedded clusters) against the XY oracle.

Angles, bond planes, cluster labels and the active-bond count must be bit
identical after every sweep.  The six fixed-point sums (Ex, Ey, Ix, Iy, Mx, My)
are sums of terms rounded to 2^-30; the two sides' FP64 sin and cos (the C
library's, the kernel's own polynomials) may differ in the last place, and a
term then changes by one unit when its value straddles a rounding boundary,
which happens with probability about 2^-21 per term.  The tests allow
8 + N / 2^16 units per sum (several times the expected count).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1208_2080_amd import binding

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

K_KT = 1.1199   # near the Kosterlitz-Thouless coupling of the square-lattice XY model


def say(msg):
    print(msg, flush=True)


def sum_tol(N: int) -> int:
    return 8 + (N >> 16)


def assert_rows_match(got, ref, N, what=""):
    got = np.atleast_2d(got)
    ref = np.atleast_2d(ref)
    assert np.array_equal(got[:, 0], ref[:, 0]), f"active bonds differ {what}: {got[:, 0]} vs {ref[:, 0]}"
    diff = np.abs(got[:, 1:] - ref[:, 1:]).max()
    assert diff <= sum_tol(N), f"observable sums differ by {diff} units {what}"


def compare_xy(L, K, seed, random_start=True, sweeps=8, tile_rows=0, dir_bits=32, labels_every=1, angles=None,
               start=0):
    say(f"case L={L} K={K} seed={seed} random={random_start} sweeps={sweeps} ty={tile_rows} bits={dir_bits}")
    lat = binding.XYLattice(L, K, seed=seed, random_start=random_start, obs_capacity=max(2, sweeps),
                            tile_rows=tile_rows, dir_bits=dir_bits)
    ref = oracle.XYOracleLattice(L, K, seed, random_start=random_start, dir_bits=dir_bits, angles=angles, sweep=start)
    if angles is not None:
        lat.load_angles(angles, start)
    assert np.array_equal(lat.angles(), ref.a), "initial angles"
    N = L * L
    for k in range(sweeps):
        t = start + k
        lat.sweep(1)
        out = ref.sweep()
        got = lat.angles()
        if not np.array_equal(got, ref.a):
            bad = np.argwhere(got != ref.a)
            raise AssertionError(f"angles differ after sweep {t} at {len(bad)} sites, first {bad[:5].tolist()}")
        if labels_every and k % labels_every == 0:
            bx, by = lat.bonds()
            assert np.array_equal(bx, oracle.pack_bonds(out["bx"])), f"+x bonds differ in sweep {t}"
            assert np.array_equal(by, oracle.pack_bonds(out["by"])), f"+y bonds differ in sweep {t}"
            assert np.array_equal(lat.labels(), out["labels"]), f"labels differ in sweep {t}"
        row = lat.measure(t, 1)[0]
        assert_rows_match(row, out["obs"], N, f"after sweep {t}")
        d_gpu = binding.xy_derived(row, L, K) if math.isfinite(K) else None
        if d_gpu is not None:
            d_ref = oracle.xy_derived(ref.a, K)
            tol = (sum_tol(N) + 2 * N * 2.0**-31 / binding.XY_UNIT) * binding.XY_UNIT
            assert abs(d_gpu["e"] - d_ref["e"]) <= 2 * tol / N * (1 + 1e-9)
            assert abs(d_gpu["m2"] - d_ref["m2"]) <= (4 * N * tol + 2 * tol * tol) / N**2 * (1 + 1e-6)
            assert abs(d_gpu["Y"] - d_ref["Y"]) <= (tol + K * (4 * N * tol + 2 * tol * tol)) / N * (1 + 1e-6)
    lat.close()
    return ref


def test_small_lattice_near_kt():
    compare_xy(64, K_KT, seed=1, sweeps=200, labels_every=10)


@pytest.mark.parametrize("L", [2, 3, 5, 17, 63, 65, 129, 200, 257])
def test_ragged_sizes(L):
    compare_xy(L, 1.0, seed=L, sweeps=6)


@pytest.mark.parametrize("ty", [32, 64, 128])
@pytest.mark.parametrize("L", [100, 256])
def test_tile_heights(ty, L):
    compare_xy(L, K_KT, seed=7, sweeps=5, tile_rows=ty)


@pytest.mark.parametrize("bits", [1, 2, 3, 5])
def test_direction_grids(bits):
    # cold start: the angles stay on the grid of 2^(bits-1) states ({0, pi} for bits <= 2)
    ref = compare_xy(96, 0.9, seed=30 + bits, random_start=False, sweeps=10, dir_bits=bits)
    assert not (ref.a.astype(np.uint64) % (2**32 >> max(bits - 1, 1))).any()
    compare_xy(70, 0.9, seed=40 + bits, random_start=True, sweeps=4, dir_bits=bits)


def test_zero_coupling_singletons():
    ref = compare_xy(80, 0.0, seed=3, sweeps=4)
    assert ref.t == 4


def test_infinite_coupling_cold_start_one_cluster():
    ref = compare_xy(150, float("inf"), seed=9, random_start=False, sweeps=4)
    assert len(np.unique(ref.a)) == 1


def test_infinite_coupling_perpendicular_spins():
    # stripes a quarter turn apart, directions on multiples of pi/2: spins at
    # right angles to the direction join no cluster even at K = inf
    L = 128
    a = np.zeros((L, L), np.uint32)
    a[:, ::2] = 2**30
    compare_xy(L, float("inf"), seed=12, sweeps=6, dir_bits=2, angles=a)


def test_multi_sweep_calls_match_single_sweeps():
    L, K = 256, K_KT
    ref = oracle.XYOracleLattice(L, K, 5)
    rows = ref.run(37)
    lat = binding.XYLattice(L, K, seed=5, obs_capacity=64)
    for n in (1, 5, 13, 18):
        lat.sweep(n)
    assert lat.sweeps_done == 37
    assert np.array_equal(lat.angles(), ref.a)
    assert_rows_match(lat.measure(0, 37), rows, L * L)
    lat.close()


def test_resume_from_checkpoint():
    L, K = 200, 0.8
    a = binding.XYLattice(L, K, seed=77, obs_capacity=64)
    a.sweep(20)
    straight = a.angles()
    obs_straight = a.measure(10, 10)
    b = binding.XYLattice(L, K, seed=77, obs_capacity=64)
    b.sweep(10)
    snap = b.angles()
    c = binding.XYLattice(L, K, seed=77, obs_capacity=64)
    c.load_angles(snap, 10)
    c.sweep(10)
    assert np.array_equal(c.angles(), straight)
    assert np.array_equal(c.measure(10, 10), obs_straight)   # the same device arithmetic: identical
    with pytest.raises(binding.SwError):
        c.measure(9, 1)
    for x in (a, b, c):
        x.close()


def test_ring_wraps():
    L, K = 64, 1.0
    ref = oracle.XYOracleLattice(L, K, 8)
    rows = ref.run(30)
    lat = binding.XYLattice(L, K, seed=8, obs_capacity=4)
    lat.sweep(30)
    assert_rows_match(lat.measure(26, 4), rows[26:], L * L)
    with pytest.raises(binding.SwError):
        lat.measure(25, 1)
    lat.close()


def test_potts_only_calls_refuse_an_xy_lattice():
    lat = binding.XYLattice(16, 1.0, seed=1, obs_capacity=4)
    lat.sweep(1)
    for call in (lat.spins, lambda: lat.load_spins(np.zeros((16, 16), np.uint8), 0),
                 lambda: lat.cluster_sums(0, 1)):
        with pytest.raises(binding.SwError):
            call()
    g = binding.Group(4, 64)
    with pytest.raises(binding.SwError) as e:
        g.sweep([lat], [1])
    assert e.value.code == binding.SW_EINVAL
    g.close()
    lat.close()


def test_L4096_bit_exact_one_sweep():
    """Several thousand tiles: one sweep from a random start against the oracle
    (angles, bonds, labels), then the measurement of the result."""
    L, K = 4096, K_KT
    compare_xy(L, K, seed=2024, sweeps=1)


def test_L8192_properties_of_a_sweep():
    """A larger lattice, checked by properties that hold at any size: every
    site keeps its angle or takes its reflection across the line perpendicular
    to the sweep's direction; every active bond joins two sites on the same
    side of that line and whose choice is the same (one choice per cluster);
    the active-bond count matches the bond planes."""
    L, K, seed = 8192, K_KT, 99
    lat = binding.XYLattice(L, K, seed=seed, obs_capacity=4)
    lat.sweep(3)
    before = lat.angles()
    lat.sweep(1)
    after = lat.angles()
    t = 3
    phi = oracle.xy_direction(seed, t, 32)
    refl = (np.uint64(2 * phi + 2**31) - before.astype(np.uint64)).astype(np.uint32)
    kept = after == before
    assert np.all(kept | (after == refl))
    bx, by = lat.bonds()
    bits_x = np.unpackbits(bx.view(np.uint8), bitorder="little").reshape(L, -1)[:, :L].astype(bool)
    bits_y = np.unpackbits(by.view(np.uint8), bitorder="little").reshape(L, -1)[:, :L].astype(bool)
    assert np.array_equal(kept[bits_x], np.roll(kept, -1, axis=1)[bits_x])
    assert np.array_equal(kept[bits_y], np.roll(kept, -1, axis=0)[bits_y])
    c = np.cos((before.astype(np.float64) - phi) * (2 * np.pi / 2**32))
    assert np.all(c[bits_x] * np.roll(c, -1, axis=1)[bits_x] > 0)
    assert np.all(c[bits_y] * np.roll(c, -1, axis=0)[bits_y] > 0)
    assert lat.measure(t, 1)[0, 0] == int(bits_x.sum()) + int(bits_y.sum())
    assert 0.0 < kept.mean() < 1.0
    lat.close()
