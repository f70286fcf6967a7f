"""GPU: lattices of L <= 128 swept whole in one workgroup's LDS (tile_rows =
SW_TILE_WHOLE, the default at these sizes) give the oracle's spins, bonds,
labels and observables, the same as the tile kernels, across kernel launches
of many sweeps, mixed with tile sweeps of the same lattice (groups), in
batches, and when the observable ring wraps."""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_2080_amd import binding
from paper_1208_2080_amd import workloads as wl

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

WHOLE = binding.SW_TILE_WHOLE


def say(msg):
    print(msg, flush=True)


def step_and_compare(lat, ref, sweeps, labels=True):
    for _ in range(sweeps):
        t = ref.t
        lat.sweep(1)
        out = ref.sweep()
        assert np.array_equal(lat.spins(), ref.s), f"spins after sweep {t}"
        if labels:
            bx, by = lat.bonds()
            assert np.array_equal(bx, oracle.pack_bonds(out["bx"])), f"+x bonds of sweep {t}"
            assert np.array_equal(by, oracle.pack_bonds(out["by"])), f"+y bonds of sweep {t}"
            assert np.array_equal(lat.labels(), out["labels"]), f"labels of sweep {t}"
        assert np.array_equal(lat.measure(t, 1)[0], out["obs"]), f"observables of sweep {t}"


@pytest.mark.parametrize("ty", [WHOLE, 64])
@pytest.mark.parametrize("L,q,K", [(2, 2, 1.5), (3, 3, 0.9), (17, 2, None), (64, 2, None), (65, 5, 0.0),
                                   (100, 3, None), (128, 2, None), (127, 255, None), (96, 4, float("inf"))])
def test_every_sweep_against_oracle(L, q, K, ty):
    K = wl.critical_coupling(q) if K is None else K
    say(f"whole/tile L={L} q={q} K={K} ty={ty}")
    lat = binding.Lattice(L, q, K, seed=L + q, obs_capacity=16, tile_rows=ty)
    ref = oracle.OracleLattice(L, q, K, L + q)
    step_and_compare(lat, ref, 6)
    lat.close()


def test_multi_sweep_launch_and_chunks():
    """One call of 5000 sweeps (two launches of the whole-lattice kernel) and
    calls of other lengths: spins and the ring's last records as the oracle's."""
    L, q, K = 16, 3, wl.critical_coupling(3)
    lat = binding.Lattice(L, q, K, seed=9, obs_capacity=64, tile_rows=WHOLE)
    ref = oracle.OracleLattice(L, q, K, 9)
    for n in (5000, 1, 37):
        rows = ref.run(n)
        lat.sweep(n)
        assert lat.sweeps_done == ref.t
        assert np.array_equal(lat.spins(), ref.s)
        k = min(n, 64)
        assert np.array_equal(lat.measure(ref.t - k, k), rows[-k:])
    lat.close()


def test_whole_and_tile_sweeps_of_one_lattice():
    """Sweeps alternate between the whole-lattice kernel (plain calls) and the
    tile kernels (group calls) on one lattice: the ring records written both
    ways read back as the oracle's, also after the ring has wrapped."""
    L, q, K = 80, 2, wl.critical_coupling(2)
    lat = binding.Lattice(L, q, K, seed=21, obs_capacity=6)
    assert lat.params.tile_rows == 0
    ref = oracle.OracleLattice(L, q, K, 21)
    g = binding.Group(1, binding.tile_count(L))
    for kind, n in [("whole", 3), ("group", 4), ("whole", 5), ("group", 2), ("whole", 1), ("group", 7),
                    ("whole", 9)]:
        rows = ref.run(n)
        if kind == "whole":
            lat.sweep(n)
        else:
            g.sweep([lat], [n])
        assert np.array_equal(lat.spins(), ref.s), f"after {kind} {n}"
        k = min(n, 6)
        assert np.array_equal(lat.measure(ref.t - k, k), rows[-k:]), f"after {kind} {n}"
        out_labels = oracle.label(*_oracle_bonds(lat, ref))
        assert np.array_equal(lat.labels(), out_labels)
    g.close()
    lat.close()


def _oracle_bonds(lat, ref):
    # the bonds of the lattice's last sweep, unpacked from its bond planes
    bx, by = lat.bonds()
    L = lat.L
    ux = np.unpackbits(bx.view(np.uint8), bitorder="little").reshape(L, -1)[:, :L]
    uy = np.unpackbits(by.view(np.uint8), bitorder="little").reshape(L, -1)[:, :L]
    return ux, uy


def test_small_batch_swept_whole():
    reps = [dict(L=L, q=q, K=wl.critical_coupling(q) * f, seed=100 + i)
            for i, (L, q, f) in enumerate([(64, 2, 1.0), (128, 3, 1.0), (5, 2, 0.9), (100, 8, 1.05),
                                           (33, 4, 1.0), (65, 2, 1.1)])]
    b = binding.Batch(reps, obs_capacity=32, tile_rows=WHOLE)
    refs = [oracle.OracleLattice(r["L"], r["q"], r["K"], r["seed"]) for r in reps]
    for kind, n in [("all", 7), ("each", [3, 0, 1, 5, 2, 4]), ("all", 1), ("each", [0, 2, 0, 0, 6, 1])]:
        counts = [n] * len(reps) if kind == "all" else n
        if kind == "all":
            b.sweep_all(n)
        else:
            b.sweep(n)
        for r, (ref, k) in enumerate(zip(refs, counts)):
            rows = ref.run(k) if k else None
            assert b.sweeps_done(r) == ref.t
            assert np.array_equal(b.spins(r), ref.s), f"replica {r} after {kind} {n}"
            if k:
                assert np.array_equal(b.measure(r, ref.t - k, k), rows), f"replica {r} after {kind} {n}"
    b.close()


def test_autotune_offers_the_whole_lattice_path():
    reps = [dict(L=64, q=2, K=wl.critical_coupling(2), seed=200 + i) for i in range(16)]
    best, ms = binding.autotune(reps, obs_capacity=8, sweeps=8)
    assert set(ms) == set(binding.tile_candidates(reps)) and WHOLE in ms
    assert ms[best] == min(ms.values())


def test_ring_wraps_and_profiled_sweeps():
    L, q, K = 64, 2, wl.critical_coupling(2)
    ref = oracle.OracleLattice(L, q, K, 8)
    rows = ref.run(30)
    lat = binding.Lattice(L, q, K, seed=8, obs_capacity=4)
    ph = lat.sweep_profiled(30)
    assert ph[0] > 0 and ph[0] == ph[4] and ph[1] == ph[2] == 0
    assert np.array_equal(lat.spins(), ref.s)
    assert np.array_equal(lat.measure(26, 4), rows[26:])
    with pytest.raises(binding.SwError):
        lat.measure(25, 1)
    lat.close()


def test_whole_lattice_path_limits():
    with pytest.raises(binding.SwError):
        binding.Lattice(129, 2, 1.0, tile_rows=WHOLE)
    with pytest.raises(binding.SwError):
        binding.Lattice(64, 2, 1.0, tile_rows=WHOLE, cluster_sums=True)
    with pytest.raises(binding.SwError):
        binding.XYLattice(64, 1.0, tile_rows=WHOLE)
    # cluster sums keep the tile kernels at small sizes
    lat = binding.Lattice(64, 2, wl.critical_coupling(2), seed=3, obs_capacity=8, cluster_sums=True)
    ref = oracle.OracleLattice(64, 2, wl.critical_coupling(2), 3)
    lat.sweep(3)
    ref.run(3)
    assert np.array_equal(lat.spins(), ref.s)
    lat.close()
