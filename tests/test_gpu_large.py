"""GPU parity at the full throughput sizes, in the launch configuration the
benchmark times (default tile height).

* L = 16384 (2^28 sites): element-by-element against the oracle for two sweeps
  (spins, bond planes and labels of the first sweep, observables of both).
* L = 65536 (2^32 sites, q = 2 and q = 3, cold start): too large for the
  oracle to sweep in seconds, so the second sweep is checked on sampled sites
  the oracle computes one by one (bond draws and activations, the new state of
  each sampled site's root) and by properties that hold at any size, over the
  whole lattice: every active bond joins two sites of one label, every label is
  at most its site's index, the observables equal those of the spins; the
  clusters of sampled sites are rebuilt by breadth-first search over the bond
  planes and must carry exactly one label, their smallest site index.
* L = 65536, q = 2 and q = 3, cold start, bit for bit: the oracle sweeps both
  lattices twice (in two host threads, while the GPU sweeps), and the spins
  (by a 64-bit hash of all 2^32 bytes) and the int64 observables must agree
  after each sweep.
"""
import collections
import threading

import numpy as np
import pytest
import torch

import oracle
from paper_1208_2080_amd import binding
from paper_1208_2080_amd import workloads as wl

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def say(msg):
    print(msg, flush=True)


def test_full_parity_L16384():
    cfg = wl.PLAIN_16384
    L, q, K, seed = cfg["L"], cfg["q"], cfg["K"], cfg["seed"]
    say(f"L={L} q={q} full parity, 2 sweeps")
    lat = binding.Lattice(L, q, K, seed=seed, random_start=cfg["random_start"], obs_capacity=1024)
    ref = oracle.OracleLattice(L, q, K, seed, random_start=cfg["random_start"])
    assert np.array_equal(lat.spins(), ref.s), "initial spins"
    for t in range(2):
        lat.sweep(1)
        out = ref.sweep()
        say(f"  sweep {t} done on both sides")
        assert np.array_equal(lat.spins(), ref.s), f"spins after sweep {t}"
        assert np.array_equal(lat.measure(t, 1)[0], out["obs"]), f"observables of sweep {t}"
        if t == 0:
            bx, by = lat.bonds()
            assert np.array_equal(bx, oracle.pack_bonds(out["bx"])), "+x bonds"
            assert np.array_equal(by, oracle.pack_bonds(out["by"])), "+y bonds"
            del bx, by
            assert np.array_equal(lat.labels(), out["labels"]), "labels"
        del out
    lat.close()


def _bit(plane, y, x):
    return bool((int(plane[y, x >> 6]) >> (x & 63)) & 1)


def _component(bx, by, L, y0, x0, cap):
    """Sites of the cluster of (y0, x0) by breadth-first search over the active
    bonds (periodic), or None if it has more than `cap` sites."""
    seen = {(y0, x0)}
    todo = collections.deque([(y0, x0)])
    while todo:
        y, x = todo.popleft()
        xl, yu = (x - 1) % L, (y - 1) % L
        nbrs = []
        if _bit(bx, y, x):
            nbrs.append((y, (x + 1) % L))
        if _bit(bx, y, xl):
            nbrs.append((y, xl))
        if _bit(by, y, x):
            nbrs.append(((y + 1) % L, x))
        if _bit(by, yu, x):
            nbrs.append((yu, x))
        for n in nbrs:
            if n not in seen:
                seen.add(n)
                if len(seen) > cap:
                    return None
                todo.append(n)
    return seen


def _sample_sites(L, n, rng):
    ys = rng.integers(0, L, n)
    xs = rng.integers(0, L, n)
    # the lattice's wrap edges and tile corners
    edge = np.array([0, 1, 63, 64, 127, 128, L // 2 - 1, L // 2, L - 65, L - 64, L - 2, L - 1])
    ey, ex = np.meshgrid(edge, edge, indexing="ij")
    return np.concatenate([ys, ey.ravel()]), np.concatenate([xs, ex.ravel()])


@pytest.mark.parametrize("name", ["HUGE_Q2", "HUGE_Q3"])
def test_sampled_and_properties_L65536(name):
    cfg = getattr(wl, name)
    L, q, K, seed = cfg["L"], cfg["q"], cfg["K"], cfg["seed"]
    W = (L + 63) // 64
    say(f"L={L} q={q} sampled + properties")
    lat = binding.Lattice(L, q, K, seed=seed, random_start=cfg["random_start"], obs_capacity=8)
    lat.sweep(1)
    before = lat.spins()
    lat.sweep(1)
    after = lat.spins()
    bx, by = lat.bonds()
    obs = lat.measure(1, 1)[0]
    say("  read spins, bonds, observables")
    lab = lat.labels()
    lat.close()
    say("  read labels")
    rng = np.random.default_rng(2024 + q)
    thr = oracle.threshold(K)

    # observables of the new configuration, over the whole lattice
    ref_obs = oracle.observe(after, q)
    n_active = int(np.bitwise_count(bx).sum()) + int(np.bitwise_count(by).sum())
    assert obs[0] == ref_obs[0] and np.array_equal(obs[2:], ref_obs[2:]), (obs, ref_obs)
    assert obs[1] == n_active
    say("  observables ok")

    # bonds, roots and new states on sampled sites, computed one by one by the oracle
    ys, xs = _sample_sites(L, 20000, rng)
    for y, x in zip(ys.tolist(), xs.tolist()):
        i = y * L + x
        wx, wy = oracle.bond_draws(seed, 1, i)
        s = before[y, x]
        ex = bool(s == before[y, (x + 1) % L] and wx < thr)
        ey = bool(s == before[(y + 1) % L, x] and wy < thr)
        assert _bit(bx, y, x) == ex and _bit(by, y, x) == ey, f"bonds of site ({y}, {x})"
        r = int(lab[y, x])
        assert r <= i and lab[r // L, r % L] == r, f"root of site ({y}, {x})"
        assert after[y, x] == oracle.newspin(seed, 1, r, q), f"new state of site ({y}, {x})"
    say("  sampled bonds, roots, states ok")

    # whole lattice: active bonds join equal labels; labels never exceed the site index
    band = 1024
    cols = np.arange(L, dtype=np.uint64)
    for y0 in range(0, L, band):
        y1 = min(L, y0 + band)
        lb = lab[y0:y1]
        mx = np.unpackbits(bx[y0:y1].view(np.uint8), axis=1, bitorder="little")[:, :L].astype(bool)
        my = np.unpackbits(by[y0:y1].view(np.uint8), axis=1, bitorder="little")[:, :L].astype(bool)
        assert not np.any(mx & (lb != np.roll(lb, -1, axis=1))), f"+x bond across labels in rows {y0}..{y1}"
        below = np.concatenate([lab[y0 + 1:y1], lab[y1 % L][None, :]], axis=0)
        assert not np.any(my & (lb != below)), f"+y bond across labels in rows {y0}..{y1}"
        idx = (np.arange(y0, y1, dtype=np.uint64)[:, None] * np.uint64(L) + cols[None, :])
        assert not np.any(lb.astype(np.uint64) > idx), f"label above its site in rows {y0}..{y1}"
    say("  whole-lattice label properties ok")

    # exact clusters of sampled sites: one label, the smallest member index
    checked = tried = 0
    for y, x in zip(*(a.tolist() for a in _sample_sites(L, 3000, rng))):
        if checked == 150:
            break
        tried += 1
        comp = _component(bx, by, L, y, x, cap=2000)
        if comp is None:
            continue
        root = min(cy * L + cx for cy, cx in comp)
        assert all(int(lab[cy, cx]) == root for cy, cx in comp), f"cluster of ({y}, {x})"
        # nothing outside the cluster carries its label in the cluster's rows
        rows = sorted({cy for cy, _ in comp})
        members = sum(int(np.count_nonzero(lab[r] == root)) for r in rows)
        assert members == len(comp), f"label {root} reaches beyond the cluster of ({y}, {x})"
        checked += 1
    say(f"  {checked} of {tried} sampled clusters rebuilt exactly (the rest exceed 2000 sites)")
    assert checked >= 30
    assert W == bx.shape[1]


def test_L4096_observables_every_sweep():
    """L = 4096 for 20 sweeps: int64 observables after every sweep and the final
    spins against the oracle."""
    cfg = wl.PLAIN_4096
    L, q, K, seed = cfg["L"], cfg["q"], cfg["K"], cfg["seed"]
    n = 20
    say(f"L={L} q={q} {n} sweeps")
    lat = binding.Lattice(L, q, K, seed=seed, random_start=cfg["random_start"], obs_capacity=n)
    lat.sweep(n)
    ref = oracle.OracleLattice(L, q, K, seed, random_start=cfg["random_start"])
    rows = ref.run(n)
    assert np.array_equal(lat.measure(0, n), rows)
    assert np.array_equal(lat.spins(), ref.s)
    lat.close()


@pytest.mark.parametrize("q", [2, 3])
def test_L65536_one_cluster_counts_need_64_bits(q):
    """K = infinity from the cold start: every bond is active, the whole
    lattice is one cluster rooted at site 0, so one state holds all 2^32 sites
    and n_active = 2^33 -- both past 32-bit range."""
    L, seed = 65536, 5
    say(f"L={L} q={q} K=inf one cluster")
    lat = binding.Lattice(L, q, float("inf"), seed=seed, random_start=False, obs_capacity=2)
    lat.sweep(1)
    obs = lat.measure(0, 1)[0]
    s_star = oracle.newspin(seed, 0, 0, q)
    expect = np.zeros(2 + q, dtype=np.int64)
    expect[1] = 2 * L * L
    expect[2 + s_star] = L * L
    assert np.array_equal(obs, expect), obs
    lat.close()


def _spin_hash(s) -> int:
    import xxhash
    return xxhash.xxh3_64_intdigest(memoryview(np.ascontiguousarray(s).reshape(-1)))


@pytest.mark.timeout(1800)
def test_L65536_bit_exact_two_sweeps(request):
    """The largest configuration (2^32 sites, cold start, q = 2 and q = 3 at
    their K_c) against the oracle after each of two sweeps: spins by a 64-bit
    hash, observables exactly.  Host RAM: the oracle holds 7 bytes per site
    per lattice (spins, two bond planes, labels: 28 GiB each, 56 GiB for both
    at once) plus one 4 GiB copy of the GPU's spins at a time; the two oracle
    lattices run in their own threads (a few minutes of one core per step), and
    each finished step is reported as it happens (outside pytest's capture, so
    that a long run shows its progress)."""
    import queue

    capture = request.config.pluginmanager.getplugin("capturemanager")

    def live(msg):
        if capture is None:
            say(msg)
            return
        with capture.global_and_fixture_disabled():
            print(msg, flush=True)

    cfgs = [wl.HUGE_Q2, wl.HUGE_Q3]
    ref_out = {}
    events = queue.Queue()

    def run_oracle(cfg):
        q = cfg["q"]
        try:
            ref = oracle.OracleLattice(cfg["L"], q, cfg["K"], cfg["seed"], random_start=cfg["random_start"])
            out = []
            for t in range(2):
                row = ref.sweep_steps(lambda step: events.put(f"  oracle q={q} sweep {t}: {step} done"))
                out.append((_spin_hash(ref.s), row))
            ref_out[q] = out
            del ref
        finally:
            events.put(None)

    threads = [threading.Thread(target=run_oracle, args=(c,)) for c in cfgs]
    for th in threads:
        th.start()
    got = {}
    for cfg in cfgs:
        L, q = cfg["L"], cfg["q"]
        live(f"L={L} q={q} cold start: 2 sweeps on the GPU")
        lat = binding.Lattice(L, q, cfg["K"], seed=cfg["seed"], random_start=cfg["random_start"], obs_capacity=4)
        res = []
        for t in range(2):
            lat.sweep(1)
            res.append((_spin_hash(lat.spins()), lat.measure(t, 1)[0]))
        got[q] = res
        lat.close()
        del lat
        torch.cuda.empty_cache()
        live(f"L={L} q={q}: GPU done")
    finished = 0
    while finished < len(threads):
        msg = events.get()   # each oracle step reports when it ends
        if msg is None:
            finished += 1
        else:
            live(msg)
    for th in threads:
        th.join()
    for cfg in cfgs:
        q = cfg["q"]
        assert q in ref_out, f"the oracle for q={q} did not finish"
        for t in range(2):
            assert got[q][t][0] == ref_out[q][t][0], f"q={q}: spins differ after sweep {t}"
            assert np.array_equal(got[q][t][1], ref_out[q][t][1]), f"q={q}: observables of sweep {t}"
        live(f"q={q}: spins and observables bit-identical after 2 sweeps")
