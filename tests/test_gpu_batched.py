"""GPU: the batched form, groups and the server give every replica exactly the
result it gets alone (and that the oracle gives)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_2080_amd import binding, serve
from paper_1208_2080_amd import workloads as wl

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def say(msg):
    print(msg, flush=True)


MIX = [dict(L=64, q=2, K=wl.critical_coupling(2), seed=11),
       dict(L=100, q=3, K=wl.critical_coupling(3), seed=12),
       dict(L=2, q=2, K=1.5, seed=13),
       dict(L=129, q=4, K=0.9 * wl.critical_coupling(4), seed=14),
       dict(L=33, q=8, K=wl.critical_coupling(8), seed=15),
       dict(L=256, q=2, K=1.1 * wl.critical_coupling(2), seed=16),
       dict(L=65, q=5, K=0.0, seed=17),
       dict(L=191, q=2, K=float("inf"), seed=18, random_start=False)]


@pytest.mark.parametrize("ty", [32, 64, 128])
def test_batch_sweep_all_matches_oracle(ty):
    say(f"batch sweep_all ty={ty}")
    b = binding.Batch(MIX, obs_capacity=32, tile_rows=ty)
    refs = [oracle.OracleLattice(r["L"], r["q"], r["K"], r["seed"], r.get("random_start", True)) for r in MIX]
    for r, ref in enumerate(refs):
        assert np.array_equal(b.spins(r), ref.s)
    for _ in range(3):
        b.sweep_all(4)
        for r, ref in enumerate(refs):
            rows = ref.run(4)
            assert np.array_equal(b.spins(r), ref.s), f"replica {r}"
            done = b.sweeps_done(r)
            assert np.array_equal(b.measure(r, done - 4, 4), rows), f"replica {r}"
    b.close()


def test_batch_sweep_all_graph_reuse_matches_oracle():
    """Cached graphs replayed after other sweep counts, after uneven sweeps and
    past the graph cache's bound keep every replica on the oracle's chain."""
    say("batch sweep_all graph reuse")
    b = binding.Batch(MIX, obs_capacity=64)
    refs = [oracle.OracleLattice(r["L"], r["q"], r["K"], r["seed"], r.get("random_start", True)) for r in MIX]

    def check(n_each):
        for r, (ref, n) in enumerate(zip(refs, n_each)):
            rows = ref.run(n) if n else None
            assert b.sweeps_done(r) == ref.t, f"replica {r}"
            assert np.array_equal(b.spins(r), ref.s), f"replica {r} after {n_each}"
            if n:
                assert np.array_equal(b.measure(r, ref.t - n, n), rows), f"replica {r} after {n_each}"

    plan = [("all", 4), ("all", 5), ("all", 4), ("each", [2] * len(MIX)), ("all", 4),
            ("each", [1, 0, 3, 0, 2, 0, 1, 0]), ("all", 5)]
    # more distinct counts than the cache keeps, then the first again
    plan += [("all", n) for n in (1, 2, 3, 6, 7, 8, 9)] + [("all", 4)]
    for kind, n in plan:
        if kind == "all":
            b.sweep_all(n)
            check([n] * len(MIX))
        else:
            b.sweep(n)
            check(n)
    b.close()


def test_autotuned_batch_matches_oracle():
    say("batch autotune")
    best, ms = binding.autotune(MIX, obs_capacity=32, sweeps=4)
    cands = binding.tile_candidates(MIX)
    assert binding.SW_TILE_WHOLE not in cands          # MIX has lattices larger than 128
    assert best in cands
    assert set(ms) == set(cands) and all(v > 0 for v in ms.values())
    assert ms[best] == min(ms.values())
    b = binding.Batch(MIX, obs_capacity=32, tile_rows="auto")
    assert b.tile_rows in cands and b.tuned_ms[b.tile_rows] == min(b.tuned_ms.values())
    refs = [oracle.OracleLattice(r["L"], r["q"], r["K"], r["seed"], r.get("random_start", True)) for r in MIX]
    b.sweep_all(5)
    for r, ref in enumerate(refs):
        rows = ref.run(5)
        assert np.array_equal(b.spins(r), ref.s), f"replica {r}"
        assert np.array_equal(b.measure(r, 0, 5), rows), f"replica {r}"
    b.close()


def test_batch_uneven_sweep_counts():
    say("batch uneven counts")
    b = binding.Batch(MIX, obs_capacity=32)
    refs = [oracle.OracleLattice(r["L"], r["q"], r["K"], r["seed"], r.get("random_start", True)) for r in MIX]
    for counts in ([3, 0, 1, 5, 2, 0, 4, 1], [0, 6, 2, 0, 1, 3, 0, 2]):
        b.sweep(counts)
        for r, (ref, n) in enumerate(zip(refs, counts)):
            rows = ref.run(n) if n else None
            assert b.sweeps_done(r) == ref.t
            assert np.array_equal(b.spins(r), ref.s), f"replica {r}"
            if n:
                assert np.array_equal(b.measure(r, ref.t - n, n), rows)
    b.close()


def test_group_equals_plain_lattices():
    say("group vs plain")
    lats = [binding.Lattice(r["L"], r["q"], r["K"], r["seed"], r.get("random_start", True), obs_capacity=16)
            for r in MIX]
    alone = [binding.Lattice(r["L"], r["q"], r["K"], r["seed"], r.get("random_start", True), obs_capacity=16)
             for r in MIX]
    tiles = sum(binding.tile_count(r["L"]) for r in MIX)
    g = binding.Group(len(MIX), tiles)
    plan = [[2, 2, 2, 2, 2, 2, 2, 2], [1, 0, 3, 0, 5, 1, 0, 2], [0, 4, 0, 4, 0, 4, 0, 4]]
    for counts in plan:
        members = [lat for lat, n in zip(lats, counts)]
        g.sweep(members, counts)
        for a, n in zip(alone, counts):
            if n:
                a.sweep(n)
        for i, (a, b) in enumerate(zip(lats, alone)):
            assert a.sweeps_done == b.sweeps_done
            assert np.array_equal(a.spins(), b.spins()), f"lattice {i}"
            if a.sweeps_done:
                n = min(a.sweeps_done, 8)
                assert np.array_equal(a.measure(a.sweeps_done - n, n), b.measure(b.sweeps_done - n, n))
    # a subset, in another order
    sub = [lats[5], lats[0], lats[3]]
    g.sweep(sub, [3, 1, 2])
    for i, n in zip((5, 0, 3), (3, 1, 2)):
        alone[i].sweep(n)
        assert np.array_equal(lats[i].spins(), alone[i].spins())
    g.close()


def test_server_jobs_identical_alone_and_in_the_mix():
    say("server mix")
    raw = wl.serving_jobs(n=16, seed=7, L_min=16, L_max=300, sweeps_min=5, sweeps_max=60, rate_per_s=400.0)
    jobs = [serve.Job(id=j["id"], L=j["L"], q=j["q"], K=j["K"], seed=j["seed"], sweeps=j["sweeps"],
                      arrival=j["arrival"]) for j in raw]
    backend = serve.GpuBackend(max_jobs=6, max_tiles=4096)
    srv = serve.SwServer(backend, hbm_budget=1 << 40, max_jobs=6, max_tiles=4096, step_sweeps=8, measure_every=3)
    budget = 4 * max(backend.footprint(j, srv.obs_capacity) for j in jobs)
    srv.hbm_budget = budget
    results, stats = srv.run(jobs, realtime=True)
    say(f"server stats {stats}")
    assert len(results) == len(jobs) and srv.peak_bytes <= budget
    for j in jobs:
        lat = binding.Lattice(j.L, j.q, j.K, seed=j.seed, obs_capacity=j.sweeps)
        lat.sweep(j.sweeps)
        assert np.array_equal(results[j.id].spins, lat.spins()), f"job {j.id}"
        assert np.array_equal(results[j.id].obs, lat.measure(0, j.sweeps)), f"job {j.id}"
        lat.close()
    ref = oracle.OracleLattice(jobs[0].L, jobs[0].q, jobs[0].K, jobs[0].seed)
    assert np.array_equal(results[jobs[0].id].obs, ref.run(jobs[0].sweeps))
    backend.close()
