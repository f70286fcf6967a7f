"""The serving scheduler on the CPU, with the oracle standing in for the device.

Checks: admission never exceeds the memory budget or the slot limit, every job
finishes (first come first served, no starvation), and every job's result is
identical to the same job run alone.
"""
import numpy as np
import pytest

import oracle
from paper_1208_2080_amd import serve
from paper_1208_2080_amd import workloads as wl


class OracleBackend:
    """The oracle as a fake device: one OracleLattice per job, stepped one by one."""

    def __init__(self):
        self.created = 0
        self.live = 0
        self.max_live = 0

    def footprint(self, job, obs_capacity):
        return job.L * job.L * 6 + obs_capacity * (2 + job.q) * 8

    def tiles(self, job):
        return -(-job.L // 64) * -(-job.L // 64)

    def create(self, job, obs_capacity):
        self.created += 1
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        lat = oracle.OracleLattice(job.L, job.q, job.K, job.seed, random_start=job.random_start)
        lat.pending = []
        return lat

    def step(self, handles, n_each):
        for h, n in zip(handles, n_each):
            h.pending.append(h.run(n))

    def mark(self):
        return None

    def wait(self, token):
        pass

    def measure(self, h, first, n, after=None):
        # the oracle runs each step at once: later steps' rows may be queued already
        rows = np.concatenate(h.pending, axis=0)
        assert rows.shape[0] >= n and h.t - rows.shape[0] == first
        h.pending = [rows[n:]] if rows.shape[0] > n else []
        return rows[:n]

    def spins(self, h, after=None):
        return h.s.copy()

    def release(self, h):
        self.live -= 1


def _jobs(n=14, seed=5):
    raw = wl.serving_jobs(n=n, seed=seed, L_min=8, L_max=48, sweeps_min=3, sweeps_max=40, rate_per_s=1e6)
    return [serve.Job(id=j["id"], L=j["L"], q=j["q"], K=j["K"], seed=j["seed"], sweeps=j["sweeps"],
                      arrival=j["arrival"]) for j in raw]


@pytest.mark.parametrize("step,every", [(1, 1), (7, 3), (64, 8), (5, 2)])
def test_results_identical_to_jobs_alone(step, every):
    jobs = _jobs()
    backend = OracleBackend()
    srv = serve.SwServer(backend, hbm_budget=1 << 40, max_jobs=4, max_tiles=10_000, step_sweeps=step,
                         measure_every=every)
    budget = 3 * max(backend.footprint(j, srv.obs_capacity) for j in jobs)
    srv.hbm_budget = budget
    results, stats = srv.run(jobs, realtime=False)
    assert sorted(results) == [j.id for j in sorted(jobs, key=lambda j: j.id)]
    assert srv.peak_bytes <= budget and backend.max_live <= 4
    for j in jobs:
        alone = oracle.OracleLattice(j.L, j.q, j.K, j.seed)
        rows = alone.run(j.sweeps)
        assert np.array_equal(results[j.id].obs, rows), j
        assert np.array_equal(results[j.id].spins, alone.s), j
        assert len(results[j.id].sweep_latencies) == -(-j.sweeps // step)
    assert stats["jobs"] == len(jobs) and stats["p99_sweep_latency_s"] >= stats["p50_sweep_latency_s"]


def test_fifo_admission_never_overtakes_the_head():
    jobs = [serve.Job(id=0, L=40, q=2, K=0.9, seed=1, sweeps=30),
            serve.Job(id=1, L=40, q=2, K=0.9, seed=2, sweeps=5),
            serve.Job(id=2, L=8, q=2, K=0.9, seed=3, sweeps=5)]
    backend = OracleBackend()
    budget = backend.footprint(jobs[0], 6) + backend.footprint(jobs[2], 6)   # 0 and 2 fit, not 0 and 1
    srv = serve.SwServer(backend, hbm_budget=budget, max_jobs=8, max_tiles=10_000, step_sweeps=5, measure_every=1)
    results, _ = srv.run(jobs, realtime=False)
    # job 2 is small enough to fit beside job 0 but must not overtake job 1
    assert results[1].admitted <= results[2].admitted
    assert len(results) == 3


def test_job_that_can_never_fit_is_refused():
    backend = OracleBackend()
    srv = serve.SwServer(backend, hbm_budget=1000, max_jobs=2, max_tiles=10, step_sweeps=5)
    with pytest.raises(ValueError):
        srv.run([serve.Job(id=0, L=64, q=2, K=0.9, seed=1, sweeps=3)], realtime=False)
