"""Continuous-batching server for Swendsen-Wang simulation jobs on one GPU.

Jobs (L, q, K, seed, number of sweeps) arrive over time.  A job is admitted
when a slot is free and its device footprint fits the HBM budget; admitted jobs
keep their lattice resident on the GPU, and every server step sweeps *all*
resident jobs together (one launch per kernel phase, ``sw_group_sweep``), so a
job that arrives while others run joins the very next step and its work
overlaps theirs on the device.  Finished jobs free their slot and memory
between steps.  Admission is first-come first-served (the head of the queue is
never overtaken), so no job starves.

Every job's random numbers are keyed only by its own seed and its own sweep
index, so its spins and observables are identical alone and in any mix.

Steps are pipelined: the next step is enqueued before the results of the
current one are read back, so the host's bookkeeping (copying observables and
final spins of finished jobs out on a second stream, admitting new jobs)
overlaps the device's work instead of leaving it idle between steps.

The device work goes through a backend object (``GpuBackend`` here); the
scheduler itself holds no arithmetic of the method.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Job:
    id: int
    L: int
    q: int
    K: float
    seed: int
    sweeps: int
    arrival: float = 0.0
    random_start: bool = True


@dataclasses.dataclass
class JobResult:
    id: int
    obs: np.ndarray            # int64 [sweeps, 2 + q]
    spins: np.ndarray          # uint8 [L, L] after the last sweep
    arrival: float
    admitted: float
    finished: float
    sweep_latencies: list      # seconds per sweep, one entry per step the job took part in


@dataclasses.dataclass
class _Resident:
    job: Job
    handle: object
    bytes: int
    tiles: int
    admitted: float
    last: float
    done: int = 0              # sweeps completed (their step has finished)
    enq: int = 0               # sweeps enqueued
    unread: int = 0            # sweeps done whose observables are still only on the device
    rows: list = dataclasses.field(default_factory=list)
    lat: list = dataclasses.field(default_factory=list)


class GpuBackend:
    """Jobs as ``binding.Lattice`` objects, stepped together through a
    ``binding.Group`` on one stream; results are read on a second stream (same
    priority) after an event that marks the end of their step."""

    def __init__(self, max_jobs: int, max_tiles: int, tile_rows: int = 0):
        import torch
        from . import binding
        self.torch = torch
        self.binding = binding
        self.tile_rows = tile_rows
        self.group = binding.Group(max_jobs, max_tiles, tile_rows)
        self.read_stream = torch.cuda.Stream(self.group.device)

    def footprint(self, job: Job, obs_capacity: int) -> int:
        return self.binding.workspace_bytes(job.L, job.q, obs_capacity, self.tile_rows)

    def tiles(self, job: Job) -> int:
        return self.binding.tile_count(job.L, job.q, self.tile_rows)

    def create(self, job: Job, obs_capacity: int):
        return self.binding.Lattice(job.L, job.q, job.K, seed=job.seed, random_start=job.random_start,
                                    obs_capacity=obs_capacity, tile_rows=self.tile_rows)

    def step(self, handles, n_each):
        self.group.sweep(handles, n_each)

    def mark(self):
        """A token for the work enqueued so far (an event on the group's stream)."""
        ev = self.torch.cuda.Event()
        ev.record(self.group.stream)
        return ev

    def wait(self, token):
        token.synchronize()

    def measure(self, handle, first: int, n: int, after=None) -> np.ndarray:
        return handle.measure_after(self.read_stream, after, first, n)

    def spins(self, handle, after=None) -> np.ndarray:
        return handle.spins_after(self.read_stream, after)

    def release(self, handle):
        # its workspace is reused only after the group stream's work; a finished
        # job is in no later step
        handle.close(sync=False)

    def close(self):
        self.group.close()


class SwServer:
    """Continuous batching under an HBM budget; see the module docstring."""

    def __init__(self, backend, hbm_budget: int, max_jobs: int, max_tiles: int, step_sweeps: int = 20,
                 measure_every: int = 8, clock=time.perf_counter):
        if step_sweeps < 1 or max_jobs < 1 or measure_every < 1:
            raise ValueError("step_sweeps, measure_every and max_jobs must be positive")
        self.backend = backend
        self.hbm_budget = int(hbm_budget)
        self.max_jobs = int(max_jobs)
        self.max_tiles = int(max_tiles)
        self.step_sweeps = int(step_sweeps)
        # observables are copied out every `measure_every` steps (and when a job
        # ends): the ring keeps that many steps of sweeps, plus the step that
        # runs while they are read
        self.measure_every = int(measure_every)
        self.obs_capacity = self.step_sweeps * (self.measure_every + 1) + 1
        self.clock = clock
        self.peak_bytes = 0
        self.steps = 0

    def admissible(self, job: Job) -> bool:
        """Can this job ever run (alone) under the budget?"""
        return (self.backend.footprint(job, self.obs_capacity) <= self.hbm_budget
                and self.backend.tiles(job) <= self.max_tiles)

    def run(self, jobs, realtime: bool = True):
        """Serve ``jobs`` (arrival times in seconds from the start) to completion.

        Returns (results by job id, stats)."""
        jobs = sorted(jobs, key=lambda j: (j.arrival, j.id))
        for j in jobs:
            if not self.admissible(j):
                raise ValueError(f"job {j.id} (L={j.L}, q={j.q}) can never fit the budget")
        pending = collections.deque(jobs)
        waiting = collections.deque()
        resident: dict[int, _Resident] = {}
        results: dict[int, JobResult] = {}
        used_bytes = used_tiles = 0
        t0 = self.clock()
        now = lambda: self.clock() - t0  # noqa: E731

        inflight = None   # (members, n_each, token) of the step on the device

        def finish(step):
            """Bookkeeping of a completed step (the next one may be running)."""
            nonlocal used_bytes, used_tiles
            members, n_each, token = step
            self.backend.wait(token)
            te = now()
            self.steps += 1
            for r, n in zip(members, n_each):
                r.done += n
                r.unread += n
                r.lat.append((te - r.last) / n)
                r.last = te
                # copy the observables out before the ring could overwrite them
                # (the step in flight adds up to step_sweeps more)
                if r.done == r.job.sweeps or r.unread + 2 * self.step_sweeps > self.obs_capacity - 1:
                    r.rows.append(self.backend.measure(r.handle, r.done - r.unread, r.unread, after=token))
                    r.unread = 0
            for r in members:
                if r.done == r.job.sweeps:
                    results[r.job.id] = JobResult(r.job.id, np.concatenate(r.rows, axis=0),
                                                  self.backend.spins(r.handle, after=token), r.job.arrival,
                                                  r.admitted, te, r.lat)
                    self.backend.release(r.handle)
                    used_bytes -= r.bytes
                    used_tiles -= r.tiles
                    del resident[r.job.id]

        while pending or waiting or resident:
            t = now()
            while pending and (pending[0].arrival <= t or not realtime):
                waiting.append(pending.popleft())
            # admission, first come first served
            while waiting and len(resident) < self.max_jobs:
                job = waiting[0]
                nb = self.backend.footprint(job, self.obs_capacity)
                nt = self.backend.tiles(job)
                if used_bytes + nb > self.hbm_budget or used_tiles + nt > self.max_tiles:
                    break
                waiting.popleft()
                handle = self.backend.create(job, self.obs_capacity)
                ta = now()
                resident[job.id] = _Resident(job, handle, nb, nt, admitted=ta, last=ta)
                used_bytes += nb
                used_tiles += nt
                self.peak_bytes = max(self.peak_bytes, used_bytes)
            # the next step: every resident job with sweeps left to enqueue
            # advances by up to step_sweeps sweeps
            members = [r for r in resident.values() if r.enq < r.job.sweeps]
            step = None
            if members:
                n_each = [min(self.step_sweeps, r.job.sweeps - r.enq) for r in members]
                self.backend.step([r.handle for r in members], n_each)
                for r, n in zip(members, n_each):
                    r.enq += n
                step = (members, n_each, self.backend.mark())
            if inflight is not None:
                finish(inflight)
            inflight = step
            if inflight is None and not resident and pending and realtime:
                time.sleep(max(0.0, min(pending[0].arrival - now(), 0.01)))
        if inflight is not None:
            finish(inflight)

        wall = now()
        lats = np.concatenate([np.asarray(res.sweep_latencies) for res in results.values()]) \
            if results else np.zeros(0)
        flips = sum(j.L * j.L * j.sweeps for j in jobs)
        stats = {
            "jobs": len(jobs),
            "steps": self.steps,
            "wall_s": wall,
            "flips_per_ns": flips / (wall * 1e9) if wall > 0 else float("nan"),
            "p50_sweep_latency_s": float(np.percentile(lats, 50)) if lats.size else float("nan"),
            "p99_sweep_latency_s": float(np.percentile(lats, 99)) if lats.size else float("nan"),
            "peak_bytes": self.peak_bytes,
            "hbm_budget": self.hbm_budget,
        }
        return results, stats
