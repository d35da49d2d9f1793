"""Serving: a request loop that runs simulation jobs with continuous batching.

A job is (L, S, beta, sweeps, seed).  Jobs arrive over time; an arrived job
is admitted as soon as its device footprint (world lines plus per-sweep
scratch, lc_footprint_parts) fits next to the resident jobs, and joins the
one resident lc_batch between two iterations.  Every iteration runs one sweep
of every resident job in one captured launch sequence; a job whose sweeps are
done leaves the batch, releasing its memory, so waiting jobs can join.  A job
larger than the whole budget is rejected (the library's LC_ETOOLARGE case).
World lines stay on the device from a job's first sweep to its last.
Each job's results equal its alone-run bit for bit: the batch changes the
schedule, never the arithmetic.

The admission policy is plain host logic (Admission); Server drives the GPU.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import Batch, Chain, lc_footprint_parts


class Admission:
    """Footprint accounting.  A resident job holds its world-line state; the
    per-sweep scratch of all resident jobs lives in one arena of the batch,
    which grows with headroom (up to a quarter more than the largest need it
    has seen, plus 1/16) and does not shrink while the batch lives.  A job is
    admitted only if the resident states, its own state and the larger of
    the arena's current size and the grown scratch of all resident jobs with
    it stay within the budget."""

    GROWTH = 1.25 * 17 / 16

    def __init__(self, budget_bytes: int, max_resident: int = 512):
        self.budget = int(budget_bytes)
        self.max_resident = int(max_resident)
        self.state = 0
        self.scratch = 0
        self.resident = 0

    @property
    def used(self) -> int:
        return self.state + self.scratch

    def need(self, state: int, scratch: int, arena_bytes: int = 0) -> float:
        return self.state + state + max(float(arena_bytes), self.GROWTH * (self.scratch + scratch))

    def fits_ever(self, state: int, scratch: int = 0) -> bool:
        return state + self.GROWTH * scratch <= self.budget

    def try_admit(self, state: int, scratch: int = 0, arena_bytes: int = 0) -> bool:
        if self.resident >= self.max_resident or self.need(state, scratch, arena_bytes) > self.budget:
            return False
        self.state += state
        self.scratch += scratch
        self.resident += 1
        return True

    def release(self, state: int, scratch: int = 0):
        self.state -= state
        self.scratch -= scratch
        self.resident -= 1


def job_bytes(job) -> int:
    st, sc = lc_footprint_parts(job.L, job.S, job.beta)
    return st + sc


def job_parts(job) -> tuple:
    """(world-line state bytes, per-sweep scratch bytes) of a job."""
    return lc_footprint_parts(job.L, job.S, job.beta)


@dataclass
class JobRecord:
    job_id: int
    arrival: float
    admitted: float
    finished: float
    sweeps: int
    ops: float
    measurement: dict
    final_state: tuple = field(repr=False, default=None)


@dataclass
class Report:
    records: list
    rejected: list
    sweep_latency_s: list
    iterations: int
    busy_s: float
    wall_s: float
    ops: float

    def summary(self) -> dict:
        lat = np.array(self.sweep_latency_s) if self.sweep_latency_s else np.zeros(1)
        turn = np.array([r.finished - r.arrival for r in self.records]) if self.records else np.zeros(1)
        wait = np.array([r.admitted - r.arrival for r in self.records]) if self.records else np.zeros(1)
        return {
            "jobs_done": len(self.records),
            "jobs_rejected": len(self.rejected),
            "iterations": self.iterations,
            "sweep_latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
            "sweep_latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
            "job_turnaround_s_p50": float(np.percentile(turn, 50)),
            "job_turnaround_s_p99": float(np.percentile(turn, 99)),
            "queue_wait_s_p50": float(np.percentile(wait, 50)),
            "ops_per_s_busy": self.ops / self.busy_s if self.busy_s > 0 else 0.0,
            "ops_per_s_wall": self.ops / self.wall_s if self.wall_s > 0 else 0.0,
            "busy_fraction": self.busy_s / self.wall_s if self.wall_s > 0 else 0.0,
        }


class Server:
    """Continuous batching of jobs on one GPU stream."""

    def __init__(self, budget_bytes: int, max_resident: int = 512, stream=None,
                 keep_states: bool = False):
        self.adm = Admission(budget_bytes, max_resident)
        self.stream = stream
        self.keep_states = keep_states

    def run(self, jobs, log=None) -> Report:
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        waiting = deque()
        resident = {}  # job_id -> [job, chain, done, nbytes, admitted, ops]
        records, rejected, lat = [], [], []
        batch = Batch(self.stream)
        busy, ops_total, iters = 0.0, 0.0, 0
        t0 = time.perf_counter()
        try:
            while pending or waiting or resident:
                now = time.perf_counter() - t0
                while pending and pending[0].arrival <= now:
                    waiting.append(pending.popleft())
                # admission: first fit over the arrived jobs, oldest first
                for job in list(waiting):
                    nb = job_parts(job)
                    if not self.adm.fits_ever(*nb):
                        waiting.remove(job)
                        rejected.append(job)
                        if log:
                            log(f"reject job {job.job_id}: {sum(nb) / 2**30:.1f} GiB")
                        continue
                    if self.adm.try_admit(*nb, arena_bytes=batch.scratch_bytes()):
                        waiting.remove(job)
                        c = Chain(job.L, job.S, job.beta, job.seed, stream=self.stream)
                        batch.add(c)
                        resident[job.job_id] = [job, c, 0, nb, time.perf_counter() - t0, 0.0]
                if not resident:
                    if batch.scratch_bytes():
                        # an empty batch gives its scratch arena back
                        batch.close()
                        batch = Batch(self.stream)
                    if pending:
                        time.sleep(max(0.0, min(0.05, pending[0].arrival - now)))
                    continue
                ts = time.perf_counter()
                batch.update(1, accumulate=True)
                dt = time.perf_counter() - ts
                busy += dt
                iters += 1
                for jid in list(resident):
                    rec = resident[jid]
                    job, c = rec[0], rec[1]
                    rec[2] += 1
                    n = c.last_sweep()["n_ops"]
                    rec[5] += n
                    ops_total += n
                    lat.append(dt)
                    if rec[2] >= job.sweeps:
                        batch.remove(c)
                        st = c.export_state() if self.keep_states else None
                        records.append(JobRecord(jid, job.arrival, rec[4], time.perf_counter() - t0,
                                                 rec[2], rec[5], c.measure(), st))
                        c.close()
                        self.adm.release(*rec[3])
                        del resident[jid]
                        if log:
                            log(f"job {jid} done after {rec[2]} sweeps")
        finally:
            for rec in resident.values():
                rec[1].close()
            batch.close()
        return Report(records, rejected, lat, iters, busy, time.perf_counter() - t0, ops_total)


def run_alone(job, stream=None, keep_state: bool = True):
    """The same job run by itself (lc_update): (measurement, final state)."""
    c = Chain(job.L, job.S, job.beta, job.seed, stream=stream)
    try:
        c.update(job.sweeps, accumulate=True)
        return c.measure(), (c.export_state() if keep_state else None)
    finally:
        c.close()
