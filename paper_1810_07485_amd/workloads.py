"""Seeded synthetic workloads: lattices and job streams, no method arithmetic.

The method's inputs are lattices (L, S, beta, seed); there is no dataset.
These generators fix the instance sets used by the batching and serving
benchmarks and their tests.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

BATCH_RNG_SEED = 20181017
SERVE_RNG_SEED = 20181018


@dataclass(frozen=True)
class Instance:
    L: int
    S: float
    beta: float
    seed: int


def batch_instances(n: int = 512, rng_seed: int = BATCH_RNG_SEED, L_min: int = 64,
                    L_max: int = 16384) -> list:
    """Independent S=1/2 chains of uneven size: L log-uniform in [L_min, L_max]
    rounded to an even value, beta uniform in [L/4, L], seed 1 + i."""
    rng = np.random.default_rng(rng_seed)
    u = rng.uniform(np.log(L_min), np.log(L_max), n)
    L = np.maximum(4, 2 * np.round(np.exp(u) / 2).astype(np.int64))
    beta = rng.uniform(L / 4.0, L)
    return [Instance(int(L[i]), 0.5, float(beta[i]), 1 + i) for i in range(n)]


@dataclass(frozen=True)
class Job:
    job_id: int
    arrival: float   # seconds after the start of the stream
    L: int
    S: float
    beta: float
    sweeps: int
    seed: int


def serving_jobs(n: int = 200, rate: float = 1.0, rng_seed: int = SERVE_RNG_SEED,
                 L_choices=(1024, 4096, 16384), S_choices=(0.5, 4.0),
                 sweep_choices=(100, 1000)) -> list:
    """A Poisson stream of simulation jobs: exponential inter-arrival times of
    mean 1/rate; S, L, beta in {L/2, L} and the sweep count drawn uniformly
    from the choices; job seed 1000 + id."""
    rng = np.random.default_rng(rng_seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    jobs = []
    for i in range(n):
        S = float(S_choices[rng.integers(len(S_choices))])
        L = int(L_choices[rng.integers(len(L_choices))])
        beta = float(L) / (2.0 if rng.integers(2) == 0 else 1.0)
        sw = int(sweep_choices[rng.integers(len(sweep_choices))])
        jobs.append(Job(i, float(t[i]), L, S, beta, sw, 1000 + i))
    return jobs
