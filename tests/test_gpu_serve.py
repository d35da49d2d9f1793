"""Serving: jobs admitted by footprint into one continuously re-formed batch
give, job by job, the same world lines and measurements as alone-runs."""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1810_07485_amd as lc
    lc.load()
    return lc


def test_each_job_same_alone_and_in_the_mix(lc):
    from paper_1810_07485_amd import serve, workloads
    jobs = workloads.serving_jobs(12, rate=40.0, L_choices=(16, 48, 128), S_choices=(0.5, 2.0),
                                  sweep_choices=(3, 9))
    big = dataclasses.replace(jobs[0], job_id=99, L=1 << 20, S=4.0, beta=float(1 << 20))
    sizes = [serve.job_bytes(j) for j in jobs]
    budget = max(sizes) * 3  # a few jobs at a time: later arrivals wait
    srv = serve.Server(budget, keep_states=True)
    rep = srv.run(jobs + [big])
    assert [j.job_id for j in rep.rejected] == [99]
    assert sorted(r.job_id for r in rep.records) == [j.job_id for j in jobs]
    assert rep.iterations > max(j.sweeps for j in jobs)
    for r in rep.records:
        job = jobs[r.job_id]
        m, st = serve.run_alone(job)
        assert r.sweeps == job.sweeps
        assert r.measurement == m, job
        for x, y in zip(r.final_state, st):
            np.testing.assert_array_equal(np.asarray(x), np.asarray(y))
    sm = rep.summary()
    assert sm["jobs_done"] == 12 and sm["jobs_rejected"] == 1
    assert sm["sweep_latency_ms_p99"] >= sm["sweep_latency_ms_p50"] > 0


def _sha(arrays):
    import hashlib
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_mix_with_split_spin_jobs_matches_oracle(lc, orc):
    """An S=4 job (8 subspins per spin, symmetrization; L=1024, beta=512) and
    an S=1/2 job (L=1024, beta=1024) served in a mix with smaller S=1/2 and
    S=2 jobs: their final world lines and measurements equal the oracle's
    (digests written by tests/golden/make_digest_golden.py from the oracle
    alone, three sweeps each)."""
    import json
    import os
    from paper_1810_07485_amd import serve, workloads
    gold_dir = os.path.join(os.path.dirname(__file__), "golden")
    jobs = workloads.serving_jobs(8, rate=40.0, L_choices=(16, 48, 128), S_choices=(0.5, 2.0, 4.0),
                                  sweep_choices=(3, 9))
    t = jobs[2].arrival
    extra = [workloads.Job(100, t, 1024, 4.0, 512.0, 3, 2001),
             workloads.Job(101, t, 1024, 0.5, 1024.0, 3, 2002)]
    gold = {}
    for j, name in zip(extra, ("digest_L1024_S4_beta512_seed2001.json",
                               "digest_L1024_beta1024_seed2002.json")):
        with open(os.path.join(gold_dir, name)) as f:
            gold[j.job_id] = json.load(f)
    sizes = [serve.job_bytes(j) for j in jobs + extra]
    srv = serve.Server(sum(sizes) * 2, keep_states=True)
    rep = srv.run(jobs + extra)
    assert not rep.rejected
    recs = {r.job_id: r for r in rep.records}
    assert any(j.S == 4.0 for j in jobs)
    for j in extra:
        g = gold[j.job_id]
        assert (g["L"], g["S"], g["beta"], g["seed"]) == (j.L, j.S, j.beta, j.seed)
        r = recs[j.job_id]
        assert _sha(r.final_state[:3]) == g["sweeps"][2]["state"], j
        stats = [s["stats"] for s in g["sweeps"][:3]]
        ref = orc.observables(stats, j.L, j.S, j.beta)
        for k in ("e", "chi_u", "chi_u_plain", "s_pi", "chi_s"):
            a, b = r.measurement[k], ref[k]
            assert a == b or abs(a - b) <= 1e-12 * max(abs(a), abs(b)), (j.job_id, k, a, b)
    for r in rep.records:
        if r.job_id in gold:
            continue
        m, st = serve.run_alone(jobs[r.job_id])
        assert r.measurement == m
        for x, y in zip(r.final_state, st):
            np.testing.assert_array_equal(np.asarray(x), np.asarray(y))
