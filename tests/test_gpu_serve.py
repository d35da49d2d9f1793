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
