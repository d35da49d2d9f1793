"""Batching: every member of a batch evolves exactly as it does alone.

Independent chains of uneven L, beta and S advanced by one launch sequence
per sweep must produce, chain by chain, the same world lines and the same
integers as when each runs alone; joining and leaving between sweeps (the
serving pattern) must not perturb the others.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CASES = [(16, 0.5, 8.0, 1), (64, 0.5, 64.0, 2), (130, 0.5, 100.5, 3), (1024, 0.5, 20.0, 4),
         (8, 1.0, 16.5, 5), (4, 4.0, 1.0, 6), (2048, 0.5, 512.0, 7), (6, 1.5, 3.0, 8)]


@pytest.fixture(scope="module")
def lc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1810_07485_amd as lc
    lc.load()
    return lc


def alone(lc, case, sweeps):
    c = lc.Chain(*case)
    stats = []
    for _ in range(sweeps):
        c.update(1)
        stats.append(c.last_sweep())
    return c.export_state(), stats, c.measure()


def same_state(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(np.asarray(x), np.asarray(y))


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_alone(lc, graph):
    sweeps = 6
    ref = [alone(lc, case, sweeps) for case in CASES]
    b = lc.Batch()
    b.set_schedule(0, graph)
    chains = [lc.Chain(*case) for case in CASES]
    for c in chains:
        b.add(c)
    stats = [[] for _ in chains]
    for _ in range(sweeps):
        b.update(1)
        for i, c in enumerate(chains):
            stats[i].append(c.last_sweep())
    for i, c in enumerate(chains):
        same_state(c.export_state(), ref[i][0])
        assert stats[i] == ref[i][1], CASES[i]
        assert c.measure() == ref[i][2]
    b.close()


def test_batch_multi_sweep_update(lc):
    """n sweeps in one call (one host synchronisation per chunk of sweeps)."""
    ref = [alone(lc, case, 9) for case in CASES[:4]]
    b = lc.Batch()
    chains = [lc.Chain(*case) for case in CASES[:4]]
    for c in chains:
        b.add(c)
    b.update(9)
    for i, c in enumerate(chains):
        same_state(c.export_state(), ref[i][0])
        assert c.last_sweep() == ref[i][1][-1]
    b.close()


def test_join_and_leave_between_sweeps(lc):
    """Chains join and leave a running batch; each matches its alone-run."""
    sweeps = {i: 4 + (i % 3) for i in range(len(CASES))}
    ref = {i: alone(lc, CASES[i], sweeps[i]) for i in sweeps}
    b = lc.Batch()
    chains = {i: lc.Chain(*CASES[i]) for i in sweeps}
    done = {i: 0 for i in sweeps}
    active = []
    pending = list(sweeps)
    step = 0
    while pending or active:
        # admit up to two new chains every other step
        if pending and step % 2 == 0:
            for _ in range(2):
                if pending:
                    i = pending.pop(0)
                    b.add(chains[i])
                    active.append(i)
        b.update(1)
        step += 1
        for i in list(active):
            done[i] += 1
            if done[i] == sweeps[i]:
                b.remove(chains[i])
                active.remove(i)
    for i in sweeps:
        same_state(chains[i].export_state(), ref[i][0])
        assert chains[i].last_sweep() == ref[i][1][-1]
        assert chains[i].measure() == ref[i][2]
    b.close()


def test_chain_alone_after_batch(lc):
    """A chain run in a batch, removed, then run alone continues exactly."""
    ref = alone(lc, CASES[3], 7)
    c = lc.Chain(*CASES[3])
    c.update(2)
    b = lc.Batch()
    b.add(c)
    b.update(3)
    b.remove(c)
    c.update(2)
    same_state(c.export_state(), ref[0])
    assert c.last_sweep() == ref[1][-1]
    b.close()


def test_footprint_packed_runner_with_autotune_equals_alone(lc):
    """Chains of the batching workload's distribution (smaller sizes): packed
    into several groups under a small scratch budget, each group autotuned;
    every chain ends where its alone-run does after the same sweep count."""
    from paper_1810_07485_amd import batching, workloads
    inst = workloads.batch_instances(24, L_min=16, L_max=512)
    specs = [(i.L, i.S, i.beta, i.seed) for i in inst]
    chains = [lc.Chain(*s) for s in specs]
    parts = [lc.lc_footprint_parts(*s[:3])[1] for s in specs]
    budget = max(parts) + sum(parts) // 5
    r = batching.BatchRunner(chains, budget)
    assert len(r.groups) >= 3 and sorted(sum(r.groups, [])) == list(range(24))
    tune = r.autotune((256, 1024), trial_sweeps=1)
    assert [g for g, _ in tune] == r.grids and set(r.grids) <= {256, 1024}
    r.update(3)
    n_sweeps = 2 * (1 + 1) + 3
    for s, c in zip(specs, chains):
        ref = lc.Chain(*s)
        ref.update(n_sweeps)
        same_state(c.export_state(), ref.export_state())
        assert c.last_sweep() == ref.last_sweep(), s
        ref.close()
    r.close()


def test_runner_tile_autotune_equals_alone(lc):
    """The packed runner choosing a linking-tile shape and a grid per group:
    every chain still ends where its alone-run does."""
    from paper_1810_07485_amd import batching, workloads
    inst = workloads.batch_instances(12, L_min=16, L_max=256)
    specs = [(i.L, i.S, i.beta, i.seed) for i in inst]
    chains = [lc.Chain(*s) for s in specs]
    parts = [lc.lc_footprint_parts(*s[:3])[1] for s in specs]
    r = batching.BatchRunner(chains, max(parts) + sum(parts) // 3)
    shapes, grids = ((0, 0), (1, 300), (16, 1500)), (128, 512)
    tune = r.autotune_tiles(shapes, grids, trial_sweeps=1)
    assert len(tune) == len(r.batches)
    assert all(sh in shapes and g in grids and ms > 0 for sh, g, ms in tune)
    r.update(2)
    n_sweeps = len(shapes) * len(grids) * 2 + 2
    for s, c in zip(specs, chains):
        ref = lc.Chain(*s)
        ref.update(n_sweeps)
        same_state(c.export_state(), ref.export_state())
        assert c.last_sweep() == ref.last_sweep(), s
        ref.close()
    r.close()


def test_chain_autotune_keeps_results(lc):
    a, b = lc.Chain(130, 0.5, 100.5, 3), lc.Chain(130, 0.5, 100.5, 3)
    best, ms = a.autotune((128, 512), trial_sweeps=2)
    assert best in (128, 512) and ms > 0
    b.update(2 * 3)
    same_state(a.export_state(), b.export_state())
    assert a.last_sweep() == b.last_sweep()


def test_exports_refuse_scratch_overwritten_by_another_engine(lc):
    """Engines on one stream share the per-sweep scratch: a chain's operator
    and label exports are refused once another engine has swept there."""
    a, b = lc.Chain(64, 0.5, 16.0, 1), lc.Chain(64, 0.5, 16.0, 2)
    a.update(1)
    n = len(a.export_labels())
    assert n == 64 + 2 * a.last_sweep()["n_ops"]
    b.update(1)
    with pytest.raises(lc.LcError):
        a.export_labels()
    with pytest.raises(lc.LcError):
        a.export_ops()
    a.update(1)
    assert len(a.export_ops()[0]) == a.last_sweep()["n_ops"]


def test_batch_workload_members_match_oracle_digests(lc):
    """All 512 chains of the batch workload run in footprint-packed batches;
    a sample of members (tests/golden/batch_members.json, written by the
    oracle alone) matches the oracle's digests after each of the first
    sweeps: every integer of the sweep and the world lines."""
    import hashlib
    import json
    import os

    import torch
    from paper_1810_07485_amd import batching, workloads

    path = os.path.join(os.path.dirname(__file__), "golden", "batch_members.json")
    with open(path) as f:
        gold = json.load(f)["members"]
    assert len(gold) >= 30
    inst = workloads.batch_instances()
    chains = [lc.Chain(i.L, i.S, i.beta, i.seed) for i in inst]
    runner = batching.BatchRunner(chains, 48 << 30)
    assert len(runner.batches) > 1 or len(chains) == 512
    nsw = min(len(m["sweeps"]) for m in gold)
    for s in range(nsw):
        runner.update(1)
        for m in gold:
            i = m["index"]
            assert (inst[i].L, inst[i].beta, inst[i].seed) == (m["L"], m["beta"], m["seed"])
            c = chains[i]
            rec = m["sweeps"][s]
            assert c.last_sweep() == rec["stats"], (i, s)
            h = hashlib.sha256()
            for a in c.export_state()[:3]:
                h.update(np.ascontiguousarray(a).tobytes())
            assert h.hexdigest() == rec["state"], (i, s)
    runner.close()
    for c in chains:
        c.close()
    torch.cuda.empty_cache()
