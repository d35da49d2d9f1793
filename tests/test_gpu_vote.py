"""Majority-vote flip rule (Sec. 3.3) on the GPU, in lockstep with the oracle.

Under LC_FLIP_VOTE every loop-graph node votes and a loop flips iff the XOR
of its nodes' votes is 1: the tally runs in the linking tiles (loops closed
there), in the fragments and the loop records (open loops) and is read back
by the flip kernels.  Every integer, the world lines, operators and labels
must equal the oracle's in its vote mode, alone, in a batch with chains of
the other rule, and through the allocation-free entry point.
"""
import pytest

from tests.test_gpu_parity import compare_sweep

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1810_07485_amd as lc
    lc.load()
    return lc


def pair(lc, orc, case, vote=True):
    g = lc.Chain(*case)
    o = orc.Chain(*case)
    if vote:
        g.set_flip_rule(lc.FLIP_VOTE)
        o.set_flip_rule(orc.FLIP_VOTE)
    return g, o


@pytest.mark.parametrize("L,S,beta,seed,sweeps", [
    (16, 0.5, 8.0, 1, 20), (512, 0.5, 37.0, 2, 5), (1024, 0.5, 256.0, 3, 3),
    (8, 1.0, 16.5, 4, 6), (6, 4.0, 9.0, 5, 3), (6, 1.5, 3.0, 6, 6)])
def test_vote_rule_lockstep(lc, orc, L, S, beta, seed, sweeps):
    g, o = pair(lc, orc, (L, S, beta, seed))
    for s in range(sweeps):
        g.update(1)
        compare_sweep(g, o, g.last_sweep(), o.sweep(), tag=f"vote L={L} S={S} sweep {s}")


def test_vote_and_label_rules_in_one_batch(lc, orc):
    cases = [((64, 0.5, 64.0, 11), True), ((64, 0.5, 64.0, 11), False), ((8, 1.0, 16.5, 12), True),
             ((256, 0.5, 40.0, 13), False)]
    b = lc.Batch()
    gs, os_ = [], []
    for case, vote in cases:
        g, o = pair(lc, orc, case, vote)
        b.add(g)
        gs.append(g)
        os_.append(o)
    for s in range(4):
        b.update(1)
        for i, (g, o) in enumerate(zip(gs, os_)):
            compare_sweep(g, o, g.last_sweep(), o.sweep(), tag=f"member {i} sweep {s}")
    b.close()


def test_vote_rule_allocation_free(lc, orc):
    g, o = pair(lc, orc, (256, 0.5, 32.0, 21))
    g.update_noalloc(5)
    for _ in range(5):
        ost = o.sweep()
    assert g.last_sweep() == ost
    for x, y in zip(g.export_state(), o.export_state()):
        assert (x == y).all() if hasattr(x, "all") else x == y
