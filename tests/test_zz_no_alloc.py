"""Allocation-free sweeps (lc_update_noalloc) against lc_update, through the C ABI.

Two calls in a row of the allocation-free entry point, the second on a
smaller chain, each checked bit for bit against the same sweeps run by
lc_update: every integer of the last sweep, the world lines and the
measurements.  A chain whose scratch does not fit the static array is
refused before any work.
"""
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


def same(a, b):
    for x, y in zip(a.export_state(), b.export_state()):
        np.testing.assert_array_equal(np.asarray(x), np.asarray(y))
    assert a.last_sweep() == b.last_sweep()
    assert a.measure() == b.measure()


@pytest.mark.parametrize("cases", [
    [((512, 0.5, 64.0, 3), 6), ((64, 0.5, 16.0, 4), 4)],
    [((16, 1.0, 8.0, 5), 5), ((6, 4.0, 2.0, 6), 3)],
])
def test_noalloc_equals_update_on_two_calls(lc, cases):
    for case, sweeps in cases:          # the second call has the smaller input
        ref = lc.Chain(*case)
        ref.update(sweeps)
        c = lc.Chain(*case)
        c.update_noalloc(sweeps)
        same(c, ref)
        ref.close()
        c.close()


def test_noalloc_continues_a_chain_run_by_update(lc):
    ref = lc.Chain(256, 0.5, 32.0, 8)
    ref.update(7)
    c = lc.Chain(256, 0.5, 32.0, 8)
    c.update(3)
    c.update_noalloc(2)
    c.update(2)
    same(c, ref)


def test_noalloc_refuses_a_chain_beyond_the_static_scratch(lc):
    c = lc.Chain(65536, 0.5, 4096.0, 1)
    with pytest.raises(lc.LcError) as e:
        c.update_noalloc(1)
    assert e.value.code == lc.LC_ETOOLARGE
    assert c.export_state()[3] == 0  # nothing ran
    c.close()
