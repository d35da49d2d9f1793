"""Degenerate inputs and error paths of the C ABI, on the GPU.

World lines without any operator (every loop is a straight line from tau = 0
to beta, so the first sweep inserts diagonal operators only into an empty
list) run in lockstep with the oracle.  Invalid calls return their documented
LC_E* code and leave the chain as it was.
"""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LC_EINVAL, LC_ECAPACITY, LC_ESTATE = -1, -4, -6


@pytest.fixture(scope="module")
def lc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1810_07485_amd as lc
    lc.load()
    return lc


def _same_state(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("L,S,beta,seed", [
    (8, 0.5, 4.0, 21),
    (130, 0.5, 64.0, 22),   # 8 windows per bond, ragged tile tail
    (6, 1.0, 3.0, 23),      # split spins: symmetrization of an empty list
    (4, 4.0, 2.0, 24),
])
def test_empty_world_lines_lockstep(lc, orc, L, S, beta, seed):
    g = lc.Chain(L, S, beta, seed)
    o = orc.Chain(L, S, beta, seed)
    n_sites = int(round(2 * S)) * L
    s0 = (np.arange(n_sites) % 2).astype(np.uint8)
    off = np.zeros(g.n_bonds + 1, np.int64)
    empty = np.zeros(0, np.uint64)
    g.import_state(s0, off, empty, 3)
    o.import_state(s0, off, empty, 3)
    _same_state(g.export_state(), o.export_state())
    for s in range(4):
        g.update(1)
        gst, ost = g.last_sweep(), o.sweep()
        for k, v in ost.items():
            assert gst[k] == v, (L, S, s, k, gst[k], v)
        _same_state(g.export_state(), o.export_state())
        np.testing.assert_array_equal(g.export_labels(), o.export_labels())


def test_error_codes_leave_the_chain_unchanged(lc):
    lib = lc.load()
    c = lc.Chain(64, 0.5, 16.0, 31)
    n = C.c_int64(0)
    with pytest.raises(lc.LcError) as e:
        c.last_sweep()                       # no sweep yet
    assert e.value.code == LC_ESTATE
    with pytest.raises(lc.LcError) as e:
        c.export_ops()
    assert e.value.code == LC_ESTATE

    c.update(3)
    before = c.export_state()
    s0, off, t, sw = before
    assert t.size > 1

    # a too-small times buffer: LC_ECAPACITY, the needed count written back
    small = np.zeros(1, np.uint64)
    n = C.c_int64(small.size)
    sw_out = C.c_int64()
    rc = lib.lc_export_state(c._h, None, None, small.ctypes.data_as(C.POINTER(C.c_uint64)),
                             C.byref(n), C.byref(sw_out))
    assert rc == LC_ECAPACITY and n.value == t.size and sw_out.value == sw

    bad_times = t.copy()
    b = int(np.argmax(np.diff(off) >= 2))    # a bond with two operators
    assert off[b + 1] - off[b] >= 2
    i = off[b]
    bad_times[i], bad_times[i + 1] = t[i + 1], t[i]
    if bad_times[i] != bad_times[i + 1]:
        with pytest.raises(lc.LcError) as e:
            c.import_state(s0, off, bad_times, sw)      # unsorted within a bond
        assert e.value.code == LC_EINVAL
    bad_off = off.copy()
    bad_off[0] = 1
    with pytest.raises(lc.LcError) as e:
        c.import_state(s0, bad_off, t, sw)
    assert e.value.code == LC_EINVAL
    bad_s0 = s0.copy()
    bad_s0[0] = 2
    with pytest.raises(lc.LcError) as e:
        c.import_state(bad_s0, off, t, sw)
    assert e.value.code == LC_EINVAL
    with pytest.raises(lc.LcError) as e:
        c.import_state(s0, off, t, -1)
    assert e.value.code == LC_EINVAL
    # operators announced by the offsets but no times array
    rc = lib.lc_import_state(c._h, s0.ctypes.data_as(C.POINTER(C.c_uint8)),
                             off.ctypes.data_as(C.POINTER(C.c_int64)), None, sw)
    assert rc == LC_EINVAL
    _same_state(c.export_state(), before)

    # a chain that belongs to a batch cannot be updated alone
    bt = lc.Batch()
    bt.add(c)
    with pytest.raises(lc.LcError) as e:
        c.update(1)
    assert e.value.code == LC_ESTATE
    bt.remove(c)
    c.update(1)
    bt.close()
    c.close()
