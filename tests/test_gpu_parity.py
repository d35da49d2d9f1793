"""Parity of the HIP path against the CPU oracle, through the C ABI.

After every sweep the world lines (spins at tau = 0+, kept operators), the
operators of the sweep with their types before and after the flip, the loop
labels and every integer of the sweep statistics must be bit-identical.
Sizes span many (bond, window) tiles with ragged tails; the split-spin
cases cover the symmetrization.
"""
import os

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


def compare_sweep(g, o, gst, ost, check_labels=True, tag=""):
    for k, v in ost.items():
        assert gst[k] == v, (tag, k, gst[k], v)
    gs0, goff, gt, gsw = g.export_state()
    os0, ooff, ot, osw = o.export_state()
    assert gsw == osw, tag
    np.testing.assert_array_equal(gs0, os0, err_msg=f"{tag} s0")
    np.testing.assert_array_equal(goff, ooff, err_msg=f"{tag} bond offsets")
    np.testing.assert_array_equal(gt, ot, err_msg=f"{tag} kept times")
    gb, gtm, gty0, gty1 = g.export_ops()
    ob, otm, oty0 = o.export_ops()
    np.testing.assert_array_equal(gb, ob, err_msg=f"{tag} op bonds")
    np.testing.assert_array_equal(gtm, otm, err_msg=f"{tag} op times")
    np.testing.assert_array_equal(gty0, oty0, err_msg=f"{tag} op types")
    if check_labels:
        np.testing.assert_array_equal(g.export_labels(), o.export_labels(), err_msg=f"{tag} labels")
        if g.two_s > 1:
            np.testing.assert_array_equal(g.export_perm(), o.export_perm(), err_msg=f"{tag} perm")


def lockstep(lc, orc, L, S, beta, seed, sweeps, check_labels=True):
    g = lc.Chain(L, S, beta, seed)
    o = orc.Chain(L, S, beta, seed)
    for s in range(sweeps):
        g.update(1)
        gst = g.last_sweep()
        ost = o.sweep()
        compare_sweep(g, o, gst, ost, check_labels, tag=f"L={L} S={S} beta={beta} sweep {s}")
    return g, o


@pytest.mark.parametrize("L,S,beta,seed,sweeps", [
    (16, 0.5, 8.0, 1, 30),        # the tiny benchmark instance
    (4, 0.5, 0.3, 2, 20),         # smallest chain, w = 0, mostly empty sites
    (6, 0.5, 2.0, 3, 20),
    (64, 0.5, 64.0, 4, 10),       # 8 windows per bond
    (130, 0.5, 100.5, 5, 8),      # non-power-of-two beta, ragged
    (512, 0.5, 37.0, 6, 5),
])
def test_parity_spin_half(lc, orc, L, S, beta, seed, sweeps):
    lockstep(lc, orc, L, S, beta, seed, sweeps)


@pytest.mark.parametrize("L,S,beta,seed,sweeps", [
    (4, 1.0, 2.0, 7, 10),
    (8, 1.0, 16.5, 8, 6),
    (6, 1.5, 3.0, 9, 6),
    (4, 4.0, 1.0, 10, 6),
    (6, 4.0, 9.0, 11, 3),
    (16, 1.0, 31.5, 12, 4),      # mean 3.9 candidates per window: some windows exceed 8
    (12, 2.0, 15.5, 13, 3),
])
def test_parity_split_spin(lc, orc, L, S, beta, seed, sweeps):
    lockstep(lc, orc, L, S, beta, seed, sweeps)


def test_parity_medium_many_tiles(lc, orc):
    """L=4096, beta=256: ~7e5 operators per sweep, 32 windows per bond."""
    lockstep(lc, orc, 4096, 0.5, 256.0, 12, 3)


def test_parity_crafted_ties(lc, orc):
    """Operators at equal times on bonds sharing a site (ordered by bond)."""
    L = 8
    s0 = np.array([1, 0, 0, 1, 0, 1, 0, 1], np.uint8)
    t1, t2, t3 = 1 << 61, 1 << 62, (1 << 63) + 5
    ops = {0: [t1, t3], 1: [t1, t2]}
    off = np.zeros(L + 1, np.int64)
    times = []
    for b in range(L):
        times += ops.get(b, [])
        off[b + 1] = len(times)
    times = np.array(times, np.uint64)
    g = lc.Chain(L, 0.5, 4.0, 3)
    o = orc.Chain(L, 0.5, 4.0, 3)
    g.import_state(s0, off, times, 10)
    o.import_state(s0, off, times, 10)
    for s in range(4):
        g.update(1)
        compare_sweep(g, o, g.last_sweep(), o.sweep(), tag=f"ties sweep {s}")


def test_checkpoint_resume_bit_exact(lc):
    """export -> import into a fresh chain -> continue == uninterrupted run."""
    a = lc.Chain(256, 0.5, 32.0, 77)
    a.update(5)
    st = a.export_state()
    b = lc.Chain(256, 0.5, 32.0, 77)
    b.import_state(*st)
    a.update(4)
    b.update(4)
    for x, y in zip(a.export_state(), b.export_state()):
        np.testing.assert_array_equal(x, y)
    assert a.last_sweep() == b.last_sweep()


def test_graph_and_direct_launch_agree(lc):
    """Graph replay and direct launches, several grid sizes: same bits."""
    ref = None
    for grid, graph in ((0, True), (0, False), (7, True), (300, False)):
        c = lc.Chain(1000, 0.5, 50.0, 5)
        c.set_schedule(grid, graph)
        c.update(6)
        st = c.export_state()
        if ref is None:
            ref = st
        else:
            for x, y in zip(ref, st):
                np.testing.assert_array_equal(x, y)
