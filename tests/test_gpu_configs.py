"""Parity of the HIP path with the oracle on the benchmark configurations.

- The tiny chain (L=16, beta=8, seed 1) for its full run of 1,000
  thermalisation and 10,000 measurement sweeps: every integer of every sweep,
  the world lines every 100 sweeps, the FP64 observables of lc_measure against
  the oracle's (1e-12 relative), and energy and susceptibility against exact
  diagonalization (3 sigma).
- lc_measure against the oracle's observables for split spins.
- Small persistent grids (7 and 64 workgroups, graph and direct launches),
  alone and in a batch: every thread walks many windows, nodes and chains.
- The largest window count of the benchmark sizes (w = 11, beta = 16,384).
"""
import json
import math
import os

import numpy as np
import pytest

from tests.test_gpu_parity import compare_sweep

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
OBS = ("e", "chi_u", "chi_u_plain", "s_pi", "chi_s")


@pytest.fixture(scope="module")
def lc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1810_07485_amd as lc
    lc.load()
    return lc


def close_rel(a, b, rel=1e-12):
    return a == b or abs(a - b) <= rel * max(abs(a), abs(b))


def check_measure(g, stats, orc, L, S, beta):
    m = g.measure()
    ref = orc.observables(stats, L, S, beta)
    assert m["n_sweeps"] == len(stats)
    for k in OBS:
        assert close_rel(m[k], ref[k]), (k, m[k], ref[k])
    assert close_rel(m["mean_ops"], sum(s["n_ops"] for s in stats) / len(stats))


def test_tiny_chain_full_run(lc, orc):
    L, S, beta, seed = 16, 0.5, 8.0, 1
    g = lc.Chain(L, S, beta, seed)
    o = orc.Chain(L, S, beta, seed)
    meas = []
    for s in range(11000):
        acc = s >= 1000
        g.update(1, accumulate=acc)
        gst, ost = g.last_sweep(), o.sweep()
        assert gst == ost, (s, gst, ost)
        if acc:
            meas.append(ost)
        if s % 100 == 99:
            for x, y in zip(g.export_state(), o.export_state()):
                np.testing.assert_array_equal(np.asarray(x), np.asarray(y), err_msg=f"sweep {s}")
            np.testing.assert_array_equal(g.export_labels(), o.export_labels(), err_msg=f"sweep {s}")
    check_measure(g, meas, orc, L, S, beta)
    # exact diagonalization: energy and uniform susceptibility within 3 sigma
    with open(os.path.join(GOLD, "ed_golden.json")) as f:
        ref = next(c for c in json.load(f)["cases"]
                   if c["L"] == L and c["S"] == S and c["beta"] == beta)
    e = np.array([0.25 - s["n_ops"] / (beta * L) for s in meas])
    chi = np.array([beta / (4 * L) * s["sum_m2"] for s in meas])
    for k, x in (("e", e), ("chi_u", chi)):
        b = x.reshape(40, -1).mean(1)
        mu, err = b.mean(), b.std(ddof=1) / math.sqrt(len(b))
        assert abs(mu - ref[k]) < 3 * err, (k, mu, err, ref[k])
    m = g.measure()
    assert close_rel(m["e"], float(e.mean()), 1e-12)


@pytest.mark.parametrize("L,S,beta,seed,sweeps", [
    (64, 0.5, 16.0, 3, 200), (8, 1.0, 4.0, 4, 200), (4, 4.0, 1.0, 5, 100), (6, 1.5, 3.0, 6, 100)])
def test_measure_matches_oracle_observables(lc, orc, L, S, beta, seed, sweeps):
    g = lc.Chain(L, S, beta, seed)
    o = orc.Chain(L, S, beta, seed)
    stats = []
    for s in range(sweeps):
        g.update(1, accumulate=True)
        ost = o.sweep()
        assert g.last_sweep() == ost, s
        stats.append(ost)
    check_measure(g, stats, orc, L, S, beta)
    g.reset_measurements()
    assert g.measure()["n_sweeps"] == 0


@pytest.mark.parametrize("grid,graph", [(7, True), (7, False), (64, True), (64, False)])
def test_small_grids_lockstep(lc, orc, grid, graph):
    """Few resident workgroups: each thread's grid-stride loop runs many
    iterations over windows and nodes, and large loops meet the wave carry of
    the per-loop accumulation."""
    L, S, beta, seed = 512, 0.5, 512.0, 31
    g = lc.Chain(L, S, beta, seed)
    g.set_schedule(grid, graph)
    o = orc.Chain(L, S, beta, seed)
    for s in range(4):
        g.update(1)
        compare_sweep(g, o, g.last_sweep(), o.sweep(), tag=f"grid {grid} sweep {s}")


def test_small_grid_batch_lockstep(lc, orc):
    """A batch at grid 7: threads move between chains of different S inside
    their loops (per-lane flushes of partial sums)."""
    cases = [(64, 0.5, 64.0, 41), (8, 1.0, 16.5, 42), (130, 0.5, 100.5, 43), (4, 4.0, 1.0, 44),
             (256, 0.5, 40.0, 45), (6, 1.5, 3.0, 46)]
    b = lc.Batch()
    b.set_schedule(7, True)
    gs = [lc.Chain(*c) for c in cases]
    os_ = [orc.Chain(*c) for c in cases]
    for c in gs:
        b.add(c)
    for s in range(5):
        b.update(1)
        for c, (g, o) in enumerate(zip(gs, os_)):
            compare_sweep(g, o, g.last_sweep(), o.sweep(), tag=f"member {c} sweep {s}")
    b.close()


def test_largest_window_count(lc, orc):
    """beta = 16,384 gives 2^11 windows per bond, as in the largest chain."""
    L, S, beta, seed = 64, 0.5, 16384.0, 1
    w, _, _ = lc.lc_debug_window_table(beta)
    assert w == 11
    g = lc.Chain(L, S, beta, seed)
    o = orc.Chain(L, S, beta, seed)
    for s in range(3):
        g.update(1)
        compare_sweep(g, o, g.last_sweep(), o.sweep(), tag=f"w=11 sweep {s}")


@pytest.mark.parametrize("L,S,beta,seed,shape", [
    (1024, 0.5, 256.0, 3, (1, 300)),     # one window per tile, small tiles
    (1024, 0.5, 256.0, 3, (16, 1700)),   # sixteen windows per tile
    (1024, 0.5, 256.0, 3, (2, 64)),      # the smallest target
    (64, 0.5, 64.0, 6, (8, 1500)),
    (8, 1.0, 16.5, 4, (2, 200)),         # split spins, two windows per tile
    (16, 4.0, 9.0, 5, (4, 1500)),        # S = 4: (2S)^2 x windows bounded by the lists
    (8, 4.0, 64.0, 2, (2, 1400)),        # S = 4, two windows: the times of the bonds the tile
                                         # does not own mostly overflow the LDS, so the walk
                                         # places events by binary searches
])
def test_tile_shapes_lockstep(lc, orc, L, S, beta, seed, shape):
    """The linking-tile shape is schedule only: every sweep equals the
    oracle's under any shape lc_set_tile accepts."""
    g = lc.Chain(L, S, beta, seed)
    g.set_tile(*shape)
    o = orc.Chain(L, S, beta, seed)
    for s in range(3):
        g.update(1)
        compare_sweep(g, o, g.last_sweep(), o.sweep(), tag=f"shape {shape} sweep {s}")


def test_tile_autotune_keeps_results(lc):
    shapes, grids = ((0, 0), (1, 400), (8, 1500)), (128, 512)
    a, b = lc.Chain(256, 0.5, 64.0, 7), lc.Chain(256, 0.5, 64.0, 7)
    shape, grid, ms = a.autotune_tiles(shapes, grids, trial_sweeps=1)
    assert shape in shapes and grid in grids and ms > 0
    b.update(len(shapes) * len(grids) * 2)
    for x, y in zip(a.export_state(), b.export_state()):
        np.testing.assert_array_equal(np.asarray(x), np.asarray(y))
    assert a.last_sweep() == b.last_sweep()
    with pytest.raises(lc.LcError):
        a.set_tile(3, 0)        # not a power of two
    with pytest.raises(lc.LcError):
        a.set_tile(4, 5000)     # beyond the LDS capacity
