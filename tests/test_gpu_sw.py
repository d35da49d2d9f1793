"""Swendsen-Wang update of the 2D Ising model (Sec. 4.1) on the GPU union-find,
through the C ABI, against the oracle (sw_oracle.c): every sweep's integers
(energy, magnetization, active bonds, clusters, sum of squared sizes,
largest), the spins after it and its cluster labels, element by element.

Lattices span one tile (64 x 64 sites), ragged tiles (L not a multiple of
64), many tiles, and the degenerate couplings K = 0 (no bond) and K large
(p = 1: every bond between equal spins).  The full-size lattice the
benchmark times (L = 8192 at K_c) is compared whole for its first sweeps.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KC = math.log(1 + math.sqrt(2)) / 2


@pytest.fixture(scope="module")
def lc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1810_07485_amd as lc
    lc.load()
    return lc


def _compare(g, o, sweeps, every=1, tag=""):
    for s in range(sweeps):
        ref = o.sweep()
        g.update(1)
        assert g.last_sweep() == ref, f"{tag} sweep {s}"
        if s % every == 0 or s == sweeps - 1:
            np.testing.assert_array_equal(g.labels(), o.labels(), err_msg=f"{tag} sweep {s}")
            np.testing.assert_array_equal(g.spins(), o.spins(), err_msg=f"{tag} sweep {s}")


@pytest.mark.parametrize("L,K,seed,sweeps", [
    (2, KC, 1, 8),        # smallest lattice: both bonds of a site join the same pair
    (3, 0.6, 2, 8),
    (16, KC, 3, 20),      # part of one tile
    (64, KC, 4, 10),      # exactly one tile
    (65, 0.3, 5, 10),     # ragged: a 1-wide column and row of tiles
    (100, KC, 6, 10),
    (130, 0.8, 7, 6),
    (256, KC, 8, 6),      # 16 tiles
    (700, 0.5, 9, 3),
])
def test_sweeps_match_the_oracle(lc, orc, L, K, seed, sweeps):
    _compare(lc.SwIsing(L, K, seed), orc.SwChain(L, K, seed), sweeps, tag=f"L={L} K={K}")


@pytest.mark.parametrize("K", [0.0, 40.0])
def test_degenerate_couplings(lc, orc, K):
    L = 96
    g, o = lc.SwIsing(L, K, 21), orc.SwChain(L, K, 21)
    _compare(g, o, 4, tag=f"K={K}")
    st = g.last_sweep()
    if K == 0.0:
        assert st["n_active"] == 0 and st["n_clusters"] == L * L
    else:
        # p = 1: the clusters are the spin domains
        assert st["n_active"] > 0


def test_multi_sweep_update_equals_single_steps(lc, orc):
    """lc_sw_update(n) with n above the 64-sweep statistics ring."""
    L, K = 48, KC
    g, o = lc.SwIsing(L, K, 31), orc.SwChain(L, K, 31)
    g.update(150)
    for _ in range(150):
        ref = o.sweep()
    assert g.last_sweep() == ref
    np.testing.assert_array_equal(g.labels(), o.labels())
    np.testing.assert_array_equal(g.spins(), o.spins())


def test_full_size_lattice(lc, orc):
    """L = 8192 at K_c, the timed workload: first two sweeps whole."""
    L = 8192
    _compare(lc.SwIsing(L, KC, 7), orc.SwChain(L, KC, 7), 2, tag="L=8192")


def test_argument_checks(lc):
    for L, K in ((1, 0.4), (1 << 21, 0.4), (16, -1.0), (16, float("nan")), (16, float("inf"))):
        with pytest.raises(lc.LcError):
            lc.SwIsing(L, K, 1)
    g = lc.SwIsing(16, 0.4, 1)
    with pytest.raises(lc.LcError):
        g.last_sweep()
    with pytest.raises(lc.LcError):
        g.labels()
    with pytest.raises(lc.LcError):
        g.update(-1)
