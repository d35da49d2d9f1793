"""Parity at the benchmark's full size (L=65,536, beta=4,096), through the C ABI.

The oracle needs minutes per sweep at this size, so its results are stored
as digests written by tests/golden/make_digest_golden.py (which calls only
the oracle): every integer of each sweep's statistics and SHA-256 digests of
the world lines, the operators and the loop labels, for as many sweeps from
the Neel start as the stored file holds.  The library runs in the
launch configuration the benchmark times (graph replay, default grid).
A later, thermalised sweep is checked on sampled operators (spins just below
each sampled operator recomputed from the exported world lines) and on
identities that hold at any size.
"""
import hashlib
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "digest_L65536_beta4096.json")


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


@pytest.fixture(scope="module")
def lc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1810_07485_amd as lc
    lc.load()
    return lc


@pytest.fixture(scope="module")
def chain(lc):
    with open(GOLD) as f:
        g = json.load(f)
    c = lc.Chain(g["L"], g["S"], g["beta"], g["seed"])
    c.gold = g
    return c


def test_thresholds_match_golden(lc, chain):
    w, mu, T = lc.lc_debug_window_table(chain.gold["beta"])
    assert w == chain.gold["window_w"] and mu == chain.gold["mu"]
    assert [str(t) for t in T] == chain.gold["thresholds"]


with open(GOLD) as _f:
    N_GOLD = len(json.load(_f)["sweeps"])
CHUNK = 10


@pytest.mark.parametrize("chunk", range((N_GOLD + CHUNK - 1) // CHUNK))
def test_sweeps_bit_exact_against_oracle_digests(chain, chunk):
    """Every stored sweep, in chunks of ten (one test each, in order): all
    integers of the sweep and the world lines after it every sweep; the
    operators and the loop labels on sweeps 0-2, the first sweep of each
    chunk and the last one (their digests hash about 7 GB per sweep)."""
    recs = chain.gold["sweeps"]
    done = getattr(chain, "gold_done", 0)
    if done != chunk * CHUNK:
        pytest.skip("the chunks run in order, from the chain's start")
    for s in range(chunk * CHUNK, min(len(recs), (chunk + 1) * CHUNK)):
        rec = recs[s]
        chain.update(1)
        chain.gold_done = s + 1
        st = chain.last_sweep()
        assert st == rec["stats"], s
        s0, off, kt, sw = chain.export_state()
        assert sw == rec["next_sweep"]
        assert sha(s0, off, kt) == rec["state"], s
        if s < 3 or s % CHUNK == 0 or s == len(recs) - 1:
            b, t, ty0, _ = chain.export_ops()
            assert sha(b.astype(np.int64), t, ty0) == rec["ops"], s
            assert sha(chain.export_labels()) == rec["labels"], s


def test_thermalised_sweep_properties(chain):
    """After more sweeps: sampled operators sit on antiparallel spins before
    and after the flip, every site keeps an even number of jumps, and the
    node, loop and energy identities hold."""
    chain.update(12)
    s0, off, kt, sw = chain.export_state()
    chain.update(1)
    st = chain.last_sweep()
    b, t, ty0, ty1 = chain.export_ops()
    L = chain.L
    assert st["n_nodes"] == L + 2 * st["n_ops"]
    assert st["n_ops"] == st["n_kept_in"] + st["n_acc"]
    assert int(ty0.sum()) == st["n_kept_in"] and int(ty1.sum()) == st["n_kept_out"]
    # kept operators are exactly the previous world lines
    np.testing.assert_array_equal(t[ty0 == 1], kt)
    # operators ordered by (bond, time)
    assert (np.diff(b) >= 0).all()
    same = np.diff(b) == 0
    assert (np.diff(t)[same] >= 0).all()
    # even number of jumps on every site after the flip
    bk = b[ty1 == 1]
    par = np.bincount(bk, minlength=L) + np.bincount((bk + 1) % L, minlength=L)
    assert (par % 2 == 0).all()
    # sampled operators: spins of both ends just below them, from s0 and the
    # off-diagonal operators of the neighbouring bonds (before the flip)
    bounds = np.searchsorted(b, np.arange(L + 1))
    rng = np.random.default_rng(5)
    for k in rng.choice(len(b), 300, replace=False):
        bb, tt = int(b[k]), int(t[k])
        x, y = bb, (bb + 1) % L
        def par_before(bond):
            lo, hi = bounds[bond], bounds[bond + 1]
            tb, ob = t[lo:hi], ty0[lo:hi]
            n = np.searchsorted(tb, tt, side="left")
            cnt = int(ob[:n].sum())
            # equal times: earlier bond index comes first
            if bond < bb:
                n2 = np.searchsorted(tb, tt, side="right")
                cnt += int(ob[n:n2].sum())
            return cnt & 1
        sx = int(s0[x]) ^ par_before((bb - 1) % L)
        sy = int(s0[y]) ^ par_before((bb + 1) % L)
        assert sx != sy, k
    e = 0.25 - st["n_ops"] / (chain.beta * L)
    assert abs(e - (0.25 - np.log(2))) < 5e-3


def _antiparallel_below(s0, off, kt, L, idx):
    """For kept operators idx of world lines (s0, off, kt), whether the two
    spins just below each are antiparallel (operators of the same bond flip
    both ends and cancel; equal times order by bond index)."""
    b = np.searchsorted(off, idx, side="right") - 1
    out = np.empty(len(idx), dtype=bool)
    for n, (k, bb) in enumerate(zip(idx, b)):
        bb = int(bb)
        tt = kt[k]
        def par_before(bond):
            tb = kt[off[bond]:off[bond + 1]]
            cnt = int(np.searchsorted(tb, tt, side="left"))
            if bond < bb:
                cnt = int(np.searchsorted(tb, tt, side="right"))
            return cnt & 1
        sx = int(s0[bb]) ^ par_before((bb - 1) % L)
        sy = int(s0[(bb + 1) % L]) ^ par_before((bb + 1) % L)
        out[n] = sx != sy
    return out


def test_largest_single_gpu_chain(lc, chain):
    """L=262,144, beta=16,384 (about 3e9 operators per sweep): per-sweep
    identities, valid world lines on sampled operators, even jump counts,
    and the energy near the Bethe value 1/4 - ln 2."""
    chain.close()  # release the medium chain
    L, beta = 262144, 16384.0
    c = lc.Chain(L, 0.5, beta, 1)
    try:
        e_seen = []
        for s in range(12):
            c.update(1)
            st = c.last_sweep()
            assert st["n_nodes"] == L + 2 * st["n_ops"], s
            assert st["n_ops"] == st["n_kept_in"] + st["n_acc"], s
            assert st["n_acc"] <= st["n_cand"] and st["n_kept_out"] <= st["n_ops"], s
            assert 0 < st["n_clusters"] <= st["n_nodes"], s
            assert st["max_size"] <= st["n_nodes"], s
            e_seen.append(0.25 - st["n_ops"] / (beta * L))
            print(f"sweep {s}: ops {st['n_ops']} loops {st['n_clusters']} e {e_seen[-1]:.6f}",
                  flush=True)
        s0, off, kt, sw = c.export_state()
        assert sw == 12 and len(kt) == st["n_kept_out"] and off[-1] == len(kt)
        assert (np.diff(off) >= 0).all()
        cnt = np.diff(off)
        assert ((cnt + np.roll(cnt, 1)) % 2 == 0).all()  # even jumps per site
        rng = np.random.default_rng(7)
        idx = np.sort(rng.choice(len(kt), 400, replace=False))
        assert _antiparallel_below(s0, off, kt, L, idx).all()
        # times sorted within each bond
        for bnd in rng.choice(L, 64, replace=False):
            tb = kt[off[bnd]:off[bnd + 1]]
            assert (tb[1:] >= tb[:-1]).all()
        assert abs(np.mean(e_seen[-4:]) - (0.25 - np.log(2))) < 2e-3
    finally:
        c.close()
