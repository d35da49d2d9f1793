"""Pins of the CPU oracle against things other than itself.

- Philox4x32-10 known-answer vectors published with the generator.
- Poisson thresholds against scipy.stats.poisson.
- Candidate law (first sweep from the Neel state accepts every candidate).
- Loop graph and labels against an independent reconstruction
  (tests/worldlines.py + scipy connected_components).
- World-line invariants before and after the flip.
- Physics: exact diagonalization, high-temperature limits, Bethe ansatz and
  the paper's printed ratios (arXiv:1810.07485, Sec. 4.4).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

from tests import worldlines as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- Philox ----
# Known-answer vectors of Philox4x32-10 (Random123 distribution, kat_vectors;
# Salmon et al., SC'11): (counter, key) -> output.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(orc, ctr, key, out):
    seed = key[0] | (key[1] << 32)
    assert orc.philox(seed, ctr) == out


def test_philox_bits_uniform(orc):
    words = np.array([orc.philox(12345, (i, 7, 0, 3)) for i in range(4000)], dtype=np.uint64)
    bits = np.unpackbits(words.astype(">u4").view(np.uint8))
    n = bits.size
    z = (bits.sum() - n / 2) / math.sqrt(n / 4)
    assert abs(z) < 4
    # byte histogram chi^2
    h = np.bincount(words.astype(">u4").view(np.uint8).ravel(), minlength=256)
    assert stats.chisquare(h).pvalue > 1e-4


# ------------------------------------------------- Poisson window table ----
@pytest.mark.parametrize("beta", [0.25, 1.0, 3.0, 8.0, 9.0, 100.0, 4096.0, 16384.0, 3000.5])
def test_window_rule_and_thresholds(orc, beta):
    w, mu, T = orc.window_table(beta)
    assert beta / 2 ** w <= 8 and (w == 0 or beta / 2 ** (w - 1) > 8)
    assert mu == beta / 2 ** (w + 1)
    cdf = stats.poisson.cdf(np.arange(len(T)), mu)
    for i, t in enumerate(T[:-1]):
        assert abs(t / 2.0 ** 64 - cdf[i]) < 1e-14
    assert T[-1] == 2 ** 64 - 1
    assert stats.poisson.sf(len(T) - 1, mu) < 1e-15


def test_first_sweep_candidates_are_poisson_uniform(orc):
    """From the initial Neel state with no operators every bond is antiparallel
    at all times, so every candidate of sweep 0 becomes an operator: their
    count per bond is Poisson(beta/2) and the times are uniform."""
    L, beta = 2048, 20.0
    ch = orc.Chain(L, 0.5, beta, 99)
    st = ch.sweep()
    assert st["n_acc"] == st["n_cand"] == st["n_ops"]
    b, t, ty = ch.export_ops()
    assert not ty.any()
    cnt = np.bincount(b, minlength=L)
    # mean and variance of Poisson(beta / 2)
    assert abs(cnt.mean() - beta / 2) < 4 * math.sqrt(beta / 2 / L)
    assert abs(cnt.var() / (beta / 2) - 1) < 0.12
    u = t.astype(np.float64) / 2.0 ** 64
    assert stats.kstest(u, "uniform").pvalue > 1e-4


# ----------------------------------------- loop graph, labels, invariants ----
def _check_sweep(orc, ch, L, two_s):
    s0, off, kt, sw = ch.export_state()
    st = ch.sweep()
    b, t, ty0 = ch.export_ops()
    lab = ch.export_labels()
    perm = ch.export_perm() if two_s > 1 else None
    # operators: kept ones are exactly the previous off-diagonal operators
    assert ty0.sum() == len(kt) == st["n_kept_in"]
    np.testing.assert_array_equal(np.sort(t[ty0 == 1]), np.sort(kt))
    # every operator has antiparallel spins below it (labeling rules i-iii)
    below, _ = wl.spins_below(L, two_s, s0, b, t, ty0)
    assert (below[:, 0] != below[:, 1]).all()
    # loops: independent rebuild of the fragment graph + scipy components
    U, V, LEN, n, nbn = wl.loop_graph(L, two_s, b, t, perm)
    assert n == st["n_nodes"] == len(lab)
    ref = wl.min_labels(U, V, n)
    np.testing.assert_array_equal(lab, ref)
    deg = np.bincount(np.concatenate([U, V]), minlength=n)
    assert (deg == 2).all()
    # estimators from the rebuilt loops
    cs = wl.cluster_stats(L, two_s, s0, ref, U, LEN, nbn)
    for k, v in cs.items():
        assert st[k] == v, k
    # staggered spin is constant along every loop (spins alternate
    # consistently): check every vertical segment of every loop
    ev = wl.site_events(L, two_s, b, t)
    stag = {}
    for i, lst in enumerate(ev):
        sgn = 1 if (i // two_s) % 2 == 0 else -1
        s = int(s0[i])
        top = i if two_s == 1 else L * two_s + i
        # segment q runs from event q (or tau = 0) to event q+1 (or beta)
        for q in range(len(lst) + 1):
            if q > 0 and ty0[lst[q - 1]]:
                s ^= 1
            lo = i if q == 0 else nbn + 2 * lst[q - 1] + 1
            hi = top if q == len(lst) else nbn + 2 * lst[q]
            val = sgn * (2 * s - 1)
            for node in (lo, hi):
                assert stag.setdefault(int(ref[node]), val) == val
    # after the flip: new operator types from the new kept list
    s1, off1, kt1, sw1 = ch.export_state()
    assert sw1 == sw + 1
    key_after = set(zip(np.repeat(np.arange(len(off1) - 1), np.diff(off1)).tolist(), kt1.tolist()))
    ty1 = np.array([(int(bb), int(tt)) in key_after for bb, tt in zip(b, t)], dtype=np.uint8)
    assert ty1.sum() == len(kt1) == st["n_kept_out"]
    # flip rule: op type changes iff exactly one of its two loops flipped
    for k in range(len(b)):
        fl = orc.flip_bit(ch.seed, sw, int(lab[nbn + 2 * k]))
        fu = orc.flip_bit(ch.seed, sw, int(lab[nbn + 2 * k + 1]))
        assert ty1[k] == ty0[k] ^ fl ^ fu
    below1, _ = wl.spins_below(L, two_s, s1, b, t, ty1)
    assert (below1[:, 0] != below1[:, 1]).all()
    if two_s == 1:
        # world lines stay periodic: even number of jumps on every site
        par = np.zeros(L, int)
        bx, by = wl.bonds(L, 1)
        np.add.at(par, bx[b[ty1 == 1]], 1)
        np.add.at(par, by[b[ty1 == 1]], 1)
        assert (par % 2 == 0).all()
    assert st["m_after"] == int((2 * s1.astype(int) - 1).sum())
    return st


@pytest.mark.parametrize("L,S,beta,seed", [(16, 0.5, 8.0, 1), (6, 0.5, 2.0, 5), (8, 1.0, 3.0, 2),
                                           (4, 2.0, 1.0, 3), (4, 4.0, 0.7, 4), (10, 1.5, 1.0, 6)])
def test_loop_graph_labels_invariants(orc, L, S, beta, seed):
    two_s = int(round(2 * S))
    ch = orc.Chain(L, S, beta, seed)
    for _ in range(4):
        _check_sweep(orc, ch, L, two_s)
    for _ in range(50):
        ch.sweep()
    for _ in range(4):
        _check_sweep(orc, ch, L, two_s)


def test_conserved_magnetization(orc):
    """sum_j s_j(tau) does not depend on tau (every jump swaps an up and a
    down spin), so the plain magnetization after the flip is the same at
    tau = 0 and just below each operator."""
    L = 32
    ch = orc.Chain(L, 0.5, 6.0, 17)
    for _ in range(20):
        ch.sweep()
    s0, _, _, _ = ch.export_state()
    ch.sweep()
    b, t, ty = ch.export_ops()
    ev = wl.site_events(L, 1, b, t)
    order = np.lexsort((np.arange(len(b)), b, t))
    s = s0.astype(int).copy()
    bx, by = wl.bonds(L, 1)
    m0 = s.sum()
    for k in order:
        if ty[k]:
            s[bx[b[k]]] ^= 1
            s[by[b[k]]] ^= 1
            assert s.sum() == m0
    assert ev is not None


def test_tie_order_crafted_state(orc):
    """Operators at exactly equal times on bonds sharing a site: the walk
    orders them by bond index.  A crafted valid state with such ties must
    keep every invariant and match the independent graph rebuild."""
    L = 8
    ch = orc.Chain(L, 0.5, 4.0, 3)
    s0 = np.array([1, 0, 0, 1, 0, 1, 0, 1], np.uint8)
    t1, t2, t3 = 1 << 61, 1 << 62, (1 << 63) + 5
    ops = {0: [t1, t3], 1: [t1, t2]}  # bond 0 at t1 and t3, bond 1 at t1 and t2
    off = np.zeros(L + 1, np.int64)
    times = []
    for bb in range(L):
        times += ops.get(bb, [])
        off[bb + 1] = len(times)
    ch.import_state(s0, off, np.array(times, np.uint64), 10)
    for _ in range(3):
        _check_sweep(orc, ch, L, 1)


def test_import_rejects_unsorted(orc):
    ch = orc.Chain(8, 0.5, 4.0, 3)
    off = np.array([0, 2, 2, 2, 2, 2, 2, 2, 2], np.int64)
    with pytest.raises(ValueError):
        ch.import_state(np.zeros(8, np.uint8), off, np.array([5, 3], np.uint64), 0)


# ---------------------------------------------------------------- physics ----
def _series(st, L, S, beta):
    two_s = int(round(2 * S))
    nb = two_s * two_s * L
    N = np.array([s["n_ops"] for s in st], float)
    return dict(
        e=nb / (4 * L) - N / (beta * L),
        chi_u=beta / (4 * L) * np.array([s["sum_m2"] for s in st], float),
        s_pi=np.array([s["sum_n0sq"] for s in st], float) / (4 * L),
        chi_s=beta / (4 * L) * np.array([float(s["sum_len2"]) for s in st]) / 2.0 ** 64,
    )


def _mean_err(x, nbins=40):
    x = np.asarray(x, float)
    n = len(x) // nbins * nbins
    b = x[:n].reshape(nbins, -1).mean(1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nbins)


def _run(orc, L, S, beta, seed, therm, meas):
    ch = orc.Chain(L, S, beta, seed)
    for _ in range(therm):
        ch.sweep()
    return [ch.sweep() for _ in range(meas)]


def _golden(L, S, beta):
    with open(os.path.join(GOLD, "ed_golden.json")) as f:
        for c in json.load(f)["cases"]:
            if c["L"] == L and c["S"] == S and c["beta"] == beta:
                return c
    raise KeyError((L, S, beta))


def test_tiny_instance_vs_exact_diagonalization(orc):
    """L=16, beta=8, seed 1, 1,000 + 10,000 sweeps: energy and uniform
    susceptibility within 3 sigma of exact diagonalization."""
    ref = _golden(16, 0.5, 8.0)
    st = _run(orc, 16, 0.5, 8.0, 1, 1000, 10000)
    ser = _series(st, 16, 0.5, 8.0)
    for k, nsig in (("e", 3), ("chi_u", 3), ("s_pi", 4), ("chi_s", 4)):
        m, e = _mean_err(ser[k])
        assert abs(m - ref[k]) < nsig * e, (k, m, e, ref[k])


@pytest.mark.parametrize("L,S,beta,seed,meas", [(4, 0.5, 0.1, 1, 20000), (6, 0.5, 1.0, 2, 20000),
                                                (8, 0.5, 8.0, 3, 20000), (12, 0.5, 2.0, 4, 8000)])
def test_small_chains_vs_exact_diagonalization(orc, L, S, beta, seed, meas):
    from oracle import ed
    ref = ed.thermal(L, S, beta, vectors=L <= 10) if L <= 10 else _golden(L, S, beta)
    st = _run(orc, L, S, beta, seed, 500, meas)
    ser = _series(st, L, S, beta)
    for k in ("e", "chi_u", "s_pi", "chi_s"):
        if k not in ref:
            continue
        m, e = _mean_err(ser[k])
        assert abs(m - ref[k]) < 4 * e, (k, m, e, ref[k])


@pytest.mark.parametrize("L,S,beta,seed,meas", [(6, 1.0, 4.0, 5, 8000), (4, 4.0, 1.0, 6, 8000)])
def test_split_spin_vs_exact_diagonalization(orc, L, S, beta, seed, meas):
    ref = _golden(L, S, beta)
    st = _run(orc, L, S, beta, seed, 500, meas)
    ser = _series(st, L, S, beta)
    for k in ("e", "chi_u", "s_pi", "chi_s"):
        m, e = _mean_err(ser[k])
        assert abs(m - ref[k]) < 4 * e, (k, m, e, ref[k])


def test_high_temperature_limits(orc):
    """beta -> 0: e -> 0 and chi_u T -> S(S+1)/3 = 1/4 (Curie law)."""
    L, beta = 16, 0.02
    st = _run(orc, L, 0.5, beta, 8, 100, 4000)
    ser = _series(st, L, 0.5, beta)
    m, e = _mean_err(ser["e"])
    assert abs(m) < 4 * e + 3 * beta / 16  # e = -3 beta/16 + O(beta^2)
    m, e = _mean_err(ser["chi_u"] / beta)
    # Curie-Weiss to first order in beta: chi T = (1/4) / (1 + beta z S(S+1)/3)
    assert abs(m - 0.25 / (1 + beta / 2)) < 4 * e + 1e-3


@pytest.mark.slow
def test_bethe_ansatz_and_paper_ratios(orc):
    """Large L, low T: e -> 1/4 - ln 2 (Bethe ansatz); operators per unit
    space-time volume -> 0.693 and loops per unit volume -> 0.398
    (Sec. 4.4: 5.64e11 operators and 3.24e11 loops at L beta = 8.14e11)."""
    L, beta = 512, 512.0
    st = _run(orc, L, 0.5, beta, 21, 60, 120)
    ser = _series(st, L, 0.5, beta)
    m, e = _mean_err(ser["e"], nbins=12)
    exact = 0.25 - math.log(2)
    assert abs(m - exact) < 3 * e + 2e-5, (m, e, exact)
    ops = np.mean([s["n_ops"] for s in st]) / (L * beta)
    loops = np.mean([s["n_clusters"] for s in st]) / (L * beta)
    # printed to three digits: 5.64e11 / 8.14e11 and 3.24e11 / 8.14e11
    assert abs(ops - 5.64 / 8.14) < 0.0015, ops
    assert abs(loops - 3.24 / 8.14) < 0.0015, loops


# ------------------------------------------------------- loop-flip bits ----
M32 = 0xFFFFFFFF


def py_philox(seed: int, ctr) -> tuple:
    """Philox4x32-10 written out in Python from its published definition
    (Salmon et al., SC'11): per round, two 32x32 -> 64-bit products of
    counter words 0 and 2; the new word 0 is hi(c2 M1) ^ c1 ^ k0, word 1 is
    lo(c2 M1), word 2 is hi(c0 M0) ^ c3 ^ k1, word 3 is lo(c0 M0); the key
    advances by the Weyl increments between rounds."""
    M0, M1, W0, W1 = 0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85
    k0, k1 = seed & M32, (seed >> 32) & M32
    c0, c1, c2, c3 = (int(x) & M32 for x in ctr)
    for r in range(10):
        if r:
            k0, k1 = (k0 + W0) & M32, (k1 + W1) & M32
        p0, p1 = M0 * c0, M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & M32, p1 & M32, ((p0 >> 32) ^ c3 ^ k1) & M32, p0 & M32
    return c0, c1, c2, c3


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_python_philox_known_answers(ctr, key, out):
    assert py_philox(key[0] | (key[1] << 32), ctr) == out


def py_flip_bit(seed: int, sweep: int, label: int) -> int:
    """Loop-flip bit of a loop whose smallest node id is `label`: 128 bits
    per Philox block of the FLIP domain (2 in the top byte of counter word
    1); block q = label / 128 is addressed by counter words 0 (low 32 bits of
    q) and 1 (bits 32..55 of q), word 3 holds the sweep; the bit is bit
    (label mod 128) of the block read as words 0..3, least significant first."""
    q, i = label >> 7, label & 127
    words = py_philox(seed, (q & M32, (2 << 24) | ((q >> 32) & 0xFFFFFF), 0, sweep & M32))
    return (words[i >> 5] >> (i & 31)) & 1


def test_flip_bits_against_independent_philox(orc):
    """The oracle's flip bit equals a bit recomputed from a separately
    written Philox (pinned above by the known-answer vectors) for labels in
    every word and bit position, block boundaries and labels beyond 2^39
    (high block bits in counter word 1)."""
    rng = np.random.default_rng(11)
    labels = list(range(0, 520)) + [127, 128, 255, 256, (1 << 32) - 1, 1 << 32, (1 << 39) + 5,
                                    (1 << 40) + 129, (1 << 50) + 77]
    labels += [int(x) for x in rng.integers(0, 1 << 45, 300)]
    for seed, sweep in ((1, 0), (0xDEADBEEFCAFEF00D, 7), (12345, 100000)):
        for lab in labels:
            assert orc.flip_bit(seed, sweep, lab) == py_flip_bit(seed, sweep, lab), (seed, sweep, lab)


def test_flip_bits_fair_and_independent(orc):
    """Each loop flips with probability 1/2 (Sec. 2, cluster flip), and the
    bits of labels c, c+1 and c+128 (same word, neighbouring bit; same bit of
    the next block) and of consecutive sweeps are independent: chi^2 tests
    on the 2x2 tables of each pair."""
    n = 20000
    base = np.arange(0, 3 * n, 3, dtype=np.int64) * 129 + 17
    f0 = np.array([orc.flip_bit(3, 5, int(c)) for c in base])
    f1 = np.array([orc.flip_bit(3, 5, int(c) + 1) for c in base])
    f128 = np.array([orc.flip_bit(3, 5, int(c) + 128) for c in base])
    fs = np.array([orc.flip_bit(3, 6, int(c)) for c in base])
    z = (f0.sum() - n / 2) / math.sqrt(n / 4)
    assert abs(z) < 4
    for other in (f1, f128, fs):
        tab = np.array([[np.sum((f0 == a) & (other == b)) for b in (0, 1)] for a in (0, 1)])
        assert stats.chi2_contingency(tab, correction=False)[1] > 1e-4, tab


# ------------------------------------------------ majority-vote flip rule ----
def py_domain_bit(seed: int, sweep: int, ident: int, dom: int) -> int:
    q, i = ident >> 7, ident & 127
    words = py_philox(seed, (q & M32, (dom << 24) | ((q >> 32) & 0xFFFFFF), 0, sweep & M32))
    return (words[i >> 5] >> (i & 31)) & 1


def test_vote_bits_against_independent_philox(orc):
    for seed, sweep in ((1, 0), (77, 3)):
        for v in list(range(300)) + [1 << 33, (1 << 40) + 5]:
            assert orc.vote_bit(seed, sweep, v) == py_domain_bit(seed, sweep, v, 4)


@pytest.mark.parametrize("L,S,beta,seed", [(16, 0.5, 8.0, 1), (8, 1.0, 3.0, 2), (4, 4.0, 0.7, 4)])
def test_vote_rule_flips_the_xor_of_each_loops_votes(orc, L, S, beta, seed):
    """Sec. 3.3's majority-vote trick: a loop flips iff the XOR of its nodes'
    votes is 1.  Checked on the oracle's exported operators and labels against
    votes recomputed with the independent Philox and loops rebuilt by scipy."""
    two_s = int(round(2 * S))
    ch = orc.Chain(L, S, beta, seed)
    ch.set_flip_rule(orc.FLIP_VOTE)
    for _ in range(20):
        ch.sweep()
    for _ in range(3):
        s0, off, kt, sw = ch.export_state()
        st = ch.sweep()
        b, t, ty0 = ch.export_ops()
        lab = ch.export_labels()
        perm = ch.export_perm() if two_s > 1 else None
        U, V, LEN, n, nbn = wl.loop_graph(L, two_s, b, t, perm)
        np.testing.assert_array_equal(lab, wl.min_labels(U, V, n))
        dec = {}
        for v in range(n):
            dec[int(lab[v])] = dec.get(int(lab[v]), 0) ^ py_domain_bit(seed, sw, v, 4)
        s1, off1, kt1, _ = ch.export_state()
        key_after = set(zip(np.repeat(np.arange(len(off1) - 1), np.diff(off1)).tolist(), kt1.tolist()))
        ty1 = np.array([(int(bb), int(tt)) in key_after for bb, tt in zip(b, t)], dtype=np.uint8)
        for k in range(len(b)):
            assert ty1[k] == ty0[k] ^ dec[int(lab[nbn + 2 * k])] ^ dec[int(lab[nbn + 2 * k + 1])]
        for x in range(len(s0)):
            assert s1[x] == s0[x] ^ dec[int(lab[x])]
        assert st["n_kept_out"] == int(ty1.sum())


@pytest.mark.parametrize("L,S,beta,seed,meas", [(8, 0.5, 8.0, 31, 20000), (6, 1.0, 4.0, 32, 8000)])
def test_vote_rule_vs_exact_diagonalization(orc, L, S, beta, seed, meas):
    """The vote rule is another Markov chain with the same stationary
    distribution: energy and susceptibility agree with exact diagonalization."""
    from oracle import ed
    ref = ed.thermal(L, S, beta, vectors=False) if S == 0.5 else _golden(L, S, beta)
    ch = orc.Chain(L, S, beta, seed)
    ch.set_flip_rule(orc.FLIP_VOTE)
    for _ in range(500):
        ch.sweep()
    st = [ch.sweep() for _ in range(meas)]
    ser = _series(st, L, S, beta)
    for k in ("e", "chi_u"):
        m, e = _mean_err(ser[k])
        assert abs(m - ref[k]) < 4 * e, (k, m, e, ref[k])
