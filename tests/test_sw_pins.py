"""Pins of the Swendsen-Wang oracle (2D Ising, the union-find benchmark of
arXiv:1810.07485 Sec. 4.1) against things other than itself.

- Bond activations recomputed with a separately written Philox and the
  threshold rule, clusters rebuilt with scipy's connected components.
- K = 0: no bond is active; K large: every bond between equal spins is.
- The exact partition function of the finite periodic lattice (Kaufman's
  four-term product formula), itself pinned by brute-force enumeration of
  small lattices, against the Monte Carlo energy.
- The improved cluster estimator of the susceptibility, <sum_c |c|^2>,
  against the plain one, <M^2>.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from tests.test_oracle_pins import M32, py_philox

KC = math.log(1 + math.sqrt(2)) / 2


# ------------------------------------------------------ exact reference ----
def brute_log_z_and_energy(m, n, K):
    """ln Z and <E>/N of the m x n periodic Ising model by enumeration."""
    N = m * n
    cfg = np.array(list(itertools.product((-1, 1), repeat=N)), dtype=np.int64).reshape(-1, m, n)
    e = -(cfg * np.roll(cfg, 1, axis=1)).sum(axis=(1, 2)) - (cfg * np.roll(cfg, 1, axis=2)).sum(axis=(1, 2))
    w = np.exp(-K * (e - e.min()))
    logz = math.log(w.sum()) - K * e.min()
    return logz, float((e * w).sum() / w.sum()) / N


def kaufman_log_z(m, n, K):
    """ln Z of the m x n periodic Ising model (Kaufman 1949): Z = 1/2
    (2 sinh 2K)^(mn/2) (Z1 + Z2 + Z3 + Z4), Z1,2 = prod_{k<n} 2 cosh|sinh(m
    g_{2k+1}/2), Z3,4 the same over g_{2k}; cosh g_l = cosh 2K cosh 2K* -
    sinh 2K sinh 2K* cos(pi l / n) with tanh K* = exp(-2K), g_0 = 2(K - K*)."""
    Ks = -0.5 * math.log(math.tanh(K))
    def gamma(l):
        if l == 0:
            return 2 * (K - Ks)
        c = math.cosh(2 * K) * math.cosh(2 * Ks) - math.sinh(2 * K) * math.sinh(2 * Ks) * math.cos(math.pi * l / n)
        return math.acosh(c)
    terms = []
    for odd in (1, 0):
        g = [gamma(2 * k + odd) for k in range(n)]
        for fn in ("cosh", "sinh"):
            logv, sign = 0.0, 1
            for x in g:
                a = m * x / 2
                if fn == "cosh":
                    logv += math.log(2) + abs(a) + math.log1p(math.exp(-2 * abs(a))) - math.log(2)
                else:
                    if a == 0:
                        sign = 0
                        break
                    sign *= 1 if a > 0 else -1
                    logv += math.log(2) + abs(a) + math.log1p(-math.exp(-2 * abs(a))) - math.log(2)
            terms.append((sign, logv))
    top = max(lv for sg, lv in terms if sg != 0)
    tot = sum(sg * math.exp(lv - top) for sg, lv in terms)
    return math.log(0.5) + (m * n / 2) * math.log(2 * math.sinh(2 * K)) + top + math.log(tot)


def kaufman_energy(m, n, K, h=1e-5):
    """<E>/N = -d ln Z / dK / N by central differences."""
    return -(kaufman_log_z(m, n, K + h) - kaufman_log_z(m, n, K - h)) / (2 * h) / (m * n)


@pytest.mark.parametrize("m,n", [(2, 2), (3, 3), (4, 4), (3, 4), (4, 3), (2, 5)])
@pytest.mark.parametrize("K", [0.2, KC, 0.7])
def test_kaufman_formula_against_enumeration(m, n, K):
    lz, e = brute_log_z_and_energy(m, n, K)
    assert abs(kaufman_log_z(m, n, K) - lz) < 1e-9 * max(1.0, abs(lz))
    assert abs(kaufman_energy(m, n, K) - e) < 1e-6


def test_kaufman_approaches_onsager():
    """At K_c the finite-lattice energy approaches Onsager's -sqrt(2) per
    site as 1/L: (e_L + sqrt 2) L is the same for L = 64 ... 1024."""
    amp = [(kaufman_energy(L, L, KC) + math.sqrt(2)) * L for L in (64, 256, 1024)]
    assert max(amp) - min(amp) < 1e-4 and -1.0 < amp[0] < -0.1
    assert abs(kaufman_energy(1024, 1024, KC) + math.sqrt(2)) < 1e-3


# ---------------------------------------------- bonds and clusters pin ----
def py_bonds(L, K, seed, sweep, s):
    T = math.floor((1.0 - math.exp(-2.0 * K)) * 2.0 ** 32) if K > 0 else 0
    act_r = np.zeros(L * L, bool)
    act_d = np.zeros(L * L, bool)
    for i in range(L * L):
        w = py_philox(seed, (i & M32, (5 << 24) | (i >> 32), 0, sweep & M32))
        y, x = divmod(i, L)
        r, d = y * L + (x + 1) % L, ((y + 1) % L) * L + x
        act_r[i] = s[i] == s[r] and w[0] < T
        act_d[i] = s[i] == s[d] and w[1] < T
    return act_r, act_d


def py_clusters(L, act_r, act_d):
    i = np.arange(L * L)
    y, x = i // L, i % L
    r, d = y * L + (x + 1) % L, ((y + 1) % L) * L + x
    u = np.concatenate([i[act_r], i[act_d]])
    v = np.concatenate([r[act_r], d[act_d]])
    A = sp.coo_matrix((np.ones(len(u)), (u, v)), shape=(L * L, L * L))
    _, comp = connected_components(A, directed=False)
    mins = np.full(comp.max() + 1, L * L)
    np.minimum.at(mins, comp, i)
    return mins[comp]


@pytest.mark.parametrize("L,K,seed", [(5, 0.3, 1), (8, KC, 2), (6, 1.5, 3)])
def test_bonds_clusters_and_flips_against_rebuild(orc, L, K, seed):
    ch = orc.SwChain(L, K, seed)
    for sweep in range(4):
        s = ch.spins()
        st = ch.sweep()
        act_r, act_d = py_bonds(L, K, seed, sweep, s)
        assert st["n_active"] == int(act_r.sum() + act_d.sum())
        lab = ch.labels()
        np.testing.assert_array_equal(lab, py_clusters(L, act_r, act_d))
        _, size = np.unique(lab, return_counts=True)
        assert st["n_clusters"] == len(size) and st["max_size"] == size.max()
        assert st["size2"] == int((size.astype(np.int64) ** 2).sum())
        sg = 2 * s.astype(np.int64) - 1
        g = sg.reshape(L, L)
        assert st["magnetization"] == int(sg.sum())
        assert st["energy"] == int(-(g * np.roll(g, -1, 1)).sum() - (g * np.roll(g, -1, 0)).sum())
        # every cluster flips with its label's bit (domain SWFLIP = 6)
        s1 = ch.spins()
        for i in range(L * L):
            c = int(lab[i])
            q, b = c >> 7, c & 127
            w = py_philox(seed, (q & M32, (6 << 24) | ((q >> 32) & 0xFFFFFF), 0, sweep))
            assert s1[i] == s[i] ^ ((w[b >> 5] >> (b & 31)) & 1)


def test_zero_and_strong_coupling(orc):
    ch = orc.SwChain(6, 0.0, 4)
    st = ch.sweep()
    assert st["n_active"] == 0 and st["n_clusters"] == 36
    ch = orc.SwChain(6, 40.0, 5)  # p = 1: the whole all-up lattice is one cluster
    st = ch.sweep()
    assert st["n_active"] == 72 and st["n_clusters"] == 1 and st["max_size"] == 36


def _mean_err(x, nbins=40):
    x = np.asarray(x, float)
    n = len(x) // nbins * nbins
    b = x[:n].reshape(nbins, -1).mean(1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nbins)


@pytest.mark.parametrize("L,K,seed", [(8, KC, 11), (16, 0.35, 12), (12, 0.6, 13)])
def test_energy_against_exact_finite_lattice(orc, L, K, seed):
    ch = orc.SwChain(L, K, seed)
    for _ in range(300):
        ch.sweep()
    st = [ch.sweep() for _ in range(12000)]
    e = np.array([s["energy"] for s in st], float) / (L * L)
    m, err = _mean_err(e)
    ref = kaufman_energy(L, L, K)
    assert abs(m - ref) < 4 * err + 1e-9, (m, err, ref)
    # improved (cluster) and plain estimators of N chi T agree
    a, ea = _mean_err(np.array([float(s["size2"]) for s in st]) / (L * L))
    b, eb = _mean_err(np.array([float(s["magnetization"]) ** 2 for s in st]) / (L * L))
    assert abs(a - b) < 4 * math.hypot(ea, eb), (a, ea, b, eb)
