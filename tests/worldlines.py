"""Independent Python reconstruction of the loop graph from exported operators.

Used by the tests to pin the oracle (and, on the GPU side, the library) with
code that shares nothing with either: given the spins at tau=0+, the
operators of a sweep in canonical (bond, time) order and, for split spins,
the symmetrization permutation, it rebuilds the world lines and the graph of
world-line fragments (arXiv:1810.07485, Sec. 2, Fig. 1(b)), then finds loops
with scipy's connected_components.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


def bonds(L: int, two_s: int):
    bx, by = [], []
    for j in range(L):
        for a in range(two_s):
            for c in range(two_s):
                bx.append(two_s * j + a)
                by.append(two_s * ((j + 1) % L) + c)
    return np.array(bx), np.array(by)


def site_events(L, two_s, op_bond, op_time):
    """Per site: operator ids in time order (ties: bond index, then op id)."""
    bx, by = bonds(L, two_s)
    ns = two_s * L
    order = np.lexsort((np.arange(len(op_bond)), op_bond, op_time))
    ev = [[] for _ in range(ns)]
    for k in order:
        ev[bx[op_bond[k]]].append(int(k))
        ev[by[op_bond[k]]].append(int(k))
    return ev


def spins_below(L, two_s, s0, op_bond, op_time, op_type):
    """Spins of the two sites of each operator just below it."""
    bx, by = bonds(L, two_s)
    ev = site_events(L, two_s, op_bond, op_time)
    below = {}
    for i, lst in enumerate(ev):
        s = int(s0[i])
        for k in lst:
            below[(k, i)] = s
            if op_type[k]:
                s ^= 1
    return np.array([[below[(k, bx[op_bond[k]])], below[(k, by[op_bond[k]])]]
                     for k in range(len(op_bond))]).reshape(-1, 2), ev


def loop_graph(L, two_s, op_bond, op_time, perm=None):
    """Edges (u, v, length) of the fragment graph and node count."""
    ns = two_s * L
    nbn = ns if two_s == 1 else 2 * ns
    ev = site_events(L, two_s, op_bond, op_time)
    U, V, LEN = [], [], []
    for i, lst in enumerate(ev):
        top = i if two_s == 1 else ns + i
        if not lst:
            U.append(i); V.append(top); LEN.append(1 << 64)
            continue
        U.append(i); V.append(nbn + 2 * lst[0]); LEN.append(int(op_time[lst[0]]))
        for a, b in zip(lst[:-1], lst[1:]):
            U.append(nbn + 2 * a + 1); V.append(nbn + 2 * b); LEN.append(int(op_time[b]) - int(op_time[a]))
        U.append(nbn + 2 * lst[-1] + 1); V.append(top); LEN.append((1 << 64) - int(op_time[lst[-1]]))
    if two_s > 1:
        for i in range(ns):
            U.append(ns + i); V.append(int(perm[i])); LEN.append(0)
    return np.array(U), np.array(V), LEN, nbn + 2 * len(op_bond), nbn


def min_labels(U, V, n):
    g = sp.coo_matrix((np.ones(len(U)), (U, V)), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    mins = np.full(comp.max() + 1, n, dtype=np.int64)
    np.minimum.at(mins, comp, np.arange(n))
    return mins[comp]


def cluster_stats(L, two_s, s0, labels, U, LEN, nbn):
    """Exact per-sweep integers from labels: the improved estimators."""
    ns = two_s * L
    roots = np.unique(labels)
    size = {int(r): 0 for r in roots}
    n0 = dict(size); m = dict(size); ln = {int(r): 0 for r in roots}
    for v in range(len(labels)):
        size[int(labels[v])] += 1
    for i in range(ns):
        n0[int(labels[i])] += 1
        m[int(labels[i])] += 2 * int(s0[i]) - 1
    for u, l in zip(U, LEN):
        ln[int(labels[u])] += l
    return dict(
        n_clusters=len(roots),
        sum_size2=sum(v * v for v in size.values()),
        sum_n0sq=sum(v * v for v in n0.values()),
        sum_m2=sum(v * v for v in m.values()),
        sum_len2=sum((v >> 32) ** 2 for v in ln.values()),
        max_size=max(size.values()),
    )


def segments(L, two_s, op_bond, op_time):
    """Vertical segments of the world lines: (first node, subspin, start tick,
    end tick), end 2^64 at beta, in the order loop_graph lists its edges."""
    ns = two_s * L
    nbn = ns if two_s == 1 else 2 * ns
    ev = site_events(L, two_s, op_bond, op_time)
    out = []
    for i, lst in enumerate(ev):
        if not lst:
            out.append((i, i, 0, 1 << 64))
            continue
        out.append((i, i, 0, int(op_time[lst[0]])))
        for a, b in zip(lst[:-1], lst[1:]):
            out.append((nbn + 2 * a + 1, i, int(op_time[a]), int(op_time[b])))
        out.append((nbn + 2 * lst[-1] + 1, i, int(op_time[lst[-1]]), 1 << 64))
    return out
