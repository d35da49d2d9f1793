"""Pins of the oracle's Fourier-mode improved estimators (the second-moment
estimators of the correlation length and the gap that arXiv:1810.07485
cites for its S = 1 results, Sec. 5), against things other than itself:

- exact diagonalization: the dynamical susceptibility chi(q, w_n) at
  (pi, 0), (pi + 2 pi/L, 0), (pi, 2 pi/beta) and S(pi + 2 pi/L) from the
  Lehmann sum over all eigenstates (oracle/ed.py), against Monte Carlo
  averages at S = 1/2 and S = 1;
- a per-sweep recomputation from the exported operators and labels with the
  independent world-line rebuild of tests/worldlines.py;
- the closed form of world lines without operators (beta -> 0): every site
  is a loop of one straight segment;
- chi(pi, 0) equals the staggered susceptibility of the integer estimators
  (which drop the low 32 bits of each loop length).
"""
import math

import numpy as np
import pytest

from oracle import ed
from tests import worldlines as wl

KEYS = ("chi_pi", "chi_pi_q1", "chi_pi_w1", "s_pi_q1")


def _mean_err(x, nbins=40):
    x = np.asarray(x, float)
    n = len(x) // nbins * nbins
    b = x[:n].reshape(nbins, -1).mean(1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nbins)


@pytest.mark.parametrize("L,S,beta,seed", [(8, 0.5, 2.0, 3), (6, 1.0, 2.0, 4), (10, 0.5, 4.0, 5)])
def test_fourier_estimators_vs_exact_diagonalization(orc, L, S, beta, seed):
    ref = ed.fourier(L, S, beta)
    ch = orc.Chain(L, S, beta, seed)
    ch.set_fourier(True)
    for _ in range(300):
        ch.sweep()
    rows = []
    for _ in range(12000):
        ch.sweep()
        f = ch.fourier()
        rows.append([f[k] for k in KEYS])
    rows = np.array(rows)
    for i, k in enumerate(KEYS):
        m, e = _mean_err(rows[:, i])
        assert abs(m - ref[k]) < 4 * e + 1e-12, (k, m, e, ref[k])


@pytest.mark.parametrize("L,S,beta,seed", [(12, 0.5, 3.0, 7), (6, 1.0, 2.5, 8)])
def test_fourier_sums_against_rebuild(orc, L, S, beta, seed):
    ts = int(round(2 * S))
    ch = orc.Chain(L, S, beta, seed)
    ch.set_fourier(True)
    for _ in range(4):
        ch.sweep()
        f = ch.fourier()
        b, t, _ = ch.export_ops()
        lab = ch.export_labels()
        d, w = 2 * math.pi / L, 2 * math.pi / beta
        q0, qd, qw, pd = {}, {}, {}, {}
        for u, x, t0, t1 in wl.segments(L, ts, b, t):
            l, j = int(lab[u]), x // ts
            ln = (t1 - t0) / 2.0 ** 64 * beta
            q0[l] = q0.get(l, 0) + ln
            qd[l] = qd.get(l, 0) + complex(math.cos(d * j), math.sin(d * j)) * ln
            eb = complex(math.cos(2 * math.pi * t1 / 2.0 ** 64), math.sin(2 * math.pi * t1 / 2.0 ** 64))
            ea = complex(math.cos(2 * math.pi * t0 / 2.0 ** 64), math.sin(2 * math.pi * t0 / 2.0 ** 64))
            qw[l] = qw.get(l, 0) + (eb - ea) / (1j * w)
        for x in range(ts * L):
            l, j = int(lab[x]), x // ts
            pd[l] = pd.get(l, 0) + complex(math.cos(d * j), math.sin(d * j))
        want = dict(chi_pi=sum(v * v for v in q0.values()) / (4 * beta * L),
                    chi_pi_q1=sum(abs(v) ** 2 for v in qd.values()) / (4 * beta * L),
                    chi_pi_w1=sum(abs(v) ** 2 for v in qw.values()) / (4 * beta * L),
                    s_pi_q1=sum(abs(v) ** 2 for v in pd.values()) / (4 * L))
        for k in KEYS:
            assert f[k] == pytest.approx(want[k], rel=1e-12, abs=1e-14), k


def test_no_operators_closed_form(orc):
    """beta -> 0: no operator is inserted; every site is one loop made of a
    single segment of length beta: chi(q, 0) = beta / 4, chi(pi, w) = 0,
    S(q) = 1/4."""
    L, beta = 10, 1e-9
    ch = orc.Chain(L, 0.5, beta, 9)
    ch.set_fourier(True)
    st = ch.sweep()
    assert st["n_ops"] == 0
    f = ch.fourier()
    assert f["chi_pi"] == pytest.approx(beta / 4, rel=1e-12)
    assert f["chi_pi_q1"] == pytest.approx(beta / 4, rel=1e-12)
    assert abs(f["chi_pi_w1"]) < 1e-12 * beta
    assert f["s_pi_q1"] == pytest.approx(0.25, rel=1e-12)


def test_zero_mode_is_the_staggered_susceptibility(orc):
    L, beta = 16, 4.0
    ch = orc.Chain(L, 0.5, beta, 10)
    ch.set_fourier(True)
    for _ in range(20):
        st = ch.sweep()
        chi_s = beta * st["sum_len2"] / 2.0 ** 64 / (4 * L)  # (len >> 32)^2, len in beta / 2^64
        assert ch.fourier()["chi_pi"] == pytest.approx(chi_s, rel=1e-6)


def test_fourier_off_by_default(orc):
    ch = orc.Chain(8, 0.5, 2.0, 1)
    ch.sweep()
    with pytest.raises(RuntimeError):
        ch.fourier()
