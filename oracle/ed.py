"""Exact diagonalization of the spin-S antiferromagnetic Heisenberg chain.

TEST INFRASTRUCTURE ONLY (pins the oracle; never used by the product path).

H = J sum_j S_j . S_{j+1}, J = 1, periodic boundaries (arXiv:1810.07485,
Sec. 2, Eq. 1; spin S as in Sec. 5).  Thermal averages at inverse temperature
beta, computed sector by sector in total S^z with dense LAPACK eigensolvers:

  e      = <H> / L
  chi_u  = beta <M^2> / L,            M   = sum_j S^z_j
  s_pi   = <Ms^2> / L,                Ms  = sum_j (-1)^j S^z_j
  chi_s  = (1/L) int_0^beta <Ms(tau) Ms(0)> dtau      (Lehmann sum)
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg as sla


def _sector_states(L: int, two_s: int, m2: int) -> np.ndarray:
    """All states with sum_j 2 m_j == m2; entries are 2 m_j in {-2S, ..., 2S}."""
    vals = list(range(-two_s, two_s + 1, 2))
    out = [s for s in itertools.product(vals, repeat=L) if sum(s) == m2]
    return np.array(out, dtype=np.int64).reshape(-1, L)


def sector_hamiltonian(L: int, two_s: int, m2: int):
    """Dense H in one total-S^z sector, with the basis (rows of 2m values)."""
    st = _sector_states(L, two_s, m2)
    n = st.shape[0]
    index = {tuple(r): i for i, r in enumerate(st)}
    H = np.zeros((n, n))
    S = two_s / 2.0
    for i, s in enumerate(st):
        m = s / 2.0
        for j in range(L):
            k = (j + 1) % L
            H[i, i] += m[j] * m[k]
            # (S+_j S-_k + S-_j S+_k) / 2
            for dj in (+2, -2):
                a, b = s[j] + dj, s[k] - dj
                if abs(a) > two_s or abs(b) > two_s:
                    continue
                mj, mk = m[j], m[k]
                if dj > 0:
                    amp = np.sqrt(S * (S + 1) - mj * (mj + 1)) * np.sqrt(S * (S + 1) - mk * (mk - 1))
                else:
                    amp = np.sqrt(S * (S + 1) - mj * (mj - 1)) * np.sqrt(S * (S + 1) - mk * (mk + 1))
                t = s.copy()
                t[j], t[k] = a, b
                H[index[tuple(t)], i] += 0.5 * amp
    return H, st


def thermal(L: int, S: float, beta: float, vectors: bool = True) -> dict:
    """Thermal observables of the spin-S chain of length L at inverse temperature beta."""
    two_s = int(round(2 * S))
    sign = np.array([(-1) ** j for j in range(L)], dtype=float)
    secs = []
    emin = np.inf
    for m2 in range(-two_s * L, two_s * L + 1, 2):
        H, st = sector_hamiltonian(L, two_s, m2)
        if vectors:
            w, V = sla.eigh(H)
        else:
            w, V = sla.eigvalsh(H), None
        secs.append((m2, w, V, st))
        emin = min(emin, w.min())
    Z = E = M2 = Ms2 = Xs = 0.0
    for m2, w, V, st in secs:
        b = np.exp(-beta * (w - emin))
        Z += b.sum()
        E += (b * w).sum()
        M2 += b.sum() * (m2 / 2.0) ** 2
        if V is not None:
            d = (st / 2.0) @ sign  # Ms is diagonal in the S^z basis
            Ms2 += (b * ((V * V).T @ (d * d))).sum()
            A = V.T @ (d[:, None] * V)
            A2 = A * A
            dE = w[:, None] - w[None, :]
            with np.errstate(divide="ignore", invalid="ignore"):
                # int_0^beta e^{-(beta-tau) E_n} e^{-tau E_m} dtau (shifted by emin)
                K = (np.exp(-beta * (w[None, :] - emin)) - np.exp(-beta * (w[:, None] - emin))) / dE
            same = np.abs(dE) < 1e-12
            K[same] = (beta * np.exp(-beta * (w[:, None] - emin)) * np.ones_like(dE))[same]
            Xs += (A2 * K).sum()
    out = dict(e=E / Z / L, chi_u=beta * M2 / Z / L)
    if vectors:
        out["s_pi"] = Ms2 / Z / L
        out["chi_s"] = Xs / Z / L
    return out


def fourier(L: int, S: float, beta: float) -> dict:
    """Dynamical susceptibility chi(q, w_n) = (1/(beta L)) int int e^{i w (tau -
    tau')} <S^z_q(tau) S^z_-q(tau')>, S^z_q = sum_j e^{i q j} S^z_j, at
    (q, w) = (pi, 0), (pi + 2 pi/L, 0), (pi, 2 pi/beta), and the equal-time
    S(pi + 2 pi/L) = <S^z_q S^z_-q> / L, by the Lehmann sum over the
    eigenstates of each total-S^z sector (S^z_q is diagonal in the S^z basis,
    so it keeps the sector):
      chi(q, w) = (1/(Z L)) sum_{m,n} |<m|S^z_q|n>|^2 (e^{-beta E_n} - e^{-beta E_m})
                  (E_m - E_n) / ((E_m - E_n)^2 + w^2),
    with beta e^{-beta E_m} for E_m = E_n at w = 0 (and 0 at w != 0)."""
    two_s = int(round(2 * S))
    j = np.arange(L)
    qs = {"chi_pi": (np.pi, 0.0), "chi_pi_q1": (np.pi + 2 * np.pi / L, 0.0),
          "chi_pi_w1": (np.pi, 2 * np.pi / beta)}
    secs, emin = [], np.inf
    for m2 in range(-two_s * L, two_s * L + 1, 2):
        H, st = sector_hamiltonian(L, two_s, m2)
        w, V = sla.eigh(H)
        secs.append((w, V, st))
        emin = min(emin, w.min())
    Z = 0.0
    acc = {k: 0.0 for k in qs}
    sq1 = 0.0
    for w, V, st in secs:
        b = np.exp(-beta * (w - emin))
        Z += b.sum()
        dE = w[:, None] - w[None, :]                      # E_m - E_n
        num = np.exp(-beta * (w[None, :] - emin)) - np.exp(-beta * (w[:, None] - emin))
        same = np.abs(dE) < 1e-12
        for k, (q, om) in qs.items():
            d = (st / 2.0) @ np.exp(1j * q * j)           # S^z_q on each basis state
            A = V.T @ (d[:, None] * V)
            A2 = np.abs(A) ** 2
            with np.errstate(divide="ignore", invalid="ignore"):
                K = num * dE / (dE * dE + om * om)
            K[same] = (beta * np.exp(-beta * (w[:, None] - emin)) * np.ones_like(dE))[same] if om == 0 else 0.0
            acc[k] += (A2 * K).sum()
            if k == "chi_pi_q1":
                sq1 += (b * A2.sum(axis=1)).sum()
    out = {k: v / Z / L for k, v in acc.items()}
    out["s_pi_q1"] = sq1 / Z / L
    return out
