"""ctypes binding of the sequential CPU oracle (``lc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; never by the product package.

The oracle is the plain definition of one continuous-time loop-cluster update
(arXiv:1810.07485, Sec. 2, the enumerated steps 1-8); see ``lc_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liblc_oracle.so")
SRC = os.path.join(HERE, "lc_oracle.c")
SRCS = [SRC, os.path.join(HERE, "sw_oracle.c")]

ORC_DOM_INIT, ORC_DOM_INS, ORC_DOM_FLIP, ORC_DOM_SYM = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no contraction of a*b+c)."""
    if force or not os.path.exists(SO):
        tmp = SO + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, *SRCS, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, SO)
    return SO


class Stats(C.Structure):
    _fields_ = [
        ("sweep", C.c_int64), ("n_ops", C.c_int64), ("n_cand", C.c_int64),
        ("n_acc", C.c_int64), ("n_kept_in", C.c_int64), ("n_kept_out", C.c_int64),
        ("n_nodes", C.c_int64), ("n_clusters", C.c_int64),
        ("sum_m2", C.c_uint64), ("sum_n0sq", C.c_uint64),
        ("sum_size2_lo", C.c_uint64), ("sum_size2_hi", C.c_uint64),
        ("sum_len2_lo", C.c_uint64), ("sum_len2_hi", C.c_uint64),
        ("m_after", C.c_int64), ("max_size", C.c_int64),
    ]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["sum_size2"] = d.pop("sum_size2_lo") | (d.pop("sum_size2_hi") << 64)
        d["sum_len2"] = d.pop("sum_len2_lo") | (d.pop("sum_len2_hi") << 64)
        return d


class SwStats(C.Structure):
    _fields_ = [("sweep", C.c_int64), ("energy", C.c_int64), ("magnetization", C.c_int64),
                ("n_active", C.c_int64), ("n_clusters", C.c_int64), ("size2_lo", C.c_uint64),
                ("size2_hi", C.c_uint64), ("max_size", C.c_int64)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["size2"] = d.pop("size2_lo") | (d.pop("size2_hi") << 64)
        return d


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            build()
        L = C.CDLL(SO)
        p64, pu64, pu8, pi32 = (C.POINTER(C.c_int64), C.POINTER(C.c_uint64),
                                C.POINTER(C.c_uint8), C.POINTER(C.c_int))
        L.orc_philox.argtypes = [C.c_uint64, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_window_table.argtypes = [C.c_double, pi32, C.POINTER(C.c_double), pu64, pi32]
        L.orc_flip_bit.argtypes = [C.c_uint64, C.c_int64, C.c_int64]
        L.orc_vote_bit.argtypes = [C.c_uint64, C.c_int64, C.c_int64]
        L.orc_set_flip_rule.argtypes = [C.c_void_p, C.c_int]
        L.orc_set_fourier.argtypes = [C.c_void_p, C.c_int]
        L.orc_fourier_last.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
        L.orc_create.argtypes = [C.c_int64, C.c_int, C.c_double, C.c_uint64,
                                 C.POINTER(C.c_void_p)]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_free.restype = None
        L.orc_sweep.argtypes = [C.c_void_p, C.POINTER(Stats)]
        L.orc_sizes.argtypes = [C.c_void_p, p64, p64, p64, p64]
        L.orc_export_state.argtypes = [C.c_void_p, pu8, p64, pu64, p64, p64]
        L.orc_import_state.argtypes = [C.c_void_p, pu8, p64, pu64, C.c_int64]
        L.orc_export_ops.argtypes = [C.c_void_p, p64, pu64, pu8, p64]
        L.orc_export_labels.argtypes = [C.c_void_p, p64, p64]
        L.orc_export_perm.argtypes = [C.c_void_p, p64, p64]
        L.orc_sw_threshold.argtypes = [C.c_double]
        L.orc_sw_threshold.restype = C.c_uint64
        L.orc_sw_create.argtypes = [C.c_int64, C.c_double, C.c_uint64, C.POINTER(C.c_void_p)]
        L.orc_sw_free.argtypes = [C.c_void_p]
        L.orc_sw_free.restype = None
        L.orc_sw_sweep.argtypes = [C.c_void_p, C.POINTER(SwStats)]
        L.orc_sw_export.argtypes = [C.c_void_p, pu8, p64]
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def philox(seed: int, ctr) -> tuple:
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    o = (C.c_uint32 * 4)()
    lib().orc_philox(C.c_uint64(seed), c, o)
    return tuple(o)


def window_table(beta: float):
    w, mu, K = C.c_int(), C.c_double(), C.c_int()
    T = (C.c_uint64 * 64)()
    rc = lib().orc_window_table(float(beta), C.byref(w), C.byref(mu), T, C.byref(K))
    if rc != 0:
        raise ValueError(f"orc_window_table rc={rc}")
    return w.value, mu.value, [T[i] for i in range(K.value)]


def flip_bit(seed: int, sweep: int, label: int) -> int:
    return int(lib().orc_flip_bit(C.c_uint64(seed), sweep, label))


def vote_bit(seed: int, sweep: int, node: int) -> int:
    return int(lib().orc_vote_bit(C.c_uint64(seed), sweep, node))


FLIP_LABEL, FLIP_VOTE = 0, 1


class Chain:
    """One Markov chain of the oracle."""

    def __init__(self, L: int, S: float, beta: float, seed: int):
        two_s = int(round(2 * S))
        self.L, self.two_s, self.beta, self.seed = int(L), two_s, float(beta), int(seed)
        h = C.c_void_p()
        rc = lib().orc_create(int(L), two_s, float(beta), C.c_uint64(seed), C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_create rc={rc}")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc_free(h)
            self._h = None

    def set_flip_rule(self, rule: int):
        """FLIP_LABEL (default) or FLIP_VOTE (XOR of the nodes' votes, Sec. 3.3)."""
        rc = lib().orc_set_flip_rule(self._h, int(rule))
        if rc != 0:
            raise ValueError(f"orc_set_flip_rule rc={rc}")

    def set_fourier(self, on: bool = True):
        """Compute the Fourier-mode estimators in the following sweeps."""
        rc = lib().orc_set_fourier(self._h, int(bool(on)))
        if rc != 0:
            raise ValueError(f"orc_set_fourier rc={rc}")

    def fourier(self) -> dict:
        """Single-sweep improved estimates of the most recent sweep:
        chi(pi, 0), chi(pi + 2 pi/L, 0), chi(pi, 2 pi/beta), S(pi + 2 pi/L)."""
        o = (C.c_double * 4)()
        rc = lib().orc_fourier_last(self._h, o)
        if rc != 0:
            raise RuntimeError(f"orc_fourier_last rc={rc}")
        return dict(chi_pi=o[0], chi_pi_q1=o[1], chi_pi_w1=o[2], s_pi_q1=o[3])

    def sizes(self):
        a, b, c, d = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        lib().orc_sizes(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d))
        return dict(n_sites=a.value, n_bonds=b.value, n_kept=c.value, sweep=d.value)

    def sweep(self) -> dict:
        st = Stats()
        rc = lib().orc_sweep(self._h, C.byref(st))
        if rc != 0:
            raise RuntimeError(f"orc_sweep rc={rc}")
        return st.as_dict()

    def export_state(self):
        sz = self.sizes()
        s0 = np.zeros(sz["n_sites"], np.uint8)
        off = np.zeros(sz["n_bonds"] + 1, np.int64)
        t = np.zeros(max(sz["n_kept"], 1), np.uint64)
        cap, sw = C.c_int64(t.size), C.c_int64()
        rc = lib().orc_export_state(self._h, _ptr(s0, C.c_uint8), _ptr(off, C.c_int64),
                                    _ptr(t, C.c_uint64), C.byref(cap), C.byref(sw))
        if rc != 0:
            raise RuntimeError(f"orc_export_state rc={rc}")
        return s0, off, t[: cap.value].copy(), sw.value

    def import_state(self, s0, bond_off, times, sweep: int):
        s0 = np.ascontiguousarray(s0, np.uint8)
        off = np.ascontiguousarray(bond_off, np.int64)
        t = np.ascontiguousarray(times, np.uint64)
        if t.size == 0:
            t = np.zeros(1, np.uint64)
        rc = lib().orc_import_state(self._h, _ptr(s0, C.c_uint8), _ptr(off, C.c_int64),
                                    _ptr(t, C.c_uint64), int(sweep))
        if rc != 0:
            raise ValueError(f"orc_import_state rc={rc}")

    def export_ops(self):
        cap = C.c_int64(0)
        lib().orc_export_ops(self._h, None, None, None, C.byref(cap))
        n = cap.value
        b = np.zeros(max(n, 1), np.int64)
        t = np.zeros(max(n, 1), np.uint64)
        ty = np.zeros(max(n, 1), np.uint8)
        cap = C.c_int64(b.size)
        rc = lib().orc_export_ops(self._h, _ptr(b, C.c_int64), _ptr(t, C.c_uint64),
                                  _ptr(ty, C.c_uint8), C.byref(cap))
        if rc != 0:
            raise RuntimeError(f"orc_export_ops rc={rc}")
        return b[:n].copy(), t[:n].copy(), ty[:n].copy()

    def export_labels(self):
        cap = C.c_int64(0)
        lib().orc_export_labels(self._h, None, C.byref(cap))
        lab = np.zeros(max(cap.value, 1), np.int64)
        n = cap.value
        cap = C.c_int64(lab.size)
        rc = lib().orc_export_labels(self._h, _ptr(lab, C.c_int64), C.byref(cap))
        if rc != 0:
            raise RuntimeError(f"orc_export_labels rc={rc}")
        return lab[:n].copy()

    def export_perm(self):
        cap = C.c_int64(0)
        lib().orc_export_perm(self._h, None, C.byref(cap))
        n = cap.value
        p = np.zeros(max(n, 1), np.int64)
        cap = C.c_int64(p.size)
        rc = lib().orc_export_perm(self._h, _ptr(p, C.c_int64), C.byref(cap))
        if rc != 0:
            raise RuntimeError(f"orc_export_perm rc={rc}")
        return p[:n].copy()


def observables(stats_list, L: int, S: float, beta: float) -> dict:
    """FP64 observables from per-sweep exact integers (Sec. 2 step 8).

    e      = N_b/(4L) - <N_ops>/(beta L)      (N_b = (2S)^2 L sub-bonds)
    chi_u  = beta/(4L) <sum_c m_c^2>            improved estimator
    chi_u0 = beta/(4L) <(sum_j (2 s_j - 1))^2>  plain estimator
    s_pi   = <sum_c n0_c^2> / (4L)
    chi_s  = beta/(4L) <sum_c ((len_c >> 32) / 2^32)^2>
    """
    n = len(stats_list)
    two_s = int(round(2 * S))
    nb = two_s * two_s * L
    sN = sum(s["n_ops"] for s in stats_list)
    sm2 = sum(s["sum_m2"] for s in stats_list)
    sma = sum(s["m_after"] ** 2 for s in stats_list)
    sn0 = sum(s["sum_n0sq"] for s in stats_list)
    sl2 = sum(s["sum_len2"] for s in stats_list)
    return dict(
        e=nb / (4.0 * L) - (sN / n) / (beta * L),
        chi_u=beta / (4.0 * L) * (sm2 / n),
        chi_u_plain=beta / (4.0 * L) * (sma / n),
        s_pi=(sn0 / n) / (4.0 * L),
        chi_s=beta / (4.0 * L) * (sl2 / 2.0**64 / n),
    )


def sw_threshold(K: float) -> int:
    return int(lib().orc_sw_threshold(float(K)))


class SwChain:
    """Swendsen-Wang update of the L x L Ising model (sw_oracle.c)."""

    def __init__(self, L: int, K: float, seed: int):
        self.L, self.K, self.seed = int(L), float(K), int(seed)
        h = C.c_void_p()
        rc = lib().orc_sw_create(self.L, self.K, C.c_uint64(self.seed), C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_sw_create rc={rc}")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc_sw_free(h)
            self._h = None

    def sweep(self) -> dict:
        st = SwStats()
        rc = lib().orc_sw_sweep(self._h, C.byref(st))
        if rc != 0:
            raise RuntimeError(f"orc_sw_sweep rc={rc}")
        return st.as_dict()

    def spins(self):
        s = np.zeros(self.L * self.L, np.uint8)
        lib().orc_sw_export(self._h, _ptr(s, C.c_uint8), None)
        return s

    def labels(self):
        lab = np.zeros(self.L * self.L, np.int64)
        rc = lib().orc_sw_export(self._h, None, _ptr(lab, C.c_int64))
        if rc != 0:
            raise RuntimeError(f"orc_sw_export rc={rc}")
        return lab
