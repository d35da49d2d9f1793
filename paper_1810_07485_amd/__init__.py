"""MI355X-native continuous-time loop-cluster QMC (arXiv:1810.07485).

Thin ctypes binding of ``liblc.so`` (C ABI in ``include/lc.h``): argument
marshalling only; every step of a sweep runs in the library's HIP kernels.
PyTorch supplies device memory (its caching allocator) and the HIP stream.

There is no CPU fallback: importing works without a GPU (so the build can be
checked), but creating a chain needs the compiled library and a device.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

from . import build as _build

__all__ = ["load", "Chain", "Batch", "SwIsing", "lc_footprint", "lc_strerror", "LcError",
           "lc_debug_philox", "lc_debug_window_table", "SweepStats", "Measurement"]

SO = _build.SO

LC_OK, LC_EINVAL, LC_ENOMEM, LC_ETOOLARGE, LC_ECAPACITY, LC_EDEVICE, LC_ESTATE = 0, -1, -2, -3, -4, -5, -6
FLIP_LABEL, FLIP_VOTE = 0, 1


class LcError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {lc_strerror(code)} ({code})")
        self.code = code


class SweepStats(C.Structure):
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


class Fourier(C.Structure):
    _fields_ = [("chi_pi", C.c_double), ("chi_pi_q1", C.c_double), ("chi_pi_w1", C.c_double),
                ("s_pi_q1", C.c_double), ("n_loops", C.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Measurement(C.Structure):
    _fields_ = [("n_sweeps", C.c_int64), ("e", C.c_double), ("chi_u", C.c_double),
                ("chi_u_plain", C.c_double), ("s_pi", C.c_double), ("chi_s", C.c_double),
                ("mean_ops", C.c_double), ("mean_clusters", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class Alloc(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


_lib = None


def load():
    """Load the compiled library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO):
        raise RuntimeError(f"{SO} is missing: run paper_1810_07485_amd/build.py (or "
                           "__graft_entry__.build()) first; there is no fallback path")
    # torch first: its bundled HIP runtime is then the one the library binds
    # to.  Loaded the other way round, the process would hold two HIP
    # runtimes, and torch's device memory and streams would be foreign to
    # the library's (every call fails with LC_EDEVICE).
    import torch  # noqa: F401
    L = C.CDLL(SO)
    p64, pu64, pu8, pi = (C.POINTER(C.c_int64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint8),
                          C.POINTER(C.c_int))
    vp = C.c_void_p
    sig = {
        "lc_footprint": ([C.c_int64, C.c_double, C.c_double, C.POINTER(C.c_size_t)], C.c_int),
        "lc_footprint_parts": ([C.c_int64, C.c_double, C.c_double, C.POINTER(C.c_size_t),
                                C.POINTER(C.c_size_t)], C.c_int),
        "lc_autotune": ([vp, pi, C.c_int, C.c_int, pi, C.POINTER(C.c_double)], C.c_int),
        "lc_batch_autotune": ([vp, pi, C.c_int, C.c_int, pi, C.POINTER(C.c_double)], C.c_int),
        "lc_init_lattice": ([C.c_int64, C.c_double, C.c_double, C.c_uint64, C.POINTER(Alloc), vp,
                             C.POINTER(vp)], C.c_int),
        "lc_update": ([vp, C.c_int64, C.c_int], C.c_int),
        "lc_update_noalloc": ([vp, C.c_int64, C.c_int], C.c_int),
        "lc_set_flip_rule": ([vp, C.c_int], C.c_int),
        "lc_measure": ([vp, C.POINTER(Measurement)], C.c_int),
        "lc_last_sweep": ([vp, C.POINTER(SweepStats)], C.c_int),
        "lc_reset_measurements": ([vp], C.c_int),
        "lc_export_state": ([vp, pu8, p64, pu64, p64, p64], C.c_int),
        "lc_import_state": ([vp, pu8, p64, pu64, C.c_int64], C.c_int),
        "lc_export_ops": ([vp, p64, pu64, pu8, pu8, p64], C.c_int),
        "lc_export_labels": ([vp, p64, p64], C.c_int),
        "lc_export_perm": ([vp, p64, p64], C.c_int),
        "lc_fourier_last": ([vp, C.POINTER(Fourier)], C.c_int),
        "lc_slice_tables": ([vp, C.c_int, p64, p64, p64, p64], C.c_int),
        "lc_free": ([vp], None),
        "lc_strerror": ([C.c_int], C.c_char_p),
        "lc_batch_create": ([C.POINTER(Alloc), vp, C.POINTER(vp)], C.c_int),
        "lc_batch_add": ([vp, vp], C.c_int),
        "lc_batch_remove": ([vp, vp], C.c_int),
        "lc_batch_size": ([vp, pi], C.c_int),
        "lc_batch_update": ([vp, C.c_int64, C.c_int], C.c_int),
        "lc_batch_set_schedule": ([vp, C.c_int, C.c_int], C.c_int),
        "lc_batch_scratch_bytes": ([vp, C.POINTER(C.c_size_t)], C.c_int),
        "lc_batch_free": ([vp], None),
        "lc_set_schedule": ([vp, C.c_int, C.c_int], C.c_int),
        "lc_set_tile": ([vp, C.c_int, C.c_int], C.c_int),
        "lc_autotune_tiles": ([vp, pi, pi, C.c_int, pi, C.c_int, C.c_int, pi, pi,
                               C.POINTER(C.c_double)], C.c_int),
        "lc_batch_autotune_tiles": ([vp, pi, pi, C.c_int, pi, C.c_int, C.c_int, pi, pi,
                                     C.POINTER(C.c_double)], C.c_int),
        "lc_capacity": ([vp, p64, C.POINTER(C.c_size_t)], C.c_int),
        "lc_phase_count": ([], C.c_int),
        "lc_phase_name": ([C.c_int], C.c_char_p),
        "lc_set_profiling": ([vp, C.c_int], C.c_int),
        "lc_profile": ([vp, C.POINTER(C.c_double), C.c_int, p64], C.c_int),
        "lc_batch_set_profiling": ([vp, C.c_int], C.c_int),
        "lc_batch_profile": ([vp, C.POINTER(C.c_double), C.c_int, p64], C.c_int),
        "lc_probe_cas": ([C.c_int, C.c_int64, C.c_int, vp, C.POINTER(C.c_double),
                          C.POINTER(C.c_double)], C.c_int),
        "lc_probe_copy": ([C.c_int64, C.c_int, vp, C.POINTER(C.c_double)], C.c_int),
        "lc_debug_philox": ([C.c_uint64, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)], C.c_int),
        "lc_debug_window_table": ([C.c_double, pi, C.POINTER(C.c_double), pu64, pi], C.c_int),
        "lc_debug_work": ([vp, p64, p64], C.c_int),
        "lc_sw_init": ([C.c_int64, C.c_double, C.c_uint64, C.POINTER(Alloc), vp, C.POINTER(vp)],
                       C.c_int),
        "lc_sw_update": ([vp, C.c_int64], C.c_int),
        "lc_sw_last": ([vp, C.POINTER(SwStats)], C.c_int),
        "lc_sw_export": ([vp, pu8, p64], C.c_int),
        "lc_sw_set_profiling": ([vp, C.c_int], C.c_int),
        "lc_sw_phase_count": ([], C.c_int),
        "lc_sw_phase_name": ([C.c_int], C.c_char_p),
        "lc_sw_profile": ([vp, C.POINTER(C.c_double), C.c_int, p64], C.c_int),
        "lc_sw_work": ([vp, p64], C.c_int),
        "lc_sw_free": ([vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def lc_strerror(code: int) -> str:
    try:
        return load().lc_strerror(code).decode()
    except RuntimeError:
        return str(code)


def _check(rc: int, what: str):
    if rc != LC_OK:
        raise LcError(rc, what)


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


# linking-tile shapes the tile tuner tries: (max windows per tile, operator target)
DEFAULT_TILE_SHAPES = ((0, 0), (4, 1500), (8, 1100), (16, 1500), (1, 1100))


def _autotune_tiles(fn, h, shapes, grids, trial_sweeps):
    shapes = list(shapes)
    win = (C.c_int * len(shapes))(*[int(w) for w, _ in shapes])
    tgt = (C.c_int * len(shapes))(*[int(t) for _, t in shapes])
    g = (C.c_int * len(grids))(*[int(x) for x in grids])
    bs, bg, ms = C.c_int(), C.c_int(), C.c_double()
    _check(fn(h, win, tgt, len(shapes), g, len(grids), int(trial_sweeps), C.byref(bs), C.byref(bg),
              C.byref(ms)), fn.__name__)
    return shapes[bs.value], bg.value, ms.value


def lc_footprint(L: int, S: float, beta: float) -> int:
    n = C.c_size_t()
    _check(load().lc_footprint(int(L), float(S), float(beta), C.byref(n)), "lc_footprint")
    return n.value


def lc_footprint_parts(L: int, S: float, beta: float) -> tuple:
    """(state bytes, scratch bytes) of one chain (see lc_footprint_parts)."""
    st, sc = C.c_size_t(), C.c_size_t()
    _check(load().lc_footprint_parts(int(L), float(S), float(beta), C.byref(st), C.byref(sc)),
           "lc_footprint_parts")
    return st.value, sc.value


def _autotune(fn, h, grids, trial_sweeps):
    g = (C.c_int * len(grids))(*[int(x) for x in grids])
    best, ms = C.c_int(), C.c_double()
    _check(fn(h, g, len(grids), int(trial_sweeps), C.byref(best), C.byref(ms)), "autotune")
    return best.value, ms.value


DEFAULT_GRIDS = (2048, 4096, 8192, 16384)


def lc_debug_philox(seed: int, ctr) -> tuple:
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    o = (C.c_uint32 * 4)()
    _check(load().lc_debug_philox(C.c_uint64(seed), c, o), "lc_debug_philox")
    return tuple(o)


def lc_debug_window_table(beta: float):
    w, mu, K = C.c_int(), C.c_double(), C.c_int()
    T = (C.c_uint64 * 64)()
    _check(load().lc_debug_window_table(float(beta), C.byref(w), C.byref(mu), T, C.byref(K)),
           "lc_debug_window_table")
    return w.value, mu.value, [T[i] for i in range(K.value)]


def lc_probe_cas(log2_words: int, n_cas: int = 1 << 26, repeats: int = 3, stream=None) -> tuple:
    """(random 8-byte CAS per second, success fraction) on 2^log2_words words."""
    r, f = C.c_double(), C.c_double()
    h = C.c_void_p(stream.cuda_stream) if stream is not None else None
    _check(load().lc_probe_cas(int(log2_words), int(n_cas), int(repeats), h, C.byref(r), C.byref(f)),
           "lc_probe_cas")
    return r.value, f.value


def lc_probe_copy(nbytes: int, repeats: int = 3, stream=None) -> float:
    """Device-to-device streaming copy: bytes read + written per second / 1e9."""
    r = C.c_double()
    h = C.c_void_p(stream.cuda_stream) if stream is not None else None
    _check(load().lc_probe_copy(int(nbytes), int(repeats), h, C.byref(r)), "lc_probe_copy")
    return r.value


class _TorchMemory:
    """Device memory and stream from PyTorch (its caching allocator)."""

    def __init__(self, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the loop-cluster library runs only on the device")
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        dev = self.stream.device

        def _alloc(nbytes, _stream, _ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, self.stream)
            except Exception as e:  # out of memory -> NULL, reported as LC_ENOMEM
                if os.environ.get("LC_VERBOSE", "0") not in ("", "0"):
                    print(f"[lc] torch allocation of {int(nbytes)} bytes failed: {e}",
                          file=sys.stderr, flush=True)
                return None

        def _free(ptr, _nbytes, _stream, _ctx):
            torch.cuda.caching_allocator_delete(ptr)

        self._fa, self._ff = ALLOC_FN(_alloc), FREE_FN(_free)
        self.alloc = Alloc(self._fa, self._ff, None)

    @property
    def handle(self):
        return C.c_void_p(self.stream.cuda_stream)


_MEMORIES = {}
_STREAMS = {}
_LIVE = weakref.WeakSet()  # chains and batches to release before interpreter teardown


@atexit.register
def _close_all():
    # batches first: they hold chains
    for o in sorted(list(_LIVE), key=lambda o: not isinstance(o, Batch)):
        o.close()


def library_stream(device=None):
    """The stream chains and batches use by default: one per device, created
    by torch at default priority.  (The legacy null stream cannot be captured
    into graphs, and engines on one stream share one scratch arena.)"""
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)
    st = _STREAMS.get(dev)
    if st is None:
        st = _STREAMS[dev] = torch.cuda.Stream(device=dev)
    return st


def _torch_memory(stream=None) -> _TorchMemory:
    """One allocator object per torch stream: engines with the same stream and
    allocator share the library's per-sweep scratch arena."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the loop-cluster library runs only on the device")
    st = stream if stream is not None else library_stream()
    key = (st.device.index, st.cuda_stream)
    m = _MEMORIES.get(key)
    if m is None:
        m = _MEMORIES[key] = _TorchMemory(st)
    return m


class Chain:
    """One Markov chain: ``lc_init_lattice`` / ``lc_update`` / ``lc_measure``."""

    def __init__(self, L: int, S: float, beta: float, seed: int, stream=None,
                 torch_memory: bool = True):
        lib = load()
        self.L, self.S, self.beta, self.seed = int(L), float(S), float(beta), int(seed)
        self.two_s = int(round(2 * S))
        self._mem = _torch_memory(stream) if torch_memory else None
        h = C.c_void_p()
        alloc = C.byref(self._mem.alloc) if self._mem else None
        strm = self._mem.handle if self._mem else None
        _check(lib.lc_init_lattice(self.L, self.S, self.beta, C.c_uint64(self.seed), alloc, strm,
                                   C.byref(h)), "lc_init_lattice")
        self._h = h
        self._lib = lib
        self.n_sites = self.two_s * self.L
        self.n_bonds = self.two_s * self.two_s * self.L
        _LIVE.add(self)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.lc_free(h)
        self._h = None

    __del__ = close

    def update(self, n_sweeps: int = 1, accumulate: bool = True):
        _check(load().lc_update(self._h, int(n_sweeps), int(bool(accumulate))), "lc_update")

    def set_flip_rule(self, rule: int):
        """FLIP_LABEL (default) or FLIP_VOTE (majority-vote XOR, lc_set_flip_rule)."""
        _check(load().lc_set_flip_rule(self._h, int(rule)), "lc_set_flip_rule")

    def update_noalloc(self, n_sweeps: int = 1, accumulate: bool = True):
        """lc_update_noalloc: the same sweeps with no allocation (static scratch)."""
        _check(load().lc_update_noalloc(self._h, int(n_sweeps), int(bool(accumulate))),
               "lc_update_noalloc")

    def fourier(self) -> dict:
        """Fourier-mode estimators of the most recent sweep (lc_fourier_last):
        chi(pi, 0), chi(pi + 2 pi/L, 0), chi(pi, 2 pi/beta), S(pi + 2 pi/L)."""
        f = Fourier()
        _check(load().lc_fourier_last(self._h, C.byref(f)), "lc_fourier_last")
        return f.as_dict()

    def capacity(self) -> tuple:
        """(kept operators per world-line buffer, scratch arena bytes), lc_capacity."""
        k, b = C.c_int64(), C.c_size_t()
        _check(load().lc_capacity(self._h, C.byref(k), C.byref(b)), "lc_capacity")
        return k.value, b.value

    def measure(self) -> dict:
        m = Measurement()
        _check(load().lc_measure(self._h, C.byref(m)), "lc_measure")
        return m.as_dict()

    def last_sweep(self) -> dict:
        s = SweepStats()
        _check(load().lc_last_sweep(self._h, C.byref(s)), "lc_last_sweep")
        return s.as_dict()

    def reset_measurements(self):
        _check(load().lc_reset_measurements(self._h), "lc_reset_measurements")

    def set_schedule(self, grid_blocks: int = 0, use_graph: bool = True):
        _check(load().lc_set_schedule(self._h, int(grid_blocks), int(bool(use_graph))),
               "lc_set_schedule")

    def set_profiling(self, on: bool = True):
        _check(load().lc_set_profiling(self._h, int(bool(on))), "lc_set_profiling")

    def autotune(self, grids=DEFAULT_GRIDS, trial_sweeps: int = 2) -> tuple:
        """Pick the fastest grid size (runs real, unaccumulated sweeps)."""
        return _autotune(load().lc_autotune, self._h, grids, trial_sweeps)

    def set_tile(self, max_windows: int = 0, target_ops: int = 0):
        """Linking-tile shape (lc_set_tile; 0, 0: the default)."""
        _check(load().lc_set_tile(self._h, int(max_windows), int(target_ops)), "lc_set_tile")

    def autotune_tiles(self, shapes=DEFAULT_TILE_SHAPES, grids=DEFAULT_GRIDS, trial_sweeps: int = 2):
        """Fastest (tile shape, grid) pair: ((max_windows, target_ops), grid, ms per sweep)."""
        return _autotune_tiles(load().lc_autotune_tiles, self._h, shapes, grids, trial_sweeps)

    def profile(self) -> tuple:
        """(dict phase -> summed ms, sweeps) since profiling was switched on."""
        return _profile(load().lc_profile, self._h)

    def work(self) -> tuple:
        """(edges between linking tiles, open fragments) of the last sweep."""
        x, f = C.c_int64(), C.c_int64()
        _check(load().lc_debug_work(self._h, C.byref(x), C.byref(f)), "lc_debug_work")
        return x.value, f.value

    def export_state(self):
        lib = load()
        n, sw = C.c_int64(0), C.c_int64()
        _check(lib.lc_export_state(self._h, None, None, None, C.byref(n), C.byref(sw)),
               "lc_export_state")
        s0 = np.zeros(self.n_sites, np.uint8)
        off = np.zeros(self.n_bonds + 1, np.int64)
        t = np.zeros(max(n.value, 1), np.uint64)
        n = C.c_int64(t.size)
        _check(lib.lc_export_state(self._h, _p(s0, C.c_uint8), _p(off, C.c_int64),
                                   _p(t, C.c_uint64), C.byref(n), C.byref(sw)), "lc_export_state")
        return s0, off, t[: n.value].copy(), sw.value

    def import_state(self, s0, bond_off, times, sweep: int):
        s0 = np.ascontiguousarray(s0, np.uint8)
        off = np.ascontiguousarray(bond_off, np.int64)
        t = np.ascontiguousarray(times, np.uint64)
        if t.size == 0:
            t = np.zeros(1, np.uint64)
        _check(load().lc_import_state(self._h, _p(s0, C.c_uint8), _p(off, C.c_int64),
                                      _p(t, C.c_uint64), int(sweep)), "lc_import_state")

    def export_ops(self):
        lib = load()
        n = C.c_int64(0)
        _check(lib.lc_export_ops(self._h, None, None, None, None, C.byref(n)), "lc_export_ops")
        k = n.value
        b = np.zeros(max(k, 1), np.int64)
        t = np.zeros(max(k, 1), np.uint64)
        t0 = np.zeros(max(k, 1), np.uint8)
        t1 = np.zeros(max(k, 1), np.uint8)
        n = C.c_int64(b.size)
        _check(lib.lc_export_ops(self._h, _p(b, C.c_int64), _p(t, C.c_uint64), _p(t0, C.c_uint8),
                                 _p(t1, C.c_uint8), C.byref(n)), "lc_export_ops")
        return b[:k].copy(), t[:k].copy(), t0[:k].copy(), t1[:k].copy()

    def export_labels(self):
        lib = load()
        n = C.c_int64(0)
        _check(lib.lc_export_labels(self._h, None, C.byref(n)), "lc_export_labels")
        k = n.value
        lab = np.zeros(max(k, 1), np.int64)
        n = C.c_int64(lab.size)
        _check(lib.lc_export_labels(self._h, _p(lab, C.c_int64), C.byref(n)), "lc_export_labels")
        return lab[:k].copy()

    def export_perm(self):
        lib = load()
        n = C.c_int64(0)
        _check(lib.lc_export_perm(self._h, None, C.byref(n)), "lc_export_perm")
        k = n.value
        p = np.zeros(max(k, 1), np.int64)
        n = C.c_int64(p.size)
        _check(lib.lc_export_perm(self._h, _p(p, C.c_int64), C.byref(n)), "lc_export_perm")
        return p[:k].copy()


class SwIsing:
    """Swendsen-Wang update of the L x L periodic Ising model at coupling K on
    the library's union-find (``lc_sw_init`` / ``lc_sw_update``)."""

    def __init__(self, L: int, K: float, seed: int, stream=None):
        lib = load()
        self.L, self.K, self.seed = int(L), float(K), int(seed)
        self._mem = _torch_memory(stream)
        h = C.c_void_p()
        _check(lib.lc_sw_init(self.L, self.K, C.c_uint64(self.seed), C.byref(self._mem.alloc),
                              self._mem.handle, C.byref(h)), "lc_sw_init")
        self._h = h
        self._lib = lib
        _LIVE.add(self)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.lc_sw_free(h)
        self._h = None

    __del__ = close

    def update(self, n_sweeps: int = 1):
        _check(self._lib.lc_sw_update(self._h, int(n_sweeps)), "lc_sw_update")

    def last_sweep(self) -> dict:
        st = SwStats()
        _check(self._lib.lc_sw_last(self._h, C.byref(st)), "lc_sw_last")
        return st.as_dict()

    def spins(self) -> np.ndarray:
        s = np.zeros(self.L * self.L, np.uint8)
        _check(self._lib.lc_sw_export(self._h, _p(s, C.c_uint8), None), "lc_sw_export")
        return s

    def labels(self) -> np.ndarray:
        lab = np.zeros(self.L * self.L, np.int64)
        _check(self._lib.lc_sw_export(self._h, None, _p(lab, C.c_int64)), "lc_sw_export")
        return lab

    def set_profiling(self, on: bool):
        _check(self._lib.lc_sw_set_profiling(self._h, int(bool(on))), "lc_sw_set_profiling")

    def profile(self) -> tuple:
        """({kernel phase: summed ms}, profiled sweeps)."""
        lib = self._lib
        k = lib.lc_sw_phase_count()
        ms, n = (C.c_double * k)(), C.c_int64()
        _check(lib.lc_sw_profile(self._h, ms, k, C.byref(n)), "lc_sw_profile")
        return {lib.lc_sw_phase_name(i).decode(): ms[i] for i in range(k)}, n.value

    def work(self) -> int:
        """Tile-local components (records) of the most recent sweep."""
        v = C.c_int64()
        _check(self._lib.lc_sw_work(self._h, C.byref(v)), "lc_sw_work")
        return v.value


def slice_tables(chain, n_slices: int):
    """lc_slice_tables: (bottom[G, ns], top[G, ns], op_labels[2 n_ops]) of the
    chain's most recent sweep cut into n_slices open-boundary time slices."""
    lib = load()
    n = C.c_int64(0)
    _check(lib.lc_slice_tables(chain._h, int(n_slices), None, None, None, C.byref(n)),
           "lc_slice_tables")
    k = n.value
    ns = chain.n_sites
    bot = np.zeros((int(n_slices), ns), np.int64)
    top = np.zeros((int(n_slices), ns), np.int64)
    lab = np.zeros(max(2 * k, 1), np.int64)
    n = C.c_int64(k)
    _check(lib.lc_slice_tables(chain._h, int(n_slices), _p(bot, C.c_int64), _p(top, C.c_int64),
                               _p(lab, C.c_int64), C.byref(n)), "lc_slice_tables")
    return bot, top, lab[: 2 * k].copy()


class Batch:
    """Many chains advanced by one launch sequence per sweep (``lc_batch_*``)."""

    def __init__(self, stream=None, torch_memory: bool = True):
        lib = load()
        self._mem = _torch_memory(stream) if torch_memory else None
        h = C.c_void_p()
        alloc = C.byref(self._mem.alloc) if self._mem else None
        strm = self._mem.handle if self._mem else None
        _check(lib.lc_batch_create(alloc, strm, C.byref(h)), "lc_batch_create")
        self._h = h
        self._lib = lib
        self.members = []
        _LIVE.add(self)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.lc_batch_free(h)
        self._h = None
        self.members = []

    __del__ = close

    def add(self, chain: Chain):
        _check(load().lc_batch_add(self._h, chain._h), "lc_batch_add")
        self.members.append(chain)

    def remove(self, chain: Chain):
        _check(load().lc_batch_remove(self._h, chain._h), "lc_batch_remove")
        self.members.remove(chain)

    def update(self, n_sweeps: int = 1, accumulate: bool = True):
        _check(load().lc_batch_update(self._h, int(n_sweeps), int(bool(accumulate))),
               "lc_batch_update")

    def set_schedule(self, grid_blocks: int = 0, use_graph: bool = True):
        _check(load().lc_batch_set_schedule(self._h, int(grid_blocks), int(bool(use_graph))),
               "lc_batch_set_schedule")

    def set_profiling(self, on: bool = True):
        _check(load().lc_batch_set_profiling(self._h, int(bool(on))), "lc_batch_set_profiling")

    def scratch_bytes(self) -> int:
        """Device bytes of the scratch arena this batch uses (lc_batch_scratch_bytes)."""
        n = C.c_size_t()
        _check(load().lc_batch_scratch_bytes(self._h, C.byref(n)), "lc_batch_scratch_bytes")
        return n.value

    def autotune(self, grids=DEFAULT_GRIDS, trial_sweeps: int = 2) -> tuple:
        """Pick the fastest grid size (runs real, unaccumulated sweeps)."""
        return _autotune(load().lc_batch_autotune, self._h, grids, trial_sweeps)

    def autotune_tiles(self, shapes=DEFAULT_TILE_SHAPES, grids=DEFAULT_GRIDS, trial_sweeps: int = 2):
        """Fastest (tile shape, grid) pair for every member: ((max_windows,
        target_ops), grid, ms per sweep)."""
        return _autotune_tiles(load().lc_batch_autotune_tiles, self._h, shapes, grids, trial_sweeps)

    def profile(self) -> tuple:
        return _profile(load().lc_batch_profile, self._h)


def phase_names() -> list:
    lib = load()
    return [lib.lc_phase_name(i).decode() for i in range(lib.lc_phase_count())]


def _profile(fn, h) -> tuple:
    names = phase_names()
    ms = (C.c_double * len(names))()
    n = C.c_int64()
    _check(fn(h, ms, len(names), C.byref(n)), "lc_profile")
    return dict(zip(names, list(ms))), n.value
