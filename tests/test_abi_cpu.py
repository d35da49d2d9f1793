"""The C-ABI library loads and exports what include/lc.h declares (no GPU).

Also checks the library's host code that needs no device: its twin of
Philox4x32-10 against the published known-answer vectors, and its Poisson
window rule against scipy.stats.poisson.
"""
import ctypes
import os
import re

import numpy as np
import pytest
from scipy import stats

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lc.h")


@pytest.fixture(scope="module")
def lib():
    import paper_1810_07485_amd as lc
    if not os.path.exists(lc.SO):
        from paper_1810_07485_amd import build
        build.build()
    return lc


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lc_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lc_init_lattice", "lc_update", "lc_measure", "lc_export_state",
                     "lc_import_state", "lc_batch_update", "lc_footprint"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    so = ctypes.CDLL(lib.SO)
    missing = [n for n in declared_functions() if not hasattr(so, n)]
    assert not missing, missing


def test_python_binding_loads(lib):
    L = lib.load()
    assert L.lc_strerror(0).decode() == "ok"
    assert lib.lc_strerror(-1) == "invalid argument"


def test_binding_shares_torchs_hip_runtime():
    """The binding loads torch before the library, so the process maps one
    HIP runtime (torch's), even when the library is loaded before the user
    imports torch.  Two runtimes would make torch's device memory and streams
    foreign to the library.  Checked in a fresh process from its memory map."""
    import subprocess
    import sys
    code = ("import paper_1810_07485_amd as lc; lc.load(); import torch; "
            "m = [l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l]; "
            "print(len(set(m)))")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "1", r.stdout


KAT = [
    ((0, 0, 0, 0), 0, (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, 0xFFFFFFFFFFFFFFFF, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), 0x299F31D0A4093822,
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,seed,out", KAT)
def test_library_philox_known_answers(lib, ctr, seed, out):
    assert lib.lc_debug_philox(seed, ctr) == out


@pytest.mark.parametrize("beta", [0.5, 8.0, 8.5, 4096.0, 16384.0, 777.25])
def test_library_window_rule(lib, beta):
    w, mu, T = lib.lc_debug_window_table(beta)
    assert beta / 2 ** w <= 8 and (w == 0 or beta / 2 ** (w - 1) > 8)
    assert mu == beta / 2 ** (w + 1)
    cdf = stats.poisson.cdf(np.arange(len(T) - 1), mu)
    assert np.all(np.abs(np.array(T[:-1], dtype=np.float64) / 2.0 ** 64 - cdf) < 1e-14)
    assert T[-1] == 2 ** 64 - 1


def test_footprint_and_argument_checks(lib):
    b = lib.lc_footprint(65536, 0.5, 4096.0)
    assert 5e9 < b < 6e10
    with pytest.raises(lib.LcError):
        lib.lc_footprint(15, 0.5, 8.0)      # odd L
    with pytest.raises(lib.LcError):
        lib.lc_footprint(16, 0.75, 8.0)     # 2S not an integer
    with pytest.raises(lib.LcError):
        lib.lc_footprint(16, 0.5, -1.0)
    with pytest.raises(lib.LcError):
        lib.lc_footprint(16, 4.5, 1.0)      # 2S > 8
    with pytest.raises(lib.LcError):
        lib.lc_footprint(1 << 32, 0.5, 1.0)   # L beyond 32-bit bond counters
    with pytest.raises(lib.LcError):
        lib.lc_footprint(1 << 27, 4.0, 1.0)   # (2S)^2 L = 2^33 sub-bonds
    assert lib.lc_footprint((1 << 26) - 2, 4.0, 0.01) > 0
