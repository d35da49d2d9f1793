"""Write exact-diagonalization reference values to ``ed_golden.json``.

Calls only ``oracle/ed.py`` (dense LAPACK eigensolvers per S^z sector).
Observables follow the definitions in that module: e = <H>/L,
chi_u = beta <M^2>/L, s_pi = <Ms^2>/L, chi_s = (1/L) int <Ms(tau) Ms(0)>.
The L=16, beta=8 entry is the tiny benchmark instance (S=1/2, periodic).

Run:  python tests/golden/make_ed_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ed  # noqa: E402

CASES = [
    (16, 0.5, 8.0),
    (12, 0.5, 2.0),
    (10, 0.5, 0.5),
    (6, 1.0, 4.0),
    (8, 1.0, 2.0),
    (4, 4.0, 1.0),
]


def main():
    out = []
    for L, S, beta in CASES:
        t0 = time.time()
        r = ed.thermal(L, S, beta, vectors=True)
        r = {k: float(v) for k, v in r.items()}
        out.append(dict(L=L, S=S, beta=beta, **r))
        print(L, S, beta, r, f"{time.time() - t0:.1f}s", flush=True)
    with open(os.path.join(HERE, "ed_golden.json"), "w") as f:
        json.dump(dict(source="oracle/ed.py exact diagonalization", cases=out), f, indent=1)


if __name__ == "__main__":
    main()
