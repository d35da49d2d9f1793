"""Write per-sweep digests of the oracle at the medium single-chain size.

Calls only ``oracle/``.  For the S=1/2 chain L=65,536, beta=4,096, seed 1,
started from its initial Neel state, it records for each of the first
sweeps: every integer of the sweep statistics and SHA-256 digests of the
world lines after the sweep (spins, per-bond offsets, kept times), of the
operators of the sweep (bond, time, type before the flip) and of the loop
labels.  The GPU test recomputes the same digests from the library.

Run:  python tests/golden/make_digest_golden.py [n_sweeps]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle  # noqa: E402

L, S, BETA, SEED = 65536, 0.5, 4096.0, 1


def sha(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 3
    ch = oracle.Chain(L, S, BETA, SEED)
    w, mu, T = oracle.window_table(BETA)
    out = dict(L=L, S=S, beta=BETA, seed=SEED, window_w=w, mu=mu,
               thresholds=[str(t) for t in T], sweeps=[])
    for s in range(n):
        t0 = time.time()
        st = ch.sweep()
        s0, off, kt, sw = ch.export_state()
        b, t, ty0 = ch.export_ops()
        lab = ch.export_labels()
        rec = dict(stats={k: int(v) for k, v in st.items()},
                   state=sha(s0, off, kt), ops=sha(b.astype(np.int64), t, ty0),
                   labels=sha(lab), next_sweep=int(sw))
        out["sweeps"].append(rec)
        print(s, f"{time.time() - t0:.0f}s", rec["stats"]["n_ops"], flush=True)
        del b, t, ty0, lab
    with open(os.path.join(HERE, "digest_L65536_beta4096.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
