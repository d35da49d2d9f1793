"""Write per-sweep digests of the oracle for one chain.

Calls only ``oracle/``.  For an S chain of L spins at inverse temperature
beta with Philox seed `seed`, started from its initial Neel state, it
records for each sweep: every integer of the sweep statistics and SHA-256
digests of the world lines after the sweep (spins, per-bond offsets, kept
times), of the operators of the sweep (bond, time, type before the flip),
of the loop labels and (split spins) of the symmetrization permutation.  The
GPU tests recompute the same digests from the library.  The file is
rewritten after every sweep, so an interrupted run leaves the sweeps it
finished; with --checkpoint DIR the oracle's own state after the last sweep
is also saved there (an .npz of its exported world lines), and a later run
with the same arguments continues from it instead of starting over.

Run:  python tests/golden/make_digest_golden.py [--checkpoint DIR] [n_sweeps] [L S beta seed [out.json]]
      (default: the medium chain L=65,536, beta=4,096, seed 1, 3 sweeps)
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


def sha(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def default_name(L, S, beta, seed):
    sp = "" if S == 0.5 else f"_S{S:g}"
    sd = "" if seed == 1 else f"_seed{seed}"
    return f"digest_L{L}{sp}_beta{beta:g}{sd}.json"


def digest_record(ch, st):
    s0, off, kt, sw = ch.export_state()
    b, t, ty0 = ch.export_ops()
    lab = ch.export_labels()
    rec = dict(stats={k: int(v) for k, v in st.items()},
               state=sha(s0, off, kt), ops=sha(b.astype(np.int64), t, ty0),
               labels=sha(lab), next_sweep=int(sw))
    if ch.two_s > 1:
        rec["perm"] = sha(ch.export_perm())
    return rec


def write(out, path):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(out, f, indent=1)
    os.replace(tmp, path)


def main():
    a = sys.argv[1:]
    ckdir = None
    if a and a[0] == "--checkpoint":
        ckdir, a = a[1], a[2:]
    n = int(a[0]) if a else 3
    if len(a) >= 5:
        L, S, beta, seed = int(a[1]), float(a[2]), float(a[3]), int(a[4])
    else:
        L, S, beta, seed = 65536, 0.5, 4096.0, 1
    path = os.path.join(HERE, a[5] if len(a) >= 6 else default_name(L, S, beta, seed))
    ch = oracle.Chain(L, S, beta, seed)
    w, mu, T = oracle.window_table(beta)
    out = dict(L=L, S=S, beta=beta, seed=seed, window_w=w, mu=mu,
               thresholds=[str(t) for t in T], sweeps=[])
    ck = None
    if ckdir:
        os.makedirs(ckdir, exist_ok=True)
        ck = os.path.join(ckdir, os.path.basename(path) + ".state.npz")
        if os.path.exists(ck) and os.path.exists(path):
            prev = json.load(open(path))
            z = np.load(ck)  # arrays only: no pickled objects
            k = int(z["sweep"])
            same = all(prev[f] == out[f] for f in ("L", "S", "beta", "seed", "window_w", "mu",
                                                   "thresholds"))
            if same and len(prev["sweeps"]) == k:
                ch.import_state(z["s0"], z["off"], z["kt"], k)
                out["sweeps"] = prev["sweeps"]
                print(f"continuing after sweep {k - 1}", flush=True)
    for s in range(len(out["sweeps"]), n):
        t0 = time.time()
        st = ch.sweep()
        out["sweeps"].append(digest_record(ch, st))
        write(out, path)
        if ck:
            s0, off, kt, sw = ch.export_state()
            tmp = ck + ".tmp.npz"
            np.savez(tmp, s0=s0, off=off, kt=kt, sweep=np.int64(sw))
            os.replace(tmp, ck)
        print(s, f"{time.time() - t0:.0f}s", st["n_ops"], flush=True)


if __name__ == "__main__":
    main()
