"""Write oracle digests for a sample of the 512-chain batch workload.

Calls only ``oracle/`` (and the seeded instance generator, which holds none
of the method's arithmetic).  The sample is every 16th chain in order of
space-time volume L beta over the smaller 480 chains, plus the chain of
largest L; with --largest only that chain is run (it needs a single core
for about half an hour and tens of GB of host memory, so it is run on its
own).  For each member, each of the first `sweeps` sweeps from its initial
state is recorded as in make_digest_golden.py: every integer of the sweep
statistics and SHA-256 digests of the world lines, the operators and the
loop labels.  Results merge into batch_members.json, one member at a time.

Run:  python tests/golden/make_batch_golden.py [--largest] [--sweeps N] [--jobs J]
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

OUT = os.path.join(HERE, "batch_members.json")


def sample_indices():
    from paper_1810_07485_amd import workloads
    inst = workloads.batch_instances()
    lb = np.array([i.L * i.beta for i in inst])
    order = np.argsort(lb, kind="stable")
    small = sorted(int(i) for i in order[:480:16])
    largest = int(np.argmax([i.L for i in inst]))
    return inst, small, largest


def run_member(args):
    idx, L, beta, seed, sweeps = args
    from oracle import oracle
    from make_digest_golden import digest_record
    ch = oracle.Chain(L, 0.5, beta, seed)
    recs = []
    t0 = time.time()
    for _ in range(sweeps):
        st = ch.sweep()
        recs.append(digest_record(ch, st))
    return dict(index=idx, L=L, S=0.5, beta=beta, seed=seed, sweeps=recs), time.time() - t0


def merge(member):
    data = {"workload": "batch_instances(512), numpy default_rng(20181017)", "members": []}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["members"] = [m for m in data["members"] if m["index"] != member["index"]] + [member]
    data["members"].sort(key=lambda m: m["index"])
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1)
    os.replace(tmp, OUT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--largest", action="store_true")
    ap.add_argument("--sweeps", type=int, default=10)
    ap.add_argument("--jobs", type=int, default=3)
    a = ap.parse_args()
    inst, small, largest = sample_indices()
    idx = [largest] if a.largest else small
    work = [(i, inst[i].L, inst[i].beta, inst[i].seed, a.sweeps) for i in idx]
    work.sort(key=lambda w: -w[1] * w[2])
    with mp.Pool(a.jobs) as pool:
        for member, el in pool.imap_unordered(run_member, work):
            merge(member)
            print(member["index"], member["L"], round(member["beta"], 1), f"{el:.0f}s", flush=True)


if __name__ == "__main__":
    main()
