#!/usr/bin/env python3
"""Throughput of the loop-cluster update on one MI355X.

Workload: the medium single chain -- S=1/2 antiferromagnetic Heisenberg
chain, J=1, L=65,536 spins, periodic, beta=4,096, Philox seed 1, random
initial Neel world lines (about 1.86e8 operators per sweep).  One step is
one full sweep of the hot path (insertion, operator merge, linking,
union-find, flip, estimators, next world lines) on device-resident state.

--workload largest runs the largest single-GPU chain instead (L=262,144,
beta=16,384, about 3e9 operators per sweep).

Prints one JSON line: operators ("graph vertices") per second over exactly
--steps sweeps after --warmup untimed sweeps, with the per-phase HIP-event
timing of those same sweeps, the roofline entry of the dominant kernel and
the CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "graph vertices/sec & MC sweeps/sec on 1 GPU, batched/served vs plain; HBM GB/s"
WORKLOADS = {
    "medium": dict(workload="S=1/2 Heisenberg chain L=65536 beta=4096 seed 1, single chain",
                   L=65536, S=0.5, beta=4096.0, seed=1),
    "largest": dict(workload="S=1/2 Heisenberg chain L=262144 beta=16384 seed 1, single chain",
                    L=262144, S=0.5, beta=16384.0, seed=1),
}
HBM_PEAK_GBS = 8000.0


def phase_bytes(n_ops, n_nodes, n_clusters, n_win, n_sites, kept_in, kept_out):
    """Algorithmic HBM bytes of each phase for one sweep (compulsory traffic:
    every array element the phase must read or write, counted once).

    n_ops operators, n_nodes loop-graph nodes, n_win (bond, window) cells,
    kept_in / kept_out off-diagonal operators before / after the sweep."""
    N, V, Cl, W, S = n_ops, n_nodes, n_clusters, n_win, n_sites
    return {
        "gen_count": 8 * kept_in + 8 * W + S + 8 * W,
        "scan_ops": 24 * W,
        "gen_write": 8 * kept_in + 8 * W + 8 * W + 9 * N,
        "init_parent": 8 * V,
        "link_ops": 8 * W + 8 * N + 16 * V,
        "link_sites": 24 * S,
        "compress": 16 * V,
        # roots: count roots per chunk (8V), assign loop index and flip bit,
        # clear the three record words (8V + 8C + 1C + 24C)
        "roots": 16 * V + 33 * Cl,
        # accum: parent word per node, time per operator, bottom spins;
        # read-modify-write of 3 words per loop record
        "accum": 8 * V + 8 * N + S + 48 * Cl,
        "cluster_sums": 24 * Cl,
        "flip": 8 * V + 2 * N + Cl + 8 * W + 2 * S,
        "scan_kept": 24 * W,
        "compact": 24 * W + 9 * N + 8 * kept_out,
        "setup": 0,
    }


def cpu_baseline(lc, L, beta, seed=1, gpu_therm=30, budget_s=12.0):
    """The oracle's rate on a bounded sample: a chain with the workload's
    beta and fewer spins (L beta = 2^24), thermalised on the GPU, imported
    into the oracle, then timed for whole oracle sweeps (>= 1, up to about
    budget_s seconds).  Single-threaded C."""
    from oracle import oracle

    g = lc.Chain(L, 0.5, beta, seed)
    g.update(gpu_therm, accumulate=False)
    st = g.export_state()
    o = oracle.Chain(L, 0.5, beta, seed)
    o.import_state(*st)
    ops, t0 = 0, time.perf_counter()
    while True:
        ops += o.sweep()["n_ops"]
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    g.close()
    return {"value": ops / el, "unit": "vertices/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle sweeps of a thermalised S=1/2 chain L={L} beta={beta:g} "
                      f"(same beta, fewer spins): {ops} operators in {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="medium",
                    help="medium: L=65536 beta=4096 (default); largest: L=262144 beta=16384")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the chain is not "
              "sharded across GPUs in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1810_07485_amd as lc

    torch.cuda.set_device(0)
    w = WORKLOADS[args.workload]
    chain = lc.Chain(w["L"], w["S"], w["beta"], w["seed"])
    chain.update(args.warmup, accumulate=False)
    chain.reset_measurements()
    chain.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chain.update(args.steps, accumulate=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    m = chain.measure()
    prof, nsw = chain.profile()
    last = chain.last_sweep()
    assert m["n_sweeps"] == args.steps == nsw
    ops_total = m["mean_ops"] * args.steps
    n_sites = chain.n_sites
    frag_total = (2 * m["mean_ops"] + n_sites) * args.steps
    wtab = lc.lc_debug_window_table(w["beta"])
    n_win = chain.n_bonds << wtab[0]
    pb = phase_bytes(m["mean_ops"], 2 * m["mean_ops"] + n_sites, m["mean_clusters"], n_win,
                     n_sites, last["n_kept_in"], last["n_kept_out"])
    phase_ms = {k: v / nsw for k, v in prof.items()}
    dom = max(phase_ms, key=phase_ms.get)
    achieved = pb[dom] / (phase_ms[dom] * 1e-3) / 1e9
    total_bytes = sum(pb.values())
    out = {
        "metric": METRIC,
        "value": ops_total / el,
        "unit": "vertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": dict(w),
        "sweeps_per_s": args.steps / el,
        "fragments_per_s": frag_total / el,
        "hbm_gbs_algorithmic": total_bytes * args.steps / el / 1e9,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": pb[dom], "avg_ms": phase_ms[dom]},
        "phase_ms": phase_ms,
        "observables": {"e": m["e"], "ops_per_L_beta": m["mean_ops"] / (w["L"] * w["beta"]),
                        "loops_per_L_beta": m["mean_clusters"] / (w["L"] * w["beta"])},
    }
    chain.close()
    if not args.no_cpu_baseline:
        Ls = max(1024, int(2 ** 24 / w["beta"]) // 2 * 2)
        out["cpu_baseline"] = cpu_baseline(lc, Ls, w["beta"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
