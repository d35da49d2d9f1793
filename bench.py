#!/usr/bin/env python3
"""Throughput of the loop-cluster update on one MI355X.

Workload: the largest single chain that fits one GPU -- S=1/2
antiferromagnetic Heisenberg chain, J=1, L=262,144 spins, periodic,
beta=16,384, Philox seed 1, random initial Neel world lines (about 3e9
operators per sweep).  One step is one full sweep of the hot path
(insertion, operator merge, linking, union-find, flip, estimators, next
world lines) on device-resident state, launched as the library runs it
(one captured HIP graph per sweep).  The per-phase times come from a
separate pass of direct launches with HIP events between the phases.

--workload medium runs the medium chain instead (L=65,536, beta=4,096,
about 1.86e8 operators per sweep).  --workload split runs an S=4
chain (8 subspins per site, L=4,096, beta=2,048, about 2.8e8 operators per
sweep; no roofline or oracle entries).  --workload batch runs 512
independent chains (L log-uniform in [64, 16,384], beta uniform in [L/4, L]):
one step is one sweep of every chain, timed as 512 sequential plain updates
and as footprint-packed, autotuned batches.  --workload serve runs the
request loop on a Poisson stream of jobs (S in {1/2, 4}, L in {1024, 4096,
16384}, beta in {L/2, L}; sweep counts scaled by --serve-sweep-scale) with
continuous batching, and reports p50/p99 per-sweep latency and throughput.
--workload sw runs the paper's union-find benchmark, the Swendsen-Wang update
of the 2D Ising model (L=8,192 periodic, K=K_c, 128 burn-in and 128 timed
sweeps; vertices are lattice sites).

Prints one JSON line: operators ("graph vertices") per second over exactly
--steps sweeps after --warmup untimed sweeps, the per-phase HIP-event timing
of a separate profiled pass, the roofline entry of the dominant kernel, the
measured random-CAS and copy ceilings of the device, and the CPU oracle's
rate on a bounded sample.  --calibrate-atomics prints only the ceilings.
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
    "split": dict(workload="S=4 Heisenberg chain (8 subspins per site) L=4096 beta=2048 seed 1, "
                           "single chain", L=4096, S=4.0, beta=2048.0, seed=1),
}
HBM_PEAK_GBS = 8000.0


def host_cpu():
    """(model name, logical cores available to this process) of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count()
    return model, n


def device_ceilings(lc):
    """Measured ceilings: random 8-byte CAS on a 32 GiB word array (larger than
    every cache, like the union-find parent words of the largest chain) and on
    a 1 MiB one (L2-resident), and a streaming 4 GiB copy."""
    hbm, f1 = lc.lc_probe_cas(32, 1 << 27, 3)
    l2, f2 = lc.lc_probe_cas(17, 1 << 27, 3)
    copy = lc.lc_probe_copy(4 << 30, 3)
    assert f1 == 1.0 and f2 == 1.0
    return {"cas_per_s_hbm": hbm, "cas_per_s_l2": l2, "copy_gbs": copy,
            "how": "lc_probe_cas: random 8-byte CAS, 2^27 per launch, on 2^32 words (32 GiB) "
                   "and on 2^17 words (1 MiB), best of 3; lc_probe_copy: 4 GiB device copy, "
                   "read + written bytes per second, best of 3"}


def phase_bytes(n_ops, n_bnodes, n_loops, n_win, n_sites, kept_in, kept_out, n_cross, n_frags):
    """Algorithmic HBM bytes of each phase for one sweep: every array element
    the phase must read or write, counted once (random accesses of the
    global union-find at one 8-byte word each).

    n_ops operators, n_bnodes boundary nodes, n_loops loops recorded for the
    global phases (roots among fragments and boundary nodes), n_win (bond,
    window) cells, kept_in / kept_out off-diagonal operators before / after
    the sweep, n_cross edges between linking tiles, n_frags open fragments."""
    N, B, Cl, W, S = n_ops, n_bnodes, n_loops, n_win, n_sites
    X, F = n_cross, n_frags
    items = F + B
    return {
        # kept times, window scans (read kstart, write opstart), acceptance masks, spins
        "gen_count": 8 * kept_in + 16 * W + 4 * W + S,
        "scan_ops": 24 * W,
        # kept times, window scans, masks, operator time and type written
        "gen_write": 8 * kept_in + 16 * W + 4 * W + 9 * N,
        # operator times and window starts read, both parent words written,
        # boundary nodes initialised, cross edges (16 B) and fragments (32 B) out
        "link_tiles": 8 * W + 8 * N + 16 * N + 8 * B + 16 * X + 32 * F,
        # cross edges read; two finds and one CAS of 8-byte words per edge
        "link_cross": 16 * X + 24 * X,
        # item nodes (fragment records, parent words) read, parents written
        "compress": 8 * F + 16 * items,
        # item parents read, roots coded, records cleared (32 B)
        "roots": 8 * F + 8 * items + 32 * Cl,
        # fragment records, two parent words per item, record atomics
        "accum": 32 * F + 16 * items + 24 * Cl,
        "cluster_sums": 32 * Cl,
        # two parent words per operator node pair (label lookups), type r/w,
        # kept counts per window, spins r/w
        "flip": 16 * N + 2 * N + 8 * W + 2 * S,
        "scan_kept": 24 * W,
        "compact": 24 * W + 9 * N + 8 * kept_out,
        "setup": 0,
    }


# per-operator bytes of the path, from the survey's model of one sweep
# (a1+a2 11.5, a3 fused into linking 8, a4+a5 16 + 48 + 32, a6+a7 28)
SURVEY_BYTES_PER_OP = 11.5 + 8 + 16 + 48 + 32 + 28


PHASE_KERNELS = {
    "gen_count": ["k_gen<false>", "k_gen_split"], "gen_write": ["k_gen<true>", "k_gen_defer"],
    "link_tiles": ["k_init_bnodes", "k_link_tile<1>"], "link_cross": ["k_link_cross"],
    "compress": ["k_compress_items"], "roots": ["k_roots_items"], "accum": ["k_accum_items", "k_accum_hash"],
    "cluster_sums": ["k_cluster_sums"], "flip": ["k_flip_tiles<256>", "k_flip_sites"],
    "compact": ["k_compact"],
}
TRAFFIC_FILES = {"medium": os.path.join(ROOT, "profiles", "hbm_traffic_L65536_beta4096.txt"),
                 "largest": os.path.join(ROOT, "profiles", "hbm_traffic_L262144_beta16384.txt")}


def measured_traffic(phase, workload):
    """HBM bytes per launch of a phase's kernels from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary of the workload (copy-calibrated), or None
    when there is none or the kernel source has changed since the counters
    were taken."""
    import hashlib
    try:
        lines = open(TRAFFIC_FILES[workload]).read().splitlines()
    except (OSError, KeyError):
        return None
    src = os.path.join(ROOT, "paper_1810_07485_amd", "csrc", "lc_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    rec, ok = {}, False
    for ln in lines:
        f = ln.split()
        if len(f) == 2 and f[0] == "kernel_source_sha256":
            ok = f[1] == sha
        elif len(f) == 6 and f[0] == "traffic":
            rec[f[1]] = int(f[4]) + int(f[5])
    ks = PHASE_KERNELS.get(phase, [])
    if not ok or not ks or any(k not in rec for k in ks):
        return None
    return sum(rec[k] for k in ks)


def cpu_baseline(L, beta, seed=1, budget_s=12.0):
    """The oracle's rate on a bounded sample: its own chain with the
    workload's beta and fewer spins (L beta = 2^24), one untimed sweep from
    the Neel state, then whole timed sweeps (>= 1, up to about budget_s
    seconds).  Single-threaded C."""
    from oracle import oracle

    o = oracle.Chain(L, 0.5, beta, seed)
    o.sweep()
    ops, t0 = 0, time.perf_counter()
    while True:
        ops += o.sweep()["n_ops"]
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    model, ncpu = host_cpu()
    return {"value": ops / el, "unit": "vertices/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "host_cores": ncpu,
            "sample": f"oracle sweeps 1.. of an S=1/2 chain L={L} beta={beta:g} from its Neel "
                      f"start (same beta, fewer spins): {ops} operators in {el:.1f} s, "
                      f"single-threaded C on one core of {ncpu} ({model})"}


def _ops_since_reset(chains):
    tot = 0.0
    for c in chains:
        m = c.measure()
        tot += m["mean_ops"] * m["n_sweeps"]
    return tot


def _timed_passes(step, chains, steps):
    import torch
    for c in chains:
        c.reset_measurements()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return el, _ops_since_reset(chains)


def bench_batch(args, lc):
    """512 chains: sequential plain updates vs footprint-packed batches."""
    import torch
    from paper_1810_07485_amd import batching, workloads

    inst = workloads.batch_instances()
    chains = [lc.Chain(i.L, i.S, i.beta, i.seed) for i in inst]
    budget = int(args.batch_budget_gib) << 30

    def plain_pass(cs=chains):
        for c in cs:
            c.update(1)

    def note(m):
        print(f"[bench batch] {m}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        plain_pass()
    note("warm-up done")
    el_p, ops_p = _timed_passes(plain_pass, chains, args.steps)
    note(f"plain: {el_p / args.steps * 1e3:.1f} ms per step")
    # small-chain subset (launch overhead dominates): plain vs one batch
    small = sorted(chains, key=lambda c: c.L * c.beta)[:256]
    el_sp, ops_sp = _timed_passes(lambda: plain_pass(small), small, args.steps)

    sb = lc.Batch()
    for c in small:
        sb.add(c)
    sgrid, _ = sb.autotune((512, 2048, 8192), 1)
    el_sb, ops_sb = _timed_passes(lambda: sb.update(1), small, args.steps)
    sb.close()
    note("small chains done")

    runner = batching.BatchRunner(chains, budget)
    tune = runner.autotune_tiles(lc.DEFAULT_TILE_SHAPES, (2048, 8192, 16384), 1)
    note("tile shapes and grids tuned")
    runner.update(1, accumulate=False)
    el_b, ops_b = _timed_passes(lambda: runner.update(1), chains, args.steps)
    n_groups = len(runner.groups)
    runner.close()
    out = {
        "metric": METRIC,
        "value": ops_b / el_b,
        "unit": "vertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el_b / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "512 independent S=1/2 chains, L log-uniform in [64,16384] even, "
                               "beta uniform in [L/4,L], seeds 1..512 (numpy default_rng(20181017)); "
                               "one step = one sweep of every chain",
                   "chains": len(chains), "scratch_budget_bytes": budget},
        "plain": {"value": ops_p / el_p, "ms_per_step": el_p / args.steps * 1e3,
                  "how": "512 sequential lc_update(1) calls per step, each chain's own graph"},
        "batched": {"groups": n_groups, "grids": [g for _, g, _ in tune],
                    "tile_shapes": [list(sh) for sh, _, _ in tune],
                    "group_ms_per_sweep": [round(ms, 3) for _, _, ms in tune],
                    "how": "footprint-packed groups, each one captured sweep; (tile shape, grid) "
                           "per group by lc_batch_autotune_tiles"},
        "speedup_vs_plain": (ops_b / el_b) / (ops_p / el_p),
        "small_chains": {"chains": len(small), "ops_per_step": ops_sp / args.steps,
                         "plain_value": ops_sp / el_sp, "batched_value": ops_sb / el_sb,
                         "grid": sgrid, "speedup": (ops_sb / el_sb) / (ops_sp / el_sp)},
        "roofline": None,
    }
    for c in chains:
        c.close()
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(4096, 4096.0)
    print(json.dumps(out), flush=True)


def bench_serve(args, lc):
    """Continuous-batching request loop on a Poisson job stream."""
    import dataclasses
    import torch
    from paper_1810_07485_amd import serve, workloads

    total = torch.cuda.get_device_properties(0).total_memory
    budget = int(0.85 * total)
    # plain single-chain throughput on one of the mix's chains (calibration)
    cal = lc.Chain(16384, 0.5, 16384.0, 7)
    cal.update(3, accumulate=False)
    el, ops = _timed_passes(lambda: cal.update(1), [cal], 3)
    cal.close()
    plain = ops / el
    jobs = workloads.serving_jobs(args.serve_jobs, rate=1.0)
    jobs = [dataclasses.replace(j, sweeps=max(1, int(round(j.sweeps * args.serve_sweep_scale))))
            for j in jobs]
    dens = {0.5: 0.693, 4.0: 33.5}  # operators per unit L beta at low temperature
    fits = [j for j in jobs if serve.job_bytes(j) <= budget]
    mean_ops = sum(dens[j.S] * j.L * j.beta * j.sweeps for j in fits) / max(1, len(fits))
    rate = 0.8 * plain / mean_ops  # jobs per second at 80 % of plain capacity
    jobs = workloads.serving_jobs(args.serve_jobs, rate=rate)
    jobs = [dataclasses.replace(j, sweeps=max(1, int(round(j.sweeps * args.serve_sweep_scale))))
            for j in jobs]
    rep = serve.Server(budget).run(jobs, log=lambda m: print(m, file=sys.stderr, flush=True))
    sm = rep.summary()
    out = {
        "metric": METRIC,
        "value": sm["ops_per_s_busy"],
        "unit": "vertices/s",
        "n_gpus": 1,
        "steps": rep.iterations,
        "warmup": 0,
        "ms_per_step": rep.busy_s / max(1, rep.iterations) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"serving: {args.serve_jobs} Poisson-arrival jobs (numpy default_rng(20181018)), "
                               "S in {1/2,4}, L in {1024,4096,16384}, beta in {L/2,L}, sweeps in {100,1000} "
                               f"scaled by {args.serve_sweep_scale}; admission by footprint within "
                               f"{budget / 2**30:.0f} GiB; one step = one iteration (one sweep of every "
                               "resident job)",
                   "arrival_rate_per_s": rate},
        "serving": sm,
        "plain": {"value": plain, "how": "one S=1/2 L=16384 beta=16384 chain alone, lc_update"},
        "roofline": None,
    }
    print(json.dumps(out), flush=True)


SW_KC = 0.44068679350977147  # ln(1 + sqrt 2) / 2
SW_L = 8192


def sw_phase_bytes(n, n_records, L):
    """Algorithmic HBM bytes of each Swendsen-Wang kernel for one sweep of n
    sites whose tiles left n_records local components (64 x 64-site tiles)."""
    R, X = n_records, 2 * L * -(-L // 64)   # X: bonds leaving a tile
    return {
        "tiles": n + 2 * n // 64 + 8 * n + 16 * R,   # spins and halo, parent words, records
        "cross": 2 * X + 16 * X,                     # both spins, both endpoints' parent words
        "compress": 8 * R + 8 * R + 8 * R + 8 * R,   # record site, root walk, parent, size cleared
        "sizes": 16 * R + 8 * R + 8 * R,             # records, parent of the site, size add
        "roots": 8 * R + 8 * R + 8 * R,              # record site, parent, size
        "flip": 8 * n + 8 * n + 2 * n,               # parent, label's parent, spin read and written
    }


def sw_cpu_baseline(budget_s=12.0):
    """The Swendsen-Wang oracle's rate on a bounded sample: L=2048 at K_c, one
    untimed sweep from the all-up start, then whole timed sweeps up to about
    budget_s seconds.  Single-threaded C."""
    from oracle import oracle

    L = 2048
    o = oracle.SwChain(L, SW_KC, 1)
    o.sweep()
    k, t0 = 0, time.perf_counter()
    while True:
        o.sweep()
        k += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    model, ncpu = host_cpu()
    return {"value": k * L * L / el, "unit": "vertices/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "host_cores": ncpu,
            "sample": f"oracle Swendsen-Wang sweeps 1..{k} of an L={L} lattice at K_c from the "
                      f"all-up start (same coupling, fewer sites): {k * L * L} site updates in "
                      f"{el:.1f} s, single-threaded C on one core of {ncpu} ({model})"}


def bench_sw(args, lc):
    """Swendsen-Wang 2D Ising on the library's union-find (the paper's
    union-find benchmark): L=8192 periodic, K=K_c, seed 1."""
    import torch

    g = lc.SwIsing(SW_L, SW_KC, 1)
    g.update(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.update(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    last = g.last_sweep()
    n = SW_L * SW_L
    g.set_profiling(True)
    E, C2 = [], []
    for _ in range(args.profile_sweeps):
        g.update(1)
        st = g.last_sweep()
        E.append(st["energy"] / n)
        C2.append(st["size2"] / n)
    prof, nsw = g.profile()
    g.set_profiling(False)
    R = g.work()
    pb = sw_phase_bytes(n, R, SW_L)
    phase_ms = {k: v / nsw for k, v in prof.items()}
    dom = max(phase_ms, key=phase_ms.get)
    achieved = pb[dom] / (phase_ms[dom] * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": n * args.steps / el,
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
        "config": {"workload": f"Swendsen-Wang 2D Ising L={SW_L} periodic, K=K_c, seed 1, all-up "
                               f"start, {args.warmup} burn-in + {args.steps} timed sweeps "
                               "(vertices = lattice sites)", "L": SW_L, "K": SW_KC},
        "sweeps_per_s": args.steps / el,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": pb[dom], "avg_ms": phase_ms[dom],
                     "timing": f"HIP events around each kernel on the library stream, {nsw} "
                               "directly launched sweeps after the timed region"},
        "path_bytes_per_sweep": sum(pb.values()),
        "hbm_gbs_algorithmic": sum(pb.values()) * args.steps / el / 1e9,
        "work": {"tile_components_per_site": R / n},
        "phase_ms": phase_ms,
        "profiled_ms_per_sweep": sum(phase_ms.values()),
        "observables": {"e_per_site": sum(E) / len(E), "mean_cluster_size": sum(C2) / len(C2),
                        "last_timed_sweep": last["sweep"],
                        "note": "means over the profiled sweeps after the timed region"},
    }
    g.close()
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = sw_cpu_baseline()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 20; largest and split 5; batch 3)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default 10; largest and split 4; batch 2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the random-CAS and copy probes")
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["batch", "serve", "sw"],
                    default="largest",
                    help="largest: L=262144 beta=16384 (default); medium: L=65536 beta=4096; "
                         "split: S=4 L=4096 beta=2048; batch: 512 chains; serve: request loop; "
                         "sw: Swendsen-Wang 2D Ising L=8192 at K_c")
    ap.add_argument("--calibrate-atomics", action="store_true",
                    help="only measure the random-CAS and copy ceilings and exit")
    ap.add_argument("--profile-sweeps", type=int, default=None,
                    help="sweeps of the separate per-phase timing pass (default 2, medium 10)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 2 GiB device to device three times (reference kernel for "
                         "the HBM byte counters) and exit")
    ap.add_argument("--batch-budget-gib", type=int, default=128,
                    help="--workload batch: per-sweep scratch budget of a footprint-packed group")
    ap.add_argument("--serve-jobs", type=int, default=24)
    ap.add_argument("--serve-sweep-scale", type=float, default=0.1)
    args = ap.parse_args()
    dflt = {"medium": (20, 10), "largest": (10, 4), "split": (5, 4), "batch": (3, 2),
            "serve": (0, 0), "sw": (128, 128)}[args.workload]
    if args.profile_sweeps is None:
        args.profile_sweeps = {"medium": 10, "sw": 32}.get(args.workload, 2)
    if args.steps is None:
        args.steps = dflt[0]
    if args.warmup is None:
        args.warmup = dflt[1]
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library runs "
              "each chain on a single GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1810_07485_amd as lc

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        x = torch.ones(1 << 28, dtype=torch.int64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": x.numel() * 8, "launches": 3}), flush=True)
        return
    if args.calibrate_atomics:
        print(json.dumps(device_ceilings(lc)), flush=True)
        return
    if args.workload == "batch":
        bench_batch(args, lc)
        return
    if args.workload == "serve":
        bench_serve(args, lc)
        return
    if args.workload == "sw":
        bench_sw(args, lc)
        return
    w = WORKLOADS[args.workload]
    chain = lc.Chain(w["L"], w["S"], w["beta"], w["seed"])
    chain.update(args.warmup, accumulate=False)
    # the chain is still equilibrating from its Neel start: keep warming up
    # (a sweep per call, at most 8) until a call no longer grows its buffers,
    # so that no reallocation falls into the timed region
    extra = 0
    cap = chain.capacity()
    while extra < 8:
        chain.update(1, accumulate=False)
        extra += 1
        cap, prev = chain.capacity(), cap
        if cap == prev:
            break
    chain.reset_measurements()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chain.update(args.steps, accumulate=True)   # graph replay, as the library runs
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    grew = chain.capacity() != cap
    m = chain.measure()
    last = chain.last_sweep()
    assert m["n_sweeps"] == args.steps
    # separate pass: direct launches with HIP events between the phases
    chain.set_profiling(True)
    chain.update(args.profile_sweeps, accumulate=False)
    prof, nsw = chain.profile()
    chain.set_profiling(False)
    ops_total = m["mean_ops"] * args.steps
    n_sites = chain.n_sites
    nbn = n_sites if w["S"] == 0.5 else 2 * n_sites  # boundary nodes
    frag_total = (2 * m["mean_ops"] + nbn) * args.steps
    wtab = lc.lc_debug_window_table(w["beta"])
    n_win = chain.n_bonds << wtab[0]
    n_cross, n_frags = chain.work()
    pb = phase_bytes(last["n_ops"], nbn, n_frags + nbn, n_win, n_sites, last["n_kept_in"],
                     last["n_kept_out"], n_cross, n_frags)
    phase_ms = {k: v / nsw for k, v in prof.items()}
    dom = max(phase_ms, key=phase_ms.get)
    achieved = pb[dom] / (phase_ms[dom] * 1e-3) / 1e9
    total_bytes = sum(pb.values())
    traffic = measured_traffic(dom, args.workload)
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
        "warmup_extra": extra,
        "buffers_grew_in_timed_region": grew,
        "fragments_per_s": frag_total / el,
        "hbm_gbs_algorithmic": total_bytes * args.steps / el / 1e9,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_gbs": (traffic / (phase_ms[dom] * 1e-3) / 1e9) if traffic else None,
                     "bytes_per_launch": pb[dom], "avg_ms": phase_ms[dom],
                     "timing": f"HIP events around each phase on the library stream, "
                               f"{nsw} directly launched sweeps after the timed region"},
        "path_roofline": {"model": "survey per-operator bytes of one sweep", "bytes_per_op":
                          SURVEY_BYTES_PER_OP, "achieved": SURVEY_BYTES_PER_OP * ops_total / el / 1e9,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": SURVEY_BYTES_PER_OP * ops_total / el / 1e9 / HBM_PEAK_GBS},
        "work": {"cross_edges_per_op": n_cross / last["n_ops"], "fragments_per_op": n_frags / last["n_ops"]},
        "phase_ms": phase_ms,
        "profiled_ms_per_sweep": sum(phase_ms.values()),
        "observables": {"e": m["e"], "ops_per_L_beta": m["mean_ops"] / (w["L"] * w["beta"]),
                        "loops_per_L_beta": m["mean_clusters"] / (w["L"] * w["beta"])},
    }
    chain.close()
    torch.cuda.empty_cache()
    if not args.no_ceilings:
        out["ceilings"] = device_ceilings(lc)
    if w["S"] != 0.5:
        # the per-phase byte model and the oracle sample are those of S = 1/2 chains
        out["roofline"] = None
    elif not args.no_cpu_baseline:
        Ls = max(1024, int(2 ** 24 / w["beta"]) // 2 * 2)
        out["cpu_baseline"] = cpu_baseline(Ls, w["beta"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
