#!/usr/bin/env python3
"""Benchmark of the multicanonical hot path on one MI355X.

Workload: plain MUCA, 2D Ising L = 64 (periodic), bit-packed spins, 4096
chains, seed 2, lnW in FP64 and uint32 acceptance thresholds, 10^4 sweeps per
iteration.  One step = one MUCA iteration: the sweep kernel over all chains
(with the LDS/atomic histogram merge) followed by muca_merge_update (FP64
accumulated-statistics recursion, flatness test, threshold rebuild and
upload).  Inputs (spins, weights) are resident in HBM before the timed
region.

Prints one JSON line: attempts/s (every Metropolis attempt counts, accepted or
not), the sweep kernel's roofline figures (HIP-event duration on the launch
stream), and the single-threaded CPU oracle timed on a bounded sample of the
same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak 32-bit integer VALU rate of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz.
PEAK_INT_OPS = 256 * 4 * 16 * 2.4e9
# Algorithmic 32-bit VALU slot-ops per Ising attempt ("Roofline"):
# Philox4x32-10 100 slots per 4 words (10 rounds x [2 wide multiplies at 4
# slots + 2 three-input XORs]) = 25 per attempt; Metropolis update 20.
OPS_PER_ATTEMPT = 45.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=10000, help="sweeps per iteration (workload: 10^4)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU oracle sample budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def cpu_baseline(seconds: float) -> dict:
    """The oracle (single-threaded C, as it stands) on a bounded sample of the
    same workload: 16 of the 4096 chains, L = 64, lnW = 0 thresholds, in
    100-sweep chunks until `seconds` have elapsed."""
    from oracle import oracle as orc
    orc.build(force=False)
    r = orc.LatticeRun(orc.ISING, 64, 16, seed=2)
    T = r.thresholds()
    sweeps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        r.sweeps(100, T)
        r.advance(100)
        sweeps += 100
    dt = time.perf_counter() - t0
    attempts = 16 * 4096 * sweeps
    return {"value": attempts / dt, "unit": "attempts/s", "cores": 1, "kind": "oracle",
            "sample": f"Ising L=64, 16 of the 4096 chains, {sweeps} sweeps ({attempts:.3g} attempts, "
                      f"{dt:.1f} s, single thread)"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1312_2213_amd import muca

    torch.cuda.set_device(0)
    L, C, seed, S = 64, 4096, 2, args.sweeps
    cfg = muca.muca_config_default("ising", L, 2, C, seed, layout=muca.MUCA_LAYOUT_BIT)
    stream = torch.cuda.current_stream()
    run = muca.Run(cfg, stream=stream)
    for _ in range(args.warmup):
        run.run_iteration(S)
        run.merge_update()
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    stats = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        run.run_iteration(S)
        evs[k][1].record(stream)
        stats.append(run.merge_update())
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    dt = t1 - t0
    attempts_per_step = C * L * L * S
    value = attempts_per_step * args.steps / dt
    kern_ms = sum(a.elapsed_time(b) for a, b in evs) / args.steps
    achieved = OPS_PER_ATTEMPT * attempts_per_step / (kern_ms * 1e-3)

    out = {
        "metric": "spin-flip attempts/s (MUCA iteration, 1 GPU)",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "plain MUCA 2D Ising L=64 periodic, bit-packed spins, 4096 chains, "
                               f"seed 2, {S} sweeps per iteration, FP64 lnW, uint32 thresholds",
                   "L": L, "chains": C, "sweeps_per_iteration": S, "parallelism": "chains, 1 GPU"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_INT_OPS / 1e12,
                     "unit": "TOP/s", "frac": achieved / PEAK_INT_OPS, "traffic": None,
                     "kernel": "lattice_sweeps<Ising, L=64, bit>", "kernel_ms": kern_ms,
                     "ops_per_attempt": OPS_PER_ATTEMPT},
        "iterations": [{k: s[k] for k in ("iteration", "flatness", "lo_visited", "hi_visited")}
                       for s in stats],
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(args.cpu_seconds)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
