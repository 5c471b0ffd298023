#!/usr/bin/env python3
"""Benchmarks of the multicanonical hot path on one MI355X.

Default workload (the headline line): plain MUCA, 2D Ising L = 64 periodic,
bit-packed spins, 4096 chains, seed 2, lnW in FP64 and uint32 acceptance
thresholds, 10^4 sweeps per iteration.  One step = one MUCA iteration: the
sweep kernel over all chains (LDS + atomic histogram merge) followed by
muca_merge_update (FP64 accumulated-statistics recursion, flatness test,
threshold rebuild and upload).  Inputs are resident in HBM before the timed
region.  The line also carries:
  roofline      the sweep kernel's figures (HIP-event duration on its stream;
                HBM traffic from the rocprofv3 counters of the same kernel
                sources, null once those sources have changed);
  more_chains   the same kernel at 131072 chains (one lane per chain,
                blocks of 512 threads: two wavefronts per SIMD), one launch;
  cpu_baseline  the single-threaded C oracle on a bounded sample of the same
                workload at weights that reject moves, on one core and as one
                process per core over disjoint chain ranges;
  time_to_flat  the batched workload (q=8 Potts L in {16,24,32,48} x 2048
                chains + 4 MUMA Ising L=32 x 512 chains at beta = 0.5), every
                instance run to a flat histogram (min/mean > 0.5): makespan
                and mean time to flat of one persistent hipGraph launch per
                round (batched), of the serving loop (served), and of the
                instances one after another with plain launches (plain);
                the multimagnetic runs' spin layout from the plain-launch
                autotuner (layouts).

Other modes (--workload): "ising64_flat" (the headline configuration run to
a flat histogram: time to flat), "potts48" (plain MUCA of the batched
workload's longest instance, q=8 Potts L=48, 2048 chains), "batched" (time
to flat, batched vs plain), "serving" (200 Poisson requests, p50/p99 time to
flat), "polymer" (N = 40, 4096 chains), "polymer_paper" (the paper's
homopolymer, N = 40 and 80), "speedup" (statistical speedup S*_p over chains
per run, Eq. 6; with --speedup-set qscan the q-state Potts crossover scan),
"muma_em" (multimagnetic run at T = 2/3 T_c with the joint (E, M) histogram
reweighted in beta, and the cost of recording it), "copy" (device copy of
known size, for counter calibration).
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
# Algorithmic 32-bit operations per Ising attempt: Philox4x32-10 10 per word
# (10 rounds x [2 wide multiplies + 2 three-input XORs] per 4 words) +
# Metropolis update 13.
OPS_PER_ATTEMPT = 23.0
# HBM bytes of one 10^4-sweep launch of the Ising L=64 kernel (4096 chains,
# 16 lanes per chain), from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled
# by a device copy of known size, and the sha256 of the sources and flags
# that built the profiled kernel: the figure is reported only while they are
# unchanged.
HBM_TRAFFIC = {"bytes_per_launch": 3339.625 * 1024 * 2.0 + 2482.125 * 1024,
               "kernel_sources_sha256": "b18bbd26c4072b73"}
KERNEL_SOURCES = ["paper_1312_2213_amd/csrc/lattice_impl.h", "paper_1312_2213_amd/csrc/muca_internal.h",
                  "paper_1312_2213_amd/csrc/philox.h", "paper_1312_2213_amd/csrc/lattice_ising.hip"]


def kernel_sources_sha256() -> str:
    """sha256 over the files that define the headline sweep kernel and the
    compiler flags of the build (first 16 hex digits)."""
    import hashlib
    from paper_1312_2213_amd import build
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    flags = [f for f in build.COMMON + build.DEVICE if not os.path.isabs(f)]  # not the checkout's path
    h.update(repr(flags).encode())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ising64",
                    choices=["ising64", "ising64_flat", "potts48", "batched", "serving", "polymer", "polymer_paper",
                             "speedup", "muma_em", "copy"])
    ap.add_argument("--sweeps", type=int, default=10000, help="sweeps per iteration (workload: 10^4)")
    ap.add_argument("--lanes-per-chain", type=int, default=0)
    ap.add_argument("--chains-per-block", type=int, default=0,
                    help="ising64: chains per block (0: the library's choice; x lanes per chain = threads)")
    ap.add_argument("--chains", type=int, default=4096, help="ising64: chains (workload: 4096)")
    ap.add_argument("--batch-lanes-per-chain", type=int, default=0, help="batched runs: 4, 16 or 0 (per run)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU oracle sample budget per leg (one core; all cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the time_to_flat sub-object")
    ap.add_argument("--batched-rounds", type=int, default=3)
    ap.add_argument("--flat-max-iters", type=int, default=3000,
                    help="time_to_flat sub-object of the headline line: iteration cap per instance")
    ap.add_argument("--max-iters", type=int, default=None,
                    help="iteration cap (default: 40 batched, 3000 serving, 1000 speedup)")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--systems", default="", help="speedup: comma-separated indices of the systems to run")
    ap.add_argument("--speedup-set", default="paper", choices=["paper", "qscan", "polymer", "time"],
                    help="speedup: the paper's spin systems, the q-state Potts crossover scan, or the "
                         "paper's homopolymer")
    ap.add_argument("--qscan-L", type=int, default=16, help="speedup --speedup-set qscan: lattice size")
    ap.add_argument("--qscan-qs", default="", help="speedup --speedup-set qscan: comma-separated q values")
    ap.add_argument("--qscan-ps", default="", help="speedup --speedup-set qscan: comma-separated chains per run")
    ap.add_argument("--replicas", type=int, default=0, help="speedup --speedup-set qscan: runs per p")
    ap.add_argument("--round-site-updates", type=int, default=1 << 16,
                    help="serving: site updates per chain in one round")
    ap.add_argument("--overlap-min-rounds", type=int, default=None,
                    help="serving: overlap the merges of requests whose iterations span at least this many rounds")
    return ap.parse_args()


CPU_CHAINS = 16  # chains per process of the CPU sample
CPU_BETA = 0.4   # canonical slope of the sample's weights: about half the moves rejected


def _cpu_weights(r):
    """Weights of the CPU sample: lnW(E) = -0.4 E, under which about half of
    the proposals from the random start are rejected (lnW = 0 would accept
    every flip, the oracle's cheapest branch pattern)."""
    import numpy as np
    from oracle import oracle as orc
    return -CPU_BETA * orc.bin_values(orc.ISING, 64, r.lo, r.hi)


def _cpu_worker(k: int, n_procs: int, seconds: float):
    """One process of the CPU sample: chains [16k, 16k + 16) of the headline
    run (seed 2, L = 64), 100-sweep chunks until `seconds` have elapsed."""
    import time as _t
    sys.path.insert(0, ROOT)
    from oracle import oracle as orc
    orc.build(force=False)
    r = orc.LatticeRun(orc.ISING, 64, CPU_CHAINS * n_procs, seed=2)
    T = r.thresholds(_cpu_weights(r))
    chains = (CPU_CHAINS * k, CPU_CHAINS * (k + 1))
    sweeps = 0
    t0 = _t.perf_counter()
    while _t.perf_counter() - t0 < seconds:
        r.sweeps(100, T, chains=chains)
        r.advance(100)
        sweeps += 100
    dt = _t.perf_counter() - t0
    return CPU_CHAINS * 4096 * sweeps, dt, r.take_accepted()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds: float) -> dict:
    """The oracle (single-threaded C, as it stands) on a bounded sample of the
    headline workload at weights that reject moves: 16 chains on one core,
    then one process per available core (at most 16) over disjoint 16-chain
    ranges, histograms independent, attempts summed (the paper's own scheme
    on CPU cores)."""
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    from oracle import oracle as orc
    orc.build(force=False)
    attempts, dt, acc = _cpu_worker(0, 1, seconds)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    P = max(1, min(avail, 16))
    with ProcessPoolExecutor(max_workers=P, mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_cpu_worker, range(P), [P] * P, [seconds] * P))
    all_attempts = sum(a for a, _, _ in parts)
    all_dt = max(d for _, d, _ in parts)
    return {"value": attempts / dt, "unit": "attempts/s", "cores": 1, "kind": "oracle",
            "sample": f"Ising L=64, seed 2, chains 0-15 of the 4096, lnW(E) = -{CPU_BETA} E "
                      f"(acceptance {acc / attempts:.2f}): {attempts:.3g} attempts in {dt:.1f} s, one thread",
            "cpu_model": cpu_model(), "cores_available": avail,
            "all_cores": {"value": all_attempts / all_dt, "unit": "attempts/s", "cores": P, "processes": P,
                          "sample": f"{P} processes, chains [16k, 16k+16) each, same weights: "
                                    f"{all_attempts:.3g} attempts in {all_dt:.1f} s"}}


def batched_instances(tune_layout: bool = True):
    """The batched workload's instances as (config, sweeps per iteration).
    The multimagnetic runs take the spin layout (bit or byte) that the
    plain-launch autotuner measures fastest for their shape (one lattice
    layout per run: its spins live in it); the batched launch then tunes
    lanes per chain and table placement per run.  Potts has one layout."""
    from paper_1312_2213_amd import muca
    from synth import WORKLOADS, sweeps_per_iteration
    out = []
    for inst in WORKLOADS["potts8_batched"]["instances"]:
        if inst["model"] == "potts":
            cfg = muca.muca_config_default("potts", inst["L"], inst["q"], inst["chains"], inst["seed"])
            sw = sweeps_per_iteration(inst["L"], inst["chains"], True)
        else:
            cfg = muca.muca_config_default("muma", inst["L"], 2, inst["chains"], inst["seed"],
                                           beta=inst["beta"], layout=muca.MUCA_LAYOUT_AUTO)
            sw = sweeps_per_iteration(inst["L"], inst["chains"], False)
            cfg.layout = muca.muca_autotune(cfg, sw)[0].layout if tune_layout else muca.MUCA_LAYOUT_BYTE
        out.append((cfg, sw))
    return out


def tuned_vs_rule_round(stream, rounds: int = 4) -> dict:
    """One batched round of the batched workload's first iteration with the
    lanes per chain and table placement chosen by the untuned rule and by the
    measured item times (muca_batch_tune): minimum over `rounds` rounds of
    each, on fresh runs of the same seeds, and the tuned choices."""
    import torch
    from paper_1312_2213_amd import muca
    specs = batched_instances()
    out = {}
    for mode in ("rule", "tuned"):
        runs = [muca.Run(c, stream=stream) for c, _ in specs]
        batch = muca.Batch(len(runs), lanes_per_chain=0, use_graph=True, autotune=mode == "tuned")
        best = None
        for k in range(rounds + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with torch.cuda.stream(stream):
                batch.run_iteration(runs, [sw for _, sw in specs], stream=stream)
            stream.synchronize()
            dt = time.perf_counter() - t0
            for r in runs:
                r.merge_update()
            if k:  # the first round loads the code (and tunes)
                best = dt if best is None else min(best, dt)
        out[f"{mode}_round_ms"] = best * 1e3
        if mode == "tuned":
            out["tuning"] = [r.batch_tuning for r in runs]
        for r in runs:
            r.free()
        batch.free()
    out["tuned_over_rule"] = out["tuned_round_ms"] / out["rule_round_ms"]
    return out


def batched_vs_plain(rounds: int, max_iters: int | None = None, batch_lpc: int = 0, autotune: bool = True) -> dict:
    """Same instances, same iterations: one batched graph launch per round vs
    plain launches one instance after another.  With max_iters, every
    instance runs until flat (or the cap) and time to flat is reported."""
    import torch
    from paper_1312_2213_amd import muca
    specs = batched_instances()
    stream = torch.cuda.Stream()

    def run_plain():
        runs = [muca.Run(c, stream=stream) for c, _ in specs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ttf = []
        iters = []
        for (c, sw), r in zip(specs, runs):
            n = 0
            while True:
                r.run_iteration(sw, stream=stream)
                st = r.merge_update()
                n += 1
                if n % 500 == 0:
                    print(f"plain: instance {len(iters)}, iteration {n}, flatness {st['flatness']:.3f}",
                          file=sys.stderr, flush=True)
                if max_iters is None:
                    if n >= rounds:
                        break
                elif st["flat"] or n >= max_iters:
                    break
            ttf.append(time.perf_counter() - t0)
            iters.append(n)
            print(f"plain: instance {len(iters) - 1} done after {n} iterations, {ttf[-1]:.1f} s",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, ttf, iters, runs

    def run_batched():
        runs = [muca.Run(c, stream=stream) for c, _ in specs]
        batch = muca.Batch(len(runs), lanes_per_chain=batch_lpc, use_graph=True, autotune=autotune)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        live = list(range(len(runs)))
        n = [0] * len(runs)
        ttf = [0.0] * len(runs)
        flat = [False] * len(runs)
        while live:
            with torch.cuda.stream(stream):
                batch.run_iteration([runs[k] for k in live], [specs[k][1] for k in live], stream=stream)
            nxt = []
            for k in live:
                st = runs[k].merge_update()
                n[k] += 1
                flat[k] = bool(st["flat"])
                done = n[k] >= rounds if max_iters is None else (st["flat"] or n[k] >= max_iters)
                if done:
                    ttf[k] = time.perf_counter() - t0
                    print(f"batched: instance {k} done after {n[k]} iterations, {ttf[k]:.1f} s",
                          file=sys.stderr, flush=True)
                else:
                    nxt.append(k)
            live = nxt
            if live and max(n) % 500 == 0:
                print(f"batched: round {max(n)}, {len(live)} instances left", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        run_batched.flat = flat
        return time.perf_counter() - t0, ttf, n, runs

    def run_served():
        """The serving loop with every instance present at t = 0: rounds of
        equal site updates per chain, so a long iteration spans several
        rounds while short instances finish theirs every round."""
        from paper_1312_2213_amd.serve import Request, Server
        reqs = []
        for k, (c, sw) in enumerate(specs):
            cfg = muca.muca_config.from_buffer_copy(c)
            if max_iters is None:
                cfg.flat_threshold = 2.0  # fixed number of iterations: never flat
            reqs.append(Request(id=k, arrival=0.0, model="lattice", L=c.L, q=c.q, chains=c.n_chains,
                                seed=c.seed, max_iters=rounds if max_iters is None else max_iters,
                                sweeps_per_iter=sw, cfg=cfg))
        def tick(rounds, n_active):
            if rounds % 2000 == 0:
                print(f"served: round {rounds}, {n_active} instances left", file=sys.stderr, flush=True)

        srv = Server(hbm_budget=1 << 40, chain_slots=1 << 20, lanes_per_chain=batch_lpc,
                     keep_results=True, stream=stream, on_round=tick, autotune=autotune,
                     log=lambda r: print(f"served: instance {r.id} done after {r.iterations} iterations, "
                                         f"{r.finished:.1f} s", file=sys.stderr, flush=True))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = srv.serve(reqs, realtime=False)
        return time.perf_counter() - t0, [r.time_to_flat for r in res], [r.iterations for r in res], res

    tuned = tuned_vs_rule_round(stream) if autotune and batch_lpc == 0 else None
    tb, ttf_b, it_b, runs_b = run_batched()
    ts, ttf_s, it_s, res_s = run_served()
    tp, ttf_p, it_p, runs_p = run_plain()
    same = all((a.last_hist() == b.last_hist()).all() for a, b in zip(runs_b, runs_p))
    same_served = all((r.hist == b.last_hist()).all() for r, b in zip(res_s, runs_p))
    attempts = sum(c.n_chains * c.L * c.L * sw * k for (c, sw), k in zip(specs, it_b))
    mean = lambda a: sum(a) / len(a)  # noqa: E731
    own_p = [t - (ttf_p[k - 1] if k else 0.0) for k, t in enumerate(ttf_p)]
    out = {"instances": "potts q=8 L=16,24,32,48 x 2048 chains + 4 x muma L=32 x 512 chains (beta 0.5)",
           "sweeps_per_iteration": [sw for _, sw in specs],
           "iterations": it_b, "identical_iterations": it_b == it_p == list(it_s),
           "identical_histograms": bool(same and same_served),
           "makespan_s": {"batched": tb, "served": ts, "plain": tp},
           "speedup_makespan": {"batched": tp / tb, "served": tp / ts},
           "attempts_per_s": {"batched": attempts / tb, "served": attempts / ts, "plain": attempts / tp},
           "autotuned": bool(autotune and batch_lpc == 0), "tuned_vs_rule": tuned,
           "layouts": ["byte" if (c.model == muca.MUCA_POTTS or c.layout == muca.MUCA_LAYOUT_BYTE) else "bit"
                       for c, _ in specs]}
    if max_iters is not None:
        out.update({"flat_threshold": 0.5, "max_iters": max_iters, "flat": run_batched.flat,
                    "mean_time_to_flat_s": {"batched": mean(ttf_b), "served": mean(ttf_s), "plain": mean(ttf_p)},
                    "speedup_mean_time_to_flat": {"batched": mean(ttf_p) / mean(ttf_b),
                                                  "served": mean(ttf_p) / mean(ttf_s)},
                    "time_to_flat_s": {"batched": ttf_b, "served": ttf_s, "plain": ttf_p},
                    "plain_own_time_s": own_p,
                    "note": "all instances submitted at t = 0; plain runs them one after another, so its "
                            "per-instance time to flat includes the queueing behind earlier instances "
                            "(plain_own_time_s without it); makespan is the like-for-like comparison"})
    else:
        out["rounds"] = rounds
    return out


def bench_ising64_flat(args):
    """The headline configuration run to a flat histogram: Ising L = 64,
    bit-packed, 4096 chains, seed 2, 10^4 sweeps per iteration, lnW = 0 at
    the start, iterations until min(H)/mean(H) > 0.5 over the reachable bins
    of E in [-8192, 8192] (or the iteration cap).  Time to flat = wall time
    from the first launch to the end of the flat merge."""
    import torch
    from paper_1312_2213_amd import muca

    torch.cuda.set_device(0)
    L, C, seed, S = 64, 4096, 2, args.sweeps
    cap = args.max_iters or 700
    cfg = muca.muca_config_default("ising", L, 2, C, seed, layout=muca.MUCA_LAYOUT_BIT,
                                   lanes_per_chain=args.lanes_per_chain)
    stream = torch.cuda.current_stream()
    run = muca.Run(cfg, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n, st = 0, None
    while n < cap:
        run.run_iteration(S)
        st = run.merge_update()
        n += 1
        print(f"iteration {n}: flatness {st['flatness']:.3f}, visited [{st['lo_visited']}, {st['hi_visited']}], "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        if st["flat"]:
            break
    dt = time.perf_counter() - t0
    attempts = C * L * L * S * n
    return {"metric": "time-to-flat-histogram (plain MUCA, 1 GPU)", "value": dt, "unit": "s",
            "higher_is_better": False, "flat": bool(st["flat"]), "iterations": n,
            "attempts_per_s": attempts / dt, "final_flatness": st["flatness"],
            "visited": [st["lo_visited"], st["hi_visited"]], "n_gpus": 1, "dtype": "u32", "data": "synthetic",
            "config": {"workload": "plain MUCA 2D Ising L=64 periodic, bit-packed spins, 4096 chains, seed 2, "
                                   f"{S} sweeps per iteration, bins E in [-8192, 8192] step 4, flatness 0.5, "
                                   f"cap {cap} iterations"}}


def bench_ising64(args):
    import torch
    from paper_1312_2213_amd import muca

    torch.cuda.set_device(0)
    L, C, seed, S = 64, args.chains, 2, args.sweeps
    cfg = muca.muca_config_default("ising", L, 2, C, seed, layout=muca.MUCA_LAYOUT_BIT,
                                   lanes_per_chain=args.lanes_per_chain, chains_per_block=args.chains_per_block)
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
    cycles = 2.4e9 * kern_ms * 1e-3 / (L * L * S)
    # HBM bytes of one launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs of
    # this kernel at this launch size, while the kernel's sources are the
    # profiled ones
    sha = kernel_sources_sha256()
    traffic = HBM_TRAFFIC["bytes_per_launch"] if (
        sha == HBM_TRAFFIC["kernel_sources_sha256"] and S == 10000 and C == 4096
        and args.lanes_per_chain in (0, 16)) else None
    # the kernel is branch-free: the same launch at weights that reject about
    # half of the moves takes the same time
    rej = muca.Run(cfg, stream=stream)
    import numpy as np
    rej.set_lnw(-CPU_BETA * (-2.0 * L * L + 4.0 * np.arange(rej.n_bins)))
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    r0.record(stream)
    rej.run_iteration(S)
    r1.record(stream)
    rej_stats = rej.merge_update()
    rej_ms = r0.elapsed_time(r1)
    rej.free()

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
        "config": {"workload": f"plain MUCA 2D Ising L=64 periodic, bit-packed spins, {C} chains, "
                               f"seed 2, {S} sweeps per iteration, FP64 lnW, uint32 thresholds",
                   "L": L, "chains": C, "sweeps_per_iteration": S, "parallelism": "chains, 1 GPU"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_INT_OPS / 1e12,
                     "unit": "TOP/s", "frac": achieved / PEAK_INT_OPS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE, copy-calibrated)",
                     "traffic_kernel_sources_sha256": HBM_TRAFFIC["kernel_sources_sha256"],
                     "kernel_sources_sha256": sha,
                     "kernel": "lattice_sweeps<Ising, L=64, bit-packed>", "kernel_ms": kern_ms,
                     "ops_per_attempt": OPS_PER_ATTEMPT, "cycles_per_attempt_per_chain": cycles,
                     "kernel_ms_rejecting_weights": rej_ms,
                     "accept_rate_rejecting_weights": rej_stats["accept_rate"]},
        "iterations": [{k: s[k] for k in ("iteration", "flatness", "lo_visited", "hi_visited")}
                       for s in stats],
    }
    if C == 4096 and S == 10000:
        out["more_chains"] = more_chains(stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    if not args.no_batched:
        out["time_to_flat"] = batched_vs_plain(None, max_iters=args.flat_max_iters,
                                               batch_lpc=args.batch_lanes_per_chain)
    return out


def more_chains(stream, C=131072, S=1000):
    """The headline kernel's model and size (Ising L = 64, bit layout, table
    staged in LDS) with enough chains to keep two wavefronts on every SIMD:
    131072 chains in the library's default shape for that count (one lane
    per chain, blocks of 512 threads), one timed launch of S sweeps after an untimed one, at
    the weights of the first merge."""
    import torch
    from paper_1312_2213_amd import muca
    L = 64
    run = muca.Run(muca.muca_config_default("ising", L, 2, C, 2, layout=muca.MUCA_LAYOUT_BIT, lanes_per_chain=1),
                   stream=stream)
    run.run_iteration(S // 10)
    run.merge_update()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    run.run_iteration(S)
    e1.record(stream)
    st = run.merge_update()
    ms = e0.elapsed_time(e1)
    _, cpb = run.blocks_shape()
    rate = C * L * L * S / (ms * 1e-3)
    run.free()
    return {"chains": C, "sweeps": S, "lanes_per_chain": 1, "threads_per_block": cpb, "kernel_ms": ms,
            "attempts_per_s": rate, "frac_alu": rate * OPS_PER_ATTEMPT / PEAK_INT_OPS,
            "accept_rate": st["accept_rate"]}


def bench_potts48(args):
    """Plain MUCA of the batched workload's longest instance: q = 8 Potts,
    L = 48, 2048 chains, seed 33, 362 sweeps per iteration (Eq. 4's 8-state
    law at p = 2048), one launch + merge per step."""
    import torch
    from paper_1312_2213_amd import muca
    from synth.workloads import sweeps_per_iteration
    torch.cuda.set_device(0)
    L, q, C, seed = 48, 8, 2048, 33
    S = sweeps_per_iteration(L, C, True)
    stream = torch.cuda.current_stream()
    run = muca.Run(muca.muca_config_default("potts", L, q, C, seed, lanes_per_chain=args.lanes_per_chain),
                   stream=stream)
    for _ in range(args.warmup):
        run.run_iteration(S)
        run.merge_update()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        run.run_iteration(S)
        evs[k][1].record(stream)
        run.merge_update()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms = sum(a.elapsed_time(b) for a, b in evs) / args.steps
    attempts = C * L * L * S
    return {"metric": "spin-flip attempts/s (plain MUCA iteration, 1 GPU)", "value": attempts * args.steps / dt,
            "unit": "attempts/s", "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": dt / args.steps * 1e3, "kernel_ms": kern_ms,
            "kernel_attempts_per_s": attempts / (kern_ms * 1e-3),
            "cycles_per_attempt_per_chain": 2.4e9 * kern_ms * 1e-3 / (L * L * S),
            "config": {"workload": f"plain MUCA 2D q=8 Potts L=48, uint8 colours, {C} chains, seed {seed}, "
                                   f"{S} sweeps per iteration"}}


def bench_serving(args):
    from paper_1312_2213_amd.serve import Request, Server, summarize
    from synth import request_stream
    reqs = [Request(id=r["id"], arrival=r["arrival"], model=r["model"], L=r["L"], q=r["q"],
                    chains=r["chains"], seed=r["seed"], max_iters=args.max_iters)
            for r in request_stream(args.requests, 4.0, 4)]
    def retired(r):
        # one JSON line per request on stderr: arrival, admission, completion
        print(json.dumps({"request": r.id, "arrival_s": r.arrival, "admitted_s": r.admitted,
                          "finished_s": r.finished, "iterations": r.iterations, "flat": r.flat,
                          "cancelled": r.cancelled, "time_to_flat_s": r.time_to_flat}), file=sys.stderr, flush=True)

    kw = {} if args.overlap_min_rounds is None else {"overlap_min_rounds": args.overlap_min_rounds}
    srv = Server(hbm_budget=64 << 20, round_site_updates=args.round_site_updates, log=retired, **kw)
    t0 = time.perf_counter()
    res = srv.serve(reqs, realtime=True)
    s = summarize(res, time.perf_counter() - t0)
    s.update({"metric": "time-to-flat-histogram p50/p99 and aggregate attempts/s (serving, 1 GPU)",
              "workload": f"{args.requests} Poisson requests at 4/s, seed 4; Ising L in {{16..64}} or "
                          "Potts q in {2..10}, L in {16,32}; 256-2048 chains; flatness 0.5; "
                          f"max {args.max_iters} iterations; HBM budget 64 MiB; "
                          f"{args.round_site_updates} site updates per chain and round",
              "rounds": srv.rounds, "peak_active": srv.peak_active,
              "overlap_min_rounds": srv.overlap_min_rounds, "overlapped_merges": srv.overlapped_merges,
              "mean_round_ms": s["makespan_s"] / max(1, srv.rounds) * 1e3,
              "mean_overlapped_merge_ms": srv.merge_seconds / srv.merges * 1e3 if srv.merges else None})
    return s


def bench_polymer_paper(args):
    """The paper's homopolymer (Eq. 7 with its parameters, no LJ cutoff) at
    N = 40 and 80, 4096 chains: one JSON line each."""
    from synth import PAPER_POLYMER
    pp = dict(PAPER_POLYMER)
    for moves in (0, 1):
        for N in (40, 80):
            out = bench_polymer(args, N=N, params=dict(pp, x_lo=-400.0, x_hi=100.0, n_bins=1000, moves=moves),
                                walk=dict(bond=pp["fene_r0"], min_dist=pp["lj_sigma"]),
                                per_sweep=N if moves == 0 else 2 * N + 1)
            out["metric"] = ("polymer displacement attempts/s, the paper's homopolymer (1 GPU)" if moves == 0 else
                             "polymer move attempts/s (shift, spherical rotation, double bridging), "
                             "the paper's homopolymer (1 GPU)")
            out["config"] = {"workload": f"bead-spring homopolymer with the paper's parameters (K=40, r0=0.7, "
                                         f"r_max=1, sigma=2^(-1/6) r0, LJ uncut), N={N}, 4096 chains, seed 5, "
                                         "1000 sweeps per iteration, 1000 bins on [-400, 100)"
                                         + (", moves: N shifts + N rotations + 1 double bridging per sweep"
                                            if moves else ", moves: N shifts per sweep")}
            print(json.dumps(out), flush=True)
    return None


def bench_muma_em(args):
    """Multimagnetic Ising at the paper's T = 2/3 T_c (beta = 1.5 beta_c):
    weights iterated until the M histogram is flat, then a production run
    that records the joint (E, M) histogram, reweighted to temperatures
    around the run's; and the cost of that recording on the sweep kernel
    (4096 chains, L = 32, 1000 sweeps, with and without)."""
    import math
    import numpy as np
    import torch
    from paper_1312_2213_amd import muca
    from synth.workloads import sweeps_per_iteration
    beta_c = 0.5 * math.log(1.0 + math.sqrt(2.0))
    beta = 1.5 * beta_c
    L, C = 16, 1024
    stream = torch.cuda.current_stream()
    run = muca.Run(muca.muca_config_default("muma", L, 2, C, 9, beta=beta, layout=muca.MUCA_LAYOUT_BIT),
                   stream=stream)
    S = sweeps_per_iteration(L, C, False)
    t0 = time.perf_counter()
    n_it, flat = 0, False
    while n_it < args.max_iters and not flat:
        run.run_iteration(S)
        flat = run.merge_update()["flat"]
        n_it += 1
    t_conv = time.perf_counter() - t0
    ne, nm = run.em_shape()
    em = torch.zeros(ne * nm, dtype=torch.int64, device="cuda")
    P = 200
    run.run_iteration_em(P, em)
    run.merge_update()
    h = em.cpu().numpy().view(np.uint64).reshape(ne, nm)
    betas = [beta * f for f in (0.9, 0.95, 1.0, 1.05, 1.1)]
    rw = run.reweight_em(h, betas)
    # recording cost: same run shape with and without the joint histogram
    big = muca.Run(muca.muca_config_default("muma", 32, 2, 4096, 3, beta=beta, layout=muca.MUCA_LAYOUT_BIT),
                   stream=stream)
    ne2, nm2 = big.em_shape()
    em2 = torch.zeros(ne2 * nm2, dtype=torch.int64, device="cuda")
    ms = {}
    for mode in ("plain", "em", "plain", "em"):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if mode == "em":
            big.run_iteration_em(1000, em2)
        else:
            big.run_iteration(1000)
        e1.record(stream)
        big.merge_update()
        ms[mode] = e0.elapsed_time(e1)
    return {"metric": "multimagnetic run with joint (E, M) histogram, reweighted in beta (1 GPU)",
            "config": {"workload": f"MUMA Ising L={L}, beta = 1.5 beta_c = {beta:.6f}, {C} chains, seed 9, "
                                   f"{S} sweeps per iteration until flat, then {P} production sweeps"},
            "iterations_to_flat": n_it, "flat": bool(flat), "seconds_to_flat": t_conv,
            "reweighted": [{"beta": b, "e": r[0], "c": r[1], "abs_m": r[2], "m2": r[3], "chi": r[4]}
                           for b, r in zip(betas, rw.tolist())],
            "em_cost": {"workload": "MUMA L=32, 4096 chains, 1000 sweeps", "plain_ms": ms["plain"],
                        "em_ms": ms["em"], "overhead": ms["em"] / ms["plain"] - 1.0}}


def bench_polymer(args, N=40, params=None, walk=None, per_sweep=None):
    import numpy as np
    import torch
    from paper_1312_2213_amd import muca
    from synth import polymer_walk
    C, S = 4096, 1000
    pos = polymer_walk(N, C, 5, **(walk or {}))
    cfg = muca.muca_config_default("polymer", 0, 2, C, 5, n_beads=N, **(params or {}))
    stream = torch.cuda.current_stream()
    run = muca.Run(cfg, positions=pos, stream=stream)
    run.run_iteration(S)
    run.merge_update()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    kern = 0.0
    for _ in range(args.steps):
        e0.record(stream)
        run.run_iteration(S)
        e1.record(stream)
        run.merge_update()
        kern += e0.elapsed_time(e1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    moves = C * (per_sweep or N) * S * args.steps
    return {"metric": "polymer displacement attempts/s (MUCA iteration, 1 GPU)", "value": moves / dt,
            "unit": "moves/s", "kernel_moves_per_s": moves / (kern * 1e-3), "ms_per_step": dt / args.steps * 1e3,
            "kernel_ms_per_step": kern / args.steps, "steps": args.steps,
            "config": {"workload": "bead-spring homopolymer N=40, 4096 chains, seed 5, 1000 sweeps per "
                                   "iteration, 2500 bins on [-200, 50)"}}


def bench_speedup(args):
    """Statistical speedup S*_p (Eq. 6) of the paper's systems: one JSON line
    per system with N_iter to flat and to full coverage per p."""
    from paper_1312_2213_amd import speedup as su
    if args.speedup_set == "polymer":
        systems = su.paper_polymer_systems()
        if args.systems:
            systems = [systems[int(k)] for k in args.systems.split(",")]
        for system, ps, replicas in systems:
            print(f"== {system.name}: p = {ps}, {replicas} runs each", file=sys.stderr, flush=True)
            res = su.run_polymer(system, ps, replicas, seed0=1, max_iters=args.max_iters,
                                 log=lambda m: print(m, file=sys.stderr, flush=True))
            print(json.dumps({"metric": "statistical speedup S*_p (iterations to flat at equal statistics)",
                              "system": system.name, "n_beads": system.n_beads, "window": [system.lo, system.hi],
                              "n_bins": system.n_bins, "sweeps_total": system.sweeps_total,
                              "therm_frac": system.therm_frac, "replicas": replicas, "max_iters": args.max_iters,
                              "seconds": res.seconds, "flat": res.table("n_iter"), "cover": res.table("n_cover"),
                              "n_iter": {str(p): v for p, v in res.n_iter.items()}}), flush=True)
        return None
    if args.speedup_set == "time":
        systems = su.time_systems()
        if args.systems:
            systems = [systems[int(k)] for k in args.systems.split(",")]
        for system, ps, replicas in systems:
            print(f"== {system.name}: p = {ps}, {replicas} runs each, alone", file=sys.stderr, flush=True)
            res = su.run_alone(system, ps, replicas, seed0=1, max_iters=args.max_iters,
                               log=lambda m: print(m, file=sys.stderr, flush=True))
            print(json.dumps({"metric": "time speedup S_p = t_1 / t_p (wall time to flat, each run alone)",
                              "system": system.name, "replicas": replicas, "max_iters": args.max_iters,
                              "seconds": res.seconds, "time": su.time_speedup(res), "flat": res.table("n_iter")}),
                  flush=True)
        return None
    if args.speedup_set == "paper":
        systems = su.paper_systems()
    else:
        kw = {}
        if args.qscan_qs:
            kw["qs"] = [int(x) for x in args.qscan_qs.split(",")]
        if args.qscan_ps:
            kw["ps"] = [int(x) for x in args.qscan_ps.split(",")]
        if args.replicas:
            kw["replicas"] = args.replicas
        systems = su.q_scan_systems(args.qscan_L, **kw)
    if args.systems:
        systems = [systems[int(k)] for k in args.systems.split(",")]
    for system, ps, replicas in systems:
        print(f"== {system.name}: p = {ps}, {replicas} runs each", file=sys.stderr, flush=True)
        res = su.run(system, ps, replicas, seed0=1, max_iters=args.max_iters,
                     log=lambda m: print(m, file=sys.stderr, flush=True))
        print(json.dumps({"metric": "statistical speedup S*_p (iterations to flat at equal statistics)",
                          "system": system.name, "q": system.q, "L": system.L,
                          "sweeps_law": "8-state Potts" if system.potts_law else "Ising",
                          "replicas": replicas, "max_iters": args.max_iters,
                          "seconds": res.seconds, "flat": res.table("n_iter"),
                          "cover": res.table("n_cover"),
                          "n_iter": {str(p): v for p, v in res.n_iter.items()}}), flush=True)
    return None


def bench_copy():
    """Device copy of 256 MiB (read 256 MiB, write 256 MiB), to scale HBM counters."""
    import torch
    n = 256 << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"workload": "copy", "bytes_read_per_copy": n, "bytes_written_per_copy": n, "copies": 3}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        sys.exit(2)
    if not os.environ.get("MUCA_AUTOTUNE_CACHE"):
        # batched item times are measured once per class and reused by every leg
        import tempfile
        os.environ["MUCA_AUTOTUNE_CACHE"] = os.path.join(tempfile.gettempdir(), f"muca_autotune_{os.getpid()}.json")
    if args.max_iters is None:
        args.max_iters = {"serving": 3000, "speedup": 1000, "muma_em": 1000, "ising64_flat": 700}.get(args.workload, 40)
    if args.workload == "ising64":
        out = bench_ising64(args)
    elif args.workload == "ising64_flat":
        out = bench_ising64_flat(args)
    elif args.workload == "potts48":
        out = bench_potts48(args)
    elif args.workload == "batched":
        out = batched_vs_plain(args.batched_rounds, max_iters=args.max_iters, batch_lpc=args.batch_lanes_per_chain)
    elif args.workload == "serving":
        out = bench_serving(args)
    elif args.workload == "polymer":
        out = bench_polymer(args)
    elif args.workload == "polymer_paper":
        out = bench_polymer_paper(args)
    elif args.workload == "speedup":
        out = bench_speedup(args)
    elif args.workload == "muma_em":
        out = bench_muma_em(args)
    else:
        out = bench_copy()
    if out is not None:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
