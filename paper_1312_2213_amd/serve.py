"""Continuous-batching server for multicanonical runs.

Requests (a lattice model, L, q, chains and seed) arrive over time.  A
request is admitted as soon as its device footprint (muca_workspace_bytes)
fits in the HBM budget and its chains fit in the chain-slot budget; its
chain state and weights then stay resident on the device until it retires.
Every round is ONE persistent batched launch over the admitted requests
that are not being merged: each advances by a chunk of sweeps sized so that
a round costs about the same number of site updates per chain for every
request (small lattices do not wait behind large ones).  When a request has
run the sweeps of its current iteration, the read-back of its merged
histogram is queued behind that round (muca_merge_begin).  A request whose
iterations span at least `overlap_min_rounds` rounds is left out of the
next round, and the host part of its merge (flatness, accumulated-statistics
recursion, new thresholds: muca_merge_finish) runs while that round is on
the device; it rejoins the round after (one skipped round per iteration, a
small share of a long iteration).  A request with shorter iterations is
merged before the next round is launched, so it never skips one.  A request
retires when its histogram is flat or after max_iters iterations.

Chunking only moves launch boundaries, so every request's result is
bit-identical to running it alone.

Sweeps per iteration follow the paper's M_opt(L, p) power laws (Eq. 4) for
p = 1, divided over the request's chains (at least 10): the Ising law for
Ising and q = 2 Potts, the 8-state Potts law for Potts q >= 3.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import muca
from synth.workloads import sweeps_per_iteration


@dataclass
class Request:
    id: int
    arrival: float
    model: str
    L: int
    q: int
    chains: int
    seed: int
    flat_threshold: float = 0.5
    max_iters: int = 1000
    sweeps_per_iter: int = 0
    cfg: object = None  # a complete muca_config (e.g. a MUMA run's beta); overrides the fields above

    def config(self):
        if self.cfg is not None:
            return self.cfg
        kw = {"flat_threshold": self.flat_threshold, "layout": muca.MUCA_LAYOUT_BIT if self.model == "ising"
              else muca.MUCA_LAYOUT_AUTO}
        return muca.muca_config_default(self.model, self.L, self.q, self.chains, self.seed, **kw)

    def __post_init__(self):
        if not self.sweeps_per_iter:
            # Potts bins are one per unit of unsatisfied bonds: for q >= 3
            # nearly all 2N + 1 are reachable, four times the Ising count,
            # so the Ising law would leave too few samples per bin to pass
            # the flatness test; q >= 3 takes the 8-state Potts law.
            potts_fit = self.model == "potts" and self.q >= 3
            self.sweeps_per_iter = sweeps_per_iteration(self.L, self.chains, potts_fit)


@dataclass
class Result:
    id: int
    arrival: float
    admitted: float | None = 0.0
    finished: float = 0.0
    iterations: int = 0
    flat: bool = False
    flatness: float = 0.0
    attempts: int = 0
    cancelled: bool = False
    lnw: np.ndarray | None = field(default=None, repr=False)
    hist: np.ndarray | None = field(default=None, repr=False)

    @property
    def time_to_flat(self) -> float:
        return self.finished - self.arrival


class _Active:
    def __init__(self, req: Request, run: muca.Run, footprint: int, res: Result):
        self.req, self.run, self.footprint, self.res = req, run, footprint, res
        self.done_in_iter = 0


class Server:
    def __init__(self, hbm_budget: int = 64 << 20, chain_slots: int = 1 << 16,
                 round_site_updates: int = 1 << 16, lanes_per_chain: int = 0, use_graph: bool = True,
                 max_active: int = 256, keep_results: bool = False, stream=None, log=None, on_round=None,
                 autotune: bool = False, overlap_min_rounds: int = 4):
        import torch
        self.overlap_min_rounds = overlap_min_rounds
        self.hbm_budget = hbm_budget
        self.chain_slots = chain_slots
        self.round_site_updates = round_site_updates
        self.keep = keep_results
        self.stream = stream or torch.cuda.Stream()
        self.batch = muca.Batch(max_active, max_items=1 << 15, lanes_per_chain=lanes_per_chain,
                                use_graph=use_graph, autotune=autotune)
        self.max_active = max_active
        self.log = log  # called with each Result as its request retires
        self.on_round = on_round  # called with (rounds so far, active requests) after each round
        self.rounds = 0
        self.peak_active = 0
        self.peak_mem = 0
        self.overlapped_merges = 0  # merges whose host part ran while a round was on the device
        self.merge_seconds = 0.0    # host time in muca_merge_finish (overlapped merges: no wait)
        self.merges = 0
        self._cancel: set[int] = set()

    def cancel(self, request_id: int):
        """Withdraws a request: if it is waiting it is never admitted, if it
        runs it leaves before the next round (its device memory is freed);
        the other requests' results are unchanged.  May be called from the
        log or on_round callbacks."""
        self._cancel.add(request_id)

    def _per_round(self, a: _Active) -> int:
        return max(1, self.round_site_updates // (a.req.L * a.req.L))

    def _chunk(self, a: _Active) -> int:
        return min(self._per_round(a), a.req.sweeps_per_iter - a.done_in_iter)

    def _overlapped(self, a: _Active) -> bool:
        """Whether this request's merges overlap the next round."""
        return -(-a.req.sweeps_per_iter // self._per_round(a)) >= self.overlap_min_rounds

    def serve(self, requests: list[Request], realtime: bool = True) -> list[Result]:
        """Runs the requests to completion; arrival times are seconds from start
        (realtime) or only an ordering (realtime=False: all present at t = 0)."""
        import torch
        pending = sorted(requests, key=lambda r: (r.arrival, r.id))
        queue: list[Request] = []
        ready: list[_Active] = []    # admitted, taking part in the next round
        merging: list[_Active] = []  # read-back queued behind the last round
        results: dict[int, Result] = {}
        used_mem = 0
        used_chains = 0
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        def drop(req: Request, res: Result | None = None):
            # a request withdrawn before admission has no admission time
            res = res or Result(req.id, req.arrival if realtime else 0.0, admitted=None)
            res.cancelled = True
            res.finished = now()
            results[req.id] = res
            if self.log:
                self.log(res)

        while pending or queue or ready or merging:
            t = now()
            while pending and (not realtime or pending[0].arrival <= t):
                queue.append(pending.pop(0))
            if self._cancel:
                for req in [r for r in pending + queue if r.id in self._cancel]:
                    (pending if req in pending else queue).remove(req)
                    drop(req)
                for a in [a for a in ready if a.req.id in self._cancel]:
                    ready.remove(a)
                    a.run.free()
                    used_mem -= a.footprint
                    used_chains -= a.req.chains
                    drop(a.req, a.res)
                if not (pending or queue or ready or merging):
                    break
            # admission, first come first served
            while queue and len(ready) + len(merging) < self.max_active:
                req = queue[0]
                cfg = req.config()
                fp = muca.muca_workspace_bytes(cfg)
                if (ready or merging) and (used_mem + fp > self.hbm_budget
                                           or used_chains + req.chains > self.chain_slots):
                    break
                queue.pop(0)
                with torch.cuda.stream(self.stream):
                    run = muca.Run(cfg, stream=self.stream)
                res = Result(req.id, req.arrival if realtime else 0.0, admitted=now())
                results[req.id] = res
                ready.append(_Active(req, run, fp, res))
                used_mem += fp
                used_chains += req.chains
            self.peak_active = max(self.peak_active, len(ready) + len(merging))
            self.peak_mem = max(self.peak_mem, used_mem)
            if not ready and not merging:
                if pending:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - now())))
                continue
            # 1. one round for the requests not being merged (returns once enqueued)
            began = []
            launched = bool(ready)
            if ready:
                chunks = [self._chunk(a) for a in ready]
                with torch.cuda.stream(self.stream):
                    self.batch.run_iteration([a.run for a in ready], chunks, stream=self.stream)
                self.rounds += 1
                still = []
                for a, ch in zip(ready, chunks):
                    a.done_in_iter += ch
                    a.res.attempts += ch * a.req.chains * a.req.L * a.req.L
                    if a.done_in_iter < a.req.sweeps_per_iter:
                        still.append(a)
                    else:
                        a.run.merge_begin()  # read-back queued behind this round
                        began.append(a)
                ready = still
            # 2. the merges begun one round earlier (their read-back precedes the
            #    round just launched, so this host work overlaps it), then those
            #    of requests with short iterations (these wait for the round)
            if launched and merging:
                self.overlapped_merges += len(merging)
            now_merged = [a for a in began if not self._overlapped(a)]
            began = [a for a in began if self._overlapped(a)]
            for a in merging + now_merged:
                t_m = time.perf_counter()
                st = a.run.merge_finish()
                if a in merging:
                    self.merge_seconds += time.perf_counter() - t_m
                    self.merges += 1
                a.done_in_iter = 0
                a.res.iterations += 1
                a.res.flatness = st["flatness"]
                if st["flat"] or a.res.iterations >= a.req.max_iters:
                    a.res.flat = bool(st["flat"])
                    a.res.finished = now()
                    if self.keep:
                        a.res.lnw = a.run.lnw()
                        a.res.hist = a.run.last_hist()
                    a.run.free()
                    if self.log:
                        self.log(a.res)
                    used_mem -= a.footprint
                    used_chains -= a.req.chains
                else:
                    ready.append(a)
            merging = began
            if self.on_round:
                self.on_round(self.rounds, len(ready) + len(merging))
        torch.cuda.synchronize()
        return [results[r.id] for r in sorted(requests, key=lambda r: r.id)]


def run_alone(req: Request, stream=None) -> Result:
    """Plain per-request loop of single launches (one launch per iteration)."""
    import torch
    t0 = time.perf_counter()
    run = muca.Run(req.config(), stream=stream)
    res = Result(req.id, 0.0)
    while True:
        run.run_iteration(req.sweeps_per_iter, stream=stream)
        st = run.merge_update()
        res.iterations += 1
        res.attempts += req.sweeps_per_iter * req.chains * req.L * req.L
        res.flatness = st["flatness"]
        if st["flat"] or res.iterations >= req.max_iters:
            res.flat = bool(st["flat"])
            break
    res.lnw = run.lnw()
    res.hist = run.last_hist()
    torch.cuda.synchronize()
    res.finished = time.perf_counter() - t0
    run.free()
    return res


def summarize(results: list[Result], makespan: float) -> dict:
    """Time to flat (arrival -> merge of the first flat iteration) over the
    requests that became flat; requests stopped by max_iters are counted
    apart, with their time to stop."""
    flat = np.array([r.time_to_flat for r in results if r.flat])
    capped = np.array([r.time_to_flat for r in results if not r.flat and not r.cancelled])
    attempts = sum(r.attempts for r in results)

    def pct(a, p):
        return float(np.percentile(a, p)) if len(a) else None

    return {"requests": len(results), "flat": int(len(flat)), "capped": int(len(capped)),
            "cancelled": sum(1 for r in results if r.cancelled),
            "p50_time_to_flat_s": pct(flat, 50), "p99_time_to_flat_s": pct(flat, 99),
            "mean_time_to_flat_s": float(flat.mean()) if len(flat) else None,
            "p50_time_to_stop_capped_s": pct(capped, 50), "makespan_s": makespan,
            "attempts": attempts, "attempts_per_s": attempts / makespan if makespan > 0 else 0.0}
