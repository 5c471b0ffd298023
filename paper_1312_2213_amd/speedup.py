"""Statistical speedup of the parallel multicanonical iteration on one GPU.

The paper's time-independent measure (Eq. 6): with p independent chains per
run and M_opt(L, p) = M_opt(L, 1) / p sweeps per chain and iteration
(Eq. 4), the total statistics per iteration is the same for every p, and

    S*_p = [N_iter M_opt(1)]_1 / [N_iter M_opt(p)]_p = p N_iter(1) / N_iter(p)

where N_iter is the number of iterations until the merged histogram is flat
(min/mean over the reachable bins above the flatness threshold), averaged
over independent runs.  The first iteration whose histogram covers every
reachable bin (min > 0) is recorded as a second convergence measure.  The paper finds S*_p close to p for the
Ising model and a saturation at large p for the 8-state Potts model and for
the multimagnetic Ising run at T = 2/3 T_c (its speedup figures; the values
are not in the text).

Here every (p, replica) run of one system starts from lnW = 0 with its own
seed, all of them advance together (one batched persistent launch per
round, every live run doing one iteration of its own sweep count), and a
run retires at its first flat iteration.  Chains are thermalised only by
the iterations themselves, as in the paper.  When the smallest p measured
is p0 > 1, S*_p is reported relative to it: (p / p0) N_iter(p0) / N_iter(p).
The reference p0 is the smallest p whose runs all converged: an Ising run
of very few chains can stay at lnW = 0 for good, since with every flip
accepted a sequential sweep maps s to -s and keeps E, so the per-sweep
histogram of each chain holds one bin and the recursion, which links
neighbouring bins, has nothing to link.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import muca
from synth.workloads import m_opt

BETA_C = 0.5 * math.log(1.0 + math.sqrt(2.0))  # 2D Ising critical coupling


@dataclass
class System:
    model: str          # "ising", "potts" or "muma"
    L: int
    q: int = 2
    beta: float = 0.0   # MUMA: fixed canonical beta of the energy factor
    potts_law: bool = False  # use the 8-state Potts power law of Eq. 4

    def sweeps(self, p: int) -> int:
        """M_opt(L, p) = ceil(M_opt(L, 1) / p), at least one sweep."""
        return max(1, math.ceil(m_opt(self.L, 1, self.potts_law) / p))

    def config(self, p: int, seed: int, flat: float):
        kw = {"flat_threshold": flat}
        if self.model == "muma":
            kw["beta"] = self.beta
        if self.model != "potts":
            kw["layout"] = muca.MUCA_LAYOUT_BIT
        return muca.muca_config_default(self.model, self.L, self.q, p, seed, **kw)

    @property
    def name(self) -> str:
        if self.model == "potts":
            return f"{self.q}-state Potts L={self.L}"
        if self.model == "muma":
            return f"multimagnetic Ising L={self.L} beta={self.beta:.4f}"
        return f"Ising L={self.L}"


@dataclass
class Result:
    system: str
    ps: list
    sweeps: list
    n_iter: dict = field(default_factory=dict)   # p -> N_iter per replica (None: capped)
    n_cover: dict = field(default_factory=dict)  # p -> first iteration with every bin visited
    trace: dict = field(default_factory=dict)    # p -> flatness of every iteration, per replica
    seconds: float = 0.0

    def table(self, measure: str = "n_iter") -> list[dict]:
        """Mean and standard error of the measure per p; S*_p relative to
        the smallest p whose runs all converged (None below it)."""
        data = getattr(self, measure)
        rows = []
        for p, m in zip(self.ps, self.sweeps):
            v = [x for x in data[p] if x is not None]
            mean = float(np.mean(v)) if v else None
            err = float(np.std(v, ddof=1) / math.sqrt(len(v))) if len(v) > 1 else None
            rows.append({"p": p, "sweeps_per_iteration": m, "runs": len(data[p]),
                         "capped": len(data[p]) - len(v), "mean": mean, "err": err,
                         "speedup": None, "speedup_err": None})
        base = next((r for r in rows if r["capped"] == 0 and r["err"] is not None), None)
        if base is not None:
            for r in rows[rows.index(base):]:
                if r["mean"] is not None and r["err"] is not None:
                    r["speedup"], r["speedup_err"] = speedup(base["p"], base["mean"], base["err"],
                                                             r["p"], r["mean"], r["err"])
        return rows


def speedup(p0: int, n0: float, e0: float, p: int, n: float, e: float) -> tuple[float, float]:
    """S*_p relative to p0 (Eq. 6 with equal total statistics per
    iteration): (p / p0) n0 / n, with the error of the two means propagated."""
    s = (p / p0) * n0 / n
    rel = math.sqrt((e0 / n0) ** 2 + (e / n) ** 2) if n0 > 0 and n > 0 else float("nan")
    return s, s * rel


def seed_of(seed0: int, k: int, r: int) -> int:
    """Seed of replica r of the k-th p value."""
    return seed0 + 1000 * k + r


def run(system: System, ps: list[int], replicas: int, seed0: int = 1, flat: float = 0.5,
        max_iters: int = 1000, stream=None, log=None) -> Result:
    """Runs `replicas` independent runs for every p until flat (or max_iters)."""
    import time

    import torch
    stream = stream or torch.cuda.Stream()
    sweeps = [system.sweeps(p) for p in ps]
    specs = [(p, m, seed_of(seed0, k, r), r) for k, (p, m) in enumerate(zip(ps, sweeps)) for r in range(replicas)]
    runs = []
    with torch.cuda.stream(stream):
        for p, _, seed, _ in specs:
            runs.append(muca.Run(system.config(p, seed, flat), stream=stream))
    batch = muca.Batch(len(runs), max_items=1 << 15, lanes_per_chain=0, use_graph=True)
    res = Result(system.name, list(ps), sweeps, {p: [None] * replicas for p in ps},
                 {p: [None] * replicas for p in ps}, {p: [[] for _ in range(replicas)] for p in ps})
    live = list(range(len(runs)))
    n = [0] * len(runs)
    t0 = time.perf_counter()
    rounds = 0
    while live:
        with torch.cuda.stream(stream):
            batch.run_iteration([runs[i] for i in live], [specs[i][1] for i in live], stream=stream)
        rounds += 1
        if log and rounds % 50 == 0:
            log(f"{system.name}: round {rounds}, {len(live)} runs left, {time.perf_counter() - t0:.0f} s")
        nxt = []
        for i in live:
            st = runs[i].merge_update()
            n[i] += 1
            p, r = specs[i][0], specs[i][3]
            res.trace[p][r].append(st["flatness"])
            if st["flatness"] > 0 and res.n_cover[p][r] is None:
                res.n_cover[p][r] = n[i]
            if st["flat"] or n[i] >= max_iters:
                res.n_iter[p][r] = n[i] if st["flat"] else None
                runs[i].free()
                if log:
                    log(f"{system.name} p={specs[i][0]} seed={specs[i][2]}: "
                        f"{n[i]} iterations{'' if st['flat'] else ' (capped)'}")
            else:
                nxt.append(i)
        live = nxt
    torch.cuda.synchronize()
    res.seconds = time.perf_counter() - t0
    batch.free()
    return res


def run_alone(system: System, ps: list[int], replicas: int, seed0: int = 1, flat: float = 0.5,
              max_iters: int = 1000, log=None) -> Result:
    """The time speedup of Eq. 5 on one GPU: every (p, replica) run alone
    (nothing else on the device), one plain launch per iteration followed by
    the merge; t_p = wall time from the first launch to the merged flat
    histogram (launches, histogram download, recursion and threshold upload
    included: the on-device counterpart of the paper's per-iteration
    communication).  Same seeds as `run`, so the same chains and N_iter.
    Result.seconds_per_run[p] holds the times of the replicas."""
    import time

    import torch
    stream = torch.cuda.Stream()
    sweeps = [system.sweeps(p) for p in ps]
    res = Result(system.name, list(ps), sweeps, {p: [None] * replicas for p in ps},
                 {p: [None] * replicas for p in ps}, {p: [[] for _ in range(replicas)] for p in ps})
    res.seconds_per_run = {p: [None] * replicas for p in ps}
    t_all = time.perf_counter()
    for k, (p, m) in enumerate(zip(ps, sweeps)):
        for r in range(replicas):
            with torch.cuda.stream(stream):
                run = muca.Run(system.config(p, seed_of(seed0, k, r), flat), stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n, st = 0, None
            while n < max_iters:
                run.run_iteration(m)
                st = run.merge_update()
                n += 1
                res.trace[p][r].append(st["flatness"])
                if st["flatness"] > 0 and res.n_cover[p][r] is None:
                    res.n_cover[p][r] = n
                if st["flat"]:
                    break
            dt = time.perf_counter() - t0
            res.n_iter[p][r] = n if st["flat"] else None
            res.seconds_per_run[p][r] = dt if st["flat"] else None
            run.free()
            if log:
                log(f"{system.name} p={p} seed={seed_of(seed0, k, r)} alone: {n} iterations, {dt:.3f} s"
                    f"{'' if st['flat'] else ' (capped)'}")
    res.seconds = time.perf_counter() - t_all
    return res


def time_speedup(res: Result) -> list[dict]:
    """S_p = t_p0 / t_p (Eq. 5, relative to the smallest fully converged p)
    with the mean wall time to flat per p and its standard error."""
    rows = []
    for p, m in zip(res.ps, res.sweeps):
        v = [x for x in res.seconds_per_run[p] if x is not None]
        mean = float(np.mean(v)) if v else None
        err = float(np.std(v, ddof=1) / math.sqrt(len(v))) if len(v) > 1 else None
        rows.append({"p": p, "sweeps_per_iteration": m, "runs": len(res.seconds_per_run[p]),
                     "capped": len(res.seconds_per_run[p]) - len(v), "t_mean_s": mean, "t_err_s": err,
                     "S_p": None, "S_p_err": None})
    base = next((r for r in rows if r["capped"] == 0 and r["t_err_s"] is not None), None)
    if base is not None:
        for r in rows[rows.index(base):]:
            if r["t_mean_s"] is not None and r["t_err_s"] is not None:
                s = base["t_mean_s"] / r["t_mean_s"]
                rel = math.sqrt((base["t_err_s"] / base["t_mean_s"]) ** 2 + (r["t_err_s"] / r["t_mean_s"]) ** 2)
                r["S_p"], r["S_p_err"] = s, s * rel
    return rows


def time_systems() -> list[tuple[System, list[int], int]]:
    """Systems of the time-speedup measurement: the 8-state Potts model at
    L = 8 (converges from p = 1) and the Ising model at L = 16 (from p = 4,
    see the remark on lnW = 0 above)."""
    pw = [2 ** k for k in range(0, 11)]
    return [(System("potts", 8, q=8, potts_law=True), pw, 8), (System("ising", 16), pw[2:], 8)]


def paper_systems() -> list[tuple[System, list[int], int]]:
    """The systems of the paper's speedup figures (Ising; 8-state Potts with
    its own power law; multimagnetic Ising at T = 2/3 T_c with the Ising
    law, extrapolated as the paper does for the remaining systems), at sizes
    whose smallest-p iterations take at most ~70 ms on one GPU:
    (system, p values, replicas)."""
    pw = [2 ** k for k in range(0, 13)]
    return [
        (System("ising", 8), pw[:11], 16),
        (System("ising", 16), pw[:11], 16),
        (System("ising", 24), pw[3:12], 8),
        (System("potts", 8, q=8, potts_law=True), pw[:11], 16),
        (System("potts", 16, q=8, potts_law=True), pw[4:12], 8),
        (System("muma", 16, beta=1.5 * BETA_C), pw[:11], 16),
    ]


def q_scan_systems(L: int = 16, qs=range(2, 11), ps=None, replicas: int = 8) -> list[tuple[System, list[int], int]]:
    """The q-state Potts crossover scan of the paper's q figure (second-order
    transition for q <= 4, weakly first order at q = 5, first order above):
    S*_p for every q at one lattice size.  The paper extrapolates M_opt per q
    without printing the values; here q = 2 takes the Ising law of Eq. 4 and
    q >= 3 the 8-state Potts law (the per-unit energy bins of q >= 3 need the
    statistics of the latter).  The paper's lattice is 64 x 64, whose
    smallest-p iterations do not fit one GPU's time budget; the default is
    16 x 16 with p = 16 .. 2048."""
    ps = list(ps) if ps is not None else [2 ** k for k in range(4, 12)]
    return [(System("potts", L, q=q, potts_law=q >= 3), ps, replicas) for q in qs]


# --------------------------------------------------------------------------
# The bead-spring homopolymer (the paper's polymer figure)
# --------------------------------------------------------------------------
@dataclass
class PolymerSystem:
    """The paper's homopolymer (Eq. 7 with its parameters) with the paper's
    move set, its energy range restricted to a window around the collapse
    transition, a fixed number of sweeps per iteration summed over the p
    chains (M(p) = ceil(M_total / p)), and thermalisation sweeps before
    every iteration (a fraction of M(p), at least one)."""
    n_beads: int
    lo: float
    hi: float
    n_bins: int
    sweeps_total: int
    therm_frac: float = 0.25
    moves: int = 1

    def sweeps(self, p: int) -> int:
        return max(1, math.ceil(self.sweeps_total / p))

    def therm(self, p: int) -> int:
        return max(1, math.ceil(self.therm_frac * self.sweeps(p)))

    def config(self, p: int, seed: int):
        from synth import PAPER_POLYMER
        return muca.muca_config_default("polymer", 0, 2, p, seed, n_beads=self.n_beads, x_lo=self.lo,
                                        x_hi=self.hi, n_bins=self.n_bins, moves=self.moves, **PAPER_POLYMER)

    @property
    def name(self) -> str:
        return f"homopolymer N={self.n_beads} E in [{self.lo:g}, {self.hi:g})"


def polymer_flatness(H) -> float:
    """min / mean over every bin of the window (all are reachable there)."""
    H = np.asarray(H, np.float64)
    return float(H.min() / H.mean()) if H.sum() > 0 else 0.0


def polymer_start(system: PolymerSystem, count: int, seed: int = 99, chains: int = 4096,
                  wide=(-220.0, 40.0, 520), max_iters: int = 400, stream=None) -> np.ndarray:
    """`count` conformations [count][N][3] whose energies lie in the window:
    a multicanonical run over a wide range from random walks, collecting the
    chains inside the window after each iteration (each chain at most once
    per iteration)."""
    from synth import PAPER_POLYMER, polymer_walk
    pp = dict(PAPER_POLYMER)
    pos = polymer_walk(system.n_beads, chains, seed, bond=pp["fene_r0"], min_dist=pp["lj_sigma"])
    cfg = muca.muca_config_default("polymer", 0, 2, chains, seed, n_beads=system.n_beads, x_lo=wide[0],
                                   x_hi=wide[1], n_bins=wide[2], moves=system.moves, **pp)
    run = muca.Run(cfg, positions=pos, stream=stream)
    got = []
    n = 0
    for _ in range(max_iters):
        run.run_iteration(200)
        run.merge_update()
        state, _, E = run.chain_state()
        sel = (E >= system.lo) & (E < system.hi)
        got.append(state[sel])
        n += int(sel.sum())
        if n >= count:
            break
    run.free()
    if n < count:
        raise RuntimeError(f"only {n} conformations in the window after {max_iters} iterations")
    return np.concatenate(got)[:count]


def run_polymer(system: PolymerSystem, ps: list[int], replicas: int, seed0: int = 1, max_iters: int = 500,
                start: np.ndarray | None = None, n_streams: int = 4, log=None) -> Result:
    """S*_p of the homopolymer: `replicas` runs per p, each from lnW = 0
    with distinct start conformations (from the window) and seeds, all runs
    advancing together (one iteration each per round, spread over a few
    streams), every run retiring at its first flat iteration."""
    import time

    import torch
    total = sum(ps) * replicas
    if start is None:
        start = polymer_start(system, total)
    if len(start) < total:
        raise ValueError(f"need {total} start conformations, got {len(start)}")
    streams = [torch.cuda.Stream() for _ in range(n_streams)]
    sweeps = [system.sweeps(p) for p in ps]
    specs, runs, off = [], [], 0
    for k, p in enumerate(ps):
        for r in range(replicas):
            st = streams[len(runs) % n_streams]
            runs.append(muca.Run(system.config(p, seed_of(seed0, k, r)), positions=start[off:off + p], stream=st))
            specs.append((p, r, st))
            off += p
    res = Result(system.name, list(ps), sweeps, {p: [None] * replicas for p in ps},
                 {p: [None] * replicas for p in ps}, {p: [[] for _ in range(replicas)] for p in ps})
    live = list(range(len(runs)))
    n = [0] * len(runs)
    t0 = time.perf_counter()
    rounds = 0
    while live:
        rounds += 1
        if log and rounds % 50 == 0:
            log(f"{system.name}: round {rounds}, {len(live)} runs live, {time.perf_counter() - t0:.1f} s")
        for i in live:
            p, _, st = specs[i]
            runs[i].thermalize(system.therm(p), stream=st)
            runs[i].run_iteration(system.sweeps(p), stream=st)
        nxt = []
        for i in live:
            p, r, _ = specs[i]
            runs[i].merge_update()
            H = runs[i].last_hist()
            f = polymer_flatness(H)
            n[i] += 1
            res.trace[p][r].append(f)
            if f > 0 and res.n_cover[p][r] is None:
                res.n_cover[p][r] = n[i]
            if f > 0.5 or n[i] >= max_iters:
                res.n_iter[p][r] = n[i] if f > 0.5 else None
                runs[i].free()
                if log:
                    log(f"{system.name} p={p} run {r}: {n[i]} iterations{'' if f > 0.5 else ' (capped)'}")
            else:
                nxt.append(i)
        live = nxt
    torch.cuda.synchronize()
    res.seconds = time.perf_counter() - t0
    return res


def paper_polymer_systems() -> list[tuple[PolymerSystem, list[int], int]]:
    """The paper's polymer figure (N = 40 and 80): windows around the
    collapse transition where the canonical energy rises steeply (T between
    about 0.9 and 1.8 for the paper's parameters, measured with this
    library), bins 2 wide, 1024 sweeps per iteration in total: (system, p
    values, replicas)."""
    pw = [2 ** k for k in range(0, 9)]
    return [
        (PolymerSystem(40, -70.0, -20.0, 25, 1024), pw, 8),
        (PolymerSystem(80, -140.0, -40.0, 50, 1024), pw[:8], 4),
    ]

