"""Batched persistent launches (one launch for runs of mixed model, L, q,
ensemble and layout) must reproduce plain per-run launches bit for bit,
graph replays included; the autotuner returns a valid, result-preserving
variant."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MIX = [  # (model, L, q, chains, seed, layout, sweeps)
    ("ising", 16, 2, 130, 41, 1, 12),
    ("ising", 24, 2, 64, 42, 2, 7),
    ("muma", 32, 2, 100, 43, 1, 5),
    ("potts", 16, 8, 70, 44, 2, 9),
    ("potts", 48, 3, 64, 45, 2, 2),
    ("ising", 64, 2, 256, 46, 1, 3),
    ("muma", 8, 2, 33, 47, 2, 20),
]


def make(spec):
    from paper_1312_2213_amd import muca
    model, L, q, chains, seed, layout, _ = spec
    kw = dict(layout=layout)
    if model == "muma":
        kw["beta"] = 0.5
    return muca.Run(muca.muca_config_default(model, L, q, chains, seed, **kw))


def snapshot(r):
    s, b, _ = r.chain_state()
    return r.last_hist().copy(), r.lnw().copy(), s, b


@pytest.mark.parametrize("graph,lpc", [(True, 4), (False, 4), (True, 16), (True, 0)])
def test_batched_equals_plain(graph, lpc):
    import torch
    from paper_1312_2213_amd import muca
    stream = torch.cuda.Stream()
    plain = [make(s) for s in MIX]
    batched = [make(s) for s in MIX]
    batch = muca.Batch(len(MIX), lanes_per_chain=lpc, use_graph=graph)
    sweeps = [s[-1] for s in MIX]
    for it in range(4):
        print(f"  iteration {it}", flush=True)
        for r, sw in zip(plain, sweeps):
            r.run_iteration(sw)
            r.merge_update()
        with torch.cuda.stream(stream):
            batch.run_iteration(batched, sweeps, stream=stream)
        for r in batched:
            r.merge_update()
        # eager device work between graph replays
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(plain, batched)):
            sa, sb = snapshot(a), snapshot(b)
            assert np.array_equal(sa[0], sb[0]), (it, k, "histogram")
            assert np.array_equal(sa[1], sb[1]), (it, k, "lnW")
            assert np.array_equal(sa[2], sb[2]) and np.array_equal(sa[3], sb[3]), (it, k, "chains")


def test_batched_equals_oracle():
    """The mixed batch, element by element against the oracle: each run's
    merged histogram, weights, thresholds, chain bins and spins after every
    iteration of one persistent launch per round (lanes per chain chosen per
    run, graph relaunches)."""
    import torch
    from oracle import oracle as orc
    from paper_1312_2213_amd import muca
    mid = {"ising": orc.ISING, "potts": orc.POTTS, "muma": orc.MUMA}
    stream = torch.cuda.Stream()
    batched = [make(s) for s in MIX]
    oracle = [orc.LatticeRun(mid[m], L, c, seed, q=q, beta=0.5 if m == "muma" else 0.0)
              for m, L, q, c, seed, _, _ in MIX]
    batch = muca.Batch(len(MIX), lanes_per_chain=0, use_graph=True)
    sweeps = [s[-1] for s in MIX]
    for it in range(3):
        print(f"  iteration {it}", flush=True)
        with torch.cuda.stream(stream):
            batch.run_iteration(batched, sweeps, stream=stream)
        for k, (g, o, sw) in enumerate(zip(batched, oracle, sweeps)):
            assert np.array_equal(g.thresholds(), o.thresholds()), (it, k, "thresholds")
            H, f, _ = o.iterate(sw)
            st = g.merge_update()
            assert np.array_equal(g.last_hist(), H), (it, k, "histogram")
            assert st["flatness"] == f, (it, k, "flatness")
            assert np.all(np.abs(g.lnw() - o.lnW) <= 1e-12 * np.maximum(1.0, np.abs(o.lnW))), (it, k, "lnW")
            s_, b_, _ = g.chain_state()
            assert np.array_equal(s_, o.spins) and np.array_equal(b_, o.bins()), (it, k, "chains")


def test_batched_subset_and_regrouping():
    """Runs can join and leave between rounds (the serving pattern)."""
    import torch
    from paper_1312_2213_amd import muca
    stream = torch.cuda.Stream()
    plain = [make(s) for s in MIX[:4]]
    batched = [make(s) for s in MIX[:4]]
    batch = muca.Batch(8, lanes_per_chain=4, use_graph=True)
    groups = [[0, 1], [0, 1, 2, 3], [2, 3], [1, 3]]
    for it, grp in enumerate(groups):
        for k in grp:
            plain[k].run_iteration(MIX[k][-1])
            plain[k].merge_update()
        with torch.cuda.stream(stream):
            batch.run_iteration([batched[k] for k in grp], [MIX[k][-1] for k in grp], stream=stream)
        for k in grp:
            batched[k].merge_update()
    for a, b in zip(plain, batched):
        sa, sb = snapshot(a), snapshot(b)
        assert all(np.array_equal(x, y) for x, y in zip(sa, sb))


def test_batched_long_launch_flushes_lds_counters():
    """A single batched launch of 3000 sweeps (64-chain work items flush
    their 16-bit LDS counters every 1023 sweeps) equals plain launches."""
    import torch
    from paper_1312_2213_amd import muca
    stream = torch.cuda.Stream()
    specs = [("ising", 8, 2, 128, 51, 1, 3000), ("potts", 8, 3, 64, 52, 2, 1500)]
    plain = [make(s) for s in specs]
    batched = [make(s) for s in specs]
    batch = muca.Batch(2, lanes_per_chain=4, use_graph=False)
    for r, s in zip(plain, specs):
        r.run_iteration(s[-1])
        r.merge_update()
    with torch.cuda.stream(stream):
        batch.run_iteration(batched, [s[-1] for s in specs], stream=stream)
    for r in batched:
        r.merge_update()
    for a, b in zip(plain, batched):
        sa, sb = snapshot(a), snapshot(b)
        assert all(np.array_equal(x, y) for x, y in zip(sa, sb))


def test_batch_rejects_polymer_and_duplicates():
    from paper_1312_2213_amd import muca
    from synth import polymer_walk
    p = muca.Run(muca.muca_config_default("polymer", 0, 2, 4, 1, n_beads=8), positions=polymer_walk(8, 4, 1))
    r = make(MIX[0])
    batch = muca.Batch(4, use_graph=False)
    with pytest.raises(muca.MucaError):
        batch.run_iteration([p], [1])
    with pytest.raises(muca.MucaError):
        batch.run_iteration([r, r], [1, 1])


def test_autotune_returns_valid_variant(tmp_path, monkeypatch):
    from paper_1312_2213_amd import muca
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("MUCA_AUTOTUNE_CACHE", str(cache))
    cfg = muca.muca_config_default("ising", 32, 2, 512, 3)
    best, ms = muca.muca_autotune(cfg, 10)
    assert ms > 0 and best.lanes_per_chain in (1, 2, 4, 16) and best.layout in (1, 2)
    assert cache.exists() and "gfx950" in cache.read_text()
    again, ms2 = muca.muca_autotune(cfg, 10)
    assert ms2 == -1.0 and (again.layout, again.lanes_per_chain, again.chains_per_block) == \
        (best.layout, best.lanes_per_chain, best.chains_per_block)
    # the tuned variant still reproduces the default variant's chains
    a = muca.Run(cfg)
    b = muca.Run(best)
    for r in (a, b):
        r.run_iteration(7)
        r.merge_update()
    assert np.array_equal(a.last_hist(), b.last_hist())
    assert np.array_equal(a.chain_state()[0], b.chain_state()[0])


def test_autotuned_batch_equals_plain_and_oracle(tmp_path, monkeypatch):
    """Lanes per chain, table placement and item order from measured item
    times (muca_batch_tune): the tuned batch still reproduces plain launches
    and the oracle; tuning leaves a run's results unchanged; a second run of
    the same class reads the cache."""
    import torch
    from oracle import oracle as orc
    from paper_1312_2213_amd import muca
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("MUCA_AUTOTUNE_CACHE", str(cache))
    mid = {"ising": orc.ISING, "potts": orc.POTTS, "muma": orc.MUMA}
    stream = torch.cuda.Stream()
    plain = [make(s) for s in MIX]
    tuned = [make(s) for s in MIX]
    oracle = [orc.LatticeRun(mid[m], L, c, seed, q=q, beta=0.5 if m == "muma" else 0.0)
              for m, L, q, c, seed, _, _ in MIX]
    batch = muca.Batch(len(MIX), lanes_per_chain=0, use_graph=True, autotune=True)
    sweeps = [s[-1] for s in MIX]
    for it in range(3):
        print(f"  iteration {it}", flush=True)
        for r, sw in zip(plain, sweeps):
            r.run_iteration(sw)
            r.merge_update()
        with torch.cuda.stream(stream):
            batch.run_iteration(tuned, sweeps, stream=stream)
        for k, (g, p, o, sw) in enumerate(zip(tuned, plain, oracle, sweeps)):
            H, _, _ = o.iterate(sw)
            g.merge_update()
            assert np.array_equal(g.last_hist(), H) and np.array_equal(p.last_hist(), H), (it, k)
            assert np.array_equal(g.lnw(), p.lnw()), (it, k)
            sg, bg = snapshot(g)[2:]
            assert np.array_equal(sg, o.spins) and np.array_equal(bg, o.bins()), (it, k)
    for r in tuned:
        t = r.batch_tuning
        assert t["rejected"] == 0 and not t["from_cache"], t
        assert t["lanes_per_chain"] in (4, 16)
        for lanes in ("4_lanes", "16_lanes"):
            assert t["us_per_sweep"][lanes]["global"] > 0, t
    assert "batch/" in cache.read_text()
    again = make(MIX[0])
    assert muca.batch_tune(again)["from_cache"]


def test_autotuned_round_no_slower_than_the_rule():
    """A round of a mixed batch shaped like the batched workload (Potts
    q = 8, L = 16 ... 48, plus multimagnetic L = 32) with the tuned choices
    takes no longer than with the untuned rule (5 % tolerance for timing
    noise; the minimum of four rounds each)."""
    import time
    import torch
    from paper_1312_2213_amd import muca
    specs = [("potts", 16, 8, 512, 61, 2, 20), ("potts", 32, 8, 512, 62, 2, 30),
             ("potts", 48, 8, 512, 63, 2, 40), ("muma", 32, 2, 256, 64, 2, 30)]
    stream = torch.cuda.Stream()
    ms = {}
    for mode in ("rule", "tuned"):
        runs = [make(s) for s in specs]
        batch = muca.Batch(len(runs), lanes_per_chain=0, use_graph=True, autotune=mode == "tuned")
        best = None
        for k in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with torch.cuda.stream(stream):
                batch.run_iteration(runs, [s[-1] for s in specs], stream=stream)
            stream.synchronize()
            dt = time.perf_counter() - t0
            for r in runs:
                r.merge_update()
            if k:
                best = dt if best is None else min(best, dt)
        ms[mode] = best * 1e3
    print(f"  round: rule {ms['rule']:.2f} ms, tuned {ms['tuned']:.2f} ms", flush=True)
    assert ms["tuned"] <= 1.05 * ms["rule"], ms
