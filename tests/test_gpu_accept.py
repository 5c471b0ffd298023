"""Acceptance rate of an iteration (accepted / attempted moves over the
recorded sweeps) against the oracle's count of accepted moves: every lattice
path (lanes per chain 1, 2, 4, 16; bit and byte rows; Ising, MUMA, Potts),
the 16-bit counter flushes of long launches, thermalisation sweeps (not
counted), batched launches, and the polymer with both move sets."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_common import pair  # noqa: E402

pytestmark = pytest.mark.gpu


def rate(o, sweeps, per_sweep):
    return o.take_accepted() / (sweeps * o.n_chains * per_sweep)


@pytest.mark.parametrize("model,L,q,layout,lpc", [("ising", 16, 2, 1, 16), ("ising", 16, 2, 2, 4),
                                                 ("ising", 24, 2, 1, 1), ("muma", 16, 2, 1, 16),
                                                 ("muma", 32, 2, 2, 2), ("potts", 16, 5, 0, 16),
                                                 ("potts", 24, 8, 0, 4), ("potts", 16, 3, 0, 2)])
def test_lattice_accept_rate(model, L, q, layout, lpc):
    print(f"{model} L={L} q={q} layout={layout} lpc={lpc}", flush=True)
    o, g = pair(model, L, 100, seed=90 + L + q, q=q, layout=layout, lpc=lpc)
    for it in range(2):
        o.sweeps(3, record=False)  # thermalisation: not counted
        o.advance(3)
        g.thermalize(3)
        H, _, _ = o.iterate(7)
        g.run_iteration(7)
        st = g.merge_update()
        assert np.array_equal(g.last_hist(), H), it
        assert st["accept_rate"] == rate(o, 7, L * L), it
        assert 0.0 < st["accept_rate"] <= 1.0


def test_long_launch_flushes_the_counter():
    """256 chains per block flush their counters every 255 sweeps."""
    o, g = pair("ising", 8, 256, seed=3, lpc=1, cpb=256)
    H, _, _ = o.iterate(700)
    g.run_iteration(700)
    st = g.merge_update()
    assert np.array_equal(g.last_hist(), H)
    assert st["accept_rate"] == rate(o, 700, 64)


def test_batched_runs_report_their_own_rates():
    import torch
    from paper_1312_2213_amd import muca
    specs = [("ising", 16, 2), ("potts", 16, 8), ("muma", 16, 2)]
    pairs = [pair(m, L, 96, seed=40 + k, q=q) for k, (m, L, q) in enumerate(specs)]
    batch = muca.Batch(len(pairs), max_items=1 << 10)
    stream = torch.cuda.Stream()
    for it in range(2):
        with torch.cuda.stream(stream):
            batch.run_iteration([g for _, g in pairs], [5, 9, 7], stream=stream)
        for (o, g), S in zip(pairs, [5, 9, 7]):
            H, _, _ = o.iterate(S)
            st = g.merge_update()
            assert np.array_equal(g.last_hist(), H)
            assert st["accept_rate"] == rate(o, S, g.n_sites), (it, g.cfg.model)
    batch.free()


@pytest.mark.parametrize("moves", [0, 1])
def test_polymer_accept_rate(moves):
    from test_gpu_polymer import pair_paper
    o, g = pair_paper(40, 65, 17, lnw_slope=-1.0, moves=moves)
    per = 40 if moves == 0 else 81
    for it in range(2):
        H = o.sweeps(6)
        o.advance(6)
        o.merge_update(H)
        g.run_iteration(6)
        st = g.merge_update()
        assert np.array_equal(g.last_hist(), H)
        assert st["accept_rate"] == rate(o, 6, per), it


def test_iteration_log(tmp_path, monkeypatch):
    """MUCA_ITER_LOG: one JSON line per merged iteration with the merge's
    statistics (flatness, visited range, acceptance) and its timing."""
    import json
    log = tmp_path / "iters.jsonl"
    monkeypatch.setenv("MUCA_ITER_LOG", str(log))
    _, g = pair("potts", 8, 64, seed=5, q=3)
    stats = []
    for _ in range(3):
        g.run_iteration(7)
        stats.append(g.merge_update())
    rows = [json.loads(l) for l in log.read_text().splitlines()]
    assert len(rows) == 3 and len({r["run"] for r in rows}) == 1
    for row, st in zip(rows, stats):
        assert row["model"] == "potts" and row["L"] == 8 and row["q"] == 3 and row["chains"] == 64
        for k in ("iteration", "sweeps", "samples", "flat", "lo_visited", "hi_visited"):
            assert row[k] == st[k], k
        assert row["flatness"] == st["flatness"] and row["accept_rate"] == st["accept_rate"]
        assert row["seconds"] > 0 and row["attempts_per_s"] > 0
