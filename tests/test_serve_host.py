"""Host logic of the serving loop, on the CPU: the device calls (runs,
batched rounds, merges) are replaced by recording stand-ins, so that the
schedule itself can be checked: admission by footprint, chunked rounds,
which requests take part in which round, when merges overlap a round, and
withdrawal of a request."""
import contextlib

import pytest

torch = pytest.importorskip("torch")
from paper_1312_2213_amd import muca, serve  # noqa: E402


class FakeRun:
    """Stands in for muca.Run: becomes flat after a number of merged
    iterations fixed by its seed."""
    log = []

    def __init__(self, cfg, stream=None):
        self.cfg = cfg
        self.flat_after = 2 + cfg.seed % 100
        self.iteration = 0
        self.begun = False
        self.freed = False
        self.pending = 0

    def merge_begin(self):
        assert not self.begun and self.pending > 0
        self.begun = True

    def merge_finish(self):
        assert self.begun
        self.begun = False
        self.pending = 0
        self.iteration += 1
        flat = self.iteration >= self.flat_after
        return {"flatness": 0.9 if flat else 0.1, "flat": int(flat)}

    def free(self):
        self.freed = True

    def lnw(self):
        return None

    def last_hist(self):
        return None


class FakeBatch:
    def __init__(self, *a, **k):
        self.rounds = []

    def run_iteration(self, runs, sweeps, stream=None):
        for r, s in zip(runs, sweeps):
            assert not r.begun and not r.freed, "a run takes part in a round while being merged or after retiring"
            r.pending += s
        self.rounds.append([(r.cfg.seed, s) for r, s in zip(runs, sweeps)])


@pytest.fixture
def fakes(monkeypatch):
    monkeypatch.setattr(muca, "Run", FakeRun)
    monkeypatch.setattr(muca, "Batch", FakeBatch)
    monkeypatch.setattr(muca, "muca_workspace_bytes", lambda cfg: 1000 * cfg.L)
    monkeypatch.setattr(torch.cuda, "stream", lambda s: contextlib.nullcontext())
    monkeypatch.setattr(torch.cuda, "synchronize", lambda: None)


def request(k, L, sweeps):
    return serve.Request(id=k, arrival=0.0, model="ising", L=L, q=2, chains=64, seed=k, sweeps_per_iter=sweeps,
                         max_iters=50)


def participation(srv, seed):
    return [i for i, rnd in enumerate(srv.batch.rounds) if any(s == seed for s, _ in rnd)]


def test_short_iterations_never_skip_a_round_and_long_ones_skip_one(fakes):
    # L = 8: 64 sites, 4096 site updates per round = 64 sweeps per round;
    # request 40: 40-sweep iterations (one round each), 42 of them;
    # request 1: 640-sweep iterations (10 rounds each, overlapped merges), 3
    reqs = [request(40, 8, 40), request(1, 8, 640)]
    srv = serve.Server(hbm_budget=1 << 30, round_site_updates=4096, stream=object(), overlap_min_rounds=4)
    out = srv.serve(reqs, realtime=False)
    assert all(r.flat for r in out)
    assert {r.id: r.iterations for r in out} == {40: 42, 1: 3}
    p0 = participation(srv, 40)
    assert p0 == list(range(len(p0)))  # every round until it retired
    p1 = participation(srv, 1)
    # 10 rounds per iteration, then one round left out while its merge runs
    gaps = [b - a for a, b in zip(p1, p1[1:]) if b - a > 1]
    assert gaps == [2, 2]
    assert srv.overlapped_merges >= 2
    # the chunks cover each iteration exactly
    assert sum(s for rnd in srv.batch.rounds for seed, s in rnd if seed == 1) == 3 * 640


def test_without_overlap_no_request_skips_a_round(fakes):
    reqs = [request(40, 8, 40), request(1, 8, 640)]
    srv = serve.Server(hbm_budget=1 << 30, round_site_updates=4096, stream=object(), overlap_min_rounds=10 ** 6)
    srv.serve(reqs, realtime=False)
    for seed in (40, 1):
        p = participation(srv, seed)
        assert p == list(range(p[0], p[0] + len(p)))
    assert srv.overlapped_merges == 0


def test_admission_by_footprint_and_withdrawal(fakes):
    # footprints 8000 and 16000 bytes; a budget of 20000 admits one of each at most
    reqs = [request(k, 8 if k % 2 else 16, 64) for k in range(6)]
    srv = serve.Server(hbm_budget=20000, round_site_updates=4096, stream=object(), keep_results=True)
    srv.on_round = lambda rounds, active: srv.cancel(4) if rounds == 1 else None
    out = srv.serve(reqs, realtime=False)
    assert srv.peak_mem <= 20000
    assert out[4].cancelled and not out[4].flat and out[4].admitted is None
    assert all(r.flat and not r.cancelled for k, r in enumerate(out) if k != 4)
    assert not participation(srv, 4)
