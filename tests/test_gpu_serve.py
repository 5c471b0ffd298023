"""Continuous batching: requests arriving while others run are admitted by
footprint, share persistent launches, and each finishes with exactly the
result it gets alone, which is the oracle's result for the same run (the
method's iteration loop: sweeps, merged histogram, recursion, new weights;
parallel-scheme paragraph and Fig. 1 caption)."""
import numpy as np
import pytest

from oracle import oracle as orc

pytestmark = pytest.mark.gpu


def reqs():
    from paper_1312_2213_amd.serve import Request
    from paper_1312_2213_amd import muca
    spec = [("ising", 16, 2, 256), ("potts", 16, 4, 320), ("ising", 24, 2, 128),
            ("potts", 16, 8, 192), ("ising", 8, 2, 64), ("potts", 32, 2, 256)]
    out = [Request(id=k, arrival=0.002 * k, model=m, L=L, q=q, chains=c, seed=500 + k, max_iters=4)
           for k, (m, L, q, c) in enumerate(spec)]
    # a request given as a complete configuration (multimagnetic, beta = 0.5)
    cfg = muca.muca_config_default("muma", 16, 2, 192, 507, beta=0.5)
    out.append(Request(id=len(out), arrival=0.003, model="muma", L=16, q=2, chains=192, seed=507,
                       max_iters=4, sweeps_per_iter=40, cfg=cfg))
    return out


def oracle_run(req):
    """The request's run (model, L, q, chains, seed, beta) in the oracle."""
    model = {"ising": orc.ISING, "potts": orc.POTTS, "muma": orc.MUMA}[req.model]
    beta = req.cfg.beta if req.cfg is not None and req.model == "muma" else 0.0
    return orc.LatticeRun(model, req.L, req.chains, req.seed, q=req.q, beta=beta)


def test_each_result_same_alone_in_the_mix_and_in_the_oracle():
    from paper_1312_2213_amd.serve import Server, run_alone
    srv = Server(hbm_budget=256 << 20, round_site_updates=4096, keep_results=True)
    mixed = srv.serve(reqs(), realtime=True)
    assert srv.rounds > len(mixed)  # chunked: several rounds per iteration
    assert srv.peak_active >= 2     # work of several requests overlapped on the device
    assert srv.overlapped_merges > 0  # host merges ran while a round was on the device
    for r, req in zip(mixed, reqs()):
        print(f"  request {req.id}: {req.model} L={req.L} q={req.q} chains={req.chains}", flush=True)
        alone = run_alone(req)
        assert r.iterations == alone.iterations and r.flat == alone.flat
        assert np.array_equal(r.hist, alone.hist), req
        assert np.array_equal(r.lnw, alone.lnw), req
        o = oracle_run(req)
        flats = [o.iterate(req.sweeps_per_iter) for _ in range(r.iterations)]
        H = flats[-1][0]
        f = [x[1] for x in flats]
        # the request stopped at the oracle's first flat iteration (or its cap)
        assert all(x <= req.flat_threshold for x in f[:-1]), (req, f)
        assert (f[-1] > req.flat_threshold) == r.flat, (req, f)
        assert np.array_equal(r.hist, H), req
        assert np.all(np.abs(r.lnw - o.lnW) <= 1e-12 * np.maximum(1.0, np.abs(o.lnW))), req


def test_admission_respects_the_memory_budget():
    from paper_1312_2213_amd import muca
    from paper_1312_2213_amd.serve import Server
    rs = reqs()
    sizes = [muca.muca_workspace_bytes(r.config()) for r in rs]
    srv = Server(hbm_budget=max(sizes), round_site_updates=4096)
    out = srv.serve(rs, realtime=False)
    assert len(out) == len(rs) and all(r.iterations >= 1 for r in out)
    assert srv.peak_mem <= max(sizes)
    assert srv.peak_active < len(rs)  # the budget forced requests to wait for memory


def test_cancelling_a_request_leaves_the_others_unchanged():
    """A request withdrawn after a few rounds leaves at once; every other
    request still ends with exactly the result it gets alone."""
    from paper_1312_2213_amd.serve import Server, run_alone
    srv = Server(hbm_budget=256 << 20, round_site_updates=4096, keep_results=True)
    srv.on_round = lambda rounds, active: srv.cancel(2) if rounds == 3 else None
    rs = reqs()
    out = srv.serve(rs, realtime=False)
    assert out[2].cancelled and not out[2].flat
    for r, req in zip(out, rs):
        if req.id == 2:
            continue
        print(f"  request {req.id}", flush=True)
        alone = run_alone(req)
        assert not r.cancelled and r.iterations == alone.iterations
        assert np.array_equal(r.hist, alone.hist) and np.array_equal(r.lnw, alone.lnw), req
