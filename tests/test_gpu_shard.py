"""Shard-sum invariance, the one-device stand-in for a run split over
several devices: a run of C chains split into two runs over consecutive
chain ranges (chain0 = 0 and k), whose pending histograms are summed on the
host and merged into both with muca_merge_update_hist, must equal the
unsplit run bit for bit: histograms, weights, thresholds and every chain."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def cfg_of(model, L, q, chains, seed, chain0=0, **kw):
    from paper_1312_2213_amd import muca
    return muca.muca_config_default(model, L, q, chains, seed, chain0=chain0, **kw)


@pytest.mark.parametrize("model,L,q,kw", [("ising", 16, 2, {"layout": 1}), ("ising", 8, 2, {"layout": 2}),
                                          ("potts", 16, 5, {}), ("muma", 16, 2, {"beta": 0.5})])
def test_two_shards_equal_the_unsplit_run(model, L, q, kw):
    from paper_1312_2213_amd import muca
    C, k, seed, sweeps = 130, 50, 77, 15
    print(f"{model} L={L}", flush=True)
    full = muca.Run(cfg_of(model, L, q, C, seed, **kw))
    a = muca.Run(cfg_of(model, L, q, k, seed, 0, **kw))
    b = muca.Run(cfg_of(model, L, q, C - k, seed, k, **kw))
    for it in range(3):
        full.run_iteration(sweeps)
        st = full.merge_update()
        for r in (a, b):
            r.run_iteration(sweeps)
        h = a.pending_hist() + b.pending_hist()
        sa, sb = a.merge_update_hist(h), b.merge_update_hist(h)
        assert np.array_equal(h, full.last_hist()), it
        assert np.array_equal(a.last_hist(), h) and np.array_equal(b.last_hist(), h)
        assert sa["flatness"] == st["flatness"] == sb["flatness"]
        assert np.array_equal(a.lnw(), full.lnw()) and np.array_equal(b.lnw(), full.lnw())
        assert np.array_equal(a.thresholds(), full.thresholds())
    fs, fb, _ = full.chain_state()
    as_, ab, _ = a.chain_state()
    bs, bb, _ = b.chain_state()
    assert np.array_equal(fs[:k], as_) and np.array_equal(fs[k:], bs)
    assert np.array_equal(fb[:k], ab) and np.array_equal(fb[k:], bb)


def test_polymer_shards_equal_the_unsplit_run():
    from paper_1312_2213_amd import muca
    from synth import polymer_walk
    C, k, N, seed = 96, 40, 16, 5
    pos = polymer_walk(N, C, seed)
    full = muca.Run(cfg_of("polymer", 0, 2, C, seed, n_beads=N), positions=pos)
    a = muca.Run(cfg_of("polymer", 0, 2, k, seed, 0, n_beads=N), positions=pos[:k])
    b = muca.Run(cfg_of("polymer", 0, 2, C - k, seed, k, n_beads=N), positions=pos[k:])
    for it in range(2):
        full.run_iteration(20)
        full.merge_update()
        for r in (a, b):
            r.run_iteration(20)
        h = a.pending_hist() + b.pending_hist()
        a.merge_update_hist(h)
        b.merge_update_hist(h)
        assert np.array_equal(h, full.last_hist()), it
        assert np.array_equal(a.lnw(), full.lnw())
    fp, fbins, fe = full.chain_state()
    ap, abins, ae = a.chain_state()
    bp, bbins, be = b.chain_state()
    assert np.array_equal(fp[:k], ap) and np.array_equal(fp[k:], bp)
    assert np.array_equal(fbins[:k], abins) and np.array_equal(fbins[k:], bbins)


def test_pending_hist_and_merged_hist_argument_checks():
    from paper_1312_2213_amd import muca
    r = muca.Run(cfg_of("ising", 8, 2, 64, 3))
    with pytest.raises(muca.MucaError):
        r.pending_hist()  # no sweeps since the last merge
    r.run_iteration(2)
    h = r.pending_hist()
    assert h.sum() == 64 * 2
    with pytest.raises(muca.MucaError):
        r.merge_update_hist(h[:-1])  # wrong length
    st = r.merge_update_hist(h)
    assert st["samples"] == 128
    with pytest.raises(muca.MucaError):
        muca.Run(cfg_of("ising", 8, 2, 64, 3, chain0=-1))
