"""The batched iteration that allocates nothing
(muca_batch_run_iteration_noalloc, work queue in the library's own device
array) against the batched iteration with a caller's workspace
(muca_batch_run_iteration): identical histograms, weights, thresholds and
chains on two calls in a row, the second with fewer runs, fewer sweeps and
so fewer work items; sizes beyond the stated maximum are refused with the
runs unchanged."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MIX = [  # (model, L, q, chains, seed, layout, sweeps)
    ("ising", 16, 2, 130, 81, 1, 12),
    ("ising", 64, 2, 256, 82, 1, 3),
    ("muma", 32, 2, 100, 83, 2, 5),
    ("potts", 16, 8, 70, 84, 2, 9),
    ("potts", 48, 3, 64, 85, 2, 2),
    ("ising", 24, 2, 64, 86, 2, 7),
]


def make(spec):
    from paper_1312_2213_amd import muca
    model, L, q, chains, seed, layout, _ = spec
    kw = dict(layout=layout)
    if model == "muma":
        kw["beta"] = 0.5
    return muca.Run(muca.muca_config_default(model, L, q, chains, seed, **kw))


def same(a, b):
    sa, ba, _ = a.chain_state()
    sb, bb, _ = b.chain_state()
    return (np.array_equal(a.last_hist(), b.last_hist()) and np.array_equal(a.lnw(), b.lnw())
            and np.array_equal(a.thresholds(), b.thresholds())
            and np.array_equal(sa, sb) and np.array_equal(ba, bb))


@pytest.mark.parametrize("lpc", [0, 4, 16])
def test_noalloc_equals_the_workspace_batch(lpc):
    import torch
    from paper_1312_2213_amd import muca
    print(f"no-alloc batched iteration, lanes per chain {lpc}", flush=True)
    stream = torch.cuda.Stream()
    ref = [make(s) for s in MIX]
    new = [make(s) for s in MIX]
    batch = muca.Batch(len(MIX), lanes_per_chain=lpc, use_graph=False)
    calls = [(list(range(len(MIX))), [s[-1] for s in MIX]),  # every run
             ([0, 3, 5], [4, 3, 2])]                            # fewer runs, sweeps and items
    for n, (idx, sw) in enumerate(calls):
        print(f"  call {n}: runs {idx}", flush=True)
        with torch.cuda.stream(stream):
            batch.run_iteration([ref[k] for k in idx], sw, stream=stream)
            muca.batch_run_iteration_noalloc([new[k] for k in idx], sw, lanes_per_chain=lpc, stream=stream)
        for k in idx:
            ref[k].merge_update()
            new[k].merge_update()
            assert same(ref[k], new[k]), (n, k)


def test_noalloc_refuses_sizes_beyond_its_maximum():
    from paper_1312_2213_amd import muca
    print("no-alloc limits", flush=True)
    many = [make(("ising", 8, 2, 64, 900 + k, 1, 1)) for k in range(muca.NOALLOC_MAX_RUNS + 1)]
    with pytest.raises(muca.MucaError, match="maximum"):
        muca.batch_run_iteration_noalloc(many, 1)
    # 16 chains per item at 16 lanes per chain: 4100 items > 4096
    big = make(("ising", 8, 2, 16 * (muca.NOALLOC_MAX_ITEMS + 4), 950, 1, 1))
    before = big.chain_state()[0].copy()
    with pytest.raises(muca.MucaError, match="capacity"):
        muca.batch_run_iteration_noalloc([big], 1, lanes_per_chain=16)
    assert np.array_equal(big.chain_state()[0], before)
    # the refused calls left the runs usable
    muca.batch_run_iteration_noalloc(many[:muca.NOALLOC_MAX_RUNS], 1)
    for r in many[:3]:
        assert r.merge_update()["samples"] == 64
