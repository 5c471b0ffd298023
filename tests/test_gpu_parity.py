"""GPU (HIP, gfx950) against the oracle on identical seeded inputs: bit-exact
histograms, spins and bins; weights and reweighted observables within 1e-12
relative (in practice identical: both sides run the same FP64 definition in
the same order with glibc libm)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_common import assert_same_state, pair  # noqa: E402

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def close(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.all(np.abs(a - b) <= RTOL * np.maximum(1.0, np.abs(b)))


def iterate_both(o, g, sweeps, iters):
    for it in range(iters):
        print(f"  iteration {it}", flush=True)
        assert np.array_equal(g.thresholds(), o.thresholds()), "thresholds differ"
        H, f, lnw_used = o.iterate(sweeps)
        g.run_iteration(sweeps)
        st = g.merge_update()
        assert np.array_equal(g.last_hist(), H), f"histogram differs in iteration {it}"
        assert abs(st["flatness"] - f) <= 1e-15
        assert close(g.lnw(), o.lnW), "lnW differs"
    return H, lnw_used


def test_init_matches():
    for model, L, q in (("ising", 8, 2), ("potts", 16, 5), ("muma", 16, 2)):
        o, g = pair(model, L, 100, seed=77, q=q)
        assert_same_state(o, g)


@pytest.mark.parametrize("layout", [1, 2])
@pytest.mark.parametrize("L", [4, 8, 16, 24])
def test_ising_iterations(L, layout):
    print(f"ising L={L} layout={layout}", flush=True)
    o, g = pair("ising", L, 130, seed=100 + L, layout=layout)
    iterate_both(o, g, 20, 3)
    assert_same_state(o, g)


@pytest.mark.parametrize("L", [32, 48, 64])
def test_ising_large_L_short(L):
    print(f"ising L={L}", flush=True)
    o, g = pair("ising", L, 70, seed=5 + L)
    iterate_both(o, g, 3, 2)
    assert_same_state(o, g)


@pytest.mark.parametrize("q,L", [(2, 8), (3, 8), (8, 16), (10, 24), (4, 32)])
def test_potts_iterations(q, L):
    print(f"potts q={q} L={L}", flush=True)
    o, g = pair("potts", L, 90, seed=200 + q, q=q)
    iterate_both(o, g, 10, 3)
    assert_same_state(o, g)


@pytest.mark.parametrize("layout", [1, 2])
@pytest.mark.parametrize("L", [8, 32])
def test_muma_iterations(L, layout):
    print(f"muma L={L} layout={layout}", flush=True)
    o, g = pair("muma", L, 100, seed=300 + L, beta=0.5, layout=layout)
    iterate_both(o, g, 10, 3)
    assert_same_state(o, g)


def test_config1_full_run():
    """Ising L=8, 16 chains, seed 1, E in [-128, 128] step 4, 12 iterations of
    2000 sweeps then the final update; reweighted u, c at three betas."""
    o, g = pair("ising", 8, 16, seed=1, lo=-128, hi=128)
    H, lnw_used = iterate_both(o, g, 2000, 12)
    betas = [0.3, 0.44, 0.6]
    assert close(g.reweight(betas), o.reweight(H, lnw_used, betas))
    assert_same_state(o, g)


def test_restricted_range_rejects_leaving_moves():
    o, g = pair("ising", 8, 64, seed=9, lo=-64, hi=48)
    iterate_both(o, g, 50, 3)
    assert_same_state(o, g)


def test_single_chain_and_ragged_tail():
    for chains in (1, 63, 65):
        o, g = pair("potts", 8, chains, seed=chains, q=3)
        iterate_both(o, g, 15, 2)
        assert_same_state(o, g)


@pytest.mark.parametrize("model,layout,q", [("ising", 1, 2), ("ising", 2, 2), ("muma", 1, 2), ("potts", 2, 6)])
def test_invariant_to_launch_shape_lanes_and_table_placement(model, layout, q):
    """Every compiled variant (lanes per chain, threads per block, threshold
    table in LDS or global memory) gives the identical Markov chains."""
    o, _ = pair(model, 16, 128, seed=4, q=q, layout=layout)
    H = o.sweeps(25)
    for lpc in (1, 2, 4, 16):
        for threads in (64, 256, 512):
            for tlds in ((0, 1) if threads <= 256 else (1,)):
                cpb = max(1, threads // lpc)
                _, g = pair(model, 16, 128, seed=4, q=q, layout=layout, cpb=cpb, tlds=tlds, lpc=lpc)
                g.run_iteration(25)
                g.merge_update()
                s, b, _ = g.chain_state()
                assert np.array_equal(g.last_hist(), H), (lpc, threads, tlds)
                assert np.array_equal(s, o.spins) and np.array_equal(b, o.bins()), (lpc, threads, tlds)


@pytest.mark.parametrize("model,layout", [("ising", 1), ("ising", 2), ("muma", 1)])
@pytest.mark.parametrize("L", [48, 64])
def test_two_word_rows_lane_splits_and_table_placement(model, L, layout):
    """Rows of two 32-site words, where a lane of 4 per chain owns several
    Philox calls of a row: identical chains for 4 and 16 lanes per chain,
    threshold table in LDS (where it fits) and in global memory."""
    print(f"{model} L={L} layout={layout}", flush=True)
    o, _ = pair(model, L, 96, seed=60 + L, layout=layout)
    H = o.sweeps(4)
    fits = not (model == "muma" and L == 64)
    for lpc in (4, 16):
        for tlds in ((0, 1) if fits else (0,)):
            _, g = pair(model, L, 96, seed=60 + L, layout=layout, tlds=tlds, lpc=lpc)
            g.run_iteration(4)
            g.merge_update()
            s, b, _ = g.chain_state()
            assert np.array_equal(g.last_hist(), H), (lpc, tlds)
            assert np.array_equal(s, o.spins) and np.array_equal(b, o.bins()), (lpc, tlds)


def test_iterations_on_alternating_streams():
    """The threshold table goes to the device asynchronously after each
    merge, on the run's stream; an iteration launched on another stream (or
    batched on one) waits for it first.  Alternating three streams and the
    batched launch must reproduce the oracle exactly."""
    import torch
    from paper_1312_2213_amd import muca
    o, g = pair("potts", 16, 300, seed=91, q=6)
    streams = [torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.current_stream()]
    batch = muca.Batch(max_runs=1)
    for it in range(9):
        H, _, _ = o.iterate(40)
        s = streams[it % 3]
        if it % 4 == 3:
            batch.run_iteration([g], [40], stream=s)
        else:
            g.run_iteration(40, stream=s)
        g.merge_update()
        assert np.array_equal(g.last_hist(), H), it
        assert close(g.lnw(), o.lnW), it
        assert np.array_equal(g.thresholds(), o.thresholds()), it
    assert_same_state(o, g)


def test_chunked_iteration_equals_one_piece():
    _, a = pair("ising", 16, 64, seed=8)
    _, b = pair("ising", 16, 64, seed=8)
    a.run_iteration(30)
    a.merge_update()
    b.run_iteration(10)
    b.run_iteration(20)
    b.merge_update()
    assert np.array_equal(a.last_hist(), b.last_hist())
    assert np.array_equal(a.lnw(), b.lnw())


def test_checkpoint_restore_is_exact():
    _, a = pair("potts", 16, 128, seed=12, q=4)
    _, b = pair("potts", 16, 128, seed=12, q=4)
    for _ in range(2):
        a.run_iteration(10)
        a.merge_update()
    blob = a.checkpoint()
    for _ in range(2):
        a.run_iteration(10)
        a.merge_update()
    b.restore(blob)
    for _ in range(2):
        b.run_iteration(10)
        b.merge_update()
    assert np.array_equal(a.last_hist(), b.last_hist())
    assert np.array_equal(a.lnw(), b.lnw())
    assert np.array_equal(a.chain_state()[0], b.chain_state()[0])


def test_ising64_full_size_sampled():
    """The bench workload's shape: L=64 bit-packed, 4096 chains.  Merged
    histogram over all chains and sampled chains' spins after 2 sweeps."""
    from oracle import oracle as orc
    o, g = pair("ising", 64, 4096, seed=2, layout=1)
    g.run_iteration(2)
    g.merge_update()
    H = o.sweeps(2)
    assert np.array_equal(g.last_hist(), H)
    s, b, _ = g.chain_state()
    for c in (0, 1, 63, 64, 1000, 4095):
        assert np.array_equal(s[c], o.spins[c]) and b[c] == o.bins()[c]


@pytest.mark.parametrize("tlds", [0, 1])
def test_potts48_full_size_table_placement(tlds):
    """q=8, L=48, 2048 chains: the 9-column threshold table (162 KiB) read
    from global memory, or its 8 non-trivial columns (144 KiB) staged in LDS."""
    o, g = pair("potts", 48, 2048, seed=33, q=8, tlds=tlds)
    g.run_iteration(2)
    g.merge_update()
    assert np.array_equal(g.last_hist(), o.sweeps(2))
    assert_same_state(o, g, chains=(0, 777, 2047))


@pytest.mark.parametrize("cpb", [256, 512])
@pytest.mark.parametrize("model,q", [("ising", 2), ("potts", 3)])
def test_lds_counters_flushed_before_16_bit_overflow(model, q, cpb):
    """256 or 512 chains per block, 2000 sweeps in one launch: with W = 1
    every Ising flip is accepted, a sweep maps s -> -s and each chain keeps
    its energy, so one bin collects far more than 2^16 counts per block.
    The packed 16-bit LDS counters must be flushed in time (every
    65535 / cpb sweeps)."""
    print(f"{model} flush cpb={cpb}", flush=True)
    o, g = pair(model, 4, cpb, seed=21, q=q, lpc=1, cpb=cpb, tlds=1)
    assert g.blocks_shape()[1] == cpb
    H, _ = iterate_both(o, g, 2000, 2)
    assert_same_state(o, g)
    if model == "ising":
        o2, g2 = pair(model, 4, cpb, seed=21, lpc=1, cpb=cpb, tlds=1)
        g2.run_iteration(2000)
        g2.merge_update()
        assert g2.last_hist().max() > 65535


def test_potts_maximum_q():
    """q = 255: colours up to 254 (high bit set) take the general byte test."""
    o, g = pair("potts", 8, 70, seed=255, q=255)
    iterate_both(o, g, 6, 3)
    assert_same_state(o, g)
    assert o.spins.max() >= 128


@pytest.mark.parametrize("model,L,q", [("ising", 4, 2), ("potts", 4, 3), ("muma", 4, 2), ("potts", 64, 4)])
def test_smallest_and_largest_lattices(model, L, q):
    print(f"{model} L={L} q={q}", flush=True)
    o, g = pair(model, L, 97, seed=40 + L, q=q, beta=0.5)
    iterate_both(o, g, 8 if L < 64 else 2, 2)
    assert_same_state(o, g)


def test_many_chains_sampled():
    """65536 chains (the whole chip at 1 lane per chain): merged histogram and
    sampled chains after 2 sweeps."""
    o, g = pair("ising", 16, 65536, seed=6, layout=1)
    g.run_iteration(2)
    g.merge_update()
    assert np.array_equal(g.last_hist(), o.sweeps(2))
    s, b, _ = g.chain_state()
    for c in (0, 1, 4095, 4096, 65535):
        assert np.array_equal(s[c], o.spins[c]) and b[c] == o.bins()[c]


def test_argument_errors_leave_the_run_usable():
    from paper_1312_2213_amd import muca
    _, g = pair("ising", 8, 64, seed=3)
    for bad in (0, -5):
        with pytest.raises(muca.MucaError):
            g.run_iteration(bad)
    with pytest.raises(muca.MucaError):
        g.merge_update()  # nothing to merge yet
    with pytest.raises(muca.MucaError):
        g.set_lnw(np.zeros(3))  # wrong length
    g.run_iteration(3)
    assert g.merge_update()["samples"] == 64 * 3
