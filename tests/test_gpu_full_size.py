"""Full-size parity at weights that reject moves.

The headline shapes (Ising L = 64 and 48 with 4096 chains, multimagnetic
L = 32 and 48 with 4096 chains, 8-state Potts L = 48 with 2048 chains) run a
few sweeps with the same non-flat weight table on the GPU and in the oracle:
a canonical slope plus a bin-to-bin ripple, so that every bin has its own
thresholds and a wrong threshold row or column offset changes the chains.
Every compiled variant of the shape (storage layout, 4 or 16 lanes per
chain, table staged in LDS or read from global memory) must give the
oracle's merged histogram, every chain's bin and spins, and the oracle's
accepted-move count, bit for bit.  Metropolis with min(1, W'/W) (Eq. 1;
Eq. 3 for the multimagnetic runs)."""
import numpy as np
import pytest

from oracle import oracle as orc

pytestmark = pytest.mark.gpu

SWEEPS = 3


def weights(model, L, lo, hi):
    """A canonical weight -beta E with a ripple of 0.3 between bins."""
    v = orc.bin_values({"ising": orc.ISING, "potts": orc.POTTS, "muma": orc.MUMA}[model], L, lo, hi)
    b = np.arange(len(v), dtype=np.float64)
    if model == "ising":
        return -0.4 * v + 0.3 * np.sin(0.7 * b)
    if model == "potts":
        return -1.0 * v + 0.3 * np.sin(0.9 * b)
    # multimagnetic: a weight in M that pulls towards |M| = N / 2 (the
    # energy factor exp(-beta E) comes with the model)
    N = L * L
    return -2e-3 * (np.abs(v) - N / 2) ** 2 / 8 + 0.3 * np.sin(0.7 * b)


_ORACLE = {}


def oracle_result(model, L, q, chains, seed):
    key = (model, L, q, chains, seed)
    if key not in _ORACLE:
        mid = {"ising": orc.ISING, "potts": orc.POTTS, "muma": orc.MUMA}[model]
        o = orc.LatticeRun(mid, L, chains, seed, q=q, beta=0.5 if model == "muma" else 0.0)
        lnw = weights(model, L, o.lo, o.hi)
        T = o.thresholds(lnw)
        H = o.sweeps(SWEEPS, T)
        acc = o.take_accepted()
        _ORACLE[key] = (lnw, T, H, acc, o.spins.copy(), o.bins().copy())
    return _ORACLE[key]


def run_variant(model, L, q, chains, seed, layout, lpc, tlds, threads=0):
    from paper_1312_2213_amd import muca
    kw = dict(layout=layout, lanes_per_chain=lpc, table_in_lds=tlds, chains_per_block=threads // lpc)
    if model == "muma":
        kw["beta"] = 0.5
    g = muca.Run(muca.muca_config_default(model, L, q, chains, seed, **kw))
    if threads:
        assert g.blocks_shape()[1] * lpc == threads
    lnw, T, H, acc, spins, bins = oracle_result(model, L, q, chains, seed)
    g.set_lnw(lnw)
    assert np.array_equal(g.thresholds(), T), "threshold tables differ"
    g.run_iteration(SWEEPS)
    st = g.merge_update()
    attempts = SWEEPS * chains * L * L
    assert np.array_equal(g.last_hist(), H), "merged histogram differs"
    assert st["accept_rate"] == acc / attempts, (st["accept_rate"], acc / attempts)
    assert 0.05 < st["accept_rate"] < 0.95, st["accept_rate"]
    s, b, _ = g.chain_state()
    assert np.array_equal(b, bins), "chain bins differ"
    bad = np.flatnonzero((s != spins).any(axis=1))
    assert bad.size == 0, f"{bad.size} chains' spins differ, first {bad[:5]}"
    g.free()


@pytest.mark.parametrize("tlds", [1, 0])
@pytest.mark.parametrize("lpc", [16, 4])
@pytest.mark.parametrize("layout", [1, 2])
@pytest.mark.parametrize("L", [64, 48])
def test_ising_full_size_rejecting_weights(L, layout, lpc, tlds):
    print(f"ising L={L} chains=4096 layout={layout} lpc={lpc} tlds={tlds}", flush=True)
    run_variant("ising", L, 2, 4096, 2, layout, lpc, tlds)


@pytest.mark.parametrize("tlds", [1, 0])
@pytest.mark.parametrize("lpc", [16, 4])
@pytest.mark.parametrize("layout", [1, 2])
@pytest.mark.parametrize("L", [32, 48])
def test_muma_full_size_rejecting_weights(L, layout, lpc, tlds):
    print(f"muma L={L} chains=4096 layout={layout} lpc={lpc} tlds={tlds}", flush=True)
    run_variant("muma", L, 2, 4096, 34, layout, lpc, tlds)


@pytest.mark.parametrize("tlds", [1, 0])
@pytest.mark.parametrize("lpc", [16, 4])
def test_potts8_L48_full_size_rejecting_weights(lpc, tlds):
    print(f"potts q=8 L=48 chains=2048 lpc={lpc} tlds={tlds}", flush=True)
    run_variant("potts", 48, 8, 2048, 33, 0, lpc, tlds)


@pytest.mark.parametrize("lpc", [16, 4, 2, 1])
def test_ising64_512_thread_blocks_rejecting_weights(lpc):
    """Blocks of 512 threads beside the staged table (two wavefronts per
    SIMD) at 8192 chains: the oracle's chains, bit for bit."""
    print(f"ising L=64 chains=8192 lpc={lpc} threads=512", flush=True)
    run_variant("ising", 64, 2, 8192, 5, 1, lpc, 1, threads=512)


@pytest.mark.parametrize("lpc", [4, 1])
def test_muma48_512_thread_blocks_rejecting_weights(lpc):
    print(f"muma L=48 chains=4096 lpc={lpc} threads=512", flush=True)
    run_variant("muma", 48, 2, 4096, 34, 1, lpc, 1, threads=512)


def test_potts8_L48_512_thread_blocks_rejecting_weights():
    print("potts q=8 L=48 chains=4096 lpc=16 threads=512", flush=True)
    run_variant("potts", 48, 8, 4096, 35, 0, 16, 1, threads=512)


def test_default_block_shape_with_many_chains():
    """32768 chains of Ising L = 64 at 4 lanes per chain: by default the
    library takes blocks of 512 threads (the staged table leaves room for
    one block per CU, and the launch has one for every CU), and its chains
    are those of 256-thread blocks at the same weights."""
    from paper_1312_2213_amd import muca
    C, L = 32768, 64
    out = []
    for cpb in (0, 64):
        g = muca.Run(muca.muca_config_default("ising", L, 2, C, 7, layout=1, lanes_per_chain=4,
                                              chains_per_block=cpb))
        out.append(g.blocks_shape()[1] * 4)
        g.set_lnw(weights("ising", L, g.cfg.lo, g.cfg.hi))
        g.run_iteration(SWEEPS)
        st = g.merge_update()
        s, b, _ = g.chain_state(0, 4096)
        out.append((g.last_hist(), st["accept_rate"], s, b))
        g.free()
    assert out[0] == 512 and out[2] == 256
    (h0, a0, s0, b0), (h1, a1, s1, b1) = out[1], out[3]
    assert np.array_equal(h0, h1) and a0 == a1 and 0.05 < a0 < 0.95
    assert np.array_equal(s0, s1) and np.array_equal(b0, b1)
