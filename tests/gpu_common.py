"""Helpers shared by the GPU parity tests: one oracle run and one HIP run of
the same configuration (same seed, range and chains)."""
import numpy as np

from oracle import oracle as orc

MODEL_ID = {"ising": orc.ISING, "potts": orc.POTTS, "muma": orc.MUMA}


def pair(model, L, chains, seed, q=2, lo=None, hi=None, beta=0.5, layout=0, cpb=0, tlds=-1, lpc=0):
    import torch  # noqa: F401
    from paper_1312_2213_amd import muca
    o = orc.LatticeRun(MODEL_ID[model], L, chains, seed, q=q, lo=lo, hi=hi,
                       beta=beta if model == "muma" else 0.0)
    kw = dict(layout=layout, chains_per_block=cpb, table_in_lds=tlds, lanes_per_chain=lpc)
    if lo is not None:
        kw["lo"] = lo
    if hi is not None:
        kw["hi"] = hi
    if model == "muma":
        kw["beta"] = beta
    cfg = muca.muca_config_default(model, L, q, chains, seed, **kw)
    g = muca.Run(cfg)
    return o, g


def gpu_spins(g, chain0=0, count=None):
    s, b, _ = g.chain_state(chain0, count)
    return s, b


def assert_same_state(o, g, chains=None):
    s, b = gpu_spins(g)
    ob = o.bins()
    if chains is None:
        assert np.array_equal(s, o.spins), "spins differ"
        assert np.array_equal(b, ob), "bins differ"
    else:
        for c in chains:
            assert np.array_equal(s[c], o.spins[c]), f"chain {c} spins differ"
            assert b[c] == ob[c], f"chain {c} bin differs"
