"""Joint (E, M) histogram of multimagnetic runs on the GPU against the
oracle: bit-exact counts for every lane split, layout and table placement,
and the reweighting to other inverse temperatures within 1e-12."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_common import assert_same_state, pair  # noqa: E402

pytestmark = pytest.mark.gpu


def em_host(em, shape):
    return em.cpu().numpy().view(np.uint64).reshape(shape)


@pytest.mark.parametrize("L,layout,lpc,tlds", [(8, 1, 0, -1), (16, 1, 16, -1), (16, 2, 4, 0), (16, 1, 1, 1),
                                               (24, 2, 2, -1), (32, 1, 16, -1), (48, 1, 4, -1), (64, 1, 16, 0)])
def test_joint_histogram_and_reweighting_equal_the_oracle(L, layout, lpc, tlds):
    import torch
    print(f"muma L={L} layout={layout} lpc={lpc} tlds={tlds}", flush=True)
    chains, sweeps = 96, 6
    o, g = pair("muma", L, chains, seed=70 + L, beta=0.44, layout=layout, lpc=lpc, tlds=tlds)
    shape = g.em_shape()
    assert shape == o.em_shape
    em = torch.zeros(shape[0] * shape[1], dtype=torch.int64, device="cuda")
    HEM = np.zeros(shape, np.uint64)
    for it in range(3):
        if it == 2:  # the last iteration alone, for the reweighting
            em.zero_()
            HEM[:] = 0
        lnw_used = o.lnW.copy()
        H = o.sweeps_em(sweeps, HEM)
        o.advance(sweeps)
        o.merge_update(H)
        g.run_iteration_em(sweeps, em)
        g.merge_update()
        assert np.array_equal(g.last_hist(), H), f"histogram differs in iteration {it}"
        assert np.array_equal(em_host(em, shape), HEM), f"joint histogram differs in iteration {it}"
    assert_same_state(o, g)
    betas = [0.3, 0.44, 0.5, 0.6]
    got = g.reweight_em(em_host(em, shape), betas)
    want = o.reweight_em(HEM, lnw_used, betas)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14)


def test_recording_leaves_the_chains_unchanged():
    import torch
    _, a = pair("muma", 16, 64, seed=5, beta=0.5)
    _, b = pair("muma", 16, 64, seed=5, beta=0.5)
    em = torch.zeros(int(np.prod(b.em_shape())), dtype=torch.int64, device="cuda")
    for _ in range(2):
        a.run_iteration(9)
        b.run_iteration_em(9, em)
        a.merge_update()
        b.merge_update()
    sa, ba, _ = a.chain_state()
    sb, bb, _ = b.chain_state()
    assert np.array_equal(sa, sb) and np.array_equal(ba, bb)
    assert np.array_equal(a.last_hist(), b.last_hist()) and np.array_equal(a.lnw(), b.lnw())
    h = em_host(em, b.em_shape())
    assert int(h.sum()) == 2 * 9 * 64


def test_argument_errors():
    import torch
    from paper_1312_2213_amd import muca
    _, ising = pair("ising", 8, 16, seed=1)
    with pytest.raises(muca.MucaError):
        ising.em_shape()
    _, g = pair("muma", 8, 16, seed=1, beta=0.4)
    ne, nm = g.em_shape()
    with pytest.raises(ValueError):
        g.run_iteration_em(1, torch.zeros(ne * nm - 1, dtype=torch.int64, device="cuda"))
    with pytest.raises(muca.MucaError):  # nothing merged yet
        g.reweight_em(np.zeros((ne, nm), np.uint64), [0.4])
    g.run_iteration_em(2, torch.zeros(ne * nm, dtype=torch.int64, device="cuda"))
    g.merge_update()
    with pytest.raises(muca.MucaError):  # size mismatch
        g.reweight_em(np.zeros((ne, nm - 1), np.uint64), [0.4])


def test_reweighted_magnetisation_matches_onsager_yang():
    """Multimagnetic Ising at T = 2/3 T_c, 16 x 16: weights iterated until
    flat, 200 production sweeps of 1024 chains with the joint histogram;
    the reweighted <|M|>/N at beta' around the run's beta equals the
    spontaneous magnetisation of the infinite lattice,
    (1 - sinh(2 beta')^-4)^(1/8), to 2e-3 (finite-size and statistical
    error at this size and temperature are far below that)."""
    import math

    import torch
    from paper_1312_2213_amd import muca
    beta_c = 0.5 * math.log(1.0 + math.sqrt(2.0))
    beta = 1.5 * beta_c
    run = muca.Run(muca.muca_config_default("muma", 16, 2, 1024, 9, beta=beta, layout=muca.MUCA_LAYOUT_BIT))
    for it in range(300):
        run.run_iteration(10)
        if run.merge_update()["flat"]:
            break
    else:
        pytest.fail("not flat in 300 iterations")
    ne, nm = run.em_shape()
    em = torch.zeros(ne * nm, dtype=torch.int64, device="cuda")
    run.run_iteration_em(200, em)
    run.merge_update()
    h = em.cpu().numpy().view(np.uint64).reshape(ne, nm)
    betas = [0.9 * beta, beta, 1.1 * beta]
    out = run.reweight_em(h, betas)
    for b, row in zip(betas, out):
        m_inf = (1.0 - math.sinh(2.0 * b) ** -4) ** 0.125
        assert abs(row[2] - m_inf) < 2e-3, (b, row[2], m_inf)
