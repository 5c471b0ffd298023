"""Pins the oracle's joint (E, M) histogram of multimagnetic runs and its
reweighting to other inverse temperatures: the histogram's M marginal is the
run's M histogram, each count sits at the energy of the configuration the
sweep left (closed forms for frozen ordered states), and the reweighted
averages of an exact joint density of states equal direct sums over all
2^16 states of a 4 x 4 lattice."""
import numpy as np
import pytest


def energy_magnetisation(s, L):
    """E = -sum over bonds (right, down) of s_i s_j, M = sum s_i, per chain."""
    g = s.reshape(-1, L, L).astype(np.int64)
    E = -(g * np.roll(g, -1, axis=2) + g * np.roll(g, -1, axis=1)).sum(axis=(1, 2))
    return E, g.sum(axis=(1, 2))


def test_marginal_and_count(orc):
    r = orc.LatticeRun(orc.MUMA, 8, 5, 11, beta=0.45)
    HEM = np.zeros(r.em_shape, np.uint64)
    H = r.sweeps_em(40, HEM)
    assert r.em_shape == (65, r.n_bins)
    assert np.array_equal(HEM.sum(axis=0), H)
    assert int(HEM.sum()) == 5 * 40


def test_each_sweep_counted_at_its_final_energy(orc):
    L = 8
    r = orc.LatticeRun(orc.MUMA, L, 6, 12, beta=0.3)
    HEM = np.zeros(r.em_shape, np.uint64)
    for _ in range(25):
        before = HEM.copy()
        r.sweeps_em(1, HEM)
        r.advance(1)
        E, M = energy_magnetisation(r.spins, L)
        assert np.array_equal(E, r.E) and np.array_equal(M, r.M)
        want = np.zeros_like(HEM)
        for e, m in zip(E, M):
            want[(e + 2 * L * L) // 4, (m - r.lo) // 2] += 1
        assert np.array_equal(HEM - before, want)


@pytest.mark.parametrize("pattern", ["up", "down", "checkerboard"])
def test_frozen_ordered_states(orc, pattern):
    """With every threshold zero no move is accepted, so each sweep counts
    the start state: all up E = -2N, M = N; all down E = -2N, M = -N;
    checkerboard E = +2N, M = 0."""
    L = 8
    N = L * L
    r = orc.LatticeRun(orc.MUMA, L, 1, 1, beta=0.2)
    y, x = np.indices((L, L))
    s = {"up": np.ones((L, L)), "down": -np.ones((L, L)),
         "checkerboard": np.where((x + y) % 2 == 0, 1, -1)}[pattern].astype(np.int8)
    r.spins[0] = s.ravel()
    r.E[0], r.M[0] = {"up": (-2 * N, N), "down": (-2 * N, -N), "checkerboard": (2 * N, 0)}[pattern]
    HEM = np.zeros(r.em_shape, np.uint64)
    r.sweeps_em(3, HEM, T=np.zeros(r.n_bins * r.n_cols, np.uint32))
    e = {"up": 0, "down": 0, "checkerboard": N}[pattern]
    b = (int(r.M[0]) - r.lo) // 2
    assert HEM[e, b] == 3 and int(HEM.sum()) == 3


def test_not_multimagnetic_is_refused(orc):
    r = orc.LatticeRun(orc.ISING, 8, 2, 1)
    with pytest.raises(RuntimeError):
        r.sweeps_em(1, np.zeros((65, r.n_bins), np.uint64))


def test_reweighting_an_exact_joint_density_of_states(orc):
    """HEM = g(E, M) of the 4 x 4 lattice (all 2^16 states enumerated),
    arbitrary weights lnW(M): the reweighted averages at beta' are the
    averages over states with weight exp(-(beta' - beta) E - lnW(M))."""
    L, N = 4, 16
    states = ((np.arange(1 << N)[:, None] >> np.arange(N)) & 1).astype(np.int8) * 2 - 1
    E, M = energy_magnetisation(states, L)
    lo = -N
    B = N + 1
    e_idx, b_idx = (E + 2 * N) // 4, (M - lo) // 2
    HEM = np.zeros((N + 1, B), np.uint64)
    np.add.at(HEM, (e_idx, b_idx), 1)
    rng = np.random.default_rng(3)
    lnW = rng.normal(0.0, 2.0, B)
    beta = 0.3
    betas = [0.0, 0.2, 0.4407, 0.7]
    got = orc.reweight_em(HEM, lnW, L, lo, beta, betas)
    for k, b2 in enumerate(betas):
        a = -(b2 - beta) * E - lnW[b_idx]
        w = np.exp(a - a.max())
        Z = w.sum()
        mE = (w * E).sum() / Z
        vE = (w * (E - mE) ** 2).sum() / Z
        mA = (w * np.abs(M)).sum() / Z
        m2 = (w * M.astype(float) ** 2).sum() / Z
        want = [mE / N, b2 * b2 * vE / N, mA / N, m2 / N ** 2, b2 * (m2 - mA * mA) / N, a.max() + np.log(Z)]
        np.testing.assert_allclose(got[k], want, rtol=1e-11, atol=1e-12)


def test_same_temperature_flat_weights_is_the_histogram_average(orc):
    HEM = np.zeros((17, 17), np.uint64)
    HEM[0, 0] = 3
    HEM[8, 8] = 5
    HEM[4, 12] = 2
    out = orc.reweight_em(HEM, np.zeros(17), 4, -16, 0.5, [0.5])[0]
    Ev = np.array([-32.0, 0.0, -16.0])
    Mv = np.array([-16.0, 0.0, 8.0])
    w = np.array([3.0, 5.0, 2.0])
    assert out[0] == pytest.approx((w * Ev).sum() / 10 / 16, rel=1e-14)
    assert out[2] == pytest.approx((w * np.abs(Mv)).sum() / 10 / 16, rel=1e-14)
    assert out[5] == pytest.approx(np.log(10.0), rel=1e-14)
