"""Pins the oracle's acceptance thresholds, reachable-bin masks, recursion,
flatness and reweighting against definitions checked by independent means."""
import math
import os

import mpmath
import numpy as np
import pytest

from oracle import exact

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return [int(l) for l in f if not l.startswith("#")]


# ---------------------------------------------------------------- thresholds
def test_threshold_rule(orc):
    M = 0xFFFFFFFF
    assert orc.threshold(0.0) == M and orc.threshold(3.0) == M
    assert orc.threshold(-1e-12) == M          # 2^32 e^D >= 2^32 - 1
    assert orc.threshold(-800.0) == 0
    rng = np.random.default_rng(1)
    with mpmath.workdps(40):
        for D in np.concatenate([-rng.exponential(2.0, 300), [-math.log(2), -1.0, -20.0]]):
            v = mpmath.ldexp(mpmath.exp(mpmath.mpf(float(D))), 32)
            t = orc.threshold(float(D))
            assert abs(t - int(mpmath.floor(v))) <= 1
            if abs(v - mpmath.nint(v)) > 1e-3:
                assert t == int(mpmath.floor(v))
    ds = -np.sort(rng.exponential(3.0, 200))[::-1]
    ts = [orc.threshold(float(d)) for d in ds]
    assert all(a <= b for a, b in zip(ts, ts[1:]))  # ascending D


def test_threshold_tables_layout(orc):
    r = orc.LatticeRun(orc.ISING, 4, 1, seed=1, lo=-24, hi=32)
    lnW = np.linspace(0.0, 3.0, r.n_bins) ** 2
    T = r.thresholds(lnW).reshape(r.n_bins, 5)
    for b in range(r.n_bins):
        for j in range(5):
            t = b + j - 2
            want = 0 if not 0 <= t < r.n_bins else orc.threshold(lnW[t] - lnW[b])
            assert T[b, j] == want
    m = orc.LatticeRun(orc.MUMA, 4, 1, seed=1, beta=0.5)
    T = m.thresholds(np.zeros(m.n_bins)).reshape(m.n_bins, 10)
    for j in range(10):
        n, up = divmod(j, 2)
        want = orc.threshold(-0.5 * (4 * n - 8))
        assert T[5, j] == want
    assert T[0, 1] == 0 and T[m.n_bins - 1, 0] == 0   # M would leave [-N, N]
    p = orc.LatticeRun(orc.POTTS, 4, 1, seed=1, q=3)
    T = p.thresholds(-0.1 * np.arange(p.n_bins)).reshape(p.n_bins, 9)
    assert T[10, 4] == 0xFFFFFFFF and T[10, 5] == orc.threshold(-0.1) and T[2, 0] == 0


# ---------------------------------------------------------------- reachable
def test_reachable_masks_match_enumeration(orc):
    bf, _ = exact.ising_dos_bruteforce(4)
    r = orc.LatticeRun(orc.ISING, 4, 1, seed=1)
    assert list(r.reachable()) == [int(int(o) > 0) for o in bf]
    p3 = load("potts_q3_L4.txt")
    p = orc.LatticeRun(orc.POTTS, 4, 1, seed=1, q=3)
    assert list(p.reachable()) == [int(o > 0) for o in p3]
    p2 = exact.potts_dos_bruteforce(4, 2)
    p = orc.LatticeRun(orc.POTTS, 4, 1, seed=1, q=2)
    assert list(p.reachable()) == [int(o > 0) for o in p2]
    d8 = load("ising_dos_L8.txt")
    r = orc.LatticeRun(orc.ISING, 8, 1, seed=1)
    assert list(r.reachable()) == [int(o > 0) for o in d8]


# ---------------------------------------------------------------- recursion
def _mask(n, zeros=()):
    m = np.ones(n, np.uint8)
    m[list(zeros)] = 0
    return m


def test_recursion_first_step_is_W_over_H(orc):
    rng = np.random.default_rng(3)
    H = rng.integers(1, 1000, 12).astype(np.uint64)
    lnR, P, lnW = orc.recursion(H, np.zeros(12), np.zeros(12), _mask(12))
    want = -np.log(H.astype(float))
    want -= want[0]
    assert np.allclose(lnW, want, rtol=0, atol=1e-12)
    # scaling H changes nothing on the first step
    _, _, lnW2 = orc.recursion(H * np.uint64(7), np.zeros(12), np.zeros(12), _mask(12))
    assert np.allclose(lnW2, lnW, atol=1e-12)


def test_recursion_constant_H_and_monotone_P(orc):
    lnR = np.linspace(-1, 1, 10)
    P = np.arange(10, dtype=float)
    H = np.full(10, 50, np.uint64)
    lnR2, P2, lnW = orc.recursion(H, lnR, P, _mask(10))
    assert np.allclose(lnR2[:9], lnR[:9]) and np.all(P2 >= P)
    assert np.allclose(P2[:9] - P[:9], 25.0)
    H[4] = 0
    _, P3, _ = orc.recursion(H, lnR, P, _mask(10))
    assert P3[3] == P[3] and P3[4] == P[4] and P3[5] == P[5] + 25.0


def test_recursion_weighted_mean_rule(orc):
    """lnR^(n+1) = (1 - k) lnR^(n) - k dlnOmega when H = Omega W exactly,
    with k = p / P_acc: the inverse-variance weighting of the estimates."""
    rng = np.random.default_rng(5)
    B = 9
    lnO = np.cumsum(rng.uniform(-2, 2, B))
    lnR0 = rng.uniform(-1, 1, B)
    P0 = rng.uniform(10, 100, B)
    lnW0 = np.concatenate([[0.0], np.cumsum(lnR0[:-1])])
    Hf = np.exp(lnO + lnW0)
    Hf *= 1e6 / Hf.max()
    H = np.round(Hf).astype(np.uint64)
    lnR, P, _ = orc.recursion(H, lnR0, P0, _mask(B))
    h = H.astype(float)
    for k in range(B - 1):
        p = h[k] * h[k + 1] / (h[k] + h[k + 1])
        kap = p / (P0[k] + p)
        est = -(math.log(h[k + 1]) - math.log(h[k]) - lnR0[k])  # estimate of lnR_exact
        assert abs(lnR[k] - ((1 - kap) * lnR0[k] + kap * est)) < 1e-12
        assert abs(P[k] - (P0[k] + p)) < 1e-9


def test_recursion_fixed_point_exact_dos(orc):
    """lnW = -lnOmega on the reachable bins is a fixed point for H = c Omega W."""
    d8 = load("ising_dos_L8.txt")
    lnO = exact.ln_dos(d8)
    r = orc.LatticeRun(orc.ISING, 8, 1, seed=1)
    m = r.reachable()
    H = np.full(r.n_bins, 1000, np.uint64) * m.astype(np.uint64)
    lnR, P, lnW = orc.recursion(H, np.zeros(r.n_bins), np.zeros(r.n_bins), m)
    assert np.allclose(lnW, 0.0)
    # first step from lnW = 0 with H proportional to Omega recovers -lnOmega
    Hf = np.where(m > 0, np.array([float(o) for o in d8]) / 2, 0)
    H = np.round(Hf).astype(np.uint64)
    H[m == 0] = 0
    _, _, lnW = orc.recursion(H, np.zeros(r.n_bins), np.zeros(r.n_bins), m)
    sel = m > 0
    dev = lnW[sel] + lnO[sel]
    assert np.ptp(dev) < 1e-9


def test_recursion_skips_unreachable_bins(orc):
    """The pair across an unreachable bin is updated; the bin itself carries
    the weight of the reachable bin below it."""
    H = np.array([10, 0, 40, 20], np.uint64)
    lnR, P, lnW = orc.recursion(H, np.zeros(4), np.zeros(4), _mask(4, [1]))
    assert abs(lnW[2] - (math.log(10) - math.log(40))) < 1e-12
    assert lnW[1] == lnW[0] == 0.0
    assert abs(lnW[3] - lnW[2] - (math.log(40) - math.log(20))) < 1e-12


def test_flatness(orc):
    H = np.array([10, 0, 20, 30], np.uint64)
    assert abs(orc.flatness(H, _mask(4, [1])) - 10 / 20) < 1e-15
    assert orc.flatness(H, _mask(4)) == 0.0
    assert orc.flatness(np.zeros(4, np.uint64), _mask(4)) == 0.0


# ---------------------------------------------------------------- reweighting
def test_reweight_exact_input_reproduces_canonical(orc):
    """Feeding H = Omega with lnW = 0 (and H = Omega W with exact weights)
    reproduces the exact canonical u and c (Eq. 2)."""
    d8 = load("ising_dos_L8.txt")
    vals = [-128 + 4 * k for k in range(65)]
    H = np.array([o >> 20 for o in d8], np.uint64)   # exact integers, DOS / 2^20
    lnO = exact.ln_dos(d8)
    for beta in (0.2, 0.44, 0.7):
        # a truncated DOS loses the low-E tail; compare with the same truncation
        tr = [int(h) for h in H]
        u, c = exact.canonical(tr, vals, beta, 64)
        out = orc.reweight(H, np.zeros(65), vals, 64, beta)
        assert abs(out[0] - u) < 1e-12 * max(1, abs(u)) and abs(out[1] - c) < 1e-11 * max(1, c)
    # exact weights: H flat (= 1000 on reachable bins), lnW = -lnOmega
    m = np.isfinite(lnO)
    Hf = np.where(m, 1000, 0).astype(np.uint64)
    lnW = np.where(m, -lnO, 0.0)
    for beta in (0.3, 0.44):
        u, c = exact.canonical(d8, vals, beta, 64)
        out = orc.reweight(Hf, lnW, vals, 64, beta)
        assert abs(out[0] - u) < 1e-12 and abs(out[1] - c) < 1e-11


def test_reweight_muma_exact(orc):
    _, em = exact.ising_dos_bruteforce(4)
    beta = 0.5
    Es = np.array([-32 + 4 * k for k in range(17)], float)
    Ms = np.array([-16 + 2 * j for j in range(17)], float)
    pm = np.array([sum(int(em[k, j]) * math.exp(-beta * Es[k]) for k in range(17)) for j in range(17)])
    H = np.full(17, 5000, np.uint64)
    lnW = -np.log(pm)
    out = orc.reweight(H, lnW, Ms, 16, beta, muma=True)
    z = pm.sum()
    assert abs(out[0] - (pm * np.abs(Ms)).sum() / z / 16) < 1e-12
    assert abs(out[1] - (pm * Ms ** 2).sum() / z / 256) < 1e-12
    assert abs(out[2]) < 1e-12


def test_potts_colours_stay_below_q_for_large_q(orc):
    """Colours 0..q-1 are unsigned bytes (q up to 255): with lnW = 0 every
    proposal is accepted, so after a few sweeps every proposal map, including
    the wrap from q-1 past 0, has been applied; colours stay in [0, q), every
    site changed colour, and the running E equals the recomputed one."""
    import numpy as np
    q = 255
    o = orc.LatticeRun(orc.POTTS, 8, 4, 31, q=q)
    assert o.spins.dtype == np.uint8
    before = o.spins.copy()
    o.sweeps(1)
    o.advance(1)
    assert np.all(o.spins != before)  # every attempt accepted: a different colour
    o.sweeps(40)
    o.advance(40)
    assert o.spins.max() < q and o.spins.max() >= 200
    for c in range(4):
        E = 0
        s = o.spins[c].reshape(8, 8).astype(int)
        E += int(np.sum(s != np.roll(s, -1, 1)) + np.sum(s != np.roll(s, -1, 0)))
        assert E == o.E[c]


# ------------------------------------------------------- accepted-move count
def test_accepted_move_count(orc):
    """lnW = 0 over the full range accepts every lattice move; zero
    thresholds accept none; thermalisation sweeps are not counted; a
    polymer shift that is accepted moves its bead, so one sweep's count is
    the number of beads that moved."""
    from synth import polymer_walk
    for model, q in ((orc.ISING, 2), (orc.POTTS, 5), (orc.MUMA, 2)):
        r = orc.LatticeRun(model, 8, 3, 2, q=q, beta=0.0)
        r.sweeps(4)
        assert r.take_accepted() == 4 * 3 * 64
        r.sweeps(4, record=False)
        assert r.take_accepted() == 0
        r.sweeps(2, T=np.zeros(r.n_bins * r.n_cols, np.uint32))
        assert r.take_accepted() == 0
    pos = polymer_walk(12, 4, 1)
    p = orc.PolymerRun(n_beads=12, n_chains=4, seed=1, pos=pos)
    before = p.pos.copy()
    p.sweeps(1)
    moved = int(np.any(p.pos != before, axis=2).sum())
    assert p.take_accepted() == moved and moved > 0


# ------------------------------------------------------------- jackknife
def test_jackknife_of_a_mean_is_the_standard_error(orc):
    """At lnW = 0 and beta = 0 the reweighted <E> is the histogram mean; with
    equal counts per block the jackknife error of a mean is the standard
    error of the block means, sqrt(sum (mu_k - mu)^2 / (m (m - 1))); equal
    blocks give zero; empty blocks are left out."""
    rng = np.random.default_rng(5)
    B, m, c = 17, 9, 400
    values = np.arange(B, dtype=np.float64) * 4.0 - 32.0
    blocks = np.zeros((m + 2, B), np.uint64)
    for k in range(m):
        blocks[k] = rng.multinomial(c, rng.dirichlet(np.ones(B)))
    vals, errs = orc.reweight_jackknife(blocks, np.zeros(B), values, 64, [0.0])
    mu = (blocks[:m] * values).sum(axis=1) / c
    want = math.sqrt(((mu - mu.mean()) ** 2).sum() / (m * (m - 1)))
    assert vals[0][2] == pytest.approx(mu.mean(), rel=1e-13)
    assert errs[0][2] == pytest.approx(want, rel=1e-10)
    same = np.tile(blocks[0], (5, 1))
    _, e0 = orc.reweight_jackknife(same, np.zeros(B), values, 64, [0.3, 0.7])
    assert np.all(np.abs(e0) < 1e-12)
