"""Pins the oracle's Markov chains against exact physics: with exact weights
the multicanonical histogram is flat (Eq. 1), with zero weights it is the
density of states, MUMA with exact magnetisation weights is flat in M (Eq. 3),
and the config-1 run reproduces the exact DOS and the exact canonical
averages after reweighting (Eq. 2).  Tolerances are several standard
deviations of the (autocorrelated) estimates; a wrong sign, index or
neighbour moves them by orders of magnitude more."""
import math
import os

import numpy as np
import pytest

from oracle import exact

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return [int(l) for l in f if not l.startswith("#")]


def run_fixed(r, lnW, sweeps, therm=50):
    T = r.thresholds(lnW)
    r.sweeps(therm, T, record=False)
    r.advance(therm)
    H = r.sweeps(sweeps, T)
    r.advance(sweeps)
    return H.astype(float)


def test_ising_exact_weights_give_flat_histogram(orc):
    bf, _ = exact.ising_dos_bruteforce(4)
    lnO = exact.ln_dos(bf)
    r = orc.LatticeRun(orc.ISING, 4, 128, seed=11)
    m = r.reachable() > 0
    H = run_fixed(r, np.where(m, -lnO, 0.0), 2000)
    assert not H[~m].any()
    rel = H[m] / H[m].mean()
    assert np.abs(rel - 1).max() < 0.12, rel


def test_ising_canonical_weights_sample_boltzmann(orc):
    """lnW(E) = -beta E turns the chain into canonical Metropolis: H is
    Omega(E) exp(-beta E).  (lnW = 0 would accept every flip: each sweep then
    flips every spin and the sweep-end energy never changes.)"""
    bf, _ = exact.ising_dos_bruteforce(4)
    beta = 0.2
    E = np.arange(-32, 33, 4, dtype=float)
    p = np.array([float(o) for o in bf]) * np.exp(-beta * E)
    p /= p.sum()
    r = orc.LatticeRun(orc.ISING, 4, 128, seed=12)
    H = run_fixed(r, -beta * E, 2000)
    big = p > 0.01
    assert np.abs(H[big] / H.sum() / p[big] - 1).max() < 0.06


def test_muma_exact_weights_flat_in_M(orc):
    _, em = exact.ising_dos_bruteforce(4)
    beta = 0.5
    Es = np.array([-32 + 4 * k for k in range(17)], float)
    pm = np.array([sum(int(em[k, j]) * math.exp(-beta * Es[k]) for k in range(17)) for j in range(17)])
    r = orc.LatticeRun(orc.MUMA, 4, 128, seed=13, beta=beta)
    H = run_fixed(r, -np.log(pm / pm.max()), 3000)
    rel = H / H.mean()
    assert np.abs(rel - 1).max() < 0.12, rel


def test_muma_zero_weights_sample_canonical_M(orc):
    _, em = exact.ising_dos_bruteforce(4)
    beta = 0.3
    Es = np.array([-32 + 4 * k for k in range(17)], float)
    pm = np.array([sum(int(em[k, j]) * math.exp(-beta * Es[k]) for k in range(17)) for j in range(17)])
    pm /= pm.sum()
    r = orc.LatticeRun(orc.MUMA, 4, 128, seed=14, beta=beta)
    H = run_fixed(r, np.zeros(17), 2000)
    big = pm > 0.02
    assert np.abs(H[big] / H.sum() / pm[big] - 1).max() < 0.08


def test_potts_q3_exact_weights_flat(orc):
    om = np.array(load("potts_q3_L4.txt"), float)
    r = orc.LatticeRun(orc.POTTS, 4, 128, seed=15, q=3)
    m = r.reachable() > 0
    lnW = np.where(m, -np.log(np.where(om > 0, om, 1)), 0.0)
    H = run_fixed(r, lnW, 3000)
    assert not H[~m].any()
    rel = H[m] / H[m].mean()
    assert np.abs(rel - 1).max() < 0.15, rel


def test_potts_q2_samples_ising_boltzmann(orc):
    bf, _ = exact.ising_dos_bruteforce(4)
    beta = 0.4   # per unsatisfied bond: Ising coupling 0.2
    r = orc.LatticeRun(orc.POTTS, 4, 128, seed=16, q=2)
    H = run_fixed(r, -beta * np.arange(r.n_bins), 2000)
    p = np.array([float(o) for o in bf]) * np.exp(-beta * 2 * np.arange(17))
    p /= p.sum()
    big = p > 0.01
    assert not H[1::2].any()
    assert np.abs(H[0::2][big] / H.sum() / p[big] - 1).max() < 0.06


def _config1_per_chain(orc):
    """Config 1 (Ising L = 8, 16 chains, seed 1, 12 iterations of 2000
    sweeps from lnW = 0) with every chain's histogram of every iteration
    kept.  Chains are independent (checked below), so running them one by
    one with the iteration's table is the same run as iterate()."""
    r = orc.LatticeRun(orc.ISING, 8, 16, seed=1, lo=-128, hi=128)
    per, flats = [], []
    for _ in range(12):
        T = r.thresholds()
        lnR_used = r.lnR.copy()
        Hc = np.zeros((r.n_chains, r.n_bins), np.uint64)
        for c in range(r.n_chains):
            r.sweeps(2000, T, chains=(c, c + 1), H=Hc[c])
        r.advance(2000)
        lnw_used = r.lnW.copy()
        H = Hc.sum(axis=0, dtype=np.uint64)
        flats.append(r.merge_update(H))
        per.append((lnR_used, lnw_used, Hc))
    return r, per, flats


def _pair_estimates(per, pairs, leave=None):
    """Accumulated-statistics estimate of -(ln Omega(b) - ln Omega(a)) for
    each pair (a, b) of consecutive reachable bins, written as the explicit
    inverse-variance mean over iterations n of lnR_used^(n) + ln h_a - ln h_b
    with weights h_a h_b / (h_a + h_b), optionally without chain `leave`."""
    num = np.zeros(len(pairs))
    den = np.zeros(len(pairs))
    for lnR_used, _, Hc in per:
        H = Hc.sum(axis=0).astype(float)
        if leave is not None:
            H = H - Hc[leave].astype(float)
        for k, (a, b) in enumerate(pairs):
            h0, h1 = H[a], H[b]
            if h0 > 0 and h1 > 0:
                p = h0 * h1 / (h0 + h1)
                num[k] += p * (lnR_used[a] + math.log(h0) - math.log(h1))
                den[k] += p
    return num / den


def test_config1_converges_to_exact_dos_within_jackknife_errors(orc):
    """Config 1: lnW^(12) + ln Omega is constant within jackknife errors over
    the 16 chains.  Tested on the increments between consecutive reachable
    bins (the quantities the recursion estimates, nearly independent of each
    other): leaving one chain out of every iteration's histogram gives 16
    replicates of each increment and its jackknife error sigma; the exact
    increment from the L = 8 density of states must lie within a few sigma
    everywhere, and the z-scores must scatter like unit normals.  The same
    statistic against the exact increments moved by one bin pair, with the
    sign of ln Omega flipped, or off by 0.1 per pair, fails by far."""
    d8 = load("ising_dos_L8.txt")
    lnO = exact.ln_dos(d8)
    r, per, flats = _config1_per_chain(orc)
    assert flats[0] == 0.0 and flats[-1] > 0.5
    idx = np.flatnonzero(r.reachable() > 0)
    pairs = list(zip(idx[:-1], idx[1:]))
    full = _pair_estimates(per, pairs)
    # the explicit mean is the oracle's recursion state
    assert np.abs(full - r.lnR[idx[:-1]]).max() < 1e-12
    C = r.n_chains
    reps = np.array([_pair_estimates(per, pairs, k) for k in range(C)])
    sig = np.sqrt((C - 1) / C * ((reps - reps.mean(axis=0)) ** 2).sum(axis=0))
    assert np.all(sig > 0)
    truth = np.array([lnO[a] - lnO[b] for a, b in pairs])
    z = (full - truth) / sig
    assert np.abs(z).max() < 4.5, z
    assert 0.4 < np.mean(z ** 2) < 2.0, np.mean(z ** 2)
    # lnW^(12) itself: the cumulative sum of those increments
    dev = (r.lnW + lnO)[idx]
    assert np.ptp(dev) < 1.0
    # plausible mistakes in the comparison are caught by the same statistic
    for wrong in (np.roll(truth, 1), -truth, truth + 0.1):
        zw = (full - wrong) / sig
        assert np.abs(zw).max() > 6 or np.mean(zw ** 2) > 4


def test_config1_reweighted_canonical_averages(orc):
    """The reweighted u, c of config 1's last iteration (Eq. 2) match the
    exact averages of the L = 8 density of states."""
    d8 = load("ising_dos_L8.txt")
    r, per, _ = _config1_per_chain(orc)
    _, lnw_used, Hc = per[-1]
    H = Hc.sum(axis=0, dtype=np.uint64)
    vals = [-128 + 4 * k for k in range(65)]
    for beta in (0.3, 0.44, 0.6):
        u, c = exact.canonical(d8, vals, beta, 64)
        out = r.reweight(H, lnw_used, [beta])[0]
        assert abs(out[0] - u) < 0.02 * abs(u)
        assert abs(out[1] - c) < 0.06 * c


def test_chains_are_independent_and_splittable(orc):
    """Running chain ranges separately and summing histograms equals one run."""
    a = orc.LatticeRun(orc.POTTS, 6, 10, seed=21, q=4)
    b = orc.LatticeRun(orc.POTTS, 6, 10, seed=21, q=4)
    T = a.thresholds(-0.05 * np.arange(a.n_bins))
    Ha = a.sweeps(30, T)
    Hb = b.sweeps(30, T, chains=(0, 4))
    Hb = b.sweeps(30, T, chains=(4, 10), H=Hb)
    assert np.array_equal(Ha, Hb) and np.array_equal(a.spins, b.spins)
