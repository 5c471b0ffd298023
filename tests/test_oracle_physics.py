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


def test_config1_converges_to_exact_dos_and_canonical(orc):
    """Ising L = 8, 16 chains, seed 1, 12 iterations of 2000 sweeps from
    lnW = 0, then the final update: lnW^(12) + ln Omega is constant and the
    reweighted u, c of the last iteration match the exact averages."""
    d8 = load("ising_dos_L8.txt")
    lnO = exact.ln_dos(d8)
    r = orc.LatticeRun(orc.ISING, 8, 16, seed=1, lo=-128, hi=128)
    flats = []
    for _ in range(12):
        H, f, lnw_used = r.iterate(2000)
        flats.append(f)
    assert flats[0] == 0.0 and flats[-1] > 0.5
    m = r.reachable() > 0
    dev = (r.lnW + lnO)[m]
    assert np.ptp(dev) < 1.0
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
