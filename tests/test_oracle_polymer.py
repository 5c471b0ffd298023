"""Pins the oracle's bead-spring polymer (Eq. 7 with the LJ cut-and-shift
and FENE parameters of the polymer workload): closed-form pair energies,
running-energy bookkeeping, and the stationary bond-length distribution of a
dimer under fixed bin weights, integrated exactly."""
import math

import numpy as np
import pytest

from synth import polymer_walk

SHIFT = 4.0 * (2.5 ** -12 - 2.5 ** -6)


def make(orc, pos, **kw):
    C, N, _ = pos.shape
    return orc.PolymerRun(n_beads=N, n_chains=C, seed=kw.pop("seed", 5), pos=pos, **kw)


def test_pair_energies_closed_form(orc):
    r = make(orc, polymer_walk(3, 1, 0))
    # dimer at the FENE rest length
    assert r.energy(np.array([[0, 0, 0], [1, 0, 0]], np.float32)) == 0.0
    e = r.energy(np.array([[0, 0, 0], [1.25, 0, 0]], np.float32))
    assert abs(e - (-5.0 * math.log(1 - 0.25))) < 1e-12
    assert r.energy(np.array([[0, 0, 0], [1.5, 0, 0]], np.float32)) == math.inf
    # trimer straight: LJ between the ends at r = 2, shifted
    e = r.energy(np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], np.float32))
    assert abs(e - (4 * (2.0 ** -12 - 2.0 ** -6) - SHIFT)) < 1e-12
    # ends at r = 1 (sigma): LJ = -shift = +0.016317
    h = math.sqrt(0.75)
    e = r.energy(np.array([[0, 0, 0], [0.5, h, 0], [1, 0, 0]], np.float32))
    x = np.array([[0, 0, 0], [0.5, h, 0], [1, 0, 0]], np.float32).astype(float)
    fb = [np.linalg.norm(x[1] - x[0]), np.linalg.norm(x[2] - x[1])]
    fene = sum(-5.0 * math.log(1 - ((b - 1) / 0.5) ** 2) for b in fb)
    assert abs(e - (fene - SHIFT)) < 1e-9 and abs(-SHIFT - 0.016316891) < 1e-9
    # beyond the cutoff
    e = r.energy(np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [2, 1.6, 0]], np.float32))
    assert np.isfinite(e)


def test_lj_minimum(orc):
    r = make(orc, polymer_walk(3, 1, 0))
    rm = 2 ** (1 / 6)
    best = min(r.energy(np.array([[0, 0, 0], [0.5 * d, math.sqrt(1 - 0.25 * d * d), 0], [d, 0, 0]],
                                 np.float32)) for d in np.linspace(1.0, 1.3, 301))
    # the two bonds stay at r0 (FENE 0) while the ends scan through the LJ well
    assert abs(best - (-1.0 - SHIFT)) < 1e-3
    assert abs(rm - 1.122462) < 1e-6


def test_initial_walk_and_running_energy(orc):
    pos = polymer_walk(40, 6, 5)
    r = make(orc, pos)
    assert np.all((r.E > -200) & (r.E < 50))
    r.lnW = -0.5 * r.bin_centres()        # canonical-like weights so moves mix
    r.sweeps(200, record=False)
    r.advance(200)
    for c in range(6):
        e = r.energy(r.pos[c])
        assert abs(e - r.E[c]) < 1e-9
        assert r.bin[c] == r.bin_of(r.E[c])
    assert not np.array_equal(r.pos, pos)


def test_dimer_bond_length_distribution(orc):
    """Two beads: the relative vector is uniform in space times the weight of
    the energy bin, so H_b is proportional to exp(lnW_b) times the integral
    of r^2 dr over the r with U_FENE(r) in bin b (U symmetric about r0)."""
    beta = 1.0
    C = 128
    pos = np.zeros((C, 2, 3), np.float32)
    pos[:, 1, 0] = 1.0
    r = make(orc, pos, seed=9)
    cent = r.bin_centres()
    r.lnW = -beta * cent
    r.sweeps(200, record=False)
    r.advance(200)
    H = r.sweeps(6000).astype(float)
    edges = -200.0 + 0.1 * np.arange(r.n_bins + 1)

    def cube_span(E):  # integral of r^2 over |r-1| <= 0.5 sqrt(1-exp(-E/5))
        a = 0.5 * np.sqrt(1 - np.exp(-np.clip(E, 0, None) / 5.0))
        return ((1 + a) ** 3 - (1 - a) ** 3) / 3

    w = (cube_span(edges[1:]) - cube_span(edges[:-1])) * np.exp(-beta * cent)
    # compare in windows of one energy unit
    sel = slice(2000, 2060)
    Hw = H[sel].reshape(-1, 10).sum(1)
    ww = w[sel].reshape(-1, 10).sum(1)
    assert H[:2000].sum() == 0
    ratio = (Hw / Hw.sum()) / (ww / ww.sum())
    assert np.abs(ratio[:3] - 1).max() < 0.03, ratio


def paper_run(orc, N, C, seed):
    from synth import PAPER_POLYMER
    pp = dict(PAPER_POLYMER)
    pos = polymer_walk(N, C, seed, bond=pp["fene_r0"], min_dist=pp["lj_sigma"])
    return orc.PolymerRun(n_beads=N, n_chains=C, seed=seed, pos=pos, x_lo=-400.0, x_hi=100.0,
                          n_bins=1000, **pp), pos


def test_paper_parameters_closed_form(orc):
    """Eq. 7 with the paper's parameters: LJ minimum -1 at r0 (sigma =
    2^(-1/6) r0, no cutoff, no shift), FENE zero at r0 and infinite at
    r_max = 1."""
    r, _ = paper_run(orc, 40, 1, 3)
    s = 2 ** (-1 / 6) * 0.7
    # trimer with the ends at r0: bonds at r0 too (equilateral), LJ(r0) = -1
    h = math.sqrt(0.75) * 0.7
    tri = np.array([[0, 0, 0], [0.35, h, 0], [0.7, 0, 0]], np.float32)
    x = tri.astype(float)
    d = np.linalg.norm(x[2] - x[0])
    lj = 4 * ((s / d) ** 12 - (s / d) ** 6)
    fene = sum(-(40 / 2) * 0.09 * math.log(1 - ((np.linalg.norm(x[k + 1] - x[k]) - 0.7) / 0.3) ** 2)
               for k in range(2))
    assert abs(r.energy(tri) - (lj + fene)) < 1e-9 and abs(lj + 1.0) < 1e-5
    # straight 4-bead chain at spacing r0: every non-bonded pair interacts,
    # also the ends at 3 r0 = 3.4 sigma (no cutoff)
    line = np.array([[0.7 * k, 0, 0] for k in range(4)], np.float32)
    x = line.astype(float)
    want = 0.0
    for a_, b_ in ((0, 2), (1, 3), (0, 3)):
        rr = np.linalg.norm(x[b_] - x[a_])
        want += 4 * ((s / rr) ** 12 - (s / rr) ** 6)
    for k in range(3):
        t = (np.linalg.norm(x[k + 1] - x[k]) - 0.7) / 0.3
        want += -(40 / 2) * 0.09 * math.log(1 - t * t)
    assert abs(r.energy(line) - want) < 1e-12 and want < -0.02
    assert r.energy(np.array([[0, 0, 0], [1.0, 0, 0]], np.float32)) == math.inf


@pytest.mark.parametrize("N", [40, 80])
def test_paper_polymer_running_energy(orc, N):
    """The per-move energy change (for N > 64 each tree slot first adds the
    terms of partners j and j + 64) keeps the running energy equal to the
    recomputed total energy."""
    r, pos = paper_run(orc, N, 3, 11)
    r.lnW = -0.5 * r.bin_centres()
    r.sweeps(60, record=False)
    r.advance(60)
    for c in range(3):
        e = r.energy(r.pos[c])
        assert abs(e - r.E[c]) < 1e-9 * max(1.0, abs(e))
        assert r.bin[c] == r.bin_of(r.E[c])
    assert not np.array_equal(r.pos, pos)
