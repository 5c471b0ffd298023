"""Host-side logic of the statistical-speedup experiment (Eqs. 4-6)."""
import math

import pytest

from paper_1312_2213_amd import speedup as su


def test_sweeps_follow_the_power_law_and_split_over_chains():
    s = su.System("ising", 16)
    m1 = 5.7 * 16 ** 2.51  # Eq. 4, Ising, p = 1
    assert s.sweeps(1) == math.ceil(m1)
    assert s.sweeps(8) == math.ceil(m1 / 8)
    assert s.sweeps(10 ** 6) == 1
    potts = su.System("potts", 8, q=8, potts_law=True)
    assert potts.sweeps(1) == math.ceil(24 * 8 ** 2.67)


def test_speedup_estimator():
    # p N(p0) / (p0 N(p)): equal iteration counts give S*_p = p / p0
    s, e = su.speedup(1, 40.0, 0.0, 16, 40.0, 0.0)
    assert s == 16 and e == 0
    s, e = su.speedup(2, 50.0, 1.0, 8, 100.0, 2.0)
    assert s == pytest.approx(2.0)
    assert e == pytest.approx(2.0 * math.sqrt(0.02 ** 2 + 0.02 ** 2))


def test_table_relative_to_smallest_fully_converged_p():
    r = su.Result("x", [1, 4, 16], [100, 25, 7], {1: [10, 12, None], 4: [11, 12, 13], 16: [12, 12, 12]},
                  {1: [2, 2, 2], 4: [1, 1, 1], 16: [1, 2, 3]})
    rows = r.table()
    assert rows[0]["capped"] == 1 and rows[0]["mean"] == 11.0 and rows[0]["speedup"] is None
    assert rows[1]["speedup"] == 1.0
    assert rows[2]["speedup"] == pytest.approx(4.0)
    cov = r.table("n_cover")
    # n_cover for p = 4 has zero spread: the reference is the first row with a defined error
    assert cov[0]["speedup"] == 1.0 and cov[2]["speedup"] == pytest.approx(16 * 2 / 2)


def test_lnw_zero_ising_sweep_keeps_the_energy():
    """The reason small-p Ising runs can stay at lnW = 0: every flip is
    accepted, so a sequential sweep maps s to -s and E is unchanged."""
    import numpy as np
    from oracle import oracle as orc
    o = orc.LatticeRun(orc.ISING, 8, 3, 5)
    E0, s0 = o.E.copy(), o.spins.copy()
    H = o.sweeps(7)
    assert np.array_equal(o.E, E0) and np.array_equal(o.spins, -s0)
    assert np.count_nonzero(H) == len(set(o.bins().tolist()))


def test_seeds_distinct():
    seeds = {su.seed_of(1, k, r) for k in range(13) for r in range(16)}
    assert len(seeds) == 13 * 16


def test_muma_at_two_thirds_tc():
    (sysm,) = [s for s, _, _ in su.paper_systems() if s.model == "muma"]
    assert sysm.beta == pytest.approx(1.5 * 0.5 * math.log(1 + math.sqrt(2)))


def test_q_scan_laws_and_grid():
    """q = 2 is the Ising model (Ising law), q >= 3 the per-unit Potts
    energies (8-state Potts law); every q on the same p grid."""
    sc = su.q_scan_systems(16)
    assert [s.q for s, _, _ in sc] == list(range(2, 11))
    assert all(s.model == "potts" and s.L == 16 for s, _, _ in sc)
    assert [s.potts_law for s, _, _ in sc] == [False] + [True] * 8
    assert all(ps == [16, 32, 64, 128, 256, 512, 1024, 2048] and r == 8 for _, ps, r in sc)
    assert sc[0][0].sweeps(16) == math.ceil(5.7 * 16 ** 2.51 / 16)
    assert sc[6][0].sweeps(16) == math.ceil(24 * 16 ** 2.67 / 16)


def test_polymer_system_sweeps_and_flatness():
    s = su.PolymerSystem(40, -70.0, -20.0, 100, 1024)
    assert [s.sweeps(p) for p in (1, 2, 3, 1024, 4096)] == [1024, 512, 342, 1, 1]
    assert [s.therm(p) for p in (1, 8, 4096)] == [256, 32, 1]
    assert su.polymer_flatness([4, 2, 6]) == pytest.approx(0.5)
    assert su.polymer_flatness([0, 0]) == 0.0
    (s40, ps, r), (s80, _, _) = su.paper_polymer_systems()
    assert s40.n_beads == 40 and s80.n_beads == 80 and ps[0] == 1 and s40.moves == 1


def test_time_speedup_table():
    r = su.Result("x", [1, 4], [100, 25], {1: [10, 10], 4: [10, 10]}, {1: [1, 1], 4: [1, 1]})
    r.seconds_per_run = {1: [2.0, 2.2], 4: [0.5, 0.6]}
    rows = su.time_speedup(r)
    assert rows[0]["S_p"] == 1.0
    assert rows[1]["S_p"] == pytest.approx(2.1 / 0.55)

