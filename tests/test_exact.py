"""Pins the exact references that the oracle is checked against: brute force,
transfer matrix and Kaufman's closed form must agree, and must reproduce the
low-temperature counts that follow from counting clusters by hand."""
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


def test_three_methods_agree_L4():
    bf, _ = exact.ising_dos_bruteforce(4)
    assert [int(x) for x in bf] == exact.ising_dos_kaufman(4) == exact.ising_dos_transfer(4)


@pytest.mark.slow
def test_transfer_equals_kaufman_L6():
    assert exact.ising_dos_transfer(6) == exact.ising_dos_kaufman(6)


@pytest.mark.parametrize("L", [8, 16])
def test_closed_forms(L):
    """Sum 2^N; Omega(E) = Omega(-E) (bipartite torus); ground state 2;
    one flipped spin 2N; domino 4N; three-site clusters, 2x2 squares and
    separated pairs give N^2 + 9N at 8 broken bonds (L >= 5)."""
    N = L * L
    dos = load(f"ising_dos_L{L}.txt")
    assert len(dos) == N + 1
    assert sum(dos) == 2 ** N
    assert dos == dos[::-1]
    assert dos[:5] == [2, 0, 2 * N, 4 * N, N * N + 9 * N]


def test_golden_L8_recomputes():
    assert load("ising_dos_L8.txt") == exact.ising_dos_kaufman(8)


def test_kaufman_lnZ_real_K_matches_enumeration():
    bf, _ = exact.ising_dos_bruteforce(4)
    with mpmath.workdps(50):
        for K in ("0.1", "0.4406868", "0.9"):
            K = mpmath.mpf(K)
            z = mpmath.fsum(int(o) * mpmath.exp(-K * (-32 + 4 * k)) for k, o in enumerate(bf))
            assert abs(exact.kaufman_lnZ(4, K) - mpmath.log(z)) < 1e-25


def test_canonical_matches_kaufman_derivatives_L8():
    """u = -(1/N) d lnZ/dK and c = (K^2/N) d^2 lnZ/dK^2 from the closed form,
    against the same averages summed over the exact DOS."""
    dos = load("ising_dos_L8.txt")
    vals = [-128 + 4 * k for k in range(65)]
    for K in (0.3, 0.44, 0.6):
        u, c = exact.canonical(dos, vals, K, 64)
        with mpmath.workdps(40):
            f = lambda k: exact.kaufman_lnZ(8, k, mpmath.mp.dps + 30)
            d1 = mpmath.diff(f, K)
            d2 = mpmath.diff(f, K, 2)
        assert abs(u - float(-d1 / 64)) < 1e-12
        assert abs(c - float(K * K * d2 / 64)) < 1e-10


def test_potts_q3_golden_and_q2_maps_to_ising():
    om = load("potts_q3_L4.txt")
    assert sum(om) == 3 ** 16 and om[0] == 3 and om[4] == 16 * 3 * 2
    assert [k for k, o in enumerate(om) if o == 0] == [1, 2, 3, 5]
    p2 = exact.potts_dos_bruteforce(4, 2)
    bf, _ = exact.ising_dos_bruteforce(4)
    # q = 2: E_unsat = (E_ising + 2N) / 2 = 2k
    assert [int(x) for x in p2[0::2]] == [int(x) for x in bf] and not p2[1::2].any()


def test_muma_joint_dos_marginals():
    bf, em = exact.ising_dos_bruteforce(4)
    assert [int(x) for x in em.sum(axis=1)] == [int(x) for x in bf]
    assert [int(x) for x in em.sum(axis=0)] == [math.comb(16, j) for j in range(17)]
