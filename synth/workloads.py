"""The five workloads, named by what they are, with their sizes."""
from __future__ import annotations

import math


def m_opt(L: int, p: int, potts: bool = False) -> float:
    """Sweeps per iteration from the paper's power laws (Eq. 4):
    Ising 5.7 L^2.51 / p, 8-state Potts 24 L^2.67 / p."""
    return (24.0 * L ** 2.67 if potts else 5.7 * L ** 2.51) / p


def sweeps_per_iteration(L: int, chains: int, potts_fit: bool) -> int:
    """max(10, ceil(M_opt(L, 1) / chains)), M_opt(L,1) from Eq. 4."""
    return max(10, math.ceil(m_opt(L, 1, potts_fit) / chains))


WORKLOADS = {
    "ising8_plain": dict(model="ising", L=8, chains=16, seed=1, lo=-128, hi=128,
                         iterations=12, sweeps=2000),
    "ising64_packed": dict(model="ising", L=64, chains=4096, seed=2, sweeps=10000,
                           flat=0.5),
    "potts8_batched": dict(instances=[dict(model="potts", q=8, L=L, chains=2048, seed=30 + k)
                                      for k, L in enumerate((16, 24, 32, 48))]
                           + [dict(model="muma", L=32, chains=512, seed=34 + k, beta=0.5)
                              for k in range(4)], flat=0.5),
    "serving200": dict(n=200, rate=4.0, seed=4, flat=0.5),
    "polymer40": dict(model="polymer", n_beads=40, chains=4096, seed=5, x_lo=-200.0,
                      x_hi=50.0, n_bins=2500, sweeps=1000, flat=0.5),
}

# The paper's bead-spring homopolymer (Eq. 7 and the parameters stated with
# it): FENE K = 40, r0 = 0.7, r_max = 1 (R = 0.3); Lennard-Jones with
# sigma = 2^(-1/6) r0 (its minimum at r0) and no cutoff; N = 40 and 80.
# The displacement cube side (0.3 sigma) is not stated in the paper: a choice here.
PAPER_POLYMER = dict(lj_eps=1.0, lj_sigma=2.0 ** (-1.0 / 6.0) * 0.7, lj_rcut=math.inf,
                     fene_k=40.0, fene_r0=0.7, fene_R=0.3, step=0.3 * 2.0 ** (-1.0 / 6.0) * 0.7)
