"""Exact references for the 2D Ising and Potts models on periodic L x L lattices.

TEST INFRASTRUCTURE ONLY (see oracle/oracle.py).

* ``ising_dos_bruteforce(L)``: enumeration of all 2^(L^2) states (L <= 4),
  giving Omega(E) and Omega(E, M).
* ``potts_dos_bruteforce(L, q)``: enumeration of all q^(L^2) states (small).
* ``ising_dos_transfer(L)``: row-to-row transfer matrix with exact integer
  polynomial entries (L <= 6).
* ``ising_dos_kaufman(L)``: exact Omega(E) for any even L from Kaufman's
  closed form of the torus partition function (Kaufman 1949; Ferdinand and
  Fisher 1969), sampled on the unit circle of y = exp(-4K) in high precision
  and inverted by a discrete Fourier transform -- the same polynomial Beale
  (1996) expands.  Every factor is written as a polynomial (Chebyshev) or a
  rational function of exp(2K) and tanh K, so no branch of a square root or a
  logarithm is ever chosen.
* ``kaufman_lnZ(L, K)``: the closed form itself at real K.
* ``canonical(dos, values, beta, nsite)``: u = <E>/N and c = beta^2 Var/N from
  an exact density of states.

The Ising energy is E = -sum_<ij> s_i s_j (J = 1); bins E = -2N + 4k.
"""
from __future__ import annotations

import itertools
import math

import mpmath
import numpy as np


# --------------------------------------------------------------------------
# Brute force
# --------------------------------------------------------------------------
def _all_spins(N: int) -> np.ndarray:
    idx = np.arange(2 ** N, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(N, dtype=np.int64)[None, :]) & 1
    return (2 * bits - 1).astype(np.int8)


def ising_dos_bruteforce(L: int):
    """Returns (Omega_E, Omega_EM): Omega_E[k] for E = -2N + 4k (k = 0..N);
    Omega_EM[k, j] for M = -N + 2j."""
    N = L * L
    assert N <= 20
    s = _all_spins(N).reshape(-1, L, L).astype(np.int32)
    E = -(s * np.roll(s, -1, axis=2)).sum(axis=(1, 2)) - (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    M = s.sum(axis=(1, 2))
    k = (E + 2 * N) // 4
    j = (M + N) // 2
    om_e = np.bincount(k, minlength=N + 1).astype(object)
    om_em = np.zeros((N + 1, N + 1), dtype=np.int64)
    np.add.at(om_em, (k, j), 1)
    return om_e, om_em


def potts_dos_bruteforce(L: int, q: int):
    """Omega[E_unsat] for E_unsat = 0..2N, by enumeration of q^N states."""
    N = L * L
    assert q ** N <= 5 * 10 ** 7
    om = np.zeros(2 * N + 1, dtype=np.int64)
    chunk = q ** min(N, 10)
    rest = N - min(N, 10)
    low = np.array(list(itertools.product(range(q), repeat=min(N, 10))), dtype=np.int8)[:, ::-1]
    for hi_idx in range(q ** rest):
        hi = np.array([(hi_idx // q ** t) % q for t in range(rest)], dtype=np.int8)
        st = np.concatenate([low, np.broadcast_to(hi, (chunk, rest))], axis=1).reshape(-1, L, L)
        e = (st != np.roll(st, -1, axis=2)).sum(axis=(1, 2)) + (st != np.roll(st, -1, axis=1)).sum(axis=(1, 2))
        om += np.bincount(e, minlength=2 * N + 1)
    return om


# --------------------------------------------------------------------------
# Transfer matrix (exact integers)
# --------------------------------------------------------------------------
def ising_dos_transfer(L: int):
    """Omega[k], E = -2N + 4k, from Tr(T^L) with T[a][b] = x^(h(a) + v(a,b)),
    x counting unsatisfied bonds (h: within row a, v: between rows a and b)."""
    assert L <= 6
    S = 1 << L
    N = L * L
    a = np.arange(S)
    rot = ((a << 1) | (a >> (L - 1))) & (S - 1)
    h = np.array([bin(int(x)).count("1") for x in (a ^ rot)])
    v = np.array([[bin(int(x ^ y)).count("1") for y in a] for x in a])
    D = 2 * N + 1
    V = np.zeros((S, S, D), dtype=np.int64)  # V[start, state, degree]
    V[a, a, 0] = 1
    shift = h[:, None] + v  # cost of going from row state b to row state c
    for _ in range(L):
        Vn = np.zeros_like(V)
        for sft in range(int(shift.max()) + 1):
            Msk = (shift == sft).astype(np.int64)
            if not Msk.any():
                continue
            part = np.einsum("ibd,bc->icd", V, Msk)
            Vn[:, :, sft:] += part[:, :, :D - sft]
        V = Vn
    poly = V[a, a, :].sum(axis=0)  # trace
    assert all(poly[1::2] == 0)
    return [int(x) for x in poly[0::2]]


# --------------------------------------------------------------------------
# Kaufman closed form
# --------------------------------------------------------------------------
def _cheb_T(m, x):
    t0, t1 = mpmath.mpf(1), x
    if m == 0:
        return t0
    for _ in range(m - 1):
        t0, t1 = t1, 2 * x * t1 - t0
    return t1


def _cheb_U(m, x):
    u0, u1 = mpmath.mpf(1), 2 * x
    if m == 0:
        return u0
    for _ in range(m - 1):
        u0, u1 = u1, 2 * x * u1 - u0
    return u1


def _kaufman_Z(L: int, s, t):
    """Z of the L x L torus as a function of s = exp(2K) and t = tanh K.

    Z = 1/2 (2 sinh 2K)^(N/2) (Z1 + Z2 + Z3 + Z4), with
    cosh g_l = cosh 2K coth 2K - cos(pi l / L), and with m = L/2
      Z1 = prod_r 2 cosh(m g_(2r+1)) = prod_r 2 T_m(c_(2r+1))
      Z3 = prod_r 2 cosh(m g_(2r))   = prod_r 2 T_m(c_(2r))
      Z2 = prod_r 2 sinh(m g_(2r+1)) = prod_r 2 U_(m-1)(c_(2r+1)) sinh g_(2r+1)
      Z4 = prod_r 2 sinh(m g_(2r))   = prod_r 2 U_(m-1)(c_(2r))   sinh g_(2r)
    The sinh g_l pair up (l, 2L - l) into c_l^2 - 1; the unpaired g_0 =
    2K + ln tanh K and g_L = 2K - ln tanh K give
    sinh g_0 = (s t - 1/(s t))/2 and sinh g_L = (s/t - t/s)/2."""
    N = L * L
    m = L // 2
    sh2 = (s - 1 / s) / 2
    ch2 = (s + 1 / s) / 2
    cc = ch2 * ch2 / sh2
    c = [cc - mpmath.cos(mpmath.pi * l / L) for l in range(2 * L)]
    Z1 = mpmath.mpf(1)
    Z2 = mpmath.mpf(1)
    Z3 = mpmath.mpf(1)
    Z4 = mpmath.mpf(1)
    for r in range(L):
        Z1 *= 2 * _cheb_T(m, c[2 * r + 1])
        Z3 *= 2 * _cheb_T(m, c[2 * r])
        Z2 *= 2 * _cheb_U(m - 1, c[2 * r + 1])
        Z4 *= 2 * _cheb_U(m - 1, c[2 * r])
    for l in range(1, L, 2):
        Z2 *= c[l] * c[l] - 1
    for l in range(2, L, 2):
        Z4 *= c[l] * c[l] - 1
    Z4 *= (s * t - 1 / (s * t)) / 2
    Z4 *= (s / t - t / s) / 2
    return (2 * sh2) ** (N // 2) * (Z1 + Z2 + Z3 + Z4) / 2


def kaufman_lnZ(L: int, K, dps: int = 50):
    """ln Z at real coupling K > 0 (L even)."""
    with mpmath.workdps(dps):
        K = mpmath.mpf(K)
        return mpmath.log(_kaufman_Z(L, mpmath.exp(2 * K), mpmath.tanh(K)))


def ising_dos_kaufman(L: int):
    """Exact Omega[k] (E = -2N + 4k, k = 0..N) as Python ints, L even."""
    assert L % 2 == 0 and L >= 2
    N = L * L
    n = N + 1
    dps = int(0.31 * N) + 40
    with mpmath.workdps(dps):
        vals = []
        for j in range(n):
            # y = exp(-4K) on the unit circle, offset by half a step
            theta = (2 * mpmath.pi * j + mpmath.pi) / n
            y = mpmath.expj(theta)
            K = -mpmath.log(y) / 4
            s = mpmath.exp(2 * K)
            t = mpmath.tanh(K)
            vals.append(_kaufman_Z(L, s, t) * mpmath.exp(-2 * N * K))
        out = []
        for k in range(n):
            acc = mpmath.mpc(0)
            for j in range(n):
                theta = (2 * mpmath.pi * j + mpmath.pi) / n
                acc += vals[j] * mpmath.expj(-theta * k)
            coef = acc / n
            re = mpmath.re(coef)
            iv = int(mpmath.nint(re))
            if abs(re - iv) > mpmath.mpf("1e-6") or abs(mpmath.im(coef)) > mpmath.mpf("1e-6"):
                raise ArithmeticError(f"coefficient {k} not integral: {coef}")
            out.append(iv)
    return out


# --------------------------------------------------------------------------
# Canonical averages from an exact density of states
# --------------------------------------------------------------------------
def canonical(dos, values, beta: float, nsite: int, dps: int = 50):
    """u = <E>/N, c = beta^2 (<E^2> - <E>^2)/N with weights Omega e^{-beta E}."""
    with mpmath.workdps(dps):
        b = mpmath.mpf(beta)
        terms = [(mpmath.mpf(int(o)), mpmath.mpf(float(v))) for o, v in zip(dos, values) if int(o) > 0]
        emin = min(v for _, v in terms)
        Z = mpmath.fsum(o * mpmath.exp(-b * (v - emin)) for o, v in terms)
        E1 = mpmath.fsum(o * v * mpmath.exp(-b * (v - emin)) for o, v in terms) / Z
        E2 = mpmath.fsum(o * v * v * mpmath.exp(-b * (v - emin)) for o, v in terms) / Z
        return float(E1 / nsite), float(b * b * (E2 - E1 * E1) / nsite)


def ln_dos(dos) -> np.ndarray:
    """ln Omega as float64 (-inf where Omega = 0)."""
    return np.array([math.log(int(o)) if int(o) > 0 else -np.inf for o in dos])
