"""Seeded input generators (numpy PCG64)."""
from __future__ import annotations

import numpy as np


def polymer_walk(n_beads: int, n_chains: int, seed: int, bond: float = 1.0,
                 min_dist: float = 1.0, max_tries: int = 10000) -> np.ndarray:
    """Random-walk conformations [chain][bead][3] (float32): bonds of length
    `bond` with directions uniform on the sphere; a bond is re-drawn until the
    new bead is at least `min_dist` from every earlier non-bonded bead."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros((n_chains, n_beads, 3), np.float64)
    for c in range(n_chains):
        for k in range(1, n_beads):
            for _ in range(max_tries):
                v = rng.normal(size=3)
                v *= bond / np.linalg.norm(v)
                x = out[c, k - 1] + v
                if k < 2 or np.min(np.linalg.norm(out[c, :k - 1] - x, axis=1)) >= min_dist:
                    out[c, k] = x
                    break
            else:
                raise RuntimeError("could not place bead")
    return out.astype(np.float32)


def request_stream(n: int, rate: float, seed: int):
    """Poisson arrivals (exponential gaps, mean 1/rate) and per-request
    parameters: Ising with L in {16,24,32,48,64} or Potts with q in
    {2,4,6,8,10} and L in {16,32}, each with probability 1/2; chains uniform
    over the multiples of 64 in [256, 2048]; request k has seed 1000 + k."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    reqs = []
    for k in range(n):
        if rng.random() < 0.5:
            model, L, q = "ising", int(rng.choice([16, 24, 32, 48, 64])), 2
        else:
            model, q, L = "potts", int(rng.choice([2, 4, 6, 8, 10])), int(rng.choice([16, 32]))
        chains = int(64 * rng.integers(4, 33))
        reqs.append({"id": k, "arrival": float(t[k]), "model": model, "L": L, "q": q,
                     "chains": chains, "seed": 1000 + k})
    return reqs
