"""Pins the oracle's spherical-rotation and double-bridging moves (the
paper's polymer move set): rotations keep every bond length, equal the
textbook rotation by 2 atan2(|a|, tau) about the stated axis, and are undone
by the mirrored word; a bridging move's energy change equals the recomputed
energy of the renumbered chain, and the move is its own inverse; over many
sweeps with all three moves the running energy stays the recomputed one."""
import math

import numpy as np
import pytest

from synth import PAPER_POLYMER, polymer_walk


def paper_run(orc, N, C=1, seed=5, moves=1, **kw):
    pp = dict(PAPER_POLYMER)
    pos = polymer_walk(N, C, seed, bond=pp["fene_r0"], min_dist=pp["lj_sigma"])
    params = dict(x_lo=-400.0, x_hi=100.0, n_bins=1000, lj_eps=pp["lj_eps"], lj_sigma=pp["lj_sigma"],
                  lj_rcut=pp["lj_rcut"], fene_k=pp["fene_k"], fene_r0=pp["fene_r0"], fene_R=pp["fene_R"],
                  step=pp["step"])
    params.update(kw)
    return orc.PolymerRun(n_beads=N, n_chains=C, seed=seed, pos=pos, moves=moves, **params)


def tau_of(word):
    u = ((word >> 8) - 8388607.5) / 8388608.0
    return u / (1.0 - abs(u))


def rodrigues(v, axis, phi):
    n = axis / np.linalg.norm(axis)
    return v * math.cos(phi) + np.cross(n, v) * math.sin(phi) + n * np.dot(n, v) * (1 - math.cos(phi))


def test_rotation_is_the_stated_rotation_and_keeps_bonds(orc):
    r = paper_run(orc, 12)
    x = r.pos[0].astype(np.float64)
    rng = np.random.default_rng(2)
    for _ in range(200):
        i = int(rng.integers(0, 12))
        w = rng.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32)
        xn = r.rotation(r.pos[0], i, w).astype(np.float64)
        tau = tau_of(int(w[0]))
        if 0 < i < 11:
            c, axis = x[i - 1], x[i + 1] - x[i - 1]
        else:
            c = x[1] if i == 0 else x[10]
            axis = np.zeros(3)
            axis[(int(w[1]) * 3) >> 32] = 1.0
        phi = 2.0 * math.atan2(np.linalg.norm(axis), tau)
        want = c + rodrigues(x[i] - c, axis, phi)
        assert np.max(np.abs(xn - want)) < 2e-6
        for nb in (i - 1, i + 1):
            if 0 <= nb < 12:
                assert abs(np.linalg.norm(xn - x[nb]) - np.linalg.norm(x[i] - x[nb])) < 2e-6


def test_mirrored_word_undoes_the_rotation(orc):
    r = paper_run(orc, 9)
    rng = np.random.default_rng(3)
    for _ in range(100):
        i = int(rng.integers(0, 9))
        w = rng.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32)
        xn = r.rotation(r.pos[0], i, w)
        moved = r.pos[0].copy()
        moved[i] = xn
        back = w.copy()
        back[0] = np.uint32(((2 ** 24 - 1 - (int(w[0]) >> 8)) << 8) | (int(w[0]) & 0xFF))
        assert tau_of(int(back[0])) == -tau_of(int(w[0]))
        xb = r.rotation(moved, i, back)
        assert np.max(np.abs(xb - r.pos[0][i])) < 2e-6


def test_bridging_energy_and_involution(orc):
    r = paper_run(orc, 20)
    x = r.pos[0].copy()
    rng = np.random.default_rng(4)
    done = 0
    for _ in range(400):
        w = rng.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32)
        got = r.bridging(x, w)
        i = (int(w[0]) * 19) >> 32
        j = (int(w[1]) * 19) >> 32
        i, j = min(i, j), max(i, j)
        if j - i < 2:
            assert got is None
            continue
        if got is None:  # a new bond outside the FENE domain
            y = x.copy()
            y[i + 1:j + 1] = x[i + 1:j + 1][::-1]
            assert r.energy(y) == math.inf
            continue
        dE, gi, gj = got
        assert (gi, gj) == (i, j)
        y = x.copy()
        y[i + 1:j + 1] = x[i + 1:j + 1][::-1]
        assert abs((r.energy(y) - r.energy(x)) - dE) < 1e-9 * max(1.0, abs(r.energy(x)))
        back = r.bridging(y, w)
        assert back is not None and back[1:] == (i, j) and abs(back[0] + dE) < 1e-9
        done += 1
    assert done >= 5  # new bonds must lie in the FENE domain: rare for an open walk


@pytest.mark.parametrize("N", [4, 13, 40])
def test_running_energy_with_all_moves(orc, N):
    r = paper_run(orc, N, C=3, seed=7)
    H = r.sweeps(60)
    assert int(H.sum()) == 3 * 60
    for c in range(3):
        e = r.energy(r.pos[c])
        assert math.isfinite(e) and abs(e - r.E[c]) < 1e-9 * max(1.0, abs(e))
        assert r.bin[c] == r.bin_of(r.E[c])


def test_full_move_set_changes_the_chain_differently(orc):
    """moves = 1 runs more proposals than the shift-only set (same seed,
    same shifts first), so the chains differ after a sweep."""
    a = paper_run(orc, 10, moves=0)
    b = paper_run(orc, 10, moves=1)
    a.sweeps(5)
    b.sweeps(5)
    assert not np.array_equal(a.pos, b.pos)
