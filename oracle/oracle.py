"""CPU oracle for parallel multicanonical simulations (arXiv:1312.2213).

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``; never by the library.

This module is a thin ctypes wrapper around ``muca_oracle.c`` (plain C,
single-threaded, FP64) plus the iteration driver written out in the paper's
order (parallel-scheme paragraph and Fig. 1 caption):

  1. p realisations start with the same weights W^(0) (lnW = 0);
  2. each runs M sweeps and fills its histogram;
  3. the histograms are merged into H^(n);
  4. the accumulated-statistics recursion gives W^(n+1), which all
     realisations use in the next iteration;
  5. repeat until the distribution is flat.

Thermalisation happens only before the first iteration (paper, paragraph on
thermalisation); chains carry their state across iterations.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "muca_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ISING, POTTS, MUMA = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, portable ISA)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Lattice(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("L", ctypes.c_int32), ("q", ctypes.c_int32),
                ("n_chains", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("lo", ctypes.c_int32), ("hi", ctypes.c_int32), ("beta", ctypes.c_double)]


class _Polymer(ctypes.Structure):
    _fields_ = [("n_beads", ctypes.c_int32), ("n_chains", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("x_lo", ctypes.c_double), ("x_hi", ctypes.c_double),
                ("n_bins", ctypes.c_int32), ("lj_eps", ctypes.c_double),
                ("lj_sigma", ctypes.c_double), ("lj_rcut", ctypes.c_double),
                ("fene_k", ctypes.c_double), ("fene_r0", ctypes.c_double),
                ("fene_R", ctypes.c_double), ("step", ctypes.c_float), ("moves", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        u32p, i32p, i8p = P(ctypes.c_uint32), P(ctypes.c_int32), P(ctypes.c_int8)
        u64p, f64p, u8p, f32p = P(ctypes.c_uint64), P(ctypes.c_double), P(ctypes.c_uint8), P(ctypes.c_float)
        L.orc_philox.argtypes = [u32p, ctypes.c_uint64, u32p]
        L.orc_nbins.argtypes = [P(_Lattice)]
        L.orc_nbins.restype = ctypes.c_int32
        L.orc_ncols.argtypes = [ctypes.c_int32]
        L.orc_ncols.restype = ctypes.c_int32
        L.orc_reachable.argtypes = [P(_Lattice), u8p]
        L.orc_measure.argtypes = [P(_Lattice), i8p, i32p, i32p]
        L.orc_init_lattice.argtypes = [P(_Lattice), i8p, i32p, i32p]
        L.orc_threshold.argtypes = [ctypes.c_double]
        L.orc_threshold.restype = ctypes.c_uint32
        L.orc_thresholds.argtypes = [P(_Lattice), f64p, u32p]
        L.orc_sweeps.argtypes = [P(_Lattice), i8p, i32p, i32p, u32p, ctypes.c_uint32,
                                 ctypes.c_int64, ctypes.c_int, u64p, ctypes.c_int32, ctypes.c_int32]
        L.orc_sweeps.restype = ctypes.c_int
        L.orc_sweeps_acc.argtypes = [P(_Lattice), i8p, i32p, i32p, u32p, ctypes.c_uint32,
                                     ctypes.c_int64, ctypes.c_int, u64p, u64p, ctypes.c_int32, ctypes.c_int32]
        L.orc_sweeps_acc.restype = ctypes.c_int
        L.orc_polymer_sweeps_acc.argtypes = [P(_Polymer), f32p, f64p, i32p, f64p, ctypes.c_uint32,
                                             ctypes.c_int64, ctypes.c_int, u64p, u64p, ctypes.c_int32,
                                             ctypes.c_int32]
        L.orc_polymer_sweeps_acc.restype = ctypes.c_int
        L.orc_sweeps_em.argtypes = [P(_Lattice), i8p, i32p, i32p, u32p, ctypes.c_uint32,
                                    ctypes.c_int64, ctypes.c_int, u64p, u64p, ctypes.c_int32, ctypes.c_int32]
        L.orc_sweeps_em.restype = ctypes.c_int
        L.orc_reweight_em.argtypes = [ctypes.c_int32, ctypes.c_int32, u64p, f64p, f64p, f64p, ctypes.c_int32,
                                      ctypes.c_double, ctypes.c_double, f64p]
        L.orc_reweight_em.restype = None
        L.orc_recursion.argtypes = [ctypes.c_int32, u8p, u64p, f64p, f64p, f64p]
        L.orc_flatness.argtypes = [ctypes.c_int32, u8p, u64p]
        L.orc_flatness.restype = ctypes.c_double
        L.orc_reweight.argtypes = [ctypes.c_int32, u64p, f64p, f64p, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_double, f64p]
        L.orc_polymer_energy.argtypes = [P(_Polymer), f32p, P(ctypes.c_int)]
        L.orc_polymer_energy.restype = ctypes.c_double
        L.orc_polymer_bin.argtypes = [P(_Polymer), ctypes.c_double]
        L.orc_polymer_bin.restype = ctypes.c_int32
        L.orc_polymer_init.argtypes = [P(_Polymer), f32p, f64p, i32p]
        L.orc_polymer_init.restype = ctypes.c_int
        L.orc_polymer_rotation.argtypes = [P(_Polymer), f32p, ctypes.c_int32, u32p, f32p]
        L.orc_polymer_rotation.restype = None
        L.orc_polymer_bridging.argtypes = [P(_Polymer), f32p, u32p, P(ctypes.c_double), P(ctypes.c_int32),
                                           P(ctypes.c_int32)]
        L.orc_polymer_bridging.restype = ctypes.c_int
        L.orc_polymer_sweeps.argtypes = [P(_Polymer), f32p, f64p, i32p, f64p, ctypes.c_uint32,
                                         ctypes.c_int64, ctypes.c_int, u64p, ctypes.c_int32,
                                         ctypes.c_int32]
        L.orc_polymer_sweeps.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# --------------------------------------------------------------------------
# Philox4x32-10
# --------------------------------------------------------------------------
def philox(ctr, seed: int) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox(_ptr(c, ctypes.c_uint32), ctypes.c_uint64(seed), _ptr(out, ctypes.c_uint32))
    return out


def threshold(D: float) -> int:
    return int(lib().orc_threshold(ctypes.c_double(D)))


# --------------------------------------------------------------------------
# Lattice MUCA / MUMA
# --------------------------------------------------------------------------
def default_range(model: int, L: int, q: int = 2):
    N = L * L
    if model == ISING:
        return -2 * N, 2 * N
    if model == POTTS:
        return 0, 2 * N
    return -N, N


def bin_values(model: int, L: int, lo: int, hi: int) -> np.ndarray:
    """Physical value of each bin: Ising E, Potts E = E_unsat - 2N (J = 1), MUMA M."""
    N = L * L
    if model == ISING:
        return np.arange(lo, hi + 1, 4, dtype=np.float64)
    if model == POTTS:
        return np.arange(lo, hi + 1, 1, dtype=np.float64) - 2 * N
    return np.arange(lo, hi + 1, 2, dtype=np.float64)


@dataclass
class LatticeRun:
    """One MUCA/MUMA instance: p chains, one shared weight table."""
    model: int
    L: int
    n_chains: int
    seed: int
    q: int = 2
    lo: int | None = None
    hi: int | None = None
    beta: float = 0.0
    sweep: int = 0                      # global sweep counter g
    iteration: int = 0
    spins: np.ndarray = field(default=None, repr=False)
    E: np.ndarray = field(default=None, repr=False)
    M: np.ndarray = field(default=None, repr=False)
    lnW: np.ndarray = field(default=None, repr=False)
    lnR: np.ndarray = field(default=None, repr=False)
    P: np.ndarray = field(default=None, repr=False)
    H: np.ndarray = field(default=None, repr=False)

    def __post_init__(self):
        d_lo, d_hi = default_range(self.model, self.L, self.q)
        if self.lo is None:
            self.lo = d_lo
        if self.hi is None:
            self.hi = d_hi
        self._c = _Lattice(self.model, self.L, self.q, self.n_chains, self.seed,
                           self.lo, self.hi, self.beta)
        B = self.n_bins
        N = self.L * self.L
        # Potts colours 0..q-1 are unsigned bytes; Ising / MUMA spins are +-1
        self.spins = np.zeros((self.n_chains, N), np.uint8 if self.model == POTTS else np.int8)
        self.E = np.zeros(self.n_chains, np.int32)
        self.M = np.zeros(self.n_chains, np.int32)
        lib().orc_init_lattice(ctypes.byref(self._c), _ptr(self.spins, ctypes.c_int8),
                               _ptr(self.E, ctypes.c_int32), _ptr(self.M, ctypes.c_int32))
        self.lnW = np.zeros(B, np.float64)
        self.lnR = np.zeros(B, np.float64)
        self.P = np.zeros(B, np.float64)
        self.H = np.zeros(B, np.uint64)
        self.accepted = 0  # accepted moves of recorded sweeps since the last take_accepted()

    def take_accepted(self) -> int:
        n, self.accepted = self.accepted, 0
        return n

    @property
    def n_bins(self) -> int:
        return int(lib().orc_nbins(ctypes.byref(self._c)))

    @property
    def n_cols(self) -> int:
        return int(lib().orc_ncols(self.model))

    def reachable(self) -> np.ndarray:
        m = np.zeros(self.n_bins, np.uint8)
        lib().orc_reachable(ctypes.byref(self._c), _ptr(m, ctypes.c_uint8))
        return m

    def bins(self) -> np.ndarray:
        step = {ISING: 4, POTTS: 1, MUMA: 2}[self.model]
        v = self.M if self.model == MUMA else self.E
        return (v - self.lo) // step

    def thresholds(self, lnW: np.ndarray | None = None) -> np.ndarray:
        lw = np.ascontiguousarray(self.lnW if lnW is None else lnW, np.float64)
        T = np.zeros(self.n_bins * self.n_cols, np.uint32)
        lib().orc_thresholds(ctypes.byref(self._c), _ptr(lw, ctypes.c_double), _ptr(T, ctypes.c_uint32))
        return T

    def sweeps(self, n: int, T: np.ndarray | None = None, record: bool = True,
               chains: tuple[int, int] | None = None, H: np.ndarray | None = None) -> np.ndarray:
        """Run n sweeps of chains [c0, c1) with thresholds T; returns the histogram."""
        if T is None:
            T = self.thresholds()
        T = np.ascontiguousarray(T, np.uint32)
        c0, c1 = (0, self.n_chains) if chains is None else chains
        if H is None:
            H = np.zeros(self.n_bins, np.uint64)
        acc = np.zeros(1, np.uint64)
        rc = lib().orc_sweeps_acc(ctypes.byref(self._c), _ptr(self.spins, ctypes.c_int8),
                                  _ptr(self.E, ctypes.c_int32), _ptr(self.M, ctypes.c_int32),
                                  _ptr(T, ctypes.c_uint32), ctypes.c_uint32(self.sweep & 0xffffffff),
                                  ctypes.c_int64(n), int(record), _ptr(H, ctypes.c_uint64),
                                  _ptr(acc, ctypes.c_uint64), c0, c1)
        self.accepted += int(acc[0])
        if rc != 0:
            raise RuntimeError("oracle chain left the binned range")
        return H

    def advance(self, n: int):
        self.sweep += n

    @property
    def em_shape(self) -> tuple[int, int]:
        """Joint (E, M) histogram of a multimagnetic run: rows e = 0..N for
        E = -2N + 4e, columns the magnetisation bins."""
        return self.L * self.L + 1, self.n_bins

    def sweeps_em(self, n: int, HEM: np.ndarray, T: np.ndarray | None = None,
                  H: np.ndarray | None = None) -> np.ndarray:
        """sweeps() of a MUMA run that also adds each sweep's (E, M bin) to HEM."""
        if T is None:
            T = self.thresholds()
        T = np.ascontiguousarray(T, np.uint32)
        if H is None:
            H = np.zeros(self.n_bins, np.uint64)
        assert HEM.dtype == np.uint64 and HEM.shape == self.em_shape and HEM.flags.c_contiguous
        rc = lib().orc_sweeps_em(ctypes.byref(self._c), _ptr(self.spins, ctypes.c_int8),
                                 _ptr(self.E, ctypes.c_int32), _ptr(self.M, ctypes.c_int32),
                                 _ptr(T, ctypes.c_uint32), ctypes.c_uint32(self.sweep & 0xffffffff),
                                 ctypes.c_int64(n), 1, _ptr(H, ctypes.c_uint64), _ptr(HEM, ctypes.c_uint64),
                                 0, self.n_chains)
        if rc != 0:
            raise RuntimeError("not a multimagnetic run" if rc == -2 else "oracle chain left the binned range")
        return H

    def reweight_em(self, HEM, lnW, betas) -> np.ndarray:
        """Canonical averages at each beta' from the joint histogram of
        sweeps run with weights lnW: rows of { <E>/N, beta'^2 Var(E)/N,
        <|M|>/N, <M^2>/N^2, beta' (<M^2> - <|M|>^2)/N, ln Z }."""
        return reweight_em(HEM, lnW, self.L, self.lo, self.beta, betas)

    def merge_update(self, H: np.ndarray) -> float:
        """Accumulated-statistics recursion on the merged histogram; returns flatness."""
        H = np.ascontiguousarray(H, np.uint64)
        mask = self.reachable()
        f = float(lib().orc_flatness(self.n_bins, _ptr(mask, ctypes.c_uint8), _ptr(H, ctypes.c_uint64)))
        lib().orc_recursion(self.n_bins, _ptr(mask, ctypes.c_uint8), _ptr(H, ctypes.c_uint64),
                            _ptr(self.lnR, ctypes.c_double), _ptr(self.P, ctypes.c_double),
                            _ptr(self.lnW, ctypes.c_double))
        self.H = H.copy()
        self.iteration += 1
        return f

    def iterate(self, n_sweeps: int) -> tuple[np.ndarray, float, np.ndarray]:
        """One MUCA iteration; returns (H^(n), flatness of H^(n), lnW^(n) used)."""
        lnw_used = self.lnW.copy()
        H = self.sweeps(n_sweeps)
        self.advance(n_sweeps)
        f = self.merge_update(H)
        return H, f, lnw_used

    def reweight(self, H, lnW, betas) -> np.ndarray:
        v = bin_values(self.model, self.L, self.lo, self.hi)
        H = np.ascontiguousarray(H, np.uint64)
        lnW = np.ascontiguousarray(lnW, np.float64)
        out = np.zeros((len(betas), 4), np.float64)
        for k, b in enumerate(betas):
            o = np.zeros(4, np.float64)
            lib().orc_reweight(self.n_bins, _ptr(H, ctypes.c_uint64), _ptr(lnW, ctypes.c_double),
                               _ptr(v, ctypes.c_double), self.L * self.L, int(self.model == MUMA),
                               ctypes.c_double(self.beta if self.model == MUMA else b),
                               _ptr(o, ctypes.c_double))
            out[k] = o
        return out


def recursion(H, lnR, P, mask):
    """Standalone recursion step (returns new lnR, P, lnW)."""
    H = np.ascontiguousarray(H, np.uint64)
    lnR = np.array(lnR, np.float64)
    P = np.array(P, np.float64)
    mask = np.ascontiguousarray(mask, np.uint8)
    lnW = np.zeros(len(H), np.float64)
    lib().orc_recursion(len(H), _ptr(mask, ctypes.c_uint8), _ptr(H, ctypes.c_uint64),
                        _ptr(lnR, ctypes.c_double), _ptr(P, ctypes.c_double), _ptr(lnW, ctypes.c_double))
    return lnR, P, lnW


def flatness(H, mask) -> float:
    H = np.ascontiguousarray(H, np.uint64)
    mask = np.ascontiguousarray(mask, np.uint8)
    return float(lib().orc_flatness(len(H), _ptr(mask, ctypes.c_uint8), _ptr(H, ctypes.c_uint64)))


def reweight(H, lnW, values, nsite, beta, muma=False):
    H = np.ascontiguousarray(H, np.uint64)
    lnW = np.ascontiguousarray(lnW, np.float64)
    v = np.ascontiguousarray(values, np.float64)
    o = np.zeros(4, np.float64)
    lib().orc_reweight(len(H), _ptr(H, ctypes.c_uint64), _ptr(lnW, ctypes.c_double),
                       _ptr(v, ctypes.c_double), nsite, int(muma), ctypes.c_double(beta),
                       _ptr(o, ctypes.c_double))
    return o


def reweight_jackknife(H_blocks, lnW, values, nsite, betas, muma=False):
    """Reweighted averages (Eq. 2, as reweight()) over the sum of the block
    histograms, and their jackknife errors: with v_k the values when block k
    is left out, over the m blocks that hold any count,
    err = sqrt((m - 1) / m * sum_k (v_k - mean_k v_k)^2).  Returns (values,
    errors), each len(betas) x 4."""
    Hb = np.asarray(H_blocks, np.uint64)
    used = [k for k in range(Hb.shape[0]) if Hb[k].sum() > 0]
    H = Hb.sum(axis=0, dtype=np.uint64)
    m = len(used)
    vals = np.zeros((len(betas), 4))
    errs = np.zeros((len(betas), 4))
    for q, beta in enumerate(betas):
        vals[q] = reweight(H, lnW, values, nsite, beta, muma)
        v = np.array([reweight(H - Hb[k], lnW, values, nsite, beta, muma) for k in used])
        mean = v.sum(axis=0) / m
        errs[q] = np.sqrt((m - 1.0) / m * ((v - mean) ** 2).sum(axis=0))
    return vals, errs


def reweight_em(HEM, lnW, L, lo, beta, betas) -> np.ndarray:
    """orc_reweight_em over the rows E = -2N + 4e and the columns
    M = lo + 2b of a multimagnetic run at inverse temperature beta."""
    N = L * L
    HEM = np.ascontiguousarray(HEM, np.uint64)
    lnW = np.ascontiguousarray(lnW, np.float64)
    NE, B = HEM.shape
    Ev = -2.0 * N + 4.0 * np.arange(NE, dtype=np.float64)
    Mv = lo + 2.0 * np.arange(B, dtype=np.float64)
    out = np.zeros((len(betas), 6), np.float64)
    for k, b2 in enumerate(betas):
        o = np.zeros(6, np.float64)
        lib().orc_reweight_em(NE, B, _ptr(HEM, ctypes.c_uint64), _ptr(lnW, ctypes.c_double),
                              _ptr(Ev, ctypes.c_double), _ptr(Mv, ctypes.c_double), N,
                              ctypes.c_double(beta), ctypes.c_double(b2), _ptr(o, ctypes.c_double))
        out[k] = o
    return out


# --------------------------------------------------------------------------
# Bead-spring polymer
# --------------------------------------------------------------------------
@dataclass
class PolymerRun:
    n_beads: int
    n_chains: int
    seed: int
    pos: np.ndarray                     # [chain][bead][3] float32 (copied)
    x_lo: float = -200.0
    x_hi: float = 50.0
    n_bins: int = 2500
    lj_eps: float = 1.0
    lj_sigma: float = 1.0
    lj_rcut: float = 2.5
    fene_k: float = 40.0
    fene_r0: float = 1.0
    fene_R: float = 0.5
    step: float = 0.3
    moves: int = 0                      # 1: shift + spherical rotation + double bridging
    sweep: int = 0
    iteration: int = 0

    def __post_init__(self):
        self._c = _Polymer(self.n_beads, self.n_chains, self.seed, self.x_lo, self.x_hi,
                           self.n_bins, self.lj_eps, self.lj_sigma, self.lj_rcut, self.fene_k,
                           self.fene_r0, self.fene_R, self.step, self.moves)
        self.pos = np.ascontiguousarray(self.pos, np.float32).reshape(
            self.n_chains, self.n_beads, 3).copy()
        self.E = np.zeros(self.n_chains, np.float64)
        self.bin = np.zeros(self.n_chains, np.int32)
        rc = lib().orc_polymer_init(ctypes.byref(self._c), _ptr(self.pos, ctypes.c_float),
                                    _ptr(self.E, ctypes.c_double), _ptr(self.bin, ctypes.c_int32))
        if rc != 0:
            raise ValueError("initial conformation outside the energy range")
        self.lnW = np.zeros(self.n_bins, np.float64)
        self.lnR = np.zeros(self.n_bins, np.float64)
        self.P = np.zeros(self.n_bins, np.float64)
        self.visited = np.zeros(self.n_bins, np.uint8)
        self.accepted = 0

    def energy(self, pos_one) -> float:
        """Total energy of one conformation [bead][3] (any number of beads)."""
        p = np.ascontiguousarray(pos_one, np.float32)
        c = _Polymer.from_buffer_copy(self._c)
        c.n_beads = p.shape[0]
        br = ctypes.c_int(0)
        e = lib().orc_polymer_energy(ctypes.byref(c), _ptr(p, ctypes.c_float), ctypes.byref(br))
        return float("inf") if br.value else float(e)

    def bin_of(self, E: float) -> int:
        return int(lib().orc_polymer_bin(ctypes.byref(self._c), ctypes.c_double(E)))

    def rotation(self, pos_one, i: int, words) -> np.ndarray:
        """The spherical-rotation proposal of bead i of one conformation."""
        p = np.ascontiguousarray(pos_one, np.float32)
        w = np.ascontiguousarray(words, np.uint32)
        out = np.zeros(3, np.float32)
        lib().orc_polymer_rotation(ctypes.byref(self._c), _ptr(p, ctypes.c_float), i, _ptr(w, ctypes.c_uint32),
                                   _ptr(out, ctypes.c_float))
        return out

    def bridging(self, pos_one, words):
        """The double-bridging proposal of one conformation: (dE, i, j) or None."""
        p = np.ascontiguousarray(pos_one, np.float32)
        w = np.ascontiguousarray(words, np.uint32)
        dE, i, j = ctypes.c_double(), ctypes.c_int32(), ctypes.c_int32()
        ok = lib().orc_polymer_bridging(ctypes.byref(self._c), _ptr(p, ctypes.c_float), _ptr(w, ctypes.c_uint32),
                                        ctypes.byref(dE), ctypes.byref(i), ctypes.byref(j))
        return (dE.value, i.value, j.value) if ok else None

    def sweeps(self, n: int, record: bool = True, chains=None, H=None):
        c0, c1 = (0, self.n_chains) if chains is None else chains
        if H is None:
            H = np.zeros(self.n_bins, np.uint64)
        acc = np.zeros(1, np.uint64)
        lib().orc_polymer_sweeps_acc(ctypes.byref(self._c), _ptr(self.pos, ctypes.c_float),
                                     _ptr(self.E, ctypes.c_double), _ptr(self.bin, ctypes.c_int32),
                                     _ptr(self.lnW, ctypes.c_double),
                                     ctypes.c_uint32(self.sweep & 0xffffffff), ctypes.c_int64(n),
                                     int(record), _ptr(H, ctypes.c_uint64), _ptr(acc, ctypes.c_uint64), c0, c1)
        self.accepted += int(acc[0])
        return H

    def take_accepted(self) -> int:
        n, self.accepted = self.accepted, 0
        return n

    def advance(self, n: int):
        self.sweep += n

    def merge_update(self, H) -> float:
        """Recursion over all bins; flatness over the bins visited so far."""
        H = np.ascontiguousarray(H, np.uint64)
        self.visited |= (H > 0).astype(np.uint8)
        f = flatness(H, self.visited)
        ones = np.ones(self.n_bins, np.uint8)
        lnW = np.zeros(self.n_bins, np.float64)
        lib().orc_recursion(self.n_bins, _ptr(ones, ctypes.c_uint8), _ptr(H, ctypes.c_uint64),
                            _ptr(self.lnR, ctypes.c_double), _ptr(self.P, ctypes.c_double),
                            _ptr(lnW, ctypes.c_double))
        self.lnW = lnW
        self.iteration += 1
        return f

    def bin_centres(self) -> np.ndarray:
        w = (self.x_hi - self.x_lo) / self.n_bins
        return self.x_lo + w * (np.arange(self.n_bins) + 0.5)
