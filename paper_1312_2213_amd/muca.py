"""Thin Python binding of libmuca.so (include/muca.h): argument marshalling only.

Every step of the multicanonical path (initialisation, sweeps, histogram
merge, weight recursion, thresholds, reweighting) runs inside the native
library.  PyTorch supplies device memory (the workspace tensor) and streams.
Importing this module fails loudly if the HIP library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch first: its HIP runtime (libamdhip64.so.7) is then the one libmuca.so
# binds to, so the process never holds two HIP/HSA runtimes.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmuca.so")

MUCA_ISING, MUCA_POTTS, MUCA_MUMA, MUCA_POLYMER = 0, 1, 2, 3
MUCA_LAYOUT_AUTO, MUCA_LAYOUT_BIT, MUCA_LAYOUT_BYTE = 0, 1, 2
MUCA_ABI_VERSION = 3
MODELS = {"ising": MUCA_ISING, "potts": MUCA_POTTS, "muma": MUCA_MUMA, "polymer": MUCA_POLYMER}


class MucaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"muca error {code}: {msg}")
        self.code = code


class muca_config(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("model", ctypes.c_int32), ("L", ctypes.c_int32),
                ("q", ctypes.c_int32), ("n_chains", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("lo", ctypes.c_int32), ("hi", ctypes.c_int32),
                ("beta", ctypes.c_double), ("flat_threshold", ctypes.c_double),
                ("chains_per_block", ctypes.c_int32), ("table_in_lds", ctypes.c_int32),
                ("n_beads", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("x_lo", ctypes.c_double), ("x_hi", ctypes.c_double),
                ("lj_eps", ctypes.c_double), ("lj_sigma", ctypes.c_double), ("lj_rcut", ctypes.c_double),
                ("fene_k", ctypes.c_double), ("fene_r0", ctypes.c_double), ("fene_R", ctypes.c_double),
                ("step", ctypes.c_float), ("lanes_per_chain", ctypes.c_int32), ("chain0", ctypes.c_int32),
                ("moves", ctypes.c_int32)]


class muca_batch_tuning(ctypes.Structure):
    _fields_ = [("us_per_sweep", (ctypes.c_double * 2) * 2), ("lanes_per_chain", ctypes.c_int32),
                ("table_in_lds", ctypes.c_int32), ("from_cache", ctypes.c_int32), ("rejected", ctypes.c_int32)]

    def as_dict(self):
        return {"us_per_sweep": {f"{l}_lanes": {"global": self.us_per_sweep[o][0], "lds": self.us_per_sweep[o][1]}
                                 for o, l in ((0, 4), (1, 16))},
                "lanes_per_chain": self.lanes_per_chain, "table_in_lds": self.table_in_lds,
                "from_cache": bool(self.from_cache), "rejected": self.rejected}


class muca_iter_stats(ctypes.Structure):
    _fields_ = [("iteration", ctypes.c_int64), ("sweeps", ctypes.c_int64), ("samples", ctypes.c_int64),
                ("flatness", ctypes.c_double), ("flat", ctypes.c_int32), ("lo_visited", ctypes.c_int32),
                ("hi_visited", ctypes.c_int32), ("reserved", ctypes.c_int32), ("accept_rate", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(no CPU fallback exists)")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    vp, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
    sig = {
        "muca_config_default": (ctypes.c_int, [i32, i32, i32, i32, u64, P(muca_config)]),
        "muca_workspace_bytes": (ctypes.c_int, [P(muca_config), P(ctypes.c_uint64)]),
        "muca_init": (ctypes.c_int, [P(muca_config), vp, u64, vp, vp, P(vp)]),
        "muca_run_iteration": (ctypes.c_int, [vp, i64, vp]),
        "muca_thermalize": (ctypes.c_int, [vp, i64, vp]),
        "muca_merge_update": (ctypes.c_int, [vp, P(muca_iter_stats)]),
        "muca_merge_begin": (ctypes.c_int, [vp]),
        "muca_merge_finish": (ctypes.c_int, [vp, P(muca_iter_stats)]),
        "muca_get_pending_hist": (ctypes.c_int, [vp, vp, i64]),
        "muca_merge_update_hist": (ctypes.c_int, [vp, vp, i64, P(muca_iter_stats)]),
        "muca_reweight": (ctypes.c_int, [vp, vp, i32, vp]),
        "muca_blocks_shape": (ctypes.c_int, [vp, P(i32), P(i32)]),
        "muca_run_iteration_blocks": (ctypes.c_int, [vp, i64, vp, vp]),
        "muca_reweight_jackknife": (ctypes.c_int, [vp, vp, i32, vp, i32, vp, vp]),
        "muca_em_shape": (ctypes.c_int, [vp, P(i32), P(i32)]),
        "muca_run_iteration_em": (ctypes.c_int, [vp, i64, vp, vp]),
        "muca_reweight_em": (ctypes.c_int, [vp, vp, i64, vp, i32, vp]),
        "muca_batch_workspace_bytes": (ctypes.c_int, [i32, i32, P(ctypes.c_uint64)]),
        "muca_batch_create": (ctypes.c_int, [i32, i32, i32, i32, vp, u64, P(vp)]),
        "muca_batch_run_iteration": (ctypes.c_int, [vp, P(vp), i32, P(ctypes.c_int64), vp]),
        "muca_batch_free": (None, [vp]),
        "muca_batch_run_iteration_noalloc": (ctypes.c_int, [P(vp), i32, P(ctypes.c_int64), i32, vp]),
        "muca_batch_tune": (ctypes.c_int, [vp, i64, vp, P(muca_batch_tuning)]),
        "muca_autotune": (ctypes.c_int, [P(muca_config), vp, u64, i64, vp, P(muca_config), P(ctypes.c_double)]),
        "muca_sizes": (ctypes.c_int, [vp, P(i32), P(i32), P(i32)]),
        "muca_get_lnw": (ctypes.c_int, [vp, vp, i32]),
        "muca_get_last_hist": (ctypes.c_int, [vp, vp, i32]),
        "muca_get_thresholds": (ctypes.c_int, [vp, vp, i64]),
        "muca_get_chain_state": (ctypes.c_int, [vp, i32, i32, vp, vp, vp]),
        "muca_set_lnw": (ctypes.c_int, [vp, vp, i32]),
        "muca_set_thresholds": (ctypes.c_int, [vp, vp, i64]),
        "muca_checkpoint": (ctypes.c_int, [vp, vp, P(ctypes.c_uint64)]),
        "muca_restore": (ctypes.c_int, [vp, vp, u64]),
        "muca_free": (None, [vp]),
        "muca_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()
EXPORTED = ("muca_config_default", "muca_workspace_bytes", "muca_init", "muca_run_iteration",
            "muca_thermalize", "muca_merge_update", "muca_merge_begin", "muca_merge_finish",
            "muca_get_pending_hist", "muca_merge_update_hist",
            "muca_reweight", "muca_blocks_shape", "muca_run_iteration_blocks", "muca_reweight_jackknife",
            "muca_em_shape", "muca_run_iteration_em", "muca_reweight_em",
            "muca_batch_workspace_bytes",
            "muca_batch_create", "muca_batch_run_iteration", "muca_batch_free",
            "muca_batch_run_iteration_noalloc", "muca_batch_tune", "muca_autotune", "muca_sizes", "muca_get_lnw", "muca_get_last_hist",
            "muca_get_thresholds", "muca_get_chain_state", "muca_set_lnw", "muca_set_thresholds",
            "muca_checkpoint", "muca_restore", "muca_free", "muca_last_error")


def _check(rc: int):
    if rc != 0:
        raise MucaError(rc, LIB.muca_last_error().decode())


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def muca_config_default(model, L=0, q=2, n_chains=1, seed=0, **overrides) -> muca_config:
    cfg = muca_config()
    m = MODELS[model] if isinstance(model, str) else int(model)
    _check(LIB.muca_config_default(m, L, q, n_chains, seed, ctypes.byref(cfg)))
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg


def muca_workspace_bytes(cfg: muca_config) -> int:
    n = ctypes.c_uint64(0)
    _check(LIB.muca_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n)))
    return n.value


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Run:
    """One MUCA/MUMA/polymer instance; holds the workspace tensor alive."""

    def __init__(self, cfg: muca_config, positions: np.ndarray | None = None, stream=None,
                 device="cuda"):
        import torch
        self.cfg = cfg
        self.stream = stream
        self.batch_tuning = None  # set by batch_tune
        nbytes = muca_workspace_bytes(cfg)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._ws_ptr = ctypes.c_void_p(aligned)
        self._ws_bytes = nbytes
        self.handle = ctypes.c_void_p()
        pos_ptr = None
        if positions is not None:
            self._pos = np.ascontiguousarray(positions, np.float32)
            pos_ptr = _ptr(self._pos)
        _check(LIB.muca_init(ctypes.byref(cfg), self._ws_ptr, nbytes, pos_ptr,
                             _stream_handle(stream), ctypes.byref(self.handle)))
        nb, nc, ns = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(LIB.muca_sizes(self.handle, ctypes.byref(nb), ctypes.byref(nc), ctypes.byref(ns)))
        self.n_bins, self.n_cols, self.n_sites = nb.value, nc.value, ns.value

    # -- the hot path ------------------------------------------------------
    def run_iteration(self, sweeps: int, stream=None):
        _check(LIB.muca_run_iteration(self.handle, int(sweeps), _stream_handle(stream or self.stream)))

    def blocks_shape(self) -> tuple[int, int]:
        """(n_blocks, chains_per_block) of the per-block histograms."""
        nb, cpb = ctypes.c_int32(), ctypes.c_int32()
        _check(LIB.muca_blocks_shape(self.handle, ctypes.byref(nb), ctypes.byref(cpb)))
        return nb.value, cpb.value

    def run_iteration_blocks(self, sweeps: int, blocks, stream=None):
        """run_iteration that also adds each chain block's histogram to
        `blocks`, a contiguous 64-bit integer device tensor of n_blocks *
        n_bins entries (accumulated into, never cleared)."""
        import torch
        nb, _ = self.blocks_shape()
        if not (isinstance(blocks, torch.Tensor) and blocks.is_cuda and blocks.dtype in (torch.uint64, torch.int64)
                and blocks.is_contiguous() and blocks.numel() == nb * self.n_bins):
            raise ValueError(f"blocks must be a contiguous 64-bit integer CUDA tensor of {nb} x {self.n_bins}")
        _check(LIB.muca_run_iteration_blocks(self.handle, int(sweeps), ctypes.c_void_p(blocks.data_ptr()),
                                             _stream_handle(stream or self.stream)))

    def reweight_jackknife(self, h_blocks, betas=None):
        """(values, jackknife errors), each n x 4 as reweight(), from host
        block histograms recorded with the last merged iteration's weights."""
        h = np.ascontiguousarray(h_blocks, np.uint64)
        nb = h.size // self.n_bins
        b = np.ascontiguousarray(np.atleast_1d(betas if betas is not None else [0.0]), np.float64)
        out = np.zeros((len(b), 4), np.float64)
        err = np.zeros((len(b), 4), np.float64)
        _check(LIB.muca_reweight_jackknife(self.handle, _ptr(h), nb, _ptr(b), len(b), _ptr(out), _ptr(err)))
        return out, err

    def em_shape(self) -> tuple[int, int]:
        """(n_e, n_m) of the joint (E, M) histogram of a multimagnetic run."""
        ne, nm = ctypes.c_int32(), ctypes.c_int32()
        _check(LIB.muca_em_shape(self.handle, ctypes.byref(ne), ctypes.byref(nm)))
        return ne.value, nm.value

    def run_iteration_em(self, sweeps: int, em, stream=None):
        """run_iteration that also counts each sweep in `em`, a contiguous
        64-bit integer device tensor of em_shape() entries (accumulated into,
        never cleared; counts are read as uint64)."""
        import torch
        ne, nm = self.em_shape()
        if not (isinstance(em, torch.Tensor) and em.is_cuda and em.dtype in (torch.uint64, torch.int64)
                and em.is_contiguous() and em.numel() == ne * nm):
            raise ValueError(f"em must be a contiguous 64-bit integer CUDA tensor of {ne} x {nm}")
        _check(LIB.muca_run_iteration_em(self.handle, int(sweeps), ctypes.c_void_p(em.data_ptr()),
                                         _stream_handle(stream or self.stream)))

    def reweight_em(self, h_em, betas) -> np.ndarray:
        """Canonical averages at each beta' from a host joint histogram
        recorded with the last merged iteration's weights: rows of
        { <E>/N, beta'^2 Var(E)/N, <|M|>/N, <M^2>/N^2, beta' (<M^2> - <|M|>^2)/N, ln Z }."""
        h = np.ascontiguousarray(h_em, np.uint64)
        b = np.ascontiguousarray(np.atleast_1d(betas), np.float64)
        out = np.zeros((len(b), 6), np.float64)
        _check(LIB.muca_reweight_em(self.handle, _ptr(h), h.size, _ptr(b), len(b), _ptr(out)))
        return out

    def thermalize(self, sweeps: int, stream=None):
        _check(LIB.muca_thermalize(self.handle, int(sweeps), _stream_handle(stream or self.stream)))

    def merge_update(self) -> dict:
        st = muca_iter_stats()
        _check(LIB.muca_merge_update(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def merge_begin(self):
        """Enqueues the histogram read-back of the iteration (returns at once)."""
        _check(LIB.muca_merge_begin(self.handle))

    def merge_finish(self) -> dict:
        """Waits for the read-back only, then recursion and new thresholds."""
        st = muca_iter_stats()
        _check(LIB.muca_merge_finish(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def pending_hist(self) -> np.ndarray:
        """Histogram of the sweeps since the last merge (a shard's part)."""
        h = np.zeros(self.n_bins, np.uint64)
        _check(LIB.muca_get_pending_hist(self.handle, _ptr(h), len(h)))
        return h

    def merge_update_hist(self, h) -> dict:
        """Merge step with the histogram summed over all shards of a run."""
        h = np.ascontiguousarray(h, np.uint64)
        st = muca_iter_stats()
        _check(LIB.muca_merge_update_hist(self.handle, _ptr(h), len(h), ctypes.byref(st)))
        return st.as_dict()

    def reweight(self, betas) -> np.ndarray:
        b = np.ascontiguousarray(np.atleast_1d(betas), np.float64)
        out = np.zeros((len(b), 4), np.float64)
        _check(LIB.muca_reweight(self.handle, _ptr(b), len(b), _ptr(out)))
        return out

    # -- accessors -----------------------------------------------------------
    def lnw(self) -> np.ndarray:
        out = np.zeros(self.n_bins, np.float64)
        _check(LIB.muca_get_lnw(self.handle, _ptr(out), self.n_bins))
        return out

    def last_hist(self) -> np.ndarray:
        out = np.zeros(self.n_bins, np.uint64)
        _check(LIB.muca_get_last_hist(self.handle, _ptr(out), self.n_bins))
        return out

    def table_size(self) -> int:
        if self.cfg.model == MUCA_POLYMER:
            return self.n_bins * self.n_bins
        return self.n_bins * self.n_cols

    def thresholds(self) -> np.ndarray:
        out = np.zeros(self.table_size(), np.uint32)
        _check(LIB.muca_get_thresholds(self.handle, _ptr(out), out.size))
        return out

    def set_lnw(self, lnw):
        a = np.ascontiguousarray(lnw, np.float64)
        _check(LIB.muca_set_lnw(self.handle, _ptr(a), len(a)))

    def set_thresholds(self, t):
        a = np.ascontiguousarray(t, np.uint32)
        _check(LIB.muca_set_thresholds(self.handle, _ptr(a), a.size))

    def chain_state(self, chain0: int = 0, count: int | None = None):
        if count is None:
            count = self.cfg.n_chains - chain0
        bins = np.zeros(count, np.int32)
        energy = np.zeros(count, np.float64)
        if self.cfg.model == MUCA_POLYMER:
            state = np.zeros((count, self.cfg.n_beads, 3), np.float32)
        else:
            # Ising / MUMA spins +-1 (int8); Potts colours 0..q-1 (uint8)
            state = np.zeros((count, self.n_sites), np.uint8 if self.cfg.model == MUCA_POTTS else np.int8)
        _check(LIB.muca_get_chain_state(self.handle, chain0, count, _ptr(state), _ptr(bins), _ptr(energy)))
        return state, bins, energy

    def checkpoint(self) -> bytes:
        n = ctypes.c_uint64(0)
        _check(LIB.muca_checkpoint(self.handle, None, ctypes.byref(n)))
        buf = (ctypes.c_uint8 * n.value)()
        _check(LIB.muca_checkpoint(self.handle, ctypes.cast(buf, ctypes.c_void_p), ctypes.byref(n)))
        return bytes(buf)

    def restore(self, blob: bytes):
        buf = (ctypes.c_uint8 * len(blob)).from_buffer_copy(blob)
        _check(LIB.muca_restore(self.handle, ctypes.cast(buf, ctypes.c_void_p), len(blob)))

    def free(self):
        if self.handle:
            LIB.muca_free(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def batch_tune(run: Run, probe_sweeps: int = 0, stream=None) -> dict:
    """Measures (or reads from MUCA_AUTOTUNE_CACHE) one batched work item's
    time for each lanes-per-chain / table-placement candidate of the run's
    class; the run keeps it for later batched launches."""
    t = muca_batch_tuning()
    _check(LIB.muca_batch_tune(run.handle, int(probe_sweeps), _stream_handle(stream or run.stream), ctypes.byref(t)))
    run.batch_tuning = t.as_dict()
    return run.batch_tuning


class Batch:
    """Persistent batched launches over several lattice runs (workspace tensor
    kept alive).  autotune=True tunes every run's class (batch_tune) before
    its first batched launch, so that lanes per chain, table placement and
    the item order come from measured item times."""

    def __init__(self, max_runs: int, max_items: int = 8192, lanes_per_chain: int = 0,
                 use_graph: bool = True, device="cuda", autotune: bool = False):
        import torch
        self.autotune = autotune
        n = ctypes.c_uint64(0)
        _check(LIB.muca_batch_workspace_bytes(max_runs, max_items, ctypes.byref(n)))
        self.workspace = torch.empty(n.value + 256, dtype=torch.uint8, device=device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        self.handle = ctypes.c_void_p()
        _check(LIB.muca_batch_create(max_runs, max_items, lanes_per_chain, int(bool(use_graph)),
                                     ctypes.c_void_p(aligned), n.value, ctypes.byref(self.handle)))

    def run_iteration(self, runs, sweeps, stream=None):
        n = len(runs)
        if self.autotune:
            for r in runs:
                if r.batch_tuning is None:
                    batch_tune(r, stream=stream)
        handles = (ctypes.c_void_p * n)(*[r.handle.value for r in runs])
        sw = (ctypes.c_int64 * n)(*[int(s) for s in (sweeps if np.ndim(sweeps) else [sweeps] * n)])
        _check(LIB.muca_batch_run_iteration(self.handle, handles, n, sw, _stream_handle(stream)))

    def free(self):
        if self.handle:
            LIB.muca_batch_free(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


NOALLOC_MAX_RUNS, NOALLOC_MAX_ITEMS = 64, 4096


def batch_run_iteration_noalloc(runs, sweeps, lanes_per_chain: int = 0, stream=None):
    """One batched iteration of `runs` without a Batch (no workspace: the
    work queue lives in the library's own device array)."""
    n = len(runs)
    handles = (ctypes.c_void_p * n)(*[r.handle.value for r in runs])
    sw = (ctypes.c_int64 * n)(*[int(s) for s in (sweeps if np.ndim(sweeps) else [sweeps] * n)])
    _check(LIB.muca_batch_run_iteration_noalloc(handles, n, sw, int(lanes_per_chain), _stream_handle(stream)))


def muca_autotune(cfg: muca_config, sweeps: int, stream=None):
    """Fastest compiled variant of cfg (timed on the device); returns (config, ms per sweep)."""
    import torch
    big = muca_config.from_buffer_copy(cfg)
    if big.model in (MUCA_ISING, MUCA_MUMA) and big.layout == MUCA_LAYOUT_AUTO:
        big.layout = MUCA_LAYOUT_BYTE
    n = muca_workspace_bytes(big)
    ws = torch.empty(n + 256, dtype=torch.uint8, device="cuda")
    aligned = (ws.data_ptr() + 255) // 256 * 256
    best = muca_config()
    ms = ctypes.c_double(0.0)
    rc = LIB.muca_autotune(ctypes.byref(cfg), ctypes.c_void_p(aligned), n, int(sweeps),
                           _stream_handle(stream), ctypes.byref(best), ctypes.byref(ms))
    _check(rc)
    torch.cuda.synchronize()
    return best, ms.value
