"""The C-ABI library loads on the CPU and exports every symbol that
include/muca.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "muca.h")
LIB = os.path.join(ROOT, "paper_1312_2213_amd", "libmuca.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(muca_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("muca_init", "muca_run_iteration", "muca_merge_update", "muca_reweight",
              "muca_batch_run_iteration", "muca_free", "muca_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libmuca.so not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_exports():
    from paper_1312_2213_amd import muca
    assert set(declared()) <= set(muca.EXPORTED)


def test_host_only_calls_without_gpu():
    """Configuration helpers never touch the device."""
    from paper_1312_2213_amd import muca
    c = muca.muca_config_default("ising", 64, 2, 4096, 2)
    assert (c.lo, c.hi, c.flat_threshold) == (-8192, 8192, 0.5)
    n = muca.muca_workspace_bytes(c)
    assert n >= 64 * 2 * 4096 * 4 + 4097 * (5 * 4 + 8)
    bad = muca.muca_config_default("ising", 12, 2, 16, 1)
    with pytest.raises(muca.MucaError):
        muca.muca_workspace_bytes(bad)
    bad = muca.muca_config_default("ising", 8, 2, 16, 1, lo=-126)
    with pytest.raises(muca.MucaError):
        muca.muca_workspace_bytes(bad)
    # shards: chain0 numbers a run's chains inside a larger run; negative or
    # past the 31-bit chain numbering is rejected
    assert c.chain0 == 0 and c.abi_version == muca.MUCA_ABI_VERSION
    for chain0, ok in ((0, True), (4096, True), (-1, False), (0x7FFFFFFF - 15, False)):
        s = muca.muca_config_default("ising", 8, 2, 16, 1, chain0=chain0)
        if ok:
            assert muca.muca_workspace_bytes(s) > 0
        else:
            with pytest.raises(muca.MucaError):
                muca.muca_workspace_bytes(s)
    old = muca.muca_config_default("ising", 8, 2, 16, 1, abi_version=1)
    with pytest.raises(muca.MucaError):
        muca.muca_workspace_bytes(old)


def test_block_shapes_checked_on_the_host():
    """Blocks of 64 .. 512 threads (a power of two); 512 only beside a
    threshold table staged in LDS."""
    from paper_1312_2213_amd import muca
    for lpc, cpb, tlds, ok in ((16, 4, -1, True), (16, 32, 1, True), (4, 128, -1, True), (1, 512, 1, True),
                               (16, 32, 0, False), (16, 64, 1, False), (4, 48, 1, False), (1, 1024, 1, False)):
        c = muca.muca_config_default("ising", 64, 2, 8192, 2, lanes_per_chain=lpc, chains_per_block=cpb,
                                     table_in_lds=tlds)
        if ok:
            assert muca.muca_workspace_bytes(c) > 0
        else:
            with pytest.raises(muca.MucaError):
                muca.muca_workspace_bytes(c)
