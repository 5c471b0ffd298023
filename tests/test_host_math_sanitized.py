"""The library's host-side arithmetic (reachable bins, thresholds, the
accumulated-statistics recursion, flatness, reweighting by Eq. 2 and its
joint (E, M) form) built on its own with AddressSanitizer and
UndefinedBehaviorSanitizer, run on seeded cases, and compared with the
oracle on the same inputs: masks and thresholds bit for bit, FP64 results
within 1e-12 relative.  CPU only."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1312_2213_amd", "csrc")
RTOL = 1e-12


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path_factory.mktemp("host_math") / "host_math_check"
    subprocess.check_call([gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "include"),
                           os.path.join(CSRC, "host_math.cpp"), os.path.join(CSRC, "host_math_check.cpp"),
                           "-o", str(exe)])
    return exe


def run(checker, tmp_path, text):
    cases = tmp_path / "cases.txt"
    cases.write_text(text)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([str(checker), str(cases)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
    return r.stdout.splitlines()


def hexs(a):
    return " ".join(float(x).hex() for x in np.asarray(a, np.float64).ravel())


def ints(a):
    return " ".join(str(int(x)) for x in np.asarray(a).ravel())


def floats(line):
    return np.array([float.fromhex(t) for t in line.split()])


def close(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return a.shape == b.shape and np.all(np.abs(a - b) <= RTOL * np.maximum(1.0, np.abs(b)))


LATTICES = [  # (model, L, q, beta)
    (orc.ISING, 8, 2, 0.0), (orc.ISING, 4, 2, 0.0), (orc.POTTS, 6, 3, 0.0), (orc.POTTS, 6, 2, 0.0),
    (orc.POTTS, 8, 8, 0.0), (orc.MUMA, 8, 2, 0.5), (orc.MUMA, 4, 2, 0.661),
]


def test_masks_and_thresholds_match_the_oracle(checker, tmp_path):
    rng = np.random.default_rng(11)
    text, expect = [], []
    for model, L, q, beta in LATTICES:
        o = orc.LatticeRun(model, L, 4, 1, q=q, beta=beta)
        B, NC = o.n_bins, o.n_cols
        step = {orc.ISING: 4, orc.POTTS: 1, orc.MUMA: 2}[model]
        text.append(f"mask {model} {q} {o.lo} {step} {L * L} {B}")
        expect.append(("mask", o.reachable()))
        # weights with steps of every size: always, never and partial acceptance
        for scale in (0.05, 1.0, 8.0):
            lnw = np.cumsum(rng.normal(0.0, scale, B))
            text.append(f"thresholds {model} {float(beta).hex()} {B} {NC} {hexs(lnw)}")
            expect.append(("T", o.thresholds(lnw)))
    out = run(checker, tmp_path, "\n".join(text) + "\n")
    assert len(out) == len(expect)
    for line, (kind, want) in zip(out, expect):
        got = np.array([int(t) for t in line.split()], np.uint64)
        assert np.array_equal(got, want.astype(np.uint64)), kind


def test_recursion_and_flatness_match_the_oracle(checker, tmp_path):
    rng = np.random.default_rng(12)
    text, expect = [], []
    for B in (1, 2, 7, 65, 300):
        for trial in range(4):
            H = rng.integers(0, 1000, B).astype(np.uint64)
            H[rng.random(B) < 0.2] = 0
            if trial == 3:
                H[:] = 0
            mask = (rng.random(B) < 0.9).astype(np.uint8)
            if trial == 2:
                mask[:] = 1
            lnR = rng.normal(0.0, 2.0, B) if trial else np.zeros(B)
            P = rng.random(B) * 50 if trial else np.zeros(B)
            text.append(f"recursion {B} {ints(mask)} {ints(H)} {hexs(lnR)} {hexs(P)}")
            expect.append(("rec", orc.recursion(H, lnR, P, mask)))
            text.append(f"flatness {B} {ints(mask)} {ints(H)}")
            expect.append(("flat", orc.flatness(H, mask)))
    out = run(checker, tmp_path, "\n".join(text) + "\n")
    assert len(out) == len(expect)
    for line, (kind, want) in zip(out, expect):
        got = floats(line)
        if kind == "rec":
            B = len(want[0])
            assert close(got[:B], want[0]) and close(got[B:2 * B], want[1]) and close(got[2 * B:], want[2])
        else:
            assert close(got, [want])


def test_reweighting_matches_the_oracle(checker, tmp_path):
    rng = np.random.default_rng(13)
    text, expect = [], []
    for model, L, q, beta in LATTICES:
        o = orc.LatticeRun(model, L, 4, 1, q=q, beta=beta)
        B, N = o.n_bins, L * L
        vals = orc.bin_values(model, L, o.lo, o.hi)
        muma = model == orc.MUMA
        for trial in range(3):
            H = rng.integers(0, 5000, B).astype(np.uint64)
            H[rng.random(B) < 0.3] = 0
            if trial == 2:
                H[:] = 0
                H[B // 2] = 7
            lnw = np.cumsum(rng.normal(0.0, 1.0, B))
            for b in ((beta,) if muma else (0.2, 0.44, 1.1)):
                text.append(f"reweight {B} {int(muma)} {N} {float(b).hex()} {ints(H)} {hexs(lnw)} {hexs(vals)}")
                expect.append(orc.reweight(H, lnw, vals, N, b, muma))
        if muma:
            NE = N + 1
            h = rng.integers(0, 50, (NE, B)).astype(np.uint64)
            h[rng.random((NE, B)) < 0.7] = 0
            for b2 in (beta * 0.9, beta, beta * 1.1):
                text.append(f"joint {NE} {B} {o.lo} 2 {N} {float(beta).hex()} {float(b2).hex()} {ints(h)} "
                            f"{hexs(lnw)}")
                expect.append(orc.reweight_em(h, lnw, L, o.lo, beta, [b2])[0])
    out = run(checker, tmp_path, "\n".join(text) + "\n")
    assert len(out) == len(expect)
    for line, want in zip(out, expect):
        assert close(floats(line), want), (line, want)


def test_checker_reports_malformed_input(checker, tmp_path):
    cases = tmp_path / "bad.txt"
    cases.write_text("recursion 3 1 1\n")
    r = subprocess.run([str(checker), str(cases)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "bad input" in r.stderr
