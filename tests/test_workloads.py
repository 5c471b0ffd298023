"""Host-side workload definitions: sweeps from Eq. 4 and the seeded request stream;
the benchmark's one-GPU contract."""
import os
import numpy as np

from synth import WORKLOADS, m_opt, request_stream, sweeps_per_iteration


def test_m_opt_power_laws():
    assert abs(m_opt(64, 1) - 5.7 * 64 ** 2.51) < 1e-6
    assert abs(m_opt(16, 4, potts=True) - 24 * 16 ** 2.67 / 4) < 1e-6
    assert sweeps_per_iteration(16, 2048, True) == 20
    assert sweeps_per_iteration(48, 2048, True) == 362
    assert sweeps_per_iteration(32, 512, False) == 67
    assert sweeps_per_iteration(8, 4096, False) == 10


def test_request_stream_is_seeded_and_shaped():
    a = request_stream(200, 4.0, 4)
    b = request_stream(200, 4.0, 4)
    assert a == b and len(a) == 200
    t = np.array([r["arrival"] for r in a])
    assert np.all(np.diff(t) > 0) and 35 < t[-1] < 70
    for r in a:
        assert r["chains"] % 64 == 0 and 256 <= r["chains"] <= 2048
        if r["model"] == "ising":
            assert r["L"] in (16, 24, 32, 48, 64)
        else:
            assert r["q"] in (2, 4, 6, 8, 10) and r["L"] in (16, 32)
    assert {r["seed"] for r in a} == set(range(1000, 1200))


def test_workload_table():
    assert WORKLOADS["ising64_packed"]["chains"] == 4096
    inst = WORKLOADS["potts8_batched"]["instances"]
    assert sum(i["chains"] for i in inst if i["model"] == "potts") == 8192
    assert sum(i["chains"] for i in inst if i["model"] == "muma") == 2048


def test_served_requests_take_the_potts_law_for_q_at_least_3():
    """Potts bins are one per unit of unsatisfied bonds (about four times
    the Ising count for q >= 3): those requests take the 8-state Potts law."""
    import math
    from paper_1312_2213_amd.serve import Request
    r4 = Request(id=0, arrival=0.0, model="potts", L=32, q=4, chains=256, seed=1)
    assert r4.sweeps_per_iter == math.ceil(24 * 32 ** 2.67 / 256)
    r2 = Request(id=1, arrival=0.0, model="potts", L=32, q=2, chains=256, seed=1)
    assert r2.sweeps_per_iter == math.ceil(5.7 * 32 ** 2.51 / 256)
    ri = Request(id=2, arrival=0.0, model="ising", L=64, q=2, chains=2048, seed=1)
    assert ri.sweeps_per_iter == math.ceil(5.7 * 64 ** 2.51 / 2048)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with status 2 and
    a message before any device work (runs on the CPU)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=root)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""
