"""Writes the exact density-of-states fixtures under tests/golden/ using only
oracle/exact.py.  Run: python tests/golden/make_golden.py

  ising_dos_L{8,16}.txt  Omega(E), E = -2N + 4k, from Kaufman's torus formula
                         (exact integers); pinned in the tests by brute force
                         and transfer matrix at small L and by closed forms.
  potts_q3_L4.txt        Omega(E_unsat), q = 3, L = 4, by enumeration.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact  # noqa: E402


def write(name, header, values):
    with open(os.path.join(HERE, name), "w") as f:
        f.write("# " + header + "\n")
        for v in values:
            f.write(f"{int(v)}\n")


if __name__ == "__main__":
    for L in (8, 16):
        write(f"ising_dos_L{L}.txt",
              f"2D Ising {L}x{L} torus, Omega(E) for E = -2N+4k, k = 0..N (N = {L * L}); "
              "Kaufman closed form, tests/golden/make_golden.py", exact.ising_dos_kaufman(L))
    write("potts_q3_L4.txt", "2D 3-state Potts 4x4 torus, Omega(E_unsat), E_unsat = 0..32; "
          "enumeration, tests/golden/make_golden.py", exact.potts_dos_bruteforce(4, 3))
