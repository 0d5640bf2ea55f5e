"""Writes primes_1024.txt: 64 seeded 1024-bit probable primes (Fermat-test moduli).

Inputs only (no expected values): drawn by the shared seeded generator and
kept by Miller-Rabin with 40 seeded rounds.  Run from the repository root:
    python tests/golden/make_primes.py
"""
import os
import sys

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
from paper_2410_18129_amd.workload import gen_primes  # noqa: E402

if __name__ == "__main__":
    ps = gen_primes(64, 1024, k=2)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "primes_1024.txt")
    with open(out, "w") as f:
        f.write("# 64 probable primes of 1024 bits, seeded (workload 2, stream 'primes'), one hex per line\n")
        for p in ps:
            f.write("%x\n" % p)
    print("wrote", out)
