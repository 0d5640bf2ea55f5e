"""Writes primes_1024.txt: 64 seeded 1024-bit probable primes (Fermat-test moduli, and the
primes of 32 RSA-2048 keys), and primes_2048.txt: 8 seeded 2048-bit probable primes (the
primes of 4 RSA-4096 keys).

Inputs only (no expected values): drawn by the shared seeded generator and
kept by Miller-Rabin with 40 seeded rounds.  Run from the repository root:
    python tests/golden/make_primes.py
"""
import os
import sys

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
from paper_2410_18129_amd.workload import gen_primes  # noqa: E402

def write(count, bits, k):
    ps = gen_primes(count, bits, k=k)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "primes_%d.txt" % bits)
    with open(out, "w") as f:
        f.write("# %d probable primes of %d bits, seeded (workload %d, stream 'primes'), one hex per line\n"
                % (count, bits, k))
        for p in ps:
            f.write("%x\n" % p)
    print("wrote", out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["1024", "2048"]
    if "1024" in which:
        write(64, 1024, 2)
    if "2048" in which:
        write(8, 2048, 3)
