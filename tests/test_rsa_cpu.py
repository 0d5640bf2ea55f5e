"""RSA keys for the CRT-RSA workload and the oracle's private-key operation, on the CPU.

The GPU's rsa_crt_batch must return c^d mod p q; the oracle computes that
directly (square-and-multiply with bit-serial reduction, no CRT).  Pins:
textbook RSA correctness (m^(e d) = m mod n) with CPython's pow, the CRT key
layout, and the oracle against both.
"""
import random

import oracle
from paper_2410_18129_amd import workload as wl


def test_keys_have_the_crt_layout():
    for bits in (1024, 2048):
        ps = wl.load_primes(bits)
        assert all(p.bit_length() == bits for p in ps)
        keys = wl.rsa_keys(ps)
        assert len(keys) >= (8 if bits == 1024 else 3)
        for k in keys:
            p, q, e, d = k["p"], k["q"], k["e"], k["d"]
            assert p != q and k["n"] == p * q
            assert (e * d) % (p - 1) == 1 and (e * d) % (q - 1) == 1
            assert k["dp"] == d % (p - 1) and k["dq"] == d % (q - 1)
            assert (k["qinv"] * q) % p == 1 and 0 < k["qinv"] < p


def test_oracle_private_operation_inverts_encryption():
    keys = wl.rsa_keys(wl.load_primes(1024))
    rng = random.Random(7)
    for k in keys[:2]:
        n = k["n"]
        for m in (0, 1, n - 1, k["p"], k["q"], rng.randrange(n)):
            c = pow(m, k["e"], n)
            got = oracle.modexp(c, k["d"], n, 2048)
            assert got == m == pow(c, k["d"], n)
            # the CRT halves, as the GPU forms them
            m1 = pow(c % k["p"], k["dp"], k["p"])
            m2 = pow(c % k["q"], k["dq"], k["q"])
            h = (k["qinv"] * (m1 - m2)) % k["p"]
            assert m2 + h * k["q"] == m


def test_messages_are_below_their_modulus():
    keys = wl.rsa_keys(wl.load_primes(1024))
    key_of = [i % len(keys) for i in range(100)]
    ms = wl.rsa_messages(wl.stream(9, "misc"), keys, key_of)
    assert all(0 <= m < keys[k]["n"] for m, k in zip(ms, key_of))
    assert max(m.bit_length() for m in ms) == 2048
