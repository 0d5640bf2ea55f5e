"""Pins for the CPU oracle (oracle/bignum.c) against what mathematics fixes.

Each pin uses something other than the oracle's own formula: CPython's
bignum routines (``*``, ``%``, ``pow``), closed forms, identities, brute force
on tiny inputs, and Fermat's little theorem on generated primes.
"""
import random

import pytest

import oracle
from paper_2410_18129_amd import workload as wl

pytestmark = pytest.mark.filterwarnings("ignore")


def _rand(rng, bits):
    return rng.getrandbits(bits) if bits > 0 else 0


def test_mul_matches_python_multiply():
    rng = random.Random(1)
    cases = [(0, 0), (1, 1), (2**32 - 1, 2**32 - 1), (2**2048 - 1, 2**2048 - 1), (2**4096 - 1, 3)]
    for bits in (1, 31, 32, 33, 64, 100, 1024, 2048, 4096):
        cases.append((_rand(rng, bits), _rand(rng, bits + 17)))
    for a, b in cases:
        assert oracle.mul(a, b) == a * b


def test_mod_matches_python_remainder():
    rng = random.Random(2)
    for bits in (3, 32, 64, 65, 1024, 2048):
        N = _rand(rng, bits) | 1 | (1 << (bits - 1))
        for x in (0, 1, N - 1, N, N + 1, 2 * N, N * N - 1, _rand(rng, 2 * bits), _rand(rng, 3 * bits + 5)):
            assert oracle.mod(x, N) == x % N


def _redc_closed_form(T, N, r):
    R = 1 << r
    q = (-T * pow(N, -1, R)) % R
    return (T + q * N) >> r


def test_redc_matches_closed_form_and_identities():
    rng = random.Random(3)
    for bits, r in ((64, 84), (1024, 1036), (1024, 1056), (2048, 2072), (3072, 3080), (4096, 4116)):
        N = _rand(rng, bits) | 1 | (1 << (bits - 1))
        R = 1 << r
        Rinv = pow(R, -1, N)
        for T in (0, 1, N - 1, N, _rand(rng, 2 * bits), (2 * N - 1) ** 2, 2**bits, (2**bits) << 28):
            C = oracle.redc(T, N, r)
            assert C == _redc_closed_form(T, N, r)
            assert (C * R - T) % N == 0  # C = T R^-1 mod N
            assert C % N == (T * Rinv) % N
            if T < 4 * N * N and R >= 4 * N:
                assert C < 2 * N  # Algorithm 5's range without a final subtraction


def test_nprime_and_r2():
    rng = random.Random(4)
    for bits, r in ((64, 84), (1024, 1036), (2048, 2072), (4096, 4116)):
        N = _rand(rng, bits) | 1 | (1 << (bits - 1))
        R = 1 << r
        Np = oracle.nprime(N, r)
        assert 0 <= Np < R and (N * Np + 1) % R == 0
        assert oracle.r2(N, r) == pow(2, 2 * r, N)


def test_montmul_is_redc_of_product():
    rng = random.Random(5)
    N = _rand(rng, 1024) | 1 | (1 << 1023)
    r = 1036
    for _ in range(5):
        a, b = rng.randrange(2 * N), rng.randrange(2 * N)
        c = oracle.montmul(a, b, N, r)
        assert (c << r) % N == (a * b) % N and c < 2 * N


def test_modexp_matches_pow_and_special_cases():
    rng = random.Random(6)
    for bits in (64, 256, 1024):
        N = _rand(rng, bits) | 1 | (1 << (bits - 1))
        a = rng.randrange(N)
        e = _rand(rng, bits)
        assert oracle.modexp(a, e, N, bits) == pow(a, e, N)
        assert oracle.modexp(a, 0, N, bits) == 1  # e = 0 with leading zeros
        assert oracle.modexp(0, 0, N, 0) == 1  # 0^0 = 1
        assert oracle.modexp(0, e | 1, N, bits) == 0
        assert oracle.modexp(a, 1, N, bits) == a
        assert oracle.modexp(N - 1, 2 * (e >> 1), N, bits) == 1
        assert oracle.modexp(N - 1, (e >> 1) * 2 + 1, N, bits) == N - 1
        assert oracle.modexp(a, 2, N, 2) == (a * a) % N


def test_modexp_brute_force_tiny():
    """All odd N < 2^7, every base, e in 0..9 against repeated multiplication."""
    for N in range(3, 128, 2):
        for a in range(N):
            acc = 1 % N
            for e in range(10):
                assert oracle.modexp(a, e, N, 4) == acc
                acc = (acc * a) % N


def test_modexp_64bit_random():
    rng = random.Random(7)
    for _ in range(200):
        N = rng.getrandbits(64) | 1 | (1 << 63)
        a, e = rng.randrange(N), rng.getrandbits(64)
        assert oracle.modexp(a, e, N, 64) == pow(a, e, N)


def test_fermat_on_generated_primes(primes_1024):
    g = wl.stream(2, "bases")
    for p in primes_1024[:16]:
        a = 1 + wl.random_below(g, wl.ints_to_words([p - 1], 16), 1024)[0]
        assert oracle.modexp(a, p - 1, p, 1024) == 1


def test_exponent_addition():
    rng = random.Random(8)
    N = rng.getrandbits(512) | 1 | (1 << 511)
    x = rng.randrange(N)
    e1, e2 = rng.getrandbits(512), rng.getrandbits(512)
    lhs = oracle.modexp(x, e1 + e2, N, 513)  # exp_bits = t + 1
    rhs = (oracle.modexp(x, e1, N, 512) * oracle.modexp(x, e2, N, 512)) % N
    assert lhs == rhs


def test_oracle_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.redc(5, 4, 8)  # even modulus
    with pytest.raises(ValueError):
        oracle.nprime(10, 8)


def test_modexp_many_matches_single_calls_and_pow():
    """The batch helper behind the CPU baseline's timing computes the same values as one call per
    instance, with base, exponent and modulus strides that differ (na != nm, ebits not a limb multiple)."""
    import ctypes
    lib = oracle._load()
    rng = random.Random(9)
    count, na, nm, ebits = 5, 3, 4, 70
    ne = (ebits + 31) // 32
    mods = [rng.getrandbits(128) | 1 | (1 << 127) for _ in range(count)]
    bases = [rng.getrandbits(96) for _ in range(count)]
    exps = [rng.getrandbits(ebits) for _ in range(count)]
    exps[1] = 0
    A = (ctypes.c_uint32 * (count * na))()
    E = (ctypes.c_uint32 * (count * ne))()
    M = (ctypes.c_uint32 * (count * nm))()
    O = (ctypes.c_uint32 * (count * nm))()
    for k in range(count):
        for i in range(na):
            A[k * na + i] = (bases[k] >> (32 * i)) & 0xFFFFFFFF
        for i in range(ne):
            E[k * ne + i] = (exps[k] >> (32 * i)) & 0xFFFFFFFF
        for i in range(nm):
            M[k * nm + i] = (mods[k] >> (32 * i)) & 0xFFFFFFFF
    assert lib.ora_modexp_many(A, na, E, ebits, M, nm, O, count) == 0
    for k in range(count):
        got = oracle.from_limbs(O[k * nm:(k + 1) * nm])
        assert got == oracle.modexp(bases[k], exps[k], mods[k], ebits) == pow(bases[k], exps[k], mods[k]), k
    # the Python wrapper the CPU baseline calls (one limb count for bases and moduli)
    assert oracle.modexp_many(bases, exps, mods, ebits) == [pow(b, e, N) for b, e, N in zip(bases, exps, mods)]
