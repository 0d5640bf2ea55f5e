"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module only draws random numbers; it holds none of the Montgomery or
exponentiation arithmetic.  The paper measures on random operands only
(Section 6: random data sets), so these draws are the workload:

  * modulus: ``bits`` uniform bits, then the top bit and bit 0 set;
  * base: uniform in [0, N) by rejection on ``bits``-bit draws;
  * exponent: ``ebits`` uniform bits;
  * lazy Montgomery operands: uniform in [0, 2N);
  * RSA keys (CRT form) from pairs of seeded primes, e = 65537, messages uniform
    below p q (key preparation is input generation, not the method).

Streams: ``numpy.random.Generator(PCG64(SeedSequence(SEED_BASE + k)))`` for
workload k, with named sub-streams spawned from it.
"""
import math

import numpy as np

SEED_BASE = 2410181290
_STREAMS = {"moduli": 0, "bases": 1, "exps": 2, "ops_a": 3, "ops_b": 4, "arrivals": 5,
            "sizes": 6, "misc": 7, "primes": 8}


def stream(k, name):
    """Independent generator for workload index ``k`` and stream ``name``."""
    ss = np.random.SeedSequence(SEED_BASE + int(k))
    child = ss.spawn(len(_STREAMS))[_STREAMS[name]]
    return np.random.Generator(np.random.PCG64(child))


def _words(bits):
    return (bits + 63) // 64


def random_words(g, bits, count):
    """count x ceil(bits/64) uint64 words holding uniform ``bits``-bit values."""
    w = _words(bits)
    arr = g.integers(0, 2 ** 64, size=(count, w), dtype=np.uint64, endpoint=False)
    top = bits - 64 * (w - 1)
    if top < 64:
        arr[:, w - 1] &= np.uint64((1 << top) - 1)
    return arr


def words_to_ints(arr):
    arr = np.ascontiguousarray(arr, dtype=np.uint64)
    return [int.from_bytes(row.tobytes(), "little") for row in arr]


def ints_to_words(vals, words):
    out = np.zeros((len(vals), words), dtype=np.uint64)
    for i, v in enumerate(vals):
        if v < 0 or v.bit_length() > 64 * words:
            raise ValueError("value does not fit")
        out[i] = np.frombuffer(int(v).to_bytes(8 * words, "little"), dtype=np.uint64)
    return out


def random_moduli(g, bits, count):
    """Odd moduli with exactly ``bits`` bits (top bit and bit 0 forced)."""
    arr = random_words(g, bits, count)
    w = arr.shape[1]
    top = bits - 64 * (w - 1)
    arr[:, w - 1] |= np.uint64(1 << (top - 1))
    arr[:, 0] |= np.uint64(1)
    return arr


def random_below(g, mods_words, bits, scale=1):
    """Uniform values in [0, scale*N) per modulus, by rejection on (bits+scale-1)-bit draws."""
    mods = words_to_ints(mods_words)
    dbits = bits + (scale - 1).bit_length()
    out = []
    for N in mods:
        lim = scale * N
        while True:
            v = int.from_bytes(random_words(g, dbits, 1)[0].tobytes(), "little")
            if v < lim:
                out.append(v)
                break
    return out


def random_below_fast(g, mods_words, bits):
    """Vectorised rejection for large batches: uniform in [0, N) per row."""
    mods = np.ascontiguousarray(mods_words)
    count, w = mods.shape
    out = np.zeros_like(mods)
    todo = np.arange(count)
    while todo.size:
        cand = random_words(g, bits, todo.size)
        # lexicographic compare from the top word down
        less = np.zeros(todo.size, dtype=bool)
        decided = np.zeros(todo.size, dtype=bool)
        for i in range(w - 1, -1, -1):
            c, m = cand[:, i], mods[todo, i]
            lt = (c < m) & ~decided
            gt = (c > m) & ~decided
            less |= lt
            decided |= lt | gt
        out[todo[less]] = cand[less]
        todo = todo[~less]
    return out


def random_exponents(g, ebits, count):
    return random_words(g, ebits, count)


def _is_probable_prime(n, g, rounds=40):
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for _ in range(rounds):
        a = 2 + int.from_bytes(random_words(g, n.bit_length() - 2, 1)[0].tobytes(), "little") % (n - 3)
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = pow(x, 2, n)
            if x == n - 1:
                break
        else:
            return False
    return True


def gen_primes(count, bits, k=2):
    """``count`` probable primes of exactly ``bits`` bits (Miller-Rabin, 40 seeded rounds).

    Generation only: the primality test picks inputs, it is not checked against.
    """
    g = stream(k, "primes")
    out = []
    while len(out) < count:
        v = int.from_bytes(random_moduli(g, bits, 1)[0].tobytes(), "little")
        if _is_probable_prime(v, g):
            out.append(v)
    return out


def size_mix(g, count, classes=(1024, 2048, 3072, 4096), probs=(0.40, 0.35, 0.15, 0.10)):
    """i.i.d. size classes with the mixed-workload proportions."""
    idx = g.choice(len(classes), size=count, p=np.asarray(probs))
    return np.asarray(classes, dtype=np.int64)[idx]


def zipf_ranks(g, count, nitems, s=1.1):
    """Truncated Zipf(s) ranks in [0, nitems)."""
    w = 1.0 / np.arange(1, nitems + 1, dtype=np.float64) ** s
    w /= w.sum()
    return g.choice(nitems, size=count, p=w)


def poisson_arrivals(g, count, rate):
    """Arrival times (seconds) of a Poisson process with ``rate`` per second."""
    return np.cumsum(g.exponential(1.0 / rate, size=count))


def rsa_keys(primes, e=65537):
    """RSA keys in CRT form from consecutive pairs of distinct primes.

    Each key is a dict with p, q, n = p q, e, d = e^{-1} mod lcm(p-1, q-1),
    dp = d mod (p-1), dq = d mod (q-1) and qinv = q^{-1} mod p (the private
    key layout of PKCS #1).  A pair whose lcm(p-1, q-1) shares a factor with
    e is skipped.
    """
    keys = []
    for i in range(0, len(primes) - 1, 2):
        p, q = primes[i], primes[i + 1]
        if p == q:
            continue
        lam = (p - 1) * (q - 1) // math.gcd(p - 1, q - 1)
        if math.gcd(e, lam) != 1:
            continue
        d = pow(e, -1, lam)
        keys.append({"p": p, "q": q, "n": p * q, "e": e, "d": d, "dp": d % (p - 1), "dq": d % (q - 1),
                     "qinv": pow(q, -1, p)})
    return keys


def rsa_messages(g, keys, key_of):
    """One message per instance, uniform below the modulus of its key (key_of[i]), by rejection."""
    out = []
    for k in key_of:
        n = keys[int(k)]["n"]
        nb = n.bit_length()
        while True:
            v = int.from_bytes(random_words(g, nb, 1)[0].tobytes(), "little")
            if v < n:
                break
        out.append(v)
    return out


def load_primes(bits):
    """The committed seeded primes of tests/golden/primes_<bits>.txt (written by make_primes.py there)."""
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden",
                        "primes_%d.txt" % bits)
    with open(path) as f:
        return [int(l, 16) for l in f if l.strip() and not l.startswith("#")]
