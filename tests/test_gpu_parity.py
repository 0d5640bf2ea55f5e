"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Bit-exact (tolerance 0): every result of this library is an integer with a
unique correct value (Montgomery REDC with q in [0, R), canonical modexp).
"""
import random

import numpy as np
import pytest

import oracle
from paper_2410_18129_amd import workload as wl
from tests import oracle_pool
from tests.gpu_util import adversarial_pairs, dev_ints, ints_dev, r_bits

pytestmark = pytest.mark.gpu

CLASSES = (64, 128, 256, 512, 1024, 2048, 3072, 4096)


@pytest.fixture(scope="module")
def mx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_18129_amd import montexp
    montexp.lib()  # raises if the library is missing: no fallback
    return montexp


def _moduli(bits, count, k=1):
    return wl.random_moduli(wl.stream(k, "moduli"), bits, count)


def _redcs(bits):
    """Reductions built for a class: truncated (Algorithm 6), plain (Algorithm 3), the word-interleaved
    CIOS (Algorithm 4; above 2048 bits with 37-limb words) and, but for the odd block count of 3072 bits,
    the truncated high half of q*N formed by one-level Karatsuba (Section 5); as keyword arguments of the
    binding."""
    r = {"trunc": {}, "plain": {"plain": True}, "cios": {"cios": True}}
    if bits != 3072:  # the block classes need an even block count (4096: four blocks of 37 limbs)
        r["kara"] = {"kara_redc": True}
    return r


_mont_redcs = _redcs


@pytest.mark.parametrize("bits", CLASSES)
def test_context_constants(mx, bits):
    mods = _moduli(bits, 70)  # 70: one full wavefront and a ragged tail
    ctx = mx.Context(mods, bits)
    rb = r_bits(bits)
    assert ctx.r_bits == rb and ctx.count == 70
    Ns = wl.words_to_ints(mods)
    for i in (0, 1, 63, 64, 69):
        N = Ns[i]
        np_, r2, r1 = ctx.export(i)
        assert np_ == oracle.nprime(N, rb)
        assert r2 == oracle.r2(N, rb)
        assert r1 == oracle.mod(1 << rb, N)
    ctx.close()


@pytest.mark.parametrize("bits", CLASSES)
@pytest.mark.parametrize("count", [1, 67])
def test_mont_mul_sqr_random(mx, bits, count):
    g = wl.stream(3, "ops_a")
    mods = _moduli(bits, count, k=3)
    Ns = wl.words_to_ints(mods)
    ctx = mx.Context(mods, bits)
    rb = ctx.r_bits
    A = wl.random_below(g, mods, bits, scale=2)
    B = wl.random_below(g, mods, bits, scale=2)
    a, b = ints_dev(A, ctx.mont_words), ints_dev(B, ctx.mont_words)
    outs = {}
    redcs = _mont_redcs(bits)
    for r, kw in redcs.items():
        outs[("mul", r)] = dev_ints(mx.mont_mul(ctx, a, b, **kw))
        outs[("sqr", r)] = dev_ints(mx.mont_sqr(ctx, a, **kw))
    idx = range(count)
    for i in idx:
        exp_mul = oracle.montmul(A[i], B[i], Ns[i], rb)
        exp_sqr = oracle.montmul(A[i], A[i], Ns[i], rb)
        for r in redcs:
            assert outs[("mul", r)][i] == exp_mul, (i, r)
            assert outs[("sqr", r)][i] == exp_sqr, (i, r)
    # every reduction gives the same integer on every instance (Theorem 1; q in [0, R) is unique)
    for r in redcs:
        assert outs[("mul", r)] == outs[("mul", "trunc")], r
        assert outs[("sqr", r)] == outs[("sqr", "trunc")], r
    ctx.close()


@pytest.mark.parametrize("bits", CLASSES)
def test_mont_mul_adversarial(mx, bits):
    mods = _moduli(bits, 4, k=4)
    Ns = wl.words_to_ints(mods)
    # N - 1 and the largest odd modulus of the class stress the top limb
    Ns[2] = (1 << bits) - 1
    Ns[3] = (1 << (bits - 1)) + 1
    pairs = []
    for N in Ns:
        pairs += [(N, a, b) for a, b in adversarial_pairs(N, bits)]
    mods2 = wl.ints_to_words([p[0] for p in pairs], (bits + 63) // 64)
    ctx = mx.Context(mods2, bits)
    rb = ctx.r_bits
    a = ints_dev([p[1] for p in pairs], ctx.mont_words)
    b = ints_dev([p[2] for p in pairs], ctx.mont_words)
    for r, kw in _mont_redcs(bits).items():
        got = dev_ints(mx.mont_mul(ctx, a, b, **kw))
        gsq = dev_ints(mx.mont_sqr(ctx, a, **kw))
        for i, (N, x, y) in enumerate(pairs):
            assert got[i] == oracle.montmul(x, y, N, rb), (i, r)
            assert gsq[i] == oracle.montmul(x, x, N, rb), (i, r)
    ctx.close()


def test_mont_ctx_idx_indirection(mx):
    bits = 256
    mods = _moduli(bits, 5, k=5)
    Ns = wl.words_to_ints(mods)
    ctx = mx.Context(mods, bits)
    import torch
    rng = random.Random(5)
    n = 130
    ci = [rng.randrange(5) for _ in range(n)]
    A = [rng.randrange(2 * Ns[c]) for c in ci]
    B = [rng.randrange(2 * Ns[c]) for c in ci]
    cidx = torch.tensor(ci, dtype=torch.int32, device="cuda")
    got = dev_ints(mx.mont_mul(ctx, ints_dev(A, ctx.mont_words), ints_dev(B, ctx.mont_words), ctx_idx=cidx))
    for i in range(n):
        assert got[i] == oracle.montmul(A[i], B[i], Ns[ci[i]], ctx.r_bits)
    ctx.close()


def _random_inputs(bits):
    count = 8 if bits >= 1024 else 70
    mods = _moduli(bits, count, k=6)
    base = wl.random_below(wl.stream(6, "bases"), mods, bits)
    exps = wl.words_to_ints(wl.random_exponents(wl.stream(6, "exps"), bits, count))
    return mods, base, exps


def _random_jobs(bits):
    mods, base, exps = _random_inputs(bits)
    return [(b, e, N, bits) for b, e, N in zip(base, exps, wl.words_to_ints(mods))]


def _submit_random():
    for bits in (2048, 3072, 4096):  # the slow classes: every instance, by the oracle pool
        oracle_pool.submit(("random", bits), _random_jobs(bits))


ORACLE_JOBS = {"test_modexp_random": _submit_random}


@pytest.mark.parametrize("bits,window", [(64, 1), (64, 3), (128, 4), (256, 2), (512, 4), (1024, 5), (2048, 5),
                                         (2048, 3), (3072, 5), (4096, 6)])
def test_modexp_random(mx, bits, window):
    mods, base, exps = _random_inputs(bits)
    count = len(base)
    Ns = wl.words_to_ints(mods)
    ctx = mx.Context(mods, bits)
    bd = ints_dev(base, ctx.words)
    ed = ints_dev(exps, ctx.words)
    res = {}
    for r, kw in _redcs(bits).items():
        res[r] = dev_ints(mx.modexp(ctx, bd, ed, bits, window=window, **kw))
    for r in res:
        assert res[r] == res["trunc"], r
    if bits <= 1024:
        want = [oracle.modexp(base[i], exps[i], Ns[i], bits) for i in range(count)]
    else:
        want = oracle_pool.results(("random", bits), lambda: _random_jobs(bits))
    assert res["trunc"] == want
    ctx.close()


def test_modexp_brute_force_64bit(mx):
    """Every window size on 64-bit moduli: special bases and exponents against the oracle."""
    bits = 64
    rng = random.Random(64)
    Ns, B, E = [], [], []
    for _ in range(40):
        N = rng.getrandbits(64) | 1 | (1 << 63)
        for a in (0, 1, 2, N - 1, rng.randrange(N)):
            for e in (0, 1, 2, 3, 16, (1 << 64) - 1, 1 << 63, rng.getrandbits(64)):
                Ns.append(N), B.append(a), E.append(e)
    for N in range(3, 64, 2):  # tiny moduli, all bases
        for a in range(N):
            Ns.append(N), B.append(a), E.append(rng.getrandbits(64))
    ctx = mx.Context(wl.ints_to_words(Ns, 1), bits)
    bd, ed = ints_dev(B, 1), ints_dev(E, 1)
    for w, kw in ((1, {}), (2, {}), (4, {}), (5, {}), (8, {}), (1, {"cios": True}), (5, {"cios": True})):
        got = dev_ints(mx.modexp(ctx, bd, ed, 64, window=w, **kw))
        for i in range(len(Ns)):
            if i % 97 == 0:
                assert got[i] == oracle.modexp(B[i], E[i], Ns[i], 64), (i, w, kw)
            assert got[i] == pow(B[i], E[i], Ns[i]), (i, w, kw)
    ctx.close()


@pytest.mark.parametrize("bits", [256, 1024])
def test_modexp_edge_exponents(mx, bits):
    mods = _moduli(bits, 4, k=7)
    Ns = wl.words_to_ints(mods)
    ctx = mx.Context(mods, bits)
    W = ctx.words
    base = [0, 1, Ns[2] - 1, Ns[3] - 1]
    for ebits, e in ((0, 0), (1, 1), (2, 2), (bits, (1 << bits) - 1), (bits, 1 << (bits - 1)), (bits + 1, 1 << bits),
                     (bits + 1, (1 << (bits + 1)) - 1), (7, 0)):
        ew = max(1, (ebits + 63) // 64)
        ed = ints_dev([e] * 4, ew)
        got = dev_ints(mx.modexp(ctx, ints_dev(base, W), ed, ebits))
        for i in range(4):
            assert got[i] == oracle.modexp(base[i], e, Ns[i], ebits), (ebits, i)
    # bits above exp_bits are ignored
    ed = ints_dev([(1 << 40) | 5] * 4, 1)
    got = dev_ints(mx.modexp(ctx, ints_dev(base, W), ed, 3))
    for i in range(4):
        assert got[i] == pow(base[i], 5, Ns[i])
    ctx.close()


def test_modexp_fermat_primes(mx, primes_1024):
    ps = primes_1024
    g = wl.stream(2, "bases")
    base = [1 + v for v in wl.random_below(g, wl.ints_to_words([p - 1 for p in ps], 16), 1024)]
    ctx = mx.Context(wl.ints_to_words(ps, 16), 1024)
    got = dev_ints(mx.modexp(ctx, ints_dev(base, 16), ints_dev([p - 1 for p in ps], 16), 1024))
    assert all(v == 1 for v in got)
    got = dev_ints(mx.modexp(ctx, ints_dev(base, 16), ints_dev(ps, 16), 1024))  # a^p = a
    assert got == base
    ctx.close()


def test_modexp_exponent_addition(mx):
    bits = 512
    mods = _moduli(bits, 66, k=8)
    Ns = wl.words_to_ints(mods)
    rng = random.Random(8)
    x = [rng.randrange(N) for N in Ns]
    e1 = [rng.getrandbits(bits) for _ in Ns]
    e2 = [rng.getrandbits(bits) for _ in Ns]
    ctx = mx.Context(mods, bits)
    xd = ints_dev(x, ctx.words)
    r12 = dev_ints(mx.modexp(ctx, xd, ints_dev([a + b for a, b in zip(e1, e2)], 9), bits + 1))
    r1 = dev_ints(mx.modexp(ctx, xd, ints_dev(e1, 8), bits))
    r2 = dev_ints(mx.modexp(ctx, xd, ints_dev(e2, 8), bits))
    for i, N in enumerate(Ns):
        assert r12[i] == (r1[i] * r2[i]) % N
    ctx.close()


def test_errors_and_noops(mx):
    import torch
    with pytest.raises(mx.MontError) as ei:
        mx.Context(np.array([[10]], dtype=np.uint64), 64)
    assert ei.value.status == mx.MX_EINVAL
    ctx = mx.Context(np.array([[11]], dtype=np.uint64), 64)
    z = torch.zeros((0, ctx.mont_words), dtype=torch.int64, device="cuda")
    mx.mont_mul(ctx, z, z)  # n = 0 is a no-op
    a = torch.zeros((2, ctx.mont_words), dtype=torch.int64, device="cuda")
    with pytest.raises(ValueError):
        mx.mont_mul(ctx, a, a)  # n exceeds the context count without ctx_idx
    one = torch.zeros((1, 1), dtype=torch.int64, device="cuda")
    with pytest.raises(mx.MontError) as ei:
        mx.modexp(ctx, one, one, 8, window=9)
    assert ei.value.status == mx.MX_EINVAL
    with pytest.raises(ValueError):
        mx.modexp(ctx, one, one, 65)  # exponent tensor narrower than exp_bits
    # MX_REDC_PLAIN and MX_REDC_CIOS exclude each other
    with pytest.raises(mx.MontError) as ei:
        mx.mont_mul(ctx, a[:1], a[:1], plain=True, cios=True)
    assert ei.value.status == mx.MX_EINVAL
    with pytest.raises(mx.MontError) as ei:
        mx.modexp(ctx, one, one, 8, plain=True, cios=True)
    assert ei.value.status == mx.MX_EINVAL
    for kw in ({"one_lane": True, "two_lanes": True}, {"one_lane": True, "four_lanes": True},
               {"two_lanes": True, "four_lanes": True}):  # one lane choice at a time
        with pytest.raises(mx.MontError) as ei:
            mx.modexp(ctx, one, one, 8, **kw)
        assert ei.value.status == mx.MX_EINVAL, kw
    with pytest.raises(mx.MontError) as ei:  # one reduction at a time
        mx.mont_sqr(ctx, a[:1], cios=True, kara_redc=True)
    assert ei.value.status == mx.MX_EINVAL
    # the Karatsuba-truncated reduction excludes the other reductions
    import ctypes
    ob = torch.zeros((1, 1), dtype=torch.int64, device="cuda")
    assert mx.lib().modexp_batch(ctx.handle, None, ctypes.c_void_p(one.data_ptr()), ctypes.c_void_p(one.data_ptr()),
                                 8, 0, ctypes.c_void_p(ob.data_ptr()), 1, mx.MX_REDC_KARATSUBA | mx.MX_REDC_CIOS,
                                 None) == mx.MX_EINVAL
    ctx.close()
    # CIOS exists for the register-resident kernels and the block classes' one-lane kernels: not for the
    # block kernels of 2048 bits
    for bits, block in ((2048, True),):
        m = _moduli(bits, 1, k=8)
        c = mx.Context(m, bits)
        x = torch.zeros((1, c.mont_words), dtype=torch.int64, device="cuda")
        with pytest.raises(mx.MontError) as ei:
            mx.mont_sqr(c, x, cios=True, block=block)
        assert ei.value.status == mx.MX_EUNSUPPORTED
        if bits == 3072:  # an odd block count: no Karatsuba halves
            with pytest.raises(mx.MontError) as ei:
                mx.mont_mul(c, x, x, kara_redc=True, block=block)
            assert ei.value.status == mx.MX_EUNSUPPORTED
        xb = torch.zeros((1, c.words), dtype=torch.int64, device="cuda")
        e1 = torch.zeros((1, 1), dtype=torch.int64, device="cuda")
        with pytest.raises(mx.MontError) as ei:
            mx.modexp(c, xb, e1, 64, cios=True, block=block)
        assert ei.value.status == mx.MX_EUNSUPPORTED
        c.close()
    # the Karatsuba-truncated reduction and the block-word CIOS run one lane per instance
    c = mx.Context(_moduli(4096, 1, k=8), 4096)
    xe = torch.zeros((1, c.words), dtype=torch.int64, device="cuda")
    e1 = torch.zeros((1, 1), dtype=torch.int64, device="cuda")
    for red in ({"kara_redc": True}, {"cios": True}):
        for kw in ({"four_lanes": True}, {"two_lanes": True}):
            with pytest.raises(mx.MontError) as ei:
                mx.modexp(c, xe, e1, 64, **red, **kw)
            assert ei.value.status == mx.MX_EUNSUPPORTED, (red, kw)
    with pytest.raises(mx.MontError) as ei:  # no Karatsuba product with CIOS
        mx.mont_sqr(c, torch.zeros((1, c.mont_words), dtype=torch.int64, device="cuda"), cios=True,
                    block="karatsuba")
    assert ei.value.status == mx.MX_EUNSUPPORTED
    c.close()
