"""GPU parity of the CRT-RSA private-key operation (rsa_crt_batch) through the C ABI.

Expected values: the message m each ciphertext c = m^e mod n was made from
(CPython pow), i.e. c^d mod n by RSA's correctness, and the oracle's direct
c^d mod n (no CRT) on samples.  Bit-exact.
"""
import random

import pytest

import oracle
from paper_2410_18129_amd import workload as wl
from tests.gpu_util import dev_ints, ints_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_18129_amd import montexp
    montexp.lib()  # raises if the library is missing: no fallback
    return montexp


def _setup(mx, bits, count, seed, with_idx=True):
    import torch
    keys = wl.rsa_keys(wl.load_primes(bits))
    W = bits // 64
    ctx_p = mx.Context(wl.ints_to_words([k["p"] for k in keys], W), bits)
    ctx_q = mx.Context(wl.ints_to_words([k["q"] for k in keys], W), bits)
    rng = random.Random(seed)
    key_of = [rng.randrange(len(keys)) for _ in range(count)] if with_idx else list(range(count))
    ms = wl.rsa_messages(wl.stream(seed, "misc"), keys, key_of)
    # messages with zero residues and Garner's borrow: 0, 1, n - 1, multiples of p and of q
    specials = (lambda k: 0, lambda k: 1, lambda k: k["n"] - 1, lambda k: k["p"], lambda k: k["q"],
                lambda k: 2 * k["q"])
    for i, f in enumerate(specials[:count]):
        ms[i] = f(keys[key_of[i]])
    cs = [pow(m, keys[k]["e"], keys[k]["n"]) for m, k in zip(ms, key_of)]
    args = dict(
        c=ints_dev(cs, 2 * W), dp=ints_dev([keys[k]["dp"] for k in key_of], W),
        dq=ints_dev([keys[k]["dq"] for k in key_of], W), qinv=ints_dev([keys[k]["qinv"] for k in key_of], W),
        key_idx=torch.tensor(key_of, dtype=torch.int32, device="cuda") if with_idx else None)
    return keys, ctx_p, ctx_q, key_of, ms, cs, args


@pytest.mark.parametrize("variant", [{}, {"window": 5}, {"plain": True}, {"cios": True}])
def test_rsa2048_crt_matches_messages_and_oracle(mx, variant):
    count = 70  # one wavefront and a ragged tail
    keys, ctx_p, ctx_q, key_of, ms, cs, args = _setup(mx, 1024, count, 21)
    got = dev_ints(mx.rsa_crt(ctx_p, ctx_q, **args, **variant))
    assert got == ms
    for i in (0, 2, 3, 6, 69):  # the oracle's c^d mod n, no CRT
        k = keys[key_of[i]]
        assert got[i] == oracle.modexp(cs[i], k["d"], k["n"], 2048), i
    ctx_p.close()
    ctx_q.close()


def test_rsa2048_crt_without_key_index_and_in_place(mx):
    count = 32  # instance i uses key i
    keys, ctx_p, ctx_q, key_of, ms, cs, args = _setup(mx, 1024, count, 22, with_idx=False)
    c = args.pop("c")
    got = dev_ints(mx.rsa_crt(ctx_p, ctx_q, c, out=c, **args))  # out may alias c
    assert got == ms
    ctx_p.close()
    ctx_q.close()


def test_rsa4096_crt(mx):
    count = 6
    keys, ctx_p, ctx_q, key_of, ms, cs, args = _setup(mx, 2048, count, 23)
    got = dev_ints(mx.rsa_crt(ctx_p, ctx_q, **args))
    assert got == ms
    k = keys[key_of[count - 1]]
    assert got[count - 1] == oracle.modexp(cs[count - 1], k["d"], k["n"], 4096)
    ctx_p.close()
    ctx_q.close()


def test_rsa_crt_errors(mx):
    import torch
    keys = wl.rsa_keys(wl.load_primes(1024))
    ctx_p = mx.Context(wl.ints_to_words([k["p"] for k in keys], 16), 1024)
    z16 = torch.zeros((0, 16), dtype=torch.int64, device="cuda")
    z32 = torch.zeros((0, 32), dtype=torch.int64, device="cuda")
    mx.rsa_crt(ctx_p, ctx_p, z32, z16, z16, z16)  # n = 0 is a no-op
    m2 = wl.random_moduli(wl.stream(24, "moduli"), 2048, 1)
    ctx_big = mx.Context(m2, 2048)
    one16 = torch.zeros((1, 16), dtype=torch.int64, device="cuda")
    one32 = torch.zeros((1, 32), dtype=torch.int64, device="cuda")
    with pytest.raises(mx.MontError) as ei:  # p and q contexts of different classes
        mx.rsa_crt(ctx_p, ctx_big, one32, one16, one16, one16)
    assert ei.value.status == mx.MX_EINVAL
    with pytest.raises(mx.MontError) as ei:
        mx.rsa_crt(ctx_p, ctx_p, one32, one16, one16, one16, plain=True, cios=True)
    assert ei.value.status == mx.MX_EINVAL
    m3 = wl.random_moduli(wl.stream(24, "moduli"), 3072, 1)
    ctx3 = mx.Context(m3, 3072)
    one48 = torch.zeros((1, 48), dtype=torch.int64, device="cuda")
    one96 = torch.zeros((1, 96), dtype=torch.int64, device="cuda")
    with pytest.raises(mx.MontError) as ei:  # 3072-bit primes are not built
        mx.rsa_crt(ctx3, ctx3, one96, one48, one48, one48)
    assert ei.value.status == mx.MX_EUNSUPPORTED
    for c in (ctx_p, ctx_big, ctx3):
        c.close()
