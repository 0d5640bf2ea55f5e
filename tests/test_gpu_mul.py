"""GPU: raw products (mp_mul_batch) -- schoolbook and Karatsuba at one and two levels -- against the
oracle's schoolbook product (Section 2; Section 3; Table 6's sizes: 4108 bits by schoolbook, 4154 by
Karatsuba, with limb counts that are not powers of two).  Bit-exact: a product is a unique integer."""
import random

import numpy as np
import pytest

import oracle
from paper_2410_18129_amd import workload as wl

pytestmark = pytest.mark.gpu

METHODS = ("schoolbook", "karatsuba", "karatsuba2")


@pytest.fixture(scope="module")
def mx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_18129_amd import montexp
    montexp.lib()  # raises if the library is missing: no fallback
    return montexp


def _operands(bits, n, seed):
    """Uniform bits-bit values, plus values that drive every carry: 0, 1, 2^bits - 1 (all-ones halves
    and quarters), the top bit alone, alternating limbs."""
    rng = random.Random(seed)
    top = (1 << bits) - 1
    special = [0, 1, top, 1 << (bits - 1), top ^ ((1 << (bits // 2)) - 1), int("10" * (bits // 2), 2) & top]
    xs = special + [rng.getrandbits(bits) for _ in range(n - len(special))]
    ys = special[::-1] + [rng.getrandbits(bits) for _ in range(n - len(special))]
    return xs, ys


@pytest.mark.parametrize("bits", [4108, 4154, 4096, 1000])
def test_products_match_oracle(mx, bits):
    import torch
    n = 200  # three tiles and a ragged tail
    xs, ys = _operands(bits, n, bits)
    W = (bits + 63) // 64
    a = torch.from_numpy(wl.ints_to_words(xs, W).view(np.int64)).cuda()
    b = torch.from_numpy(wl.ints_to_words(ys, W).view(np.int64)).cuda()
    want = [oracle.mul(x, y) for x, y in zip(xs, ys)]
    want_sq = [oracle.mul(x, x) for x in xs]
    for m in METHODS:
        got = wl.words_to_ints(mx.mp_mul(a, b, bits, method=m).cpu().numpy().view(np.uint64))
        assert got == want, (bits, m, next(i for i in range(n) if got[i] != want[i]))
        sq = wl.words_to_ints(mx.mp_mul(a, None, bits, method=m).cpu().numpy().view(np.uint64))
        assert sq == want_sq, (bits, m, "square")


def test_bits_above_the_operand_size_are_ignored(mx):
    import torch
    bits, n = 4108, 64
    xs, ys = _operands(bits, n, 7)
    W = (bits + 63) // 64
    junk = [v | (((1 << (64 * W - bits)) - 1) << bits) for v in xs]  # the unused top bits of the last word set
    a = torch.from_numpy(wl.ints_to_words(junk, W).view(np.int64)).cuda()
    b = torch.from_numpy(wl.ints_to_words(ys, W).view(np.int64)).cuda()
    for m in METHODS:
        got = wl.words_to_ints(mx.mp_mul(a, b, bits, method=m).cpu().numpy().view(np.uint64))
        assert got == [oracle.mul(x, y) for x, y in zip(xs, ys)], m


def test_small_workspace_runs_several_launches(mx):
    import torch
    bits, n = 4154, 300
    xs, ys = _operands(bits, n, 9)
    W = (bits + 63) // 64
    a = torch.from_numpy(wl.ints_to_words(xs, W).view(np.int64)).cuda()
    b = torch.from_numpy(wl.ints_to_words(ys, W).view(np.int64)).cuda()
    one_tile = mx.mp_mul_ws_bytes(bits, 64, "karatsuba2")
    ws = torch.empty(one_tile + 100, dtype=torch.uint8, device="cuda")  # holds one tile: five launches
    got = wl.words_to_ints(mx.mp_mul(a, b, bits, method="karatsuba2", ws=ws).cpu().numpy().view(np.uint64))
    assert got == [oracle.mul(x, y) for x, y in zip(xs, ys)]
    with pytest.raises(mx.MontError) as ei:
        mx.mp_mul(a, b, bits, ws=torch.empty(one_tile // 2, dtype=torch.uint8, device="cuda"))
    assert ei.value.status == mx.MX_EINVAL


@pytest.mark.parametrize("bits", [4108, 4154])
def test_full_size_16384_products(mx, bits):
    """The bench's launch: 16384 seeded instances; the three methods agree on every instance and the
    oracle checks every 16th instance (one per quarter tile)."""
    n = 16384
    g = wl.stream(3, "ops_a")
    a_w = wl.random_words(g, bits, n)
    b_w = wl.random_words(g, bits, n)
    a, b = mx.to_device(a_w), mx.to_device(b_w)
    outs = {m: mx.mp_mul(a, b, bits, method=m).cpu().numpy() for m in METHODS}
    assert np.array_equal(outs["schoolbook"], outs["karatsuba"])
    assert np.array_equal(outs["schoolbook"], outs["karatsuba2"])
    A, B = wl.words_to_ints(a_w[::16]), wl.words_to_ints(b_w[::16])
    got = wl.words_to_ints(outs["karatsuba2"][::16].view(np.uint64))
    assert got == [oracle.mul(x, y) for x, y in zip(A, B)]
