"""GPU parity at the full sizes and in the launch configurations that bench.py times.

The inputs are the bench's own seeded inputs (the same generators and seeds).
Outputs are checked one by one against the oracle on samples, and on every
instance through properties that hold at any size:
- the truncated, plain and word-interleaved reductions give the same integers;
- the schoolbook and Karatsuba block kernels give the same integers;
- the persistent mixed launch, replayed from a HIP graph, gives what
  single-class launches give;
- RSA outputs m satisfy m^e = c (mod n).
Each modexp result is unique (canonical), so these comparisons are exact.
"""
import numpy as np
import pytest

import oracle
from paper_2410_18129_amd import workload as wl
from tests.gpu_util import dev_ints

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_18129_amd import montexp
    montexp.lib()  # raises if the library is missing: no fallback
    return montexp


def _batch(mx, bits, n, k):
    """The bench's inputs for one size class: seeded moduli, bases below N, bits-bit exponents."""
    mods = wl.random_moduli(wl.stream(k, "moduli"), bits, n)
    base = wl.random_below_fast(wl.stream(k, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(k, "exps"), bits, n)
    return mods, base, exps, mx.Context(mods, bits), mx.to_device(base), mx.to_device(exps)


def _row(arr, i):
    return wl.words_to_ints(np.ascontiguousarray(arr[i:i + 1]).view(np.uint64))[0]


def _oracle_check(out, mods, base, exps, bits, idx):
    for i in idx:
        assert _row(out, i) == oracle.modexp(_row(base, i), _row(exps, i), _row(mods, i), bits), (bits, i)


def test_headline_65536_x_2048_w5(mx):
    n, bits = 65536, 2048
    mods, base, exps, ctx, b, e = _batch(mx, bits, n, 2)
    res = {tag: mx.modexp(ctx, b, e, bits, window=5, **kw).cpu().numpy()
           for tag, kw in (("trunc", {}), ("plain", {"plain": True}), ("cios", {"cios": True}))}
    assert np.array_equal(res["trunc"], res["plain"])
    assert np.array_equal(res["trunc"], res["cios"])
    _oracle_check(res["trunc"], mods, base, exps, bits, (0, 32768, n - 1))
    ctx.close()


def test_16384_x_4096_w6_schoolbook_and_karatsuba(mx):
    n, bits = 16384, 4096
    mods, base, exps, ctx, b, e = _batch(mx, bits, n, 3)
    sb = mx.modexp(ctx, b, e, bits, window=6, block=True).cpu().numpy()
    ka = mx.modexp(ctx, b, e, bits, window=6, block="karatsuba").cpu().numpy()
    assert np.array_equal(sb, ka)
    _oracle_check(sb, mods, base, exps, bits, (n - 1,))
    ctx.close()


def test_mixed_200k_persistent_launch_from_graph(mx):
    import torch
    sizes = wl.size_mix(wl.stream(4, "sizes"), 200000)
    batches = []
    for c in (1024, 2048, 3072, 4096):
        n = int((sizes == c).sum())
        mods, base, exps, ctx, b, e = _batch(mx, c, n, 4 + c)
        batches.append({"ctx": ctx, "base": b, "exp": e, "exp_bits": c, "out": torch.zeros_like(b),
                        "window": 3 if c <= 2048 else 5, "host": (mods, base, exps)})
    plan = mx.MixedPlan([{k: v for k, v in bb.items() if k != "host"} for bb in batches])
    alone = {bb["exp_bits"]: mx.modexp(bb["ctx"], bb["base"], bb["exp"], bb["exp_bits"],
                                       window=bb["window"]).cpu().numpy() for bb in batches}
    for launch in range(2):  # the first call captures the graph, the second replays it
        for bb in batches:
            bb["out"].zero_()  # eager work between the launches
        plan.launch(graph=True)
        torch.cuda.synchronize()
        for bb in batches:
            assert np.array_equal(bb["out"].cpu().numpy(), alone[bb["exp_bits"]]), (launch, bb["exp_bits"])
    for bb in batches:
        c = bb["exp_bits"]
        got = alone[c]
        mods, base, exps = bb["host"]
        _oracle_check(got, mods, base, exps, c, (0, got.shape[0] - 1) if c <= 2048 else (got.shape[0] - 1,))
    plan.close()
    for bb in batches:
        bb["ctx"].close()


def test_rsa2048_crt_65536_operations(mx):
    import torch
    nr = 65536
    keys = wl.rsa_keys(wl.load_primes(1024))
    g = wl.stream(10, "misc")
    key_of = g.integers(0, len(keys), size=nr)
    cs = wl.rsa_messages(g, keys, key_of)
    ctx_p = mx.Context(wl.ints_to_words([k["p"] for k in keys], 16), 1024)
    ctx_q = mx.Context(wl.ints_to_words([k["q"] for k in keys], 16), 1024)

    def dev_words(vals, words):
        return torch.from_numpy(wl.ints_to_words(vals, words).view(np.int64)).to("cuda")

    out = mx.rsa_crt(ctx_p, ctx_q, dev_words(cs, 32), dev_words([keys[k]["dp"] for k in key_of], 16),
                     dev_words([keys[k]["dq"] for k in key_of], 16), dev_words([keys[k]["qinv"] for k in key_of], 16),
                     window=3, key_idx=torch.from_numpy(key_of.astype(np.int32)).to("cuda"))
    got = dev_ints(out)
    for i in range(nr):  # RSA: (c^d)^e = c (mod n)
        k = keys[key_of[i]]
        assert got[i] < k["n"] and pow(got[i], k["e"], k["n"]) == cs[i], i
    for i in (0, nr - 1):
        k = keys[key_of[i]]
        assert got[i] == oracle.modexp(cs[i], k["d"], k["n"], 2048), i
    ctx_p.close()
    ctx_q.close()
