"""GPU parity at the full sizes and in the launch configurations that bench.py times.

The inputs are the bench's own seeded inputs (the same generators and seeds).
Outputs are checked one by one against the oracle on samples that reach every
tile of each launch (tests/oracle_pool.py: tile t contributes the instance at
lane t mod 64, so the lane positions are covered too), and on every instance
through properties that hold at any size:
- the truncated, plain and word-interleaved reductions give the same integers;
- the schoolbook and Karatsuba block kernels give the same integers;
- the persistent mixed launch, replayed from a HIP graph, gives what
  single-class launches give;
- RSA outputs m satisfy m^e = c (mod n).
Each modexp result is unique (canonical), so these comparisons are exact.
The oracle's values are computed by the worker pool while earlier tests run.
"""
import functools

import numpy as np
import pytest

from paper_2410_18129_amd import workload as wl
from tests import oracle_pool
from tests.gpu_util import dev_ints

pytestmark = pytest.mark.gpu

HEADLINE = (65536, 2048, 2)          # instances, bits, workload seed index
C3 = (16384, 4096, 3)
MIXED_N = 200000
RSA_N = 65536


@pytest.fixture(scope="module")
def mx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_18129_amd import montexp
    montexp.lib()  # raises if the library is missing: no fallback
    return montexp


@functools.lru_cache(maxsize=None)
def _host(bits, n, k):
    """The bench's inputs for one size class: seeded moduli, bases below N, bits-bit exponents."""
    mods = wl.random_moduli(wl.stream(k, "moduli"), bits, n)
    base = wl.random_below_fast(wl.stream(k, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(k, "exps"), bits, n)
    return mods, base, exps


def _row(arr, i):
    return wl.words_to_ints(np.ascontiguousarray(arr[i:i + 1]).view(np.uint64))[0]


def _jobs(bits, n, k, idx):
    mods, base, exps = _host(bits, n, k)
    return [(_row(base, i), _row(exps, i), _row(mods, i), bits) for i in idx]


def _headline_idx():
    n = HEADLINE[0]
    return oracle_pool.spread(n, n // 64)  # one instance in every wavefront's tile


def _c3_idx():
    return oracle_pool.spread(C3[0], 256)


@functools.lru_cache(maxsize=None)
def _mixed_counts():
    sizes = wl.size_mix(wl.stream(4, "sizes"), MIXED_N)
    return {c: int((sizes == c).sum()) for c in (1024, 2048, 3072, 4096)}


def _mixed_idx(c):
    """Oracle samples of the mixed launch: every 64-instance tile of the 1024-bit batch, every second
    tile of the 2048-bit batch, 256 instances spread over the tiles of the 3072- and 4096-bit batches."""
    n = _mixed_counts()[c]
    tiles = (n + 63) // 64
    count = {1024: tiles, 2048: (tiles + 1) // 2}.get(c, 256)
    return oracle_pool.spread(n, count, salt=c // 1024)


@functools.lru_cache(maxsize=None)
def _rsa_inputs():
    keys = wl.rsa_keys(wl.load_primes(1024))
    g = wl.stream(10, "misc")
    key_of = g.integers(0, len(keys), size=RSA_N)
    return keys, key_of, wl.rsa_messages(g, keys, key_of)


def _rsa_idx():
    return oracle_pool.spread(RSA_N, 64, salt=5)


def _rsa_jobs():
    keys, key_of, cs = _rsa_inputs()
    return [(cs[i], keys[key_of[i]]["d"], keys[key_of[i]]["n"], 2048) for i in _rsa_idx()]


def _submit_headline():
    oracle_pool.submit("headline", _jobs(HEADLINE[1], HEADLINE[0], HEADLINE[2], _headline_idx()))


def _submit_c3():
    oracle_pool.submit("c3", _jobs(C3[1], C3[0], C3[2], _c3_idx()))


def _submit_mixed():
    for c, n in _mixed_counts().items():
        oracle_pool.submit(("mixed", c), _jobs(c, n, 4 + c, _mixed_idx(c)))


ORACLE_JOBS = {
    "test_headline_65536_x_2048_w5": _submit_headline,
    "test_16384_x_4096_w6_schoolbook_and_karatsuba": _submit_c3,
    "test_mixed_200k_persistent_launch_from_graph": _submit_mixed,
    "test_rsa2048_crt_65536_operations": lambda: oracle_pool.submit("rsa", _rsa_jobs()),
}


def _oracle_check(out, key, idx, jobs_fn, what):
    want = oracle_pool.results(key, jobs_fn)
    assert len(want) == len(idx)
    bad = [i for i, v in zip(idx, want) if _row(out, i) != v]
    assert not bad, "%s: %d of %d oracle samples differ, first at instance %d" % (what, len(bad), len(idx), bad[0])


def test_headline_65536_x_2048_w5(mx):
    n, bits, k = HEADLINE
    mods, base, exps = _host(bits, n, k)
    ctx = mx.Context(mods, bits)
    b, e = mx.to_device(base), mx.to_device(exps)
    res = {tag: mx.modexp(ctx, b, e, bits, window=5, **kw).cpu().numpy()
           for tag, kw in (("trunc", {}), ("plain", {"plain": True}), ("cios", {"cios": True}))}
    assert np.array_equal(res["trunc"], res["plain"])
    assert np.array_equal(res["trunc"], res["cios"])
    idx = _headline_idx()
    assert len(idx) == n // 64
    _oracle_check(res["trunc"], "headline", idx, lambda: _jobs(bits, n, k, idx), "65536 x 2048 w5")
    ctx.close()


def test_16384_x_4096_w6_schoolbook_and_karatsuba(mx):
    n, bits, k = C3
    mods, base, exps = _host(bits, n, k)
    ctx = mx.Context(mods, bits)
    b, e = mx.to_device(base), mx.to_device(exps)
    sb = mx.modexp(ctx, b, e, bits, window=6, block=True).cpu().numpy()
    ka = mx.modexp(ctx, b, e, bits, window=6, block="karatsuba").cpu().numpy()
    assert np.array_equal(sb, ka)
    ci = mx.modexp(ctx, b, e, bits, window=6, cios=True).cpu().numpy()  # block-word CIOS
    assert np.array_equal(sb, ci)
    idx = _c3_idx()
    _oracle_check(sb, "c3", idx, lambda: _jobs(bits, n, k, idx), "16384 x 4096 w6")
    ctx.close()


def test_mixed_200k_persistent_launch_from_graph(mx):
    import torch
    batches = []
    for c, n in _mixed_counts().items():
        mods, base, exps = _host(c, n, 4 + c)
        ctx = mx.Context(mods, c)
        b = mx.to_device(base)
        batches.append({"ctx": ctx, "base": b, "exp": mx.to_device(exps), "exp_bits": c, "out": torch.zeros_like(b),
                        "window": 3 if c <= 2048 else 5})
    plan = mx.MixedPlan(batches)
    alone = {bb["exp_bits"]: mx.modexp(bb["ctx"], bb["base"], bb["exp"], bb["exp_bits"],
                                       window=bb["window"]).cpu().numpy() for bb in batches}
    for launch in range(2):  # the first call captures the graph, the second replays it
        for bb in batches:
            bb["out"].zero_()  # eager work between the launches
        plan.launch(graph=True)
        torch.cuda.synchronize()
        for bb in batches:
            assert np.array_equal(bb["out"].cpu().numpy(), alone[bb["exp_bits"]]), (launch, bb["exp_bits"])
    for c, n in _mixed_counts().items():
        idx = _mixed_idx(c)
        _oracle_check(alone[c], ("mixed", c), idx, lambda: _jobs(c, n, 4 + c, idx), "mixed %d-bit" % c)
    plan.close()
    for bb in batches:
        bb["ctx"].close()


def test_rsa2048_crt_65536_operations(mx):
    import torch
    nr = RSA_N
    keys, key_of, cs = _rsa_inputs()
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
    idx = _rsa_idx()
    want = oracle_pool.results("rsa", _rsa_jobs)  # c^d mod pq by the oracle's square-and-multiply (no CRT)
    assert [got[i] for i in idx] == want
    ctx_p.close()
    ctx_q.close()
