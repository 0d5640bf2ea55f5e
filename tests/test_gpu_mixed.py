"""GPU: block kernels vs register-resident kernels, the mixed-size persistent
launch (alone == in the mix, graph replays), and the autotuner."""
import random

import numpy as np
import pytest

import oracle
from paper_2410_18129_amd import workload as wl
from tests import oracle_pool
from tests.gpu_util import dev_ints, ints_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_18129_amd import montexp
    montexp.lib()
    return montexp


@pytest.mark.parametrize("bits", [1024, 2048])
def test_block_kernels_match_register_kernels(mx, bits):
    n = 70
    mods = wl.random_moduli(wl.stream(11, "moduli"), bits, n)
    ctx = mx.Context(mods, bits)
    g = wl.stream(11, "ops_a")
    A = wl.random_below(g, mods, bits, scale=2)
    B = wl.random_below(g, mods, bits, scale=2)
    a, b = ints_dev(A, ctx.mont_words), ints_dev(B, ctx.mont_words)
    for plain in (False, True):
        assert dev_ints(mx.mont_mul(ctx, a, b, plain=plain, block=True)) == dev_ints(mx.mont_mul(ctx, a, b, plain=plain))
        assert dev_ints(mx.mont_sqr(ctx, a, plain=plain, block=True)) == dev_ints(mx.mont_sqr(ctx, a, plain=plain))
    base = wl.random_below_fast(wl.stream(11, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(11, "exps"), bits, n)
    bd, ed = mx.to_device(base), mx.to_device(exps)
    r_blk = dev_ints(mx.modexp(ctx, bd, ed, bits, window=4, block=True))
    assert r_blk == dev_ints(mx.modexp(ctx, bd, ed, bits, window=4))
    M, Bs, Es = wl.words_to_ints(mods), wl.words_to_ints(base), wl.words_to_ints(exps)
    assert r_blk[0] == oracle.modexp(Bs[0], Es[0], M[0], bits)
    ctx.close()


@pytest.mark.parametrize("window", [1, 2, 3, 8])
def test_block_kernel_small_and_large_windows(mx, window):
    # the block kernels' table scan reads eight entries per iteration: windows 1 and 2
    # (fewer than eight entries) re-read entry 0 under a zero mask; window 8 is the largest
    bits, n = 1024, 67
    mods = wl.random_moduli(wl.stream(12, "moduli"), bits, n)
    ctx = mx.Context(mods, bits)
    base = wl.random_below_fast(wl.stream(12, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(12, "exps"), bits, n)
    bd, ed = mx.to_device(base), mx.to_device(exps)
    r_blk = dev_ints(mx.modexp(ctx, bd, ed, bits, window=window, block=True))
    assert r_blk == dev_ints(mx.modexp(ctx, bd, ed, bits, window=window))
    M, Bs, Es = wl.words_to_ints(mods), wl.words_to_ints(base), wl.words_to_ints(exps)
    for i in (0, 33, n - 1):
        assert r_blk[i] == oracle.modexp(Bs[i], Es[i], M[i], bits)
    ctx.close()


def test_block_kernel_one_two_and_four_lanes_per_instance_agree(mx):
    # batches of at most 32768 instances run four lanes per instance, larger ones one: the same
    # instances computed by a 33001-instance batch (one lane) and by a 20001-instance and a
    # 4001-instance slice of it (four lanes), then with one, two and four lanes forced
    bits, n = 1024, 33001
    mods = wl.random_moduli(wl.stream(13, "moduli"), bits, n)
    ctx = mx.Context(mods, bits)
    base = wl.random_below_fast(wl.stream(13, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(13, "exps"), bits, n)
    bd, ed = mx.to_device(base), mx.to_device(exps)
    one = dev_ints(mx.modexp(ctx, bd, ed, bits, window=3, block=True))
    import torch
    lo, hi = 29000, 33001
    idx = torch.arange(lo, hi, dtype=torch.int32, device=bd.device)
    four = dev_ints(mx.modexp(ctx, bd[lo:hi].contiguous(), ed[lo:hi].contiguous(), bits, window=3, block=True,
                              ctx_idx=idx))
    assert four == one[lo:hi]  # four lanes per instance
    lo2 = n - 20001
    idx2 = torch.arange(lo2, n, dtype=torch.int32, device=bd.device)
    assert dev_ints(mx.modexp(ctx, bd[lo2:].contiguous(), ed[lo2:].contiguous(), bits, window=3, block=True,
                              ctx_idx=idx2)) == one[lo2:]  # four lanes per instance
    forced = dev_ints(mx.modexp(ctx, bd[lo:hi].contiguous(), ed[lo:hi].contiguous(), bits, window=3, block=True,
                                ctx_idx=idx, one_lane=True))  # MX_ONE_LANE: one lane per instance at any size
    assert forced == one[lo:hi]
    capped = dev_ints(mx.modexp(ctx, bd[lo2:].contiguous(), ed[lo2:].contiguous(), bits, window=3, block=True,
                                ctx_idx=idx2, two_lanes=True))  # MX_TWO_LANES: two lanes where four would run
    assert capped == one[lo2:]
    big = dev_ints(mx.modexp(ctx, bd, ed, bits, window=3, block=True, four_lanes=True))  # MX_FOUR_LANES at 33001
    assert big == one
    M, Bs, Es = wl.words_to_ints(mods), wl.words_to_ints(base), wl.words_to_ints(exps)
    for i in (0, 32767, 32768, n - 1):
        assert one[i] == oracle.modexp(Bs[i], Es[i], M[i], bits)
    ctx.close()


@pytest.mark.parametrize("bits", [2048, 3072])
def test_four_lane_block_kernel_matches_register_or_one_lane(mx, bits):
    """The four-lane block kernel (columns split by residue, arrays in LDS) at 2048 bits (two blocks) and
    3072 bits (three: a limb count that is not a multiple of four, so the split table scan masks its last
    limbs) gives the register-resident kernel's (2048) or the one-lane block kernel's (3072) results on a
    batch with a ragged tail, and the oracle's on samples."""
    n = 200
    mods = wl.random_moduli(wl.stream(17, "moduli"), bits, n)
    ctx = mx.Context(mods, bits)
    base = wl.random_below_fast(wl.stream(17, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(17, "exps"), bits, n)
    bd, ed = mx.to_device(base), mx.to_device(exps)
    four = dev_ints(mx.modexp(ctx, bd, ed, bits, window=4, block=True, four_lanes=True))
    ref = dev_ints(mx.modexp(ctx, bd, ed, bits, window=4) if bits == 2048 else
                   mx.modexp(ctx, bd, ed, bits, window=4, one_lane=True))
    assert four == ref
    M, Bs, Es = wl.words_to_ints(mods), wl.words_to_ints(base), wl.words_to_ints(exps)
    for i in (0, 15, 16, 101, n - 1):
        assert four[i] == oracle.modexp(Bs[i], Es[i], M[i], bits), i
    ctx.close()


def test_block_flag_unsupported_class(mx):
    ctx = mx.Context(wl.random_moduli(wl.stream(12, "moduli"), 256, 1), 256)
    a = ints_dev([1], ctx.mont_words)
    with pytest.raises(mx.MontError) as ei:
        mx.mont_mul(ctx, a, a, block=True)
    assert ei.value.status == mx.MX_EUNSUPPORTED
    ctx.close()


def _mixed_host(bits, n, k):
    mods = wl.random_moduli(wl.stream(k, "moduli"), bits, n)
    base = wl.random_below_fast(wl.stream(k, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(k, "exps"), bits, n)
    return mods, base, exps


PLAN_COUNTS = {1024: 130, 2048: 70, 3072: 65, 4096: 71}


def _plan_idx(bits):
    """Oracle samples of the small mixed plan: every instance up to 2048 bits, 16 spread over the others."""
    n = PLAN_COUNTS[bits]
    return list(range(n)) if bits <= 2048 else sorted({(k * n) // 16 for k in range(16)} | {n - 1})


def _plan_jobs(bits):
    mods, base, exps = _mixed_host(bits, PLAN_COUNTS[bits], 13)
    M, B, E = wl.words_to_ints(mods), wl.words_to_ints(base), wl.words_to_ints(exps)
    return [(B[i], E[i], M[i], bits) for i in _plan_idx(bits)]


def _submit_plan():
    for bits in PLAN_COUNTS:
        oracle_pool.submit(("plan", bits), _plan_jobs(bits))


ORACLE_JOBS = {"test_mixed_plan_matches_single_class_and_oracle": _submit_plan,
               "test_autotuned_plan_matches_single_class_and_oracle": _submit_plan}


def _mixed_inputs(mx, counts, k=13):
    import torch
    batches, ref = [], []
    for bits, n in counts.items():
        mods, base, exps = _mixed_host(bits, n, k)
        ctx = mx.Context(mods, bits)
        b = {"ctx": ctx, "base": mx.to_device(base), "exp": mx.to_device(exps), "exp_bits": bits,
             "out": torch.zeros((n, ctx.words), dtype=torch.int64, device="cuda")}
        batches.append(b)
        ref.append((mods, base, exps))
    return batches, ref


def test_mixed_plan_matches_single_class_and_oracle(mx):
    import torch
    counts = PLAN_COUNTS
    batches, ref = _mixed_inputs(mx, counts)
    batches[1]["block"] = False
    plan = mx.MixedPlan(batches)
    # tiles of 64 instances; 4096-bit schoolbook tiles hold 32 (two lanes per instance)
    assert plan.njobs == sum((n + (31 if bits == 4096 else 63)) // (32 if bits == 4096 else 64)
                             for bits, n in counts.items())
    plan.launch()
    torch.cuda.synchronize()
    for b, (mods, base, exps), bits in zip(batches, ref, counts):
        got = dev_ints(b["out"])
        alone = dev_ints(mx.modexp(b["ctx"], b["base"], b["exp"], bits, window=plan.windows[list(counts).index(bits)]))
        assert got == alone, bits  # the same result alone and in the mix
        want = oracle_pool.results(("plan", bits), lambda: _plan_jobs(bits))
        assert [got[i] for i in _plan_idx(bits)] == want, bits
    plan.close()
    for b in batches:
        b["ctx"].close()


def test_mixed_plan_graph_replays(mx):
    import torch
    counts = {1024: 100, 2048: 64}
    batches, ref = _mixed_inputs(mx, counts, k=14)
    batches[0]["block"] = True
    plan = mx.MixedPlan(batches)
    expect = []
    for b, bits in zip(batches, counts):
        expect.append(dev_ints(mx.modexp(b["ctx"], b["base"], b["exp"], bits, window=plan.windows[len(expect)],
                                         block=b.get("block", False))))
    for rep in range(3):
        for b in batches:
            b["out"].zero_()
        torch.cuda.synchronize()
        plan.launch(graph=True)
        torch.cuda.synchronize()
        for b, e in zip(batches, expect):
            assert dev_ints(b["out"]) == e, rep
    # the graph reads the buffers at replay time: new exponents give new results
    b0 = batches[0]
    b0["exp"].copy_(torch.roll(b0["exp"], 1, 0))
    plan.launch(graph=True)
    torch.cuda.synchronize()
    again = dev_ints(mx.modexp(b0["ctx"], b0["base"], b0["exp"], 1024, window=plan.windows[0], block=True))
    assert dev_ints(b0["out"]) == again
    plan.close()
    for b in batches:
        b["ctx"].close()


def test_mixed_plan_rejects_bad_batches(mx):
    import torch
    ctx = mx.Context(wl.random_moduli(wl.stream(15, "moduli"), 512, 4), 512)
    t = torch.zeros((4, ctx.words), dtype=torch.int64, device="cuda")
    with pytest.raises(mx.MontError) as ei:
        mx.MixedPlan([{"ctx": ctx, "base": t, "exp": t, "exp_bits": 512, "out": t}])
    assert ei.value.status == mx.MX_EUNSUPPORTED
    ctx.close()


def test_autotuner_measures_and_caches_tile_times(mx, tmp_path):
    from paper_2410_18129_amd import autotune
    cache = str(tmp_path / "cache.json")
    t = autotune.tile_times([1024], path=cache, waves=16, reps=1)
    assert set(t[1024]) == {autotune._key(w, f) for w, f in autotune.CANDIDATES[1024]}
    assert all(v > 0 for v in t[1024].values())
    assert autotune.tile_times([1024], path=cache, waves=16) == t  # cached, no re-measure


def test_autotuned_plan_matches_single_class_and_oracle(mx, tmp_path):
    """A plan built from the tuner's choice (window, family, lanes per class) gives what single-class launches
    with the same window and family give, and the oracle's values."""
    import torch
    from paper_2410_18129_amd import autotune
    counts = {1024: 130, 2048: 70, 3072: 65, 4096: 71}
    waves = 32
    # two candidates per large class keep the test short (one, two or four lanes per instance)
    cands = {1024: [(3, 0), (4, 0)], 2048: [(3, 0), (3, mx.MX_IMPL_BLOCK)],
             3072: [(4, mx.MX_IMPL_BLOCK | mx.MX_ONE_LANE), (4, mx.MX_IMPL_BLOCK | mx.MX_FOUR_LANES)],
             4096: [(4, mx.MX_IMPL_BLOCK | mx.MX_TWO_LANES), (4, mx.MX_IMPL_BLOCK | mx.MX_FOUR_LANES)]}
    times = {b: autotune.measure_class(b, waves=waves, reps=1, candidates=c) for b, c in cands.items()}
    sched, span = autotune.choose(counts, times, waves)
    assert span > 0 and set(sched) == set(counts)
    batches, ref = _mixed_inputs(mx, counts, k=13)
    for b, bits in zip(batches, counts):
        b.update(autotune.batch_args(sched[bits]))
    plan = mx.MixedPlan(batches)
    assert plan.njobs == sum(-(-n // sched[bits]["tile_instances"]) for bits, n in counts.items())
    plan.launch(graph=True)
    torch.cuda.synchronize()
    for b, bits in zip(batches, counts):
        s = sched[bits]
        fam = s["flags"] & (mx.MX_IMPL_BLOCK | mx.MX_MUL_KARATSUBA)
        alone = dev_ints(mx.modexp(b["ctx"], b["base"], b["exp"], bits, window=s["window"],
                                   block="karatsuba" if fam == mx.MX_MUL_KARATSUBA else bool(fam)))
        got = dev_ints(b["out"])
        assert got == alone, (bits, s)
        want = oracle_pool.results(("plan", bits), lambda: _plan_jobs(bits))
        assert [got[i] for i in _plan_idx(bits)] == want, bits
    plan.close()
    for b in batches:
        b["ctx"].close()


def test_mixed_plan_lane_flags(mx):
    """MX_ONE_LANE / MX_TWO_LANES / MX_FOUR_LANES pick the tile of a block batch (64, 32 or 16 instances; the
    four-lane tiles keep their arrays in LDS); two and four lanes exist for the 3072- and 4096-bit schoolbook
    tiles only.  Every choice gives the single-class results."""
    import torch
    counts = {3072: 65, 4096: 71}
    batches, _ = _mixed_inputs(mx, counts, k=13)
    alone = [dev_ints(mx.modexp(b["ctx"], b["base"], b["exp"], bits, window=4, one_lane=True))
             for b, bits in zip(batches, counts)]
    for flags, tiles in ((mx.MX_ONE_LANE, 2 + 2), (mx.MX_TWO_LANES, 3 + 3), (mx.MX_FOUR_LANES, 5 + 5)):
        for b in batches:
            b["flags"] = flags
            b["window"] = 4
            b["out"].zero_()
        plan = mx.MixedPlan(batches)
        assert plan.njobs == tiles
        plan.launch()
        torch.cuda.synchronize()
        for b, want, bits in zip(batches, alone, counts):
            assert dev_ints(b["out"]) == want, (bits, flags)
        plan.close()
    ctx = mx.Context(wl.random_moduli(wl.stream(15, "moduli"), 2048, 4), 2048)
    t = torch.zeros((4, ctx.words), dtype=torch.int64, device="cuda")
    for flags in (mx.MX_TWO_LANES, mx.MX_FOUR_LANES):
        with pytest.raises(mx.MontError) as ei:
            mx.MixedPlan([{"ctx": ctx, "base": t, "exp": t, "exp_bits": 2048, "out": t, "flags": flags}])
        assert ei.value.status == mx.MX_EUNSUPPORTED
    with pytest.raises(mx.MontError) as ei:
        mx.MixedPlan([{"ctx": ctx, "base": t, "exp": t, "exp_bits": 2048, "out": t,
                       "flags": mx.MX_ONE_LANE | mx.MX_FOUR_LANES}])
    assert ei.value.status == mx.MX_EINVAL
    ctx.close()
    for b in batches:
        b["ctx"].close()


@pytest.mark.parametrize("bits", [2048, 4096])
def test_karatsuba_matches_schoolbook(mx, bits):
    from tests.gpu_util import adversarial_pairs
    n = 66
    mods = wl.random_moduli(wl.stream(16, "moduli"), bits, n)
    M = wl.words_to_ints(mods)
    g = wl.stream(16, "ops_a")
    A = wl.random_below(g, mods, bits, scale=2)
    B = wl.random_below(g, mods, bits, scale=2)
    # adversarial operands on the first contexts: all-ones halves drive the half-sum carries
    for k, (x, y) in enumerate(adversarial_pairs(M[0], bits)[:10]):
        A[k], B[k] = x % (2 * M[k]), y % (2 * M[k])
    ctx = mx.Context(mods, bits)
    a, b = ints_dev(A, ctx.mont_words), ints_dev(B, ctx.mont_words)
    for plain in (False, True):
        kmul = dev_ints(mx.mont_mul(ctx, a, b, plain=plain, block="karatsuba"))
        ksqr = dev_ints(mx.mont_sqr(ctx, a, plain=plain, block="karatsuba"))
        assert kmul == dev_ints(mx.mont_mul(ctx, a, b, plain=plain, block=True))
        assert ksqr == dev_ints(mx.mont_sqr(ctx, a, plain=plain, block=True))
    for i in (0, 5, n - 1):
        assert kmul[i] == oracle.montmul(A[i], B[i], M[i], ctx.r_bits)
        assert ksqr[i] == oracle.montmul(A[i], A[i], M[i], ctx.r_bits)
    base = wl.random_below_fast(wl.stream(16, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(16, "exps"), bits, n)
    bd, ed = mx.to_device(base), mx.to_device(exps)
    rk = dev_ints(mx.modexp(ctx, bd, ed, bits, window=4, block="karatsuba"))
    assert rk == dev_ints(mx.modexp(ctx, bd, ed, bits, window=4, block=True))
    Bs, Es = wl.words_to_ints(base), wl.words_to_ints(exps)
    assert rk[1] == pow(Bs[1], Es[1], M[1])
    ctx.close()


@pytest.mark.parametrize("bits", [2048, 4096])
def test_block_karatsuba_truncated_reduction(mx, bits):
    """The truncated q N by one-level Karatsuba in the block kernels (Section 5, Karatsuba paragraph): the
    same integers as the schoolbook-truncated block kernels and the oracle, for products, squares and
    exponentiations, with the schoolbook or the Karatsuba product."""
    from tests.gpu_util import adversarial_pairs
    n = 67
    mods = wl.random_moduli(wl.stream(18, "moduli"), bits, n)
    M = wl.words_to_ints(mods)
    g = wl.stream(18, "ops_a")
    A = wl.random_below(g, mods, bits, scale=2)
    B = wl.random_below(g, mods, bits, scale=2)
    for k, (x, y) in enumerate(adversarial_pairs(M[0], bits)):
        A[k], B[k] = x % (2 * M[k]), y % (2 * M[k])
    ctx = mx.Context(mods, bits)
    a, b = ints_dev(A, ctx.mont_words), ints_dev(B, ctx.mont_words)
    for impl in (True, "karatsuba"):
        kmul = dev_ints(mx.mont_mul(ctx, a, b, block=impl, kara_redc=True))
        ksqr = dev_ints(mx.mont_sqr(ctx, a, block=impl, kara_redc=True))
        assert kmul == dev_ints(mx.mont_mul(ctx, a, b, block=True)), impl
        assert ksqr == dev_ints(mx.mont_sqr(ctx, a, block=True)), impl
    for i in range(n):
        assert kmul[i] == oracle.montmul(A[i], B[i], M[i], ctx.r_bits), i
        assert ksqr[i] == oracle.montmul(A[i], A[i], M[i], ctx.r_bits), i
    base = wl.random_below_fast(wl.stream(18, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(18, "exps"), bits, n)
    bd, ed = mx.to_device(base), mx.to_device(exps)
    rk = dev_ints(mx.modexp(ctx, bd, ed, bits, window=4, block=True, kara_redc=True))
    assert rk == dev_ints(mx.modexp(ctx, bd, ed, bits, window=4, block=True))
    Bs, Es = wl.words_to_ints(base), wl.words_to_ints(exps)
    for i in (0, n - 1):
        assert rk[i] == oracle.modexp(Bs[i], Es[i], M[i], bits), i
    ctx.close()


@pytest.mark.parametrize("bits", [1024, 3072])
def test_karatsuba_needs_even_block_count(mx, bits):
    ctx = mx.Context(wl.random_moduli(wl.stream(17, "moduli"), bits, 1), bits)
    a = ints_dev([1], ctx.mont_words)
    with pytest.raises(mx.MontError) as ei:
        mx.mont_mul(ctx, a, a, block="karatsuba")
    assert ei.value.status == mx.MX_EUNSUPPORTED
    ctx.close()
