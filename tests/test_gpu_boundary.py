"""GPU: the C ABI's workspace rules.

- batch calls never allocate: a context's workspace comes from mont_ctx_init
  (one launch of its moduli at the default window) or mont_ctx_reserve;
- a workspace that holds fewer instances than the batch runs it in several
  launches with the same results; one that holds no tile gives MX_ENOMEM;
- calls on one context from two streams take turns on its workspace (results
  as if run one after the other);
- rsa_crt_batch_ws (caller workspace) equals rsa_crt_batch.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2410_18129_amd import workload as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_18129_amd import montexp
    montexp.lib()  # raises if the library is missing: no fallback
    return montexp


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _raw_modexp(mx, ctx, b, e, ebits, w, out, idx=None, stream=None):
    """modexp_batch through the C ABI without the binding's reserve call."""
    return mx.lib().modexp_batch(ctx.handle, _p(idx), _p(b), _p(e), ebits, w, _p(out), b.shape[0], 0,
                                 ctypes.c_void_p(stream.cuda_stream) if stream is not None else None)


def test_workspace_sizes_and_chunked_launches(mx):
    import torch
    bits = 2048
    mods = wl.random_moduli(wl.stream(40, "moduli"), bits, 64)
    ctx = mx.Context(mods, bits)
    # init reserves one launch of the 64 moduli at the default window (3)
    assert ctx.device_bytes() >= mx.modexp_ws_bytes(ctx, 64, 3)
    n = 200  # four tiles through ctx_idx: more than the initial workspace holds at window 3
    idx = (torch.arange(n, dtype=torch.int32, device="cuda") * 7) % 64
    base = wl.random_below_fast(wl.stream(40, "bases"), mods[(np.arange(n) * 7) % 64], bits)
    b = mx.to_device(base)
    e = mx.to_device(wl.random_exponents(wl.stream(40, "exps"), bits, n))
    out = torch.zeros_like(b)
    assert _raw_modexp(mx, ctx, b, e, bits, 3, out, idx) == mx.MX_OK  # runs as several launches
    torch.cuda.synchronize()
    # window 5 needs more per tile than the initial workspace holds: refused, nothing launched
    o5 = torch.zeros_like(b)
    assert _raw_modexp(mx, ctx, b, e, bits, 5, o5, idx) == mx.MX_ENOMEM
    assert b"mont_ctx_reserve" in mx.lib().mont_last_error()
    torch.cuda.synchronize()
    assert torch.count_nonzero(o5).item() == 0
    # after a reserve of one launch, the same call is one launch with the same results as window 3
    ctx.reserve(mx.modexp_ws_bytes(ctx, n, 5))
    assert _raw_modexp(mx, ctx, b, e, bits, 5, o5, idx) == mx.MX_OK
    torch.cuda.synchronize()
    assert torch.equal(out, o5)
    M = wl.words_to_ints(mods)
    got, B, E = wl.words_to_ints(out.cpu().numpy().view(np.uint64)), wl.words_to_ints(base), \
        wl.words_to_ints(e.cpu().numpy().view(np.uint64))
    for i in (0, 63, 64, 130, n - 1):
        assert got[i] == oracle.modexp(B[i], E[i], M[(i * 7) % 64], bits), i
    ctx.close()


def test_two_streams_take_turns_on_one_context(mx):
    import torch
    bits, n = 1024, 256
    mods = wl.random_moduli(wl.stream(41, "moduli"), bits, n)
    ctx = mx.Context(mods, bits)
    ins = []
    for k in range(4):
        b = mx.to_device(wl.random_below_fast(wl.stream(41 + k, "bases"), mods, bits))
        e = mx.to_device(wl.random_exponents(wl.stream(41 + k, "exps"), bits, n))
        ins.append((b, e))
    ref = [mx.modexp(ctx, b, e, bits, window=4) for b, e in ins]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = [torch.zeros_like(ins[0][0]) for _ in ins]
    for rep in range(3):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        for k, (b, e) in enumerate(ins):  # no synchronisation between the calls of the two streams
            st = s1 if k % 2 == 0 else s2
            with torch.cuda.stream(st):
                assert _raw_modexp(mx, ctx, b, e, bits, 4, outs[k], stream=st) == mx.MX_OK
        torch.cuda.synchronize()
        for k in range(len(ins)):
            assert torch.equal(outs[k], ref[k]), (rep, k)
    ctx.close()


def test_rsa_crt_with_caller_workspace(mx):
    import torch
    keys = wl.rsa_keys(wl.load_primes(1024))
    g = wl.stream(42, "misc")
    n = 300
    key_of = g.integers(0, len(keys), size=n)
    cs = wl.rsa_messages(g, keys, key_of)
    ctx_p = mx.Context(wl.ints_to_words([k["p"] for k in keys], 16), 1024)
    ctx_q = mx.Context(wl.ints_to_words([k["q"] for k in keys], 16), 1024)

    def dev(vals, words):
        return torch.from_numpy(wl.ints_to_words(vals, words).view(np.int64)).to("cuda")

    args = (dev(cs, 32), dev([keys[k]["dp"] for k in key_of], 16), dev([keys[k]["dq"] for k in key_of], 16),
            dev([keys[k]["qinv"] for k in key_of], 16))
    kidx = torch.from_numpy(key_of.astype(np.int32)).to("cuda")
    ref = mx.rsa_crt(ctx_p, ctx_q, *args, window=4, key_idx=kidx)
    need = mx.rsa_crt_ws_bytes(ctx_p, n, window=4)
    for ws_bytes in (need, need // 3):  # one paired launch; or the halves in several launches
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        got = mx.rsa_crt(ctx_p, ctx_q, *args, window=4, key_idx=kidx, ws=ws)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), ws_bytes
    vals = wl.words_to_ints(ref.cpu().numpy().view(np.uint64))
    for i in (0, n - 1):
        k = keys[key_of[i]]
        assert vals[i] == oracle.modexp(cs[i], k["d"], k["n"], 2048)
    tiny = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(mx.MontError) as ei:
        mx.rsa_crt(ctx_p, ctx_q, *args, window=4, key_idx=kidx, ws=tiny)
    assert ei.value.status == mx.MX_EINVAL
    ctx_p.close()
    ctx_q.close()


def test_check_inputs_flag(mx):
    """MX_CHECK_INPUTS: in-range inputs give the usual results; out-of-range ones give MX_EINVAL naming the count
    and the first instance, with nothing else launched."""
    import torch
    bits, n = 1024, 100
    mods = wl.random_moduli(wl.stream(43, "moduli"), bits, n)
    ctx = mx.Context(mods, bits)
    M = wl.words_to_ints(mods)
    base = wl.random_below(wl.stream(43, "bases"), mods, bits)
    e = mx.to_device(wl.random_exponents(wl.stream(43, "exps"), bits, n))
    b = torch.from_numpy(wl.ints_to_words(base, ctx.words).view(np.int64)).cuda()
    ref = mx.modexp(ctx, b, e, bits, window=4)
    assert torch.equal(mx.modexp(ctx, b, e, bits, window=4, check_inputs=True), ref)
    bad = list(base)
    bad[17], bad[60] = M[17], M[60] + 5  # base = N and base > N
    bb = torch.from_numpy(wl.ints_to_words(bad, ctx.words).view(np.int64)).cuda()
    out = torch.zeros_like(bb)
    with pytest.raises(mx.MontError) as ei:
        mx.modexp(ctx, bb, e, bits, window=4, out=out, check_inputs=True)
    assert ei.value.status == mx.MX_EINVAL and "2 of 100" in str(ei.value) and "instance 17" in str(ei.value)
    assert torch.count_nonzero(out).item() == 0
    # Montgomery operands: a, b < 2N
    A = wl.random_below(wl.stream(43, "ops_a"), mods, bits, scale=2)
    a = torch.from_numpy(wl.ints_to_words(A, ctx.mont_words).view(np.int64)).cuda()
    assert torch.equal(mx.mont_mul(ctx, a, a, check_inputs=True), mx.mont_mul(ctx, a, a))
    A[99] = 2 * M[99]
    a2 = torch.from_numpy(wl.ints_to_words(A, ctx.mont_words).view(np.int64)).cuda()
    with pytest.raises(mx.MontError) as ei:
        mx.mont_sqr(ctx, a2, check_inputs=True)
    assert ei.value.status == mx.MX_EINVAL and "1 of 100" in str(ei.value) and "instance 99" in str(ei.value)
    ctx.close()
