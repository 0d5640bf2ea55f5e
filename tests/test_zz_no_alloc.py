"""GPU: the allocation-free exponentiation entry point against modexp_batch.

modexp_batch_noalloc keeps its workspace in a fixed device array of the
library (one per GPU) instead of allocating one.  It must give exactly what
modexp_batch gives (results are unique integers: tolerance 0), call after call
on the same array, including after a call of another size class that left its
own values in the array, and must refuse batches whose workspace exceeds the
array before anything is launched.
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


def _inputs(mx, bits, n, k):
    mods = wl.random_moduli(wl.stream(k, "moduli"), bits, n)
    base = wl.random_below_fast(wl.stream(k, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(k, "exps"), bits, n)
    return mods, mx.Context(mods, bits), mx.to_device(base), mx.to_device(exps)


def _noalloc(mx, ctx, b, e, ebits, window, out, n=None, flags=0):
    import torch
    n = b.shape[0] if n is None else n
    return mx.lib().modexp_batch_noalloc(ctx.handle, None, ctypes.c_void_p(b.data_ptr()),
                                         ctypes.c_void_p(e.data_ptr()), ebits, window,
                                         ctypes.c_void_p(out.data_ptr()), n, flags,
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_noalloc_matches_modexp_batch_call_after_call(mx):
    import torch
    # (bits, n, window, flags, seed): the second call is smaller than the first on the same class, the
    # third is another class after it (the array holds the previous call's values), the fourth a block
    # kernel (3072 bits, its own layout of the array)
    calls = [(2048, 4000, 5, 0, 31), (2048, 1000, 5, 0, 32), (1024, 700, 4, 0, 33), (3072, 300, 5, 0, 34),
             (2048, 129, 3, mx.MX_REDC_PLAIN, 35)]
    for bits, n, w, flags, k in calls:
        mods, ctx, b, e = _inputs(mx, bits, n, k)
        ref = mx.modexp(ctx, b, e, bits, window=w, plain=bool(flags & mx.MX_REDC_PLAIN))
        out = torch.full_like(b, -1)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        assert _noalloc(mx, ctx, b, e, bits, w, out, flags=flags) == mx.MX_OK, mx.lib().mont_last_error()
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] >= free0 - (1 << 20)  # nothing allocated on the device
        assert torch.equal(out, ref), (bits, n, w)
        got = wl.words_to_ints(out.cpu().numpy().view(np.uint64))
        M, B, E = wl.words_to_ints(mods), wl.words_to_ints(b.cpu().numpy().view(np.uint64)), \
            wl.words_to_ints(e.cpu().numpy().view(np.uint64))
        for i in (0, n - 1):
            assert got[i] == oracle.modexp(B[i], E[i], M[i], bits), (bits, i)
        ctx.close()


def test_noalloc_refuses_batches_beyond_the_array(mx):
    import torch
    mods, ctx, b, e = _inputs(mx, 2048, 64, 36)
    # 16384 instances at window 5 need 1.4e8 bytes of workspace, more than the array holds; the
    # buffers are the full size, so the call stays in bounds whatever it does
    big = 16384
    bb = b.repeat(big // 64, 1).contiguous()
    eb = e.repeat(big // 64, 1).contiguous()
    out = torch.zeros_like(bb)
    idx = torch.arange(big, dtype=torch.int32, device="cuda") % 64
    st = mx.lib().modexp_batch_noalloc(ctx.handle, ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(bb.data_ptr()),
                                       ctypes.c_void_p(eb.data_ptr()), 2048, 5, ctypes.c_void_p(out.data_ptr()), big,
                                       0, None)
    assert st == mx.MX_EINVAL
    assert b"maximum" in mx.lib().mont_last_error()
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0  # nothing was launched
    ctx.close()
