"""GPU serving: continuous batching over resident contexts; each result is the
same alone and in the mix (bit-exact), admission by memory budget."""
import numpy as np
import pytest

import oracle
from paper_2410_18129_amd import serving, workload as wl

pytestmark = pytest.mark.gpu

SMALL_MODULI = {1024: 16, 2048: 14, 3072: 6, 4096: 4}


@pytest.fixture(scope="module")
def mx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_18129_amd import montexp
    montexp.lib()
    return montexp


def test_serving_results_match_alone(mx):
    import torch
    tr = serving.Trace(1500, 30000.0, k=41, moduli=SMALL_MODULI)
    maxb = {1024: 256, 2048: 256, 3072: 64, 4096: 64}
    ex = serving.GpuExecutor(tr, maxb, mem_budget=2 << 30, max_slots=3)
    res = serving.Server(ex, tr.classes, maxb).run(tr, timeout_s=120)
    assert not res.failed.any() and not np.isnan(res.finish).any()
    assert len(res.batches) > 4  # requests were batched dynamically, not all at once
    for c in tr.classes:
        got = wl.words_to_ints(ex.out[c].cpu().numpy().view(np.uint64))
        # alone: every request of the class in one launch, and a sample one by one
        whole = mx.modexp(ex.ctx[c], ex.base[c], ex.exp[c], c, window=ex.windows[c], ctx_idx=ex.cidx[c])
        assert got == wl.words_to_ints(whole.cpu().numpy().view(np.uint64)), c
        for i in (0, tr.count[c] // 2, tr.count[c] - 1):
            one = mx.modexp(ex.ctx[c], ex.base[c][i:i + 1], ex.exp[c][i:i + 1], c, window=ex.windows[c],
                            ctx_idx=ex.cidx[c][i:i + 1])
            assert got[i] == wl.words_to_ints(one.cpu().numpy().view(np.uint64))[0]
        i = tr.count[c] - 1
        M = wl.words_to_ints(tr.mods[c])[int(tr.mod_id[tr.cls == c][i])]
        B, E = wl.words_to_ints(tr.base[c][i:i + 1])[0], wl.words_to_ints(tr.exp[c][i:i + 1])[0]
        if c <= 2048:
            assert got[i] == oracle.modexp(B, E, M, c)
        else:
            assert got[i] == pow(B, E, M)
    st = res.stats()
    assert st["p99_ms"] >= st["p50_ms"] > 0
    ex.close()
    torch.cuda.synchronize()


def test_serving_memory_budget_too_small(mx):
    tr = serving.Trace(200, 10000.0, k=42, moduli=SMALL_MODULI)
    with pytest.raises(MemoryError):
        serving.GpuExecutor(tr, {1024: 4096, 2048: 4096, 3072: 4096, 4096: 4096}, mem_budget=1 << 20)


def test_modexp_ws_matches_library_workspace(mx):
    import torch
    bits, n = 2048, 130
    mods = wl.random_moduli(wl.stream(43, "moduli"), bits, n)
    base = wl.random_below_fast(wl.stream(43, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(43, "exps"), bits, n)
    ctx = mx.Context(mods, bits)
    bd, ed = mx.to_device(base), mx.to_device(exps)
    ref = mx.modexp(ctx, bd, ed, bits, window=4)
    need = mx.modexp_ws_bytes(ctx, n, 4)
    ws = torch.empty(need // 2, dtype=torch.uint8, device="cuda")  # half: the call splits the batch
    out = mx.modexp_ws(ctx, bd, ed, bits, ws, window=4)
    assert torch.equal(out, ref)
    with pytest.raises(mx.MontError):
        mx.modexp_ws(ctx, bd, ed, bits, torch.empty(16, dtype=torch.uint8, device="cuda"), window=4)
    ctx.close()
