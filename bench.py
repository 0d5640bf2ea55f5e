"""Benchmark: 2048-bit batched constant-time modexp on one MI355X.

One step = one launch of the whole hot path (context-resident moduli,
conversion to Montgomery form, window table, 410 windows of 5 squarings + a
masked table scan + a multiplication, conversion back, canonical output)
over a batch of 65536 synthetic instances with inputs resident in HBM.

Prints one JSON line (see the design doc for every field).  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2048-bit modexp/s (truncated vs plain Montgomery), % int-mul peak; p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--bits", type=int, default=2048)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--window", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline leg")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-reduction comparison")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle instances (0 = 2 per core)")
    return ap.parse_args()


def cpu_baseline(bits, sample, cores):
    """The oracle (plain C schoolbook + bit-serial reduction + square-and-multiply)
    on a bounded sample of the same workload, one process per core."""
    import multiprocessing as mp
    import numpy as np
    from paper_2410_18129_amd import workload as wl
    g = wl.stream(2, "moduli")
    mods = wl.random_moduli(g, bits, sample)
    base = wl.random_below_fast(wl.stream(2, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(2, "exps"), bits, sample)
    M, B, E = wl.words_to_ints(mods), wl.words_to_ints(base), wl.words_to_ints(exps)
    chunks = [(B[i::cores], E[i::cores], M[i::cores], bits) for i in range(cores)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_chunk, chunks)
    dt = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "modexp/s", "cores": cores, "kind": "oracle",
            "sample": "%d x %d-bit modexp (2048-bit exponents), %d worker processes, %.1f s wall" %
                      (sample, bits, cores, dt)}


def _oracle_chunk(args):
    import oracle
    b, e, m, bits = args
    if b:
        oracle.modexp_many(b, e, m, bits)
    return len(b)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus %d requested); every instance is "
              "independent, see DESIGN.md for how the batch would shard" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2410_18129_amd import counts, montexp as mx, workload as wl

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    mx.lib()
    dev = torch.device("cuda:0")
    bits, n, w = a.bits, a.batch, a.window
    g = wl.stream(2, "moduli")
    mods = wl.random_moduli(g, bits, n)
    base = wl.random_below_fast(wl.stream(2, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(2, "exps"), bits, n)
    ctx = mx.Context(mods, bits)
    bd = mx.to_device(base, dev)
    ed = mx.to_device(exps, dev)
    out = torch.empty_like(bd)
    stream = torch.cuda.current_stream()

    def run(plain, steps, warmup):
        for _ in range(warmup):
            mx.modexp(ctx, bd, ed, bits, window=w, out=out, plain=plain, stream=stream)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for e0, e1 in evs:
            e0.record(stream)
            mx.modexp(ctx, bd, ed, bits, window=w, out=out, plain=plain, stream=stream)
            e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms = [e0.elapsed_time(e1) for e0, e1 in evs]
        return wall, kms

    wall, kms = run(False, a.steps, a.warmup)
    ms_step = wall * 1e3 / a.steps
    value = n * a.steps / wall
    prod = counts.modexp_products(bits, bits, w, trunc=True)
    kavg = sum(kms) / len(kms)
    achieved = prod * n / (kavg * 1e-3)
    res = {
        "metric": METRIC, "value": value, "unit": "modexp/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "%d-bit constant-time fixed-window modexp, batch %d, window %d, truncated "
                               "Montgomery reduction, %d-bit exponents" % (bits, n, w, bits),
                   "global_batch": n, "bits": bits, "window": w, "limb_bits": 28, "limbs": counts.limbs(bits),
                   "parallelism": "one instance per lane, single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": counts.PEAK_MAD_PER_S / 1e12,
                     "unit": "Tmad/s", "frac": achieved / counts.PEAK_MAD_PER_S, "traffic": None,
                     "kernel": "k_modexp<74,32,true>", "kernel_ms": kavg,
                     "work_per_launch": "%d x %d 28x28-bit products" % (n, prod)},
    }
    if not a.no_plain:
        wall_p, kms_p = run(True, max(2, a.steps // 2), 1)
        vp = n * len(kms_p) / wall_p
        prod_p = counts.modexp_products(bits, bits, w, trunc=False)
        kp = sum(kms_p) / len(kms_p)
        res["plain"] = {"value": vp, "unit": "modexp/s", "kernel_ms": kp,
                        "frac": prod_p * n / (kp * 1e-3) / counts.PEAK_MAD_PER_S}
        res["trunc_speedup"] = value / vp
    # modmul/s on the same moduli (streaming REDC(a*b), values in [0, 2N))
    A = mx.to_device(wl.random_below_fast(wl.stream(2, "ops_a"), mods, bits), dev)
    A = torch.nn.functional.pad(A, (0, ctx.mont_words - ctx.words))
    B = torch.roll(A, 1, 0).contiguous()
    O = torch.empty_like(A)
    for _ in range(3):
        mx.mont_mul(ctx, A, B, out=O, stream=stream)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        mx.mont_mul(ctx, A, B, out=O, stream=stream)
    torch.cuda.synchronize()
    res["modmul_per_s"] = n * reps / (time.perf_counter() - t0)
    if not a.no_cpu:
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        cores = max(1, min(cores, 16))
        sample = a.cpu_sample or 2 * cores
        res["cpu_baseline"] = cpu_baseline(bits, sample, cores)
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
