"""Benchmark of the batched truncated-Montgomery exponentiation on one MI355X.

One step = one launch of the whole hot path (context-resident moduli,
conversion into Montgomery form, window table, every window's squarings +
constant-time table scan + multiplication, conversion back, canonical
output) over 65536 seeded 2048-bit instances, window 5, inputs resident in
HBM.  The JSON line also carries the other workloads (8 x 1024-bit; 16384 x
4096-bit schoolbook vs Karatsuba; the 200k mixed-size persistent launch; the
serving loop's p50/p99) and the oracle timed on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2048-bit modexp/s (truncated vs plain Montgomery and CIOS), % int-mul peak; p99 latency"
KERNEL_SOURCES = ("mx_core.hpp", "mx_kernels.hpp")  # the headline kernel's code (mx_class.hip only launches it)
SERVE_SLOTS = 2  # serving: execution slots per size class


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--bits", type=int, default=2048)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--window", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="headline only (no other workloads)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline leg")
    ap.add_argument("--only", choices=("headline", "c3"), default=None,
                    help="one launch configuration alone, for profiling: the headline exponentiation (window "
                         "--window) or the 16384 x 4096-bit block exponentiation at window 6")
    ap.add_argument("--plain", action="store_true",
                    help="with --only headline: the plain reduction (Algorithm 3) instead of the truncated one")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 256 MiB device-to-device three times (calibrates FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def copy_probe():
    import torch
    n = 256 << 20
    a = torch.ones(n // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "copies": 3}))


def progress(msg):
    """One line on stderr when a measured section ends (the JSON result goes to stdout)."""
    print("bench.py: %s" % msg, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2410_18129_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_id):
    """HBM bytes per launch from the committed counter summary, if it was taken on these sources."""
    path = os.path.join(ROOT, "profiles", "modexp2048_w5_traffic.md")
    try:
        txt = open(path).read()
    except OSError:
        return None
    m = re.search(r"source hash: `([0-9a-f]+)`", txt)
    t = re.search(r"HBM bytes per launch \(scaled\): `([0-9.eE+]+)`", txt)
    if not m or not t or m.group(1) != kernel_id:
        return None
    return float(t.group(1))


def _oracle_jobs_rate(jobs, cores, min_s):
    """Rate of the oracle on `jobs` [(base, exp, N, ebits)], one process per core, repeating the whole
    sample until min_s seconds of wall time have passed; (instances per second, repeats, wall seconds)."""
    import multiprocessing as mp
    chunks = [jobs[i::cores] for i in range(cores)]
    chunks = [c for c in chunks if c]
    reps, t0 = 0, time.perf_counter()
    with mp.get_context("fork").Pool(len(chunks)) as pool:
        while True:
            pool.map(_oracle_chunk, chunks)
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= min_s:
                break
    return len(jobs) * reps / dt, reps, dt


def _oracle_chunk(jobs):
    import oracle
    for b, e, m, ebits in jobs:
        oracle.modexp(b, e, m, ebits)
    return len(jobs)


def _sample_jobs(bits, n_total, k, idx):
    """(base, exp, N, ebits) of the instances idx of workload k's seeded n_total-instance batch."""
    from paper_2410_18129_amd import workload as wl
    mods = wl.random_moduli(wl.stream(k, "moduli"), bits, n_total)
    base = wl.random_below_fast(wl.stream(k, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(k, "exps"), bits, n_total)
    M, B, E = wl.words_to_ints(mods[idx]), wl.words_to_ints(base[idx]), wl.words_to_ints(exps[idx])
    return [(b, e, m, bits) for b, e, m in zip(B, E, M)]


def cpu_baseline(cores, min_s=10.0):
    """The oracle (plain C schoolbook + bit-serial reduction + square-and-multiply) on bounded samples
    of the workloads, one process per core, each leg at least min_s seconds of wall time: all 8
    instances of the 1024-bit workload (repeated), 512 of the 65536 x 2048-bit headline (the value),
    64 of the 16384 x 4096-bit workload and 1000 of the 200k mixed workload stratified by class
    (400 / 350 / 150 / 100)."""
    import numpy as np
    from paper_2410_18129_amd import workload as wl
    legs = {}
    spread = lambda n, m: np.arange(m) * (n // m)
    r, reps, dt = _oracle_jobs_rate(_sample_jobs(2048, 65536, 2, spread(65536, 512)), cores, min_s)
    main = {"value": r, "unit": "modexp/s", "cores": cores, "kind": "oracle",
            "sample": "512 of the 65536 seeded 2048-bit instances (2048-bit exponents, every 128th), %d worker "
                      "processes, %d pass(es), %.1f s wall" % (cores, reps, dt)}
    r1, reps1, dt1 = _oracle_jobs_rate(_sample_jobs(1024, 8, 1, np.arange(8)), cores, min_s)
    legs["c1_1024x8"] = {"modexp_per_s": r1, "sample": "all 8 instances, %d passes, %.1f s wall" % (reps1, dt1)}
    r3, reps3, dt3 = _oracle_jobs_rate(_sample_jobs(4096, 16384, 3, spread(16384, 64)), cores, min_s)
    legs["c3_4096x16384"] = {"modexp_per_s": r3, "sample": "64 instances, every 256th, %d pass(es), %.1f s wall"
                                                           % (reps3, dt3)}
    sizes = wl.size_mix(wl.stream(4, "sizes"), 200000)
    jobs = []
    for c, m in ((1024, 400), (2048, 350), (3072, 150), (4096, 100)):
        n_c = int((sizes == c).sum())
        jobs += _sample_jobs(c, n_c, 4 + c, spread(n_c, m))
    r4, reps4, dt4 = _oracle_jobs_rate(jobs, cores, min_s)
    legs["c4_mixed_200k"] = {"modexp_per_s": r4, "sample": "1000 instances stratified 400/350/150/100 by class, "
                                                           "%d pass(es), %.1f s wall" % (reps4, dt4)}
    main["legs"] = legs
    return main


class Batch:
    """Seeded inputs for one size class, resident on the device."""

    def __init__(self, mx, bits, n, k, dev):
        from paper_2410_18129_amd import workload as wl
        import torch
        self.bits, self.n = bits, n
        mods = wl.random_moduli(wl.stream(k, "moduli"), bits, n)
        self.ctx = mx.Context(mods, bits)
        self.base = mx.to_device(wl.random_below_fast(wl.stream(k, "bases"), mods, bits), dev)
        self.exp = mx.to_device(wl.random_exponents(wl.stream(k, "exps"), bits, n), dev)
        self.out = torch.empty_like(self.base)


def time_launches(fn, steps, warmup, stream):
    """Wall time of `steps` launches after `warmup`, and each launch's kernel time (events on the stream)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [e0.elapsed_time(e1) for e0, e1 in evs]


def main():
    a = parse()
    if a.copy_probe:
        copy_probe()
        return
    if a.gpus != 1:
        print("bench.py: runs on one GPU only (--gpus %d requested); the instances are independent, so a "
              "multi-GPU run would shard the batch by instance with no exchange on the hot path" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    if not a.quick:
        # the serving workload runs 4 x SERVE_SLOTS streams concurrently: give each its own hardware
        # queue (HIP reads this once, at its first device call; 4 by default)
        os.environ["GPU_MAX_HW_QUEUES"] = str(4 * SERVE_SLOTS + 1)
    import torch
    from paper_2410_18129_amd import counts, montexp as mx
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    mx.lib()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    bits, n, w = a.bits, a.batch, a.window
    if a.only:
        only_line(a, mx, counts, dev, stream)
        return

    # ---- headline: config 2, 65536 x 2048-bit, window 5, truncated ---------
    b2 = Batch(mx, bits, n, 2, dev)

    def step(plain=False, win=w, cios=False, kara_redc=False):
        mx.modexp(b2.ctx, b2.base, b2.exp, bits, window=win, out=b2.out, plain=plain, cios=cios, kara_redc=kara_redc,
                  stream=stream)

    wall, kms = time_launches(step, a.steps, a.warmup, stream)
    value = n * a.steps / wall
    kavg = sum(kms) / len(kms)
    prod = counts.modexp_products(bits, bits, w, trunc=True)
    achieved = prod * n / (kavg * 1e-3)
    khash = kernel_hash()
    traffic = measured_traffic(khash)
    res = {
        "metric": METRIC, "value": value, "unit": "modexp/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": wall * 1e3 / a.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "%d-bit constant-time fixed-window modexp, batch %d, window %d, truncated "
                               "Montgomery reduction, %d-bit exponents (seeded random odd moduli, bases < N)"
                               % (bits, n, w, bits),
                   "global_batch": n, "bits": bits, "window": w, "limb_bits": 28, "limbs": counts.limbs(bits),
                   "parallelism": "one instance per lane, one GPU"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": counts.PEAK_MAD_PER_S / 1e12,
                     "unit": "Tmad/s", "frac": achieved / counts.PEAK_MAD_PER_S, "traffic": traffic,
                     "kernel": "k_modexp<74,32,true>", "kernel_ms": kavg, "source_hash": khash,
                     "work_per_launch": "%d instances x %d 28x28-bit products" % (n, prod)},
    }
    wall_p, kms_p = time_launches(lambda: step(plain=True), max(2, a.steps // 2), 1, stream)
    vp = n * len(kms_p) / wall_p
    prod_p = counts.modexp_products(bits, bits, w, trunc=False)
    kp = sum(kms_p) / len(kms_p)
    res["plain"] = {"value": vp, "unit": "modexp/s", "kernel_ms": kp,
                    "frac": prod_p * n / (kp * 1e-3) / counts.PEAK_MAD_PER_S}
    res["trunc_speedup"] = value / vp
    # the word-interleaved multiplication (Algorithm 4, CIOS) on the same inputs
    wall_c, kms_c = time_launches(lambda: step(cios=True), max(2, a.steps // 2), 1, stream)
    vc = n * len(kms_c) / wall_c
    kc = sum(kms_c) / len(kms_c)
    res["cios"] = {"value": vc, "unit": "modexp/s", "kernel_ms": kc,
                   "frac": counts.modexp_products(bits, bits, w, cios=True) * n / (kc * 1e-3) / counts.PEAK_MAD_PER_S}
    res["trunc_vs_cios"] = value / vc
    # the truncated high half of q*N by one-level Karatsuba (Section 5): the same products, more additions
    wall_k, kms_k = time_launches(lambda: step(kara_redc=True), max(2, a.steps // 2), 1, stream)
    vk = n * len(kms_k) / wall_k
    res["kara_redc"] = {"value": vk, "unit": "modexp/s", "kernel_ms": sum(kms_k) / len(kms_k)}
    res["trunc_vs_kara_redc"] = value / vk
    # the window the library picks for this class (3: the table stays in the last-level cache)
    tuned = {}
    for plain in (False, True):
        wl3, k3 = time_launches(lambda: step(plain=plain, win=3), max(2, a.steps // 2), 1, stream)
        tuned["plain" if plain else "trunc"] = n * len(k3) / wl3
        if not plain:
            p3 = counts.modexp_products(bits, bits, 3, trunc=True)
            tuned["frac"] = p3 * n / (sum(k3) / len(k3) * 1e-3) / counts.PEAK_MAD_PER_S
    tuned["trunc_speedup"] = tuned["trunc"] / tuned["plain"]
    res["window3"] = tuned
    progress("headline, plain, CIOS and window-3 launches done")
    # modmul / modsqr per second on the same moduli (values in [0, 2N))
    A = torch.nn.functional.pad(b2.base, (0, b2.ctx.mont_words - b2.ctx.words))
    B = torch.roll(A, 1, 0).contiguous()
    O = torch.empty_like(A)
    nl = counts.limbs(bits)
    for op, fn in (("mul", lambda kw: mx.mont_mul(b2.ctx, A, B, out=O, stream=stream, **kw)),
                   ("sqr", lambda kw: mx.mont_sqr(b2.ctx, A, out=O, stream=stream, **kw))):
        rates = {}
        for r, kw in (("trunc", {}), ("plain", {"plain": True}), ("cios", {"cios": True}),
                      ("kara", {"kara_redc": True})):
            wl_, kk = time_launches(lambda: fn(kw), 20, 3, stream)
            rates[r] = n * 20 / wl_
            if r == "trunc":
                res["mod%s_per_s" % op] = rates[r]
                res["mod%s_frac" % op] = (counts.op_products(nl, True)[op] * n / (sum(kk) / len(kk) * 1e-3)
                                          / counts.PEAK_MAD_PER_S)
        res["mod%s_trunc_speedup" % op] = rates["trunc"] / rates["plain"]
        res["mod%s_cios_per_s" % op] = rates["cios"]
        res["mod%s_trunc_vs_cios" % op] = rates["trunc"] / rates["cios"]
        # the truncated high half of q*N by one-level Karatsuba (the same products, more additions)
        res["mod%s_kara_redc_per_s" % op] = rates["kara"]
        res["mod%s_trunc_vs_kara_redc" % op] = rates["trunc"] / rates["kara"]
    b2.ctx.close()
    progress("modmul / modsqr done")
    del b2

    if not a.quick:
        res["workloads"] = other_workloads(a, mx, counts, dev, stream)
        crt = res["workloads"]["rsa2048_crt"]
        # an RSA-2048 private-key operation without the CRT is one 2048-bit exponentiation (window 3 above)
        crt["vs_direct_2048_w3"] = crt["ops_per_s_trunc"] / res["window3"]["trunc"]
    if not a.no_cpu:
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        cores = max(1, min(cores, 16))
        res["cpu_baseline"] = cpu_baseline(cores)
        progress("oracle CPU baseline done")
    print(json.dumps(res), flush=True)


def only_line(a, mx, counts, dev, stream):
    """One configuration's launches alone (for a profiler run): prints its kernel time per launch."""
    if a.only == "headline":
        b = Batch(mx, a.bits, a.batch, 2, dev)
        fn = lambda: mx.modexp(b.ctx, b.base, b.exp, a.bits, window=a.window, out=b.out, plain=a.plain,
                               stream=stream)
        work = counts.modexp_products(a.bits, a.bits, a.window) * b.n  # the truncated method's products
        name = "%d x %d-bit modexp, window %d%s" % (b.n, a.bits, a.window, ", plain reduction" if a.plain else "")
    else:
        b = Batch(mx, 4096, 16384, 3, dev)
        fn = lambda: mx.modexp(b.ctx, b.base, b.exp, 4096, window=6, out=b.out, block=True, stream=stream)
        work = counts.modexp_products(4096, 4096, 6) * b.n
        name = "16384 x 4096-bit modexp, window 6, block schoolbook"
    wall, kms = time_launches(fn, a.steps, a.warmup, stream)
    kavg = sum(kms) / len(kms)
    print(json.dumps({"only": name, "steps": a.steps, "warmup": a.warmup, "ms_per_step": wall * 1e3 / a.steps,
                      "kernel_ms": kavg, "kernel_ms_each": kms,
                      "frac": work / (kavg * 1e-3) / counts.PEAK_MAD_PER_S}), flush=True)
    b.ctx.close()


def rsa_crt_workload(mx, counts, dev, stream, nr=65536):
    """RSA-2048 private-key operations by the CRT (two 1024-bit exponentiations and Garner's recombination
    per operation) over 32 seeded keys, ciphertexts uniform below each key's modulus."""
    import numpy as np
    import torch
    from paper_2410_18129_amd import workload as wl
    keys = wl.rsa_keys(wl.load_primes(1024))
    g = wl.stream(10, "misc")
    key_of = g.integers(0, len(keys), size=nr)
    cs = wl.rsa_messages(g, keys, key_of)
    ctx_p = mx.Context(wl.ints_to_words([k["p"] for k in keys], 16), 1024)
    ctx_q = mx.Context(wl.ints_to_words([k["q"] for k in keys], 16), 1024)

    def dev_words(vals, words):
        return torch.from_numpy(wl.ints_to_words(vals, words).view(np.int64)).to(dev)

    c = dev_words(cs, 32)
    dp = dev_words([keys[k]["dp"] for k in key_of], 16)
    dq = dev_words([keys[k]["dq"] for k in key_of], 16)
    qi = dev_words([keys[k]["qinv"] for k in key_of], 16)
    kidx = torch.from_numpy(key_of.astype(np.int32)).to(dev)
    o = torch.empty_like(c)
    res = {"instances": nr, "keys": len(keys), "window": 3}
    for tag, kw in (("trunc", {}), ("plain", {"plain": True})):
        wl_, k = time_launches(lambda: mx.rsa_crt(ctx_p, ctx_q, c, dp, dq, qi, window=3, out=o, key_idx=kidx,
                                                  stream=stream, **kw), 3, 1, stream)
        res["ops_per_s_" + tag] = nr * 3 / wl_
        res["ms_per_batch_" + tag] = sum(k) / len(k)
    # work: two 1024-bit exponentiations with 1024-bit exponents per operation (the CRT steps are O(n^2))
    res["frac"] = (2 * counts.modexp_products(1024, 1024, 3) * nr / (res["ms_per_batch_trunc"] * 1e-3)
                   / counts.PEAK_MAD_PER_S)
    res["trunc_speedup"] = res["ops_per_s_trunc"] / res["ops_per_s_plain"]
    ctx_p.close()
    ctx_q.close()
    return res


def other_workloads(a, mx, counts, dev, stream):
    import torch
    from paper_2410_18129_amd import serving
    from paper_2410_18129_amd import workload as wl
    out = {}
    # ---- config 1: 8 x 1024-bit ------------------------------------------------
    b1 = Batch(mx, 1024, 8, 1, dev)
    c1 = {}
    # the latency of one exponentiation: one lane per instance (register-resident), or four lanes per
    # instance (the block kernel with its arrays in LDS)
    for tag, kw in (("trunc", {}), ("plain", {"plain": True}), ("cios", {"cios": True}),
                    ("trunc_four_lanes", {"block": True})):
        wl_, k = time_launches(lambda: mx.modexp(b1.ctx, b1.base, b1.exp, 1024, window=5, out=b1.out, stream=stream,
                                                 **kw), 5, 2, stream)
        c1["modexp_ms_" + tag] = min(k)
    out["c1_1024x8"] = c1
    progress("8 x 1024-bit done")
    b1.ctx.close()
    # ---- config 3: 16384 x 4096-bit, schoolbook vs one-level Karatsuba -------------
    b3 = Batch(mx, 4096, 16384, 3, dev)
    c3 = {}
    for impl in (True, "karatsuba"):
        tag = "karatsuba" if impl == "karatsuba" else "schoolbook"
        wl_, k = time_launches(lambda: mx.modexp(b3.ctx, b3.base, b3.exp, 4096, window=6, out=b3.out, block=impl,
                                                 stream=stream), 2, 1, stream)
        c3["modexp_per_s_" + tag] = b3.n * 2 / wl_
        c3["frac_" + tag] = (counts.modexp_products(4096, 4096, 6) * b3.n / (sum(k) / len(k) * 1e-3) /
                             counts.PEAK_MAD_PER_S)
        A = torch.nn.functional.pad(b3.base, (0, b3.ctx.mont_words - b3.ctx.words))
        O = torch.empty_like(A)
        wl_, _ = time_launches(lambda: mx.mont_mul(b3.ctx, A, A, out=O, block=impl, stream=stream), 5, 1, stream)
        c3["modmul_per_s_" + tag] = b3.n * 5 / wl_
    # the Karatsuba kernel runs one lane per instance; the schoolbook at one lane too, for a like-for-like ratio
    wl_, k = time_launches(lambda: mx.modexp(b3.ctx, b3.base, b3.exp, 4096, window=6, out=b3.out, block=True,
                                             one_lane=True, stream=stream), 2, 1, stream)
    c3["modexp_per_s_schoolbook_one_lane"] = b3.n * 2 / wl_
    c3["schoolbook_vs_karatsuba_one_lane"] = c3["modexp_per_s_schoolbook_one_lane"] / c3["modexp_per_s_karatsuba"]
    # the truncated q N by one-level Karatsuba in the block kernel (one lane per instance, row f2)
    wl_, k = time_launches(lambda: mx.modexp(b3.ctx, b3.base, b3.exp, 4096, window=6, out=b3.out, block=True,
                                             kara_redc=True, stream=stream), 2, 1, stream)
    c3["modexp_per_s_kara_redc_one_lane"] = b3.n * 2 / wl_
    c3["schoolbook_vs_kara_redc_one_lane"] = (c3["modexp_per_s_schoolbook_one_lane"] /
                                              c3["modexp_per_s_kara_redc_one_lane"])
    # word-interleaved Montgomery multiplication (Algorithm 4) with 37-limb words, one lane per instance (row f1)
    wl_, k = time_launches(lambda: mx.modexp(b3.ctx, b3.base, b3.exp, 4096, window=6, out=b3.out, cios=True,
                                             stream=stream), 2, 1, stream)
    c3["modexp_per_s_cios_one_lane"] = b3.n * 2 / wl_
    c3["schoolbook_vs_cios_one_lane"] = c3["modexp_per_s_schoolbook_one_lane"] / c3["modexp_per_s_cios_one_lane"]
    # raw products at Table 6's largest sizes (limb counts 147 and 149), schoolbook and Karatsuba at one
    # and two levels, 16384 seeded instances each
    g = wl.stream(3, "ops_a")
    raw = {}
    for pbits in (4108, 4154):
        a_ = mx.to_device(wl.random_words(g, pbits, b3.n), dev)
        b_ = mx.to_device(wl.random_words(g, pbits, b3.n), dev)
        o_ = torch.empty((b3.n, mx.words_for(2 * pbits)), dtype=torch.int64, device=dev)
        line = {}
        for lv, m in enumerate(("schoolbook", "karatsuba", "karatsuba2")):
            ws_ = torch.empty(mx.mp_mul_ws_bytes(pbits, b3.n, m), dtype=torch.uint8, device=dev)
            wl_, k = time_launches(lambda: mx.mp_mul(a_, b_, pbits, method=m, out=o_, ws=ws_, stream=stream), 10, 2,
                                   stream)
            kms = sum(k) / len(k)
            line[m] = {"products_per_s": b3.n * 10 / wl_, "kernel_ms": kms,
                       "frac": counts.mul_products(pbits, lv) * b3.n / (kms * 1e-3) / counts.PEAK_MAD_PER_S,
                       "partial_products": counts.mul_products(pbits, lv)}
            del ws_
        line["karatsuba_vs_schoolbook"] = line["karatsuba"]["products_per_s"] / line["schoolbook"]["products_per_s"]
        line["karatsuba2_vs_schoolbook"] = (line["karatsuba2"]["products_per_s"] /
                                            line["schoolbook"]["products_per_s"])
        raw[str(pbits)] = line
    c3["raw_products_16384"] = raw
    out["c3_4096x16384"] = c3
    progress("16384 x 4096-bit done")
    out["rsa2048_crt"] = rsa_crt_workload(mx, counts, dev, stream)
    progress("CRT-RSA done")
    b3.ctx.close()
    del b3
    # ---- config 4: 200k mixed sizes, one persistent launch, schedule per class from the autotuner ----
    from paper_2410_18129_amd import autotune
    sizes = wl.size_mix(wl.stream(4, "sizes"), 200000)
    nb = {c: int((sizes == c).sum()) for c in (1024, 2048, 3072, 4096)}
    t0 = time.perf_counter()
    sched, model_ms = autotune.plan_for_mix(nb)
    tune_s = time.perf_counter() - t0
    progress("autotuner done (%.1f s)" % tune_s)
    batches = [Batch(mx, c, nb[c], 4 + c, dev) for c in nb]

    def mixed_line(args_of):
        plan = mx.MixedPlan([dict({"ctx": bb.ctx, "base": bb.base, "exp": bb.exp, "exp_bits": bb.bits, "out": bb.out},
                                  **args_of(bb.bits)) for bb in batches])
        wl_, k = time_launches(lambda: plan.launch(stream=stream, graph=True), 2, 1, stream)
        work = sum(counts.modexp_products(bb.bits, bb.bits, w) * bb.n for bb, w in zip(batches, plan.windows))
        line = {"modexp_per_s": 200000 * 2 / wl_, "ms_per_launch": wl_ * 1e3 / 2, "windows": plan.windows,
                "jobs": plan.njobs, "persistent_waves": plan.nslots,
                "frac": work / (sum(k) / len(k) * 1e-3) / counts.PEAK_MAD_PER_S}
        plan.close()
        return line

    c4 = mixed_line(lambda bits: autotune.batch_args(sched[bits]))
    c4.update({"counts": nb, "hip_graph": True, "schedule": {str(b): sched[b] for b in sched},
               "schedule_source": "autotuner: tile times of every candidate (window, kernel family, lanes per "
                                  "instance) measured in the persistent kernel, choice by the modelled makespan",
               "model_ms": model_ms, "tune_s": tune_s})
    # the hand-set schedule of earlier measurements (windows 3 / 5, default lanes), for comparison
    hand = mixed_line(lambda bits: {"window": 3 if bits <= 2048 else 5})
    c4["handset_ms_per_launch"] = hand["ms_per_launch"]
    out["c4_mixed_200k"] = c4
    progress("200k mixed launch done")
    offline = c4["modexp_per_s"]
    for bb in batches:
        bb.ctx.close()
    del batches
    torch.cuda.synchronize()
    # ---- config 5: serving, Poisson arrivals over 2000 resident moduli ---------------------
    rates = (50e3, 100e3, 200e3, 300e3, 400e3)
    # at least 200k requests per rate, and a trace of at least 3 s (several batch durations of the
    # slowest class), so that throughput is not just the fill and drain of a burst
    span_s, nmin = 3.0, 200000
    # SERVE_SLOTS execution slots (a stream and a workspace each) per class, each stream on its own
    # hardware queue; batches of a class are paced about a batch duration / SERVE_SLOTS apart
    maxb = {1024: 65536, 2048: 65536, 3072: 32768, 4096: 32768}
    sweep = []
    for r in rates:
        nreq = int(max(nmin, r * span_s))
        tr = serving.Trace(nreq, r, k=5)
        ex = serving.GpuExecutor(tr, maxb, mem_budget=8 << 30, windows={1024: 3, 2048: 3, 3072: 5, 4096: 5},
                                 max_slots=SERVE_SLOTS)
        st = serving.Server(ex, tr.classes, maxb).run(tr, timeout_s=300)
        s = st.stats()
        s["vs_offline"] = s["throughput"] / offline
        sweep.append(s)
        ex.close()
        del ex, tr
        torch.cuda.synchronize()
        progress("serving at %.0f req/s done" % r)
    out["c5_serving"] = {"moduli": 2000, "slots_per_class": SERVE_SLOTS,
                         "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "0")), "sweep": sweep,
                         "offline_mixed_modexp_per_s": offline}
    return out


if __name__ == "__main__":
    main()
