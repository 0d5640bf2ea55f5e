"""Constant-time evidence for the exponentiation kernels from hardware counters.

Algorithm 7's fixed-window exponentiation is constant-time when its instruction
stream and its memory requests do not depend on the secret exponent (nor on the
base): every window runs the same squarings and multiplication, and the table
entry is selected by a full masked scan.  This probe launches one
exponentiation kernel once per input class, in a fixed order, on a batch that
gives every SIMD of the GPU a wavefront.  Under ``rocprofv3 --pmc`` each launch
is one dispatch with its own counters; ``compare`` reads rocprofv3's counter
CSV and reports, per counter, whether every input class gave the same value.

Input classes (same seeded moduli in every class):
  random, random2   uniform bases below N and uniform exponents (two draws)
  random_repeat     the inputs of `random` again: the run-to-run spread of a counter
  exp_zero, exp_ones   exponent 0 ... 0 and 1 ... 1 (all exp_bits bits), random bases
  base_zero, base_one  base 0 and base 1, random exponents

    rocprofv3 --pmc <counters> -d DIR -o ct -- python3 -m paper_2410_18129_amd.ctprobe run --bits 2048
    python3 -m paper_2410_18129_amd.ctprobe compare DIR [DIR ...]
"""
import argparse
import csv
import glob
import os
import sys

import numpy as np

CASES = ("random", "random_repeat", "random2", "exp_zero", "exp_ones", "base_zero", "base_one")
# (batch, window) per class: 65536 lanes, one wavefront per SIMD; the 4096-bit block kernel runs four
# lanes per instance at this batch size
CONFIGS = {1024: (131072, 5), 2048: (65536, 5), 3072: (65536, 5), 4096: (16384, 6)}


def _inputs(bits, n, case):
    from . import workload as wl
    mods = wl.random_moduli(wl.stream(20, "moduli"), bits, n)
    k = 21 if case == "random2" else 20
    base = wl.random_below_fast(wl.stream(k, "bases"), mods, bits)
    exps = wl.random_exponents(wl.stream(k, "exps"), bits, n)
    if case == "exp_zero":
        exps[:] = np.uint64(0)
    elif case == "exp_ones":
        exps[:] = np.uint64(0xFFFFFFFFFFFFFFFF)
        top = bits - 64 * (exps.shape[1] - 1)
        if top < 64:
            exps[:, -1] = np.uint64((1 << top) - 1)
    elif case == "base_zero":
        base[:] = np.uint64(0)
    elif case == "base_one":
        base[:] = np.uint64(0)
        base[:, 0] = np.uint64(1)
    return mods, base, exps


def run(bits, block):
    import torch
    from . import montexp as mx
    n, w = CONFIGS[bits]
    dev = torch.device("cuda:0")
    ctx = None
    for case in CASES:
        mods, base, exps = _inputs(bits, n, case)
        if ctx is None:
            ctx = mx.Context(mods, bits)
        b, e = mx.to_device(base, dev), mx.to_device(exps, dev)
        out = mx.modexp(ctx, b, e, bits, window=w, block=block)
        torch.cuda.synchronize()
        print("ctprobe: %d-bit n=%d w=%d case %s launched (dispatch %d of the exponentiation kernel)"
              % (bits, n, w, case, CASES.index(case)), flush=True)
        del out
    ctx.close()


def _read(dirs):
    """{kernel name: [{counter: value}, ...] in dispatch order} from rocprofv3 counter CSVs."""
    rows = {}
    for d in dirs:
        for path in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
            with open(path) as f:
                for r in csv.DictReader(f):
                    k = r.get("Kernel_Name", "")
                    if "k_modexp" not in k:
                        continue
                    disp = int(r.get("Dispatch_Id", r.get("Correlation_Id", 0)))
                    rows.setdefault(k, {}).setdefault(disp, {})[r["Counter_Name"]] = float(r["Counter_Value"])
    return {k: [v[d] for d in sorted(v)] for k, v in rows.items()}


def compare(dirs):
    """Prints one table per kernel: each counter under every input class, and how they compare.

    A counter that differs between `random` and `random_repeat` (the same inputs launched twice)
    depends on timing (cache hits of concurrent wavefronts), not on the data; for those the spread
    across all classes is printed beside the spread between the two identical launches.  Returns
    True when every counter that is the same for identical launches is the same for every class."""
    data = _read(dirs)
    ok_all = True
    for kern, disps in data.items():
        if len(disps) != len(CASES):
            print("%s: %d dispatches, expected %d (one per input class)" % (kern, len(disps), len(CASES)))
            ok_all = False
            continue
        counters = sorted(set().union(*[d.keys() for d in disps]))
        print("kernel %s" % kern)
        print("| counter | " + " | ".join(CASES) + " | across classes |")
        print("|---" * (len(CASES) + 2) + "|")
        for c in counters:
            vals = [d.get(c) for d in disps]
            if len(set(vals)) == 1:
                verdict = "equal"
            else:
                lo, hi = min(vals), max(vals)
                rep = abs(vals[0] - vals[1]) / max(vals[0], 1.0)
                if rep > 0:
                    verdict = "timing-dependent: spread %.3f %%, identical launches %.3f %%" % (
                        100.0 * (hi - lo) / max(lo, 1.0), 100.0 * rep)
                else:
                    verdict = "DIFFERS"
                    ok_all = False
            print("| %s | %s | %s |" % (c, " | ".join("%.0f" % v if v is not None else "-" for v in vals), verdict))
        print()
    print("every counter that is the same for identical launches is the same for every input class: %s"
          % ("yes" if ok_all else "NO"))
    return ok_all


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--bits", type=int, default=2048, choices=sorted(CONFIGS))
    r.add_argument("--block", action="store_true", help="the block kernels (the only ones above 2048 bits)")
    c = sub.add_parser("compare")
    c.add_argument("dirs", nargs="+")
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.bits, a.block or a.bits > 2048)
    else:
        sys.exit(0 if compare(a.dirs) else 1)


if __name__ == "__main__":
    main()
