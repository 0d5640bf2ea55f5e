"""Per-size-class plan choice (window and kernel family) for the mixed launch.

The measurement runs in the library (mx_tune_modexp: seeded sample inputs,
every candidate window, register-resident and block kernels where both
exist, best of several runs).  This module only caches the winners in a
JSON file keyed by GPU architecture and size class, so later plans reuse
them without re-measuring.
"""
import json
import os

from . import montexp as mx
from . import workload as wl

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "montexp", "plan_cache.json")
# windows whose per-slot workspace fits the mixed launch (see mx_mixed_plan_create)
CANDIDATES = {1024: (3, 4, 5), 2048: (3, 4, 5), 3072: (3, 4, 5), 4096: (3, 4, 5)}


def _arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def load(path=DEFAULT_CACHE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save(cache, path=DEFAULT_CACHE):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_class(bits, n=4096, reps=2, seed_k=9):
    """Measures the candidates for one class on n seeded moduli; returns the plan dict."""
    mods = wl.random_moduli(wl.stream(seed_k, "moduli"), bits, n)
    ctx = mx.Context(mods, bits)
    try:
        w, flags, ms = mx.tune_modexp(ctx, n, bits, windows=CANDIDATES.get(bits, (3, 4, 5)), try_block=True,
                                      reps=reps)
    finally:
        ctx.close()
    return {"window": w, "block": bool(flags & mx.MX_IMPL_BLOCK), "karatsuba": bool(flags & mx.MX_MUL_KARATSUBA),
            "ms_per_tile": ms, "sample": n}


def plan_for(classes, path=DEFAULT_CACHE, retune=False, n=4096):
    """{bits: plan} for the given classes, measuring the ones not cached for this GPU."""
    cache = load(path)
    arch = _arch()
    entry = cache.setdefault(arch, {})
    changed = False
    for b in classes:
        if retune or str(b) not in entry:
            entry[str(b)] = tune_class(b, n=n)
            changed = True
    if changed:
        save(cache, path)
    return {b: entry[str(b)] for b in classes}
