"""Autotuner of the mixed-size persistent launch.

For every size class it picks the window, the kernel family (register-resident,
block schoolbook, block Karatsuba) and the lanes per instance, which fixes the
tile a wavefront takes from the job list (64 / lanes instances).

1. Tile times, measured and cached per GPU architecture: for each candidate
   schedule of a class, a one-batch mixed plan holding exactly one tile per
   persistent wave is launched (best of a few launches).  Every wave runs one
   tile, so the launch time is the tile time inside the persistent kernel
   itself, at the occupancy of the real launch.
2. The choice, modelled per workload: each class keeps its fastest schedule
   per lane count (time per instance); every combination of those is scored by
   the makespan of the plan's own schedule (tiles in decreasing cost order, each
   taken by the next free wave) with the measured tile times, and the shortest
   wins.  Fewer instances per tile (two lanes) cost more in total but shorten
   the longest tiles, which can end the launch sooner.

The measurements run in the library (mixed plans, HIP events on the launch
stream); this module only generates the seeded sample inputs, caches the times
in a JSON file and runs the scheduling model.
"""
import heapq
import itertools
import json
import os

from . import montexp as mx
from . import workload as wl

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "montexp", "plan_cache.json")
FAMILY = {0: "register", mx.MX_IMPL_BLOCK: "block", mx.MX_MUL_KARATSUBA: "karatsuba"}
# (window, flags) candidates per class; windows whose per-wave workspaces fit the plan's 2 GiB limit
_B, _K, _1, _2, _4 = mx.MX_IMPL_BLOCK, mx.MX_MUL_KARATSUBA, mx.MX_ONE_LANE, mx.MX_TWO_LANES, mx.MX_FOUR_LANES
CANDIDATES = {
    1024: [(w, f) for f in (0, _B) for w in (3, 4, 5)],
    2048: [(w, f) for f in (0, _B, _K) for w in (3, 4, 5)],
    3072: [(w, f) for f in (_B | _1, _B | _2, _B | _4) for w in (4, 5)],
    4096: [(w, f) for f in (_B | _1, _B | _2, _B | _4, _K) for w in (4, 5)],
}


def lanes_of(bits, flags):
    """Lanes per instance of a schedule (the plan's rule: two for 4096-bit schoolbook tiles by default)."""
    if flags & mx.MX_FOUR_LANES:
        return 4
    if flags & mx.MX_TWO_LANES:
        return 2
    if flags & (mx.MX_ONE_LANE | mx.MX_MUL_KARATSUBA) or bits != 4096:
        return 1
    return 2


def _arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _waves():
    import torch
    return 4 * torch.cuda.get_device_properties(0).multi_processor_count  # one per SIMD


def load(path=DEFAULT_CACHE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save(cache, path=DEFAULT_CACHE):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _key(window, flags):
    return "w%d_f%d" % (window, flags)


def measure_class(bits, waves=None, reps=2, seed_k=9, candidates=None):
    """{candidate key: ms per tile} for one class: each candidate as a one-batch plan of one tile per wave."""
    import torch
    waves = waves or _waves()
    cands = candidates or CANDIDATES[bits]
    n = waves * 64  # the one-lane batch; two-lane candidates use its first half
    mods = wl.random_moduli(wl.stream(seed_k, "moduli"), bits, n)
    ctx = mx.Context(mods, bits)
    base = mx.to_device(wl.random_below_fast(wl.stream(seed_k, "bases"), mods, bits))
    exps = mx.to_device(wl.random_exponents(wl.stream(seed_k, "exps"), bits, n))
    out = torch.empty_like(base)
    stream = torch.cuda.current_stream()
    res = {}
    try:
        for w, flags in cands:
            m = n // lanes_of(bits, flags)
            plan = mx.MixedPlan([{"ctx": ctx, "base": base[:m], "exp": exps[:m], "exp_bits": bits, "out": out[:m],
                                  "window": w, "flags": flags}])
            try:
                assert plan.njobs == waves and plan.nslots == waves, (plan.njobs, plan.nslots)
                plan.launch(stream=stream)  # warm-up
                best = float("inf")
                for _ in range(reps):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    plan.launch(stream=stream)
                    e1.record(stream)
                    e1.synchronize()
                    best = min(best, e0.elapsed_time(e1))
                res[_key(w, flags)] = best
            finally:
                plan.close()
    finally:
        ctx.close()
    return res


def tile_times(classes, path=DEFAULT_CACHE, retune=False, waves=None, reps=2):
    """{bits: {candidate key: ms per tile}}, measuring the classes not cached for this GPU and wave count."""
    cache = load(path)
    waves = waves or _waves()
    entry = cache.setdefault("%s/%d" % (_arch(), waves), {})
    changed = False
    for b in classes:
        if retune or str(b) not in entry:
            entry[str(b)] = measure_class(b, waves=waves, reps=reps)
            changed = True
    if changed:
        save(cache, path)
    return {b: entry[str(b)] for b in classes}


def makespan(tiles, waves):
    """Length of the plan's schedule: tiles (durations) in decreasing order, each to the next free wave."""
    free = [0.0] * min(waves, max(1, len(tiles)))
    heapq.heapify(free)
    for t in sorted(tiles, reverse=True):
        heapq.heappush(free, heapq.heappop(free) + t)
    return max(free) if tiles else 0.0


def choose(counts, times, waves):
    """The schedule per class minimising the modelled makespan for `counts` {bits: instances}.

    Returns ({bits: schedule dict}, modelled ms)."""
    options = {}
    for bits in counts:
        per_lanes = {}
        for key, ms in times[bits].items():
            w, f = (int(x[1:]) for x in key.split("_"))
            lanes = lanes_of(bits, f)
            cost = ms * lanes / 64.0  # per instance
            if lanes not in per_lanes or cost < per_lanes[lanes][0]:
                per_lanes[lanes] = (cost, w, f, ms)
        options[bits] = [(lanes, v[1], v[2], v[3]) for lanes, v in sorted(per_lanes.items())]
    best = None
    for combo in itertools.product(*[options[b] for b in counts]):
        tiles = []
        for bits, (lanes, w, f, ms) in zip(counts, combo):
            per_tile = 64 // lanes
            tiles += [ms] * (-(-counts[bits] // per_tile))
        span = makespan(tiles, waves)
        if best is None or span < best[0]:
            best = (span, combo)
    plan = {}
    for bits, (lanes, w, f, ms) in zip(counts, best[1]):
        fam = FAMILY[f & (mx.MX_IMPL_BLOCK | mx.MX_MUL_KARATSUBA)]
        plan[bits] = {"window": w, "flags": f, "family": fam, "lanes": lanes, "tile_instances": 64 // lanes,
                      "ms_per_tile": ms}
    return plan, best[0]


def plan_for_mix(counts, path=DEFAULT_CACHE, retune=False, waves=None, reps=2):
    """Autotuned schedule per class for a mixed workload {bits: instances}: ({bits: schedule}, modelled ms)."""
    waves = waves or _waves()
    return choose(counts, tile_times(list(counts), path=path, retune=retune, waves=waves, reps=reps), waves)


def batch_args(schedule):
    """The MixedPlan batch keys of one class's schedule."""
    return {"window": schedule["window"], "flags": schedule["flags"], "tile_cost": schedule["ms_per_tile"]}
