"""Continuous-batching modexp server over device-resident Montgomery contexts.

Requests (size class, modulus id, base, exponent) arrive over time.  The
scheduler keeps one FIFO per size class and a fixed pool of execution slots
per class.  A slot owns the device memory one in-flight batch needs (its
exponentiation workspace) and a stream; the pool is sized from a memory
budget at start-up, so admission is by memory: a batch is launched only
when a slot of its class is free, otherwise its requests wait.  Whenever a
slot is free and requests are waiting, the waiting requests (up to the
class's batch cap) are launched at once, so requests that arrive while
other batches run join the next batch while those batches are still on the
GPU, and batches on different slots overlap on the device (continuous
batching).  Latency is completion (host clock, when the slot's event has
fired) minus arrival.

The scheduler is independent of the device: an executor provides
``slots(cls)``, ``launch(slot, cls, lo, hi)`` (requests lo..hi-1 of the
class, in arrival order), ``poll(slot) -> None | True | Exception``.
``GpuExecutor`` runs the library's constant-time exponentiation; the tests
drive the same scheduler with a CPU fake.
"""
import time
from collections import deque

import numpy as np

from . import montexp as mx
from . import workload as wl

MIX = (1024, 2048, 3072, 4096)
MIX_P = (0.40, 0.35, 0.15, 0.10)
MODULI_PER_CLASS = {1024: 800, 2048: 700, 3072: 300, 4096: 200}  # 2000 resident moduli


class Trace:
    """A seeded request stream: Poisson arrivals, the size mix, Zipf(1.1) modulus reuse.

    Per class c the requests are numbered 0..count[c]-1 in arrival order;
    ``cls[k]``, ``local[k]`` map global request k to that numbering.
    """

    def __init__(self, n, rate, k=5, classes=MIX, probs=MIX_P, moduli=MODULI_PER_CLASS, zipf_s=1.1):
        self.n, self.rate, self.classes = n, rate, tuple(classes)
        self.arrival = wl.poisson_arrivals(wl.stream(k, "arrivals"), n, rate)
        self.cls = wl.size_mix(wl.stream(k, "sizes"), n, classes, probs)
        self.mods = {}
        self.mod_id = np.zeros(n, dtype=np.int32)
        self.local = np.zeros(n, dtype=np.int64)
        self.count = {}
        gm = wl.stream(k, "moduli")
        gz = wl.stream(k, "misc")
        for c in self.classes:
            idx = np.nonzero(self.cls == c)[0]
            self.count[c] = len(idx)
            self.local[idx] = np.arange(len(idx))
            self.mods[c] = wl.random_moduli(gm, c, moduli[c])
            self.mod_id[idx] = wl.zipf_ranks(gz, len(idx), moduli[c], zipf_s).astype(np.int32)
        self.base, self.exp = {}, {}
        gb, ge = wl.stream(k, "bases"), wl.stream(k, "exps")
        for c in self.classes:
            idx = np.nonzero(self.cls == c)[0]
            m = self.mods[c][self.mod_id[idx]]
            self.base[c] = wl.random_below_fast(gb, m, c)
            self.exp[c] = wl.random_exponents(ge, c, len(idx))
        # cumulative arrivals per class: arrived_by[c][k] = requests of c among the first k
        self.arrived_by = {c: np.concatenate([[0], np.cumsum(self.cls == c)]) for c in self.classes}


class Server:
    """Continuous-batching scheduler (see the module docstring).

    Pacing: a batch costs about the same time whatever its size (every lane
    runs one whole exponentiation), so a class with k slots starts a new batch
    at most every (observed batch duration) / k seconds, unless a full batch is
    waiting.  Without pacing, a trickle of arrivals would occupy every slot
    with a tiny batch and the next arrivals would wait a whole batch duration.
    """

    def __init__(self, executor, classes, max_batch, idle_sleep=20e-6, pace=True):
        self.ex, self.classes = executor, tuple(classes)
        self.max_batch = dict(max_batch)
        self.idle_sleep = idle_sleep
        self.pace = pace

    def run(self, trace, timeout_s=600.0):
        """Replays the trace in real time; returns per-request finish times and status."""
        n = trace.n
        finish = np.full(n, np.nan)
        failed = np.zeros(n, dtype=bool)
        batches = []  # (cls, lo, hi, launch time)
        head = {c: 0 for c in self.classes}  # next request (class numbering) not yet launched
        free = {c: deque(self.ex.slots(c)) for c in self.classes}
        nslot = {c: max(1, len(free[c])) for c in self.classes}
        dur = {c: 0.0 for c in self.classes}  # running estimate of a batch's duration per class
        last = {c: -1e30 for c in self.classes}  # launch time of the class's latest batch
        busy = []  # (slot, cls, lo, hi, launch time)
        # global request ids of class c in class order, to write finish times
        gid = {c: np.nonzero(trace.cls == c)[0] for c in self.classes}
        done = 0
        nxt = 0
        t0 = time.perf_counter()
        while done < n:
            now = time.perf_counter() - t0
            if now > timeout_s:
                raise TimeoutError("serving trace did not drain in %.0f s" % timeout_s)
            nxt = int(np.searchsorted(trace.arrival, now, side="right"))
            progressed = False
            # retire finished batches
            still = []
            for slot, c, lo, hi, tl in busy:
                st = self.ex.poll(slot)
                if st is None:
                    still.append((slot, c, lo, hi, tl))
                    continue
                t = time.perf_counter() - t0
                dur[c] = t - tl if dur[c] == 0.0 else 0.7 * dur[c] + 0.3 * (t - tl)
                ids = gid[c][lo:hi]
                finish[ids] = t
                if st is not True:
                    failed[ids] = True
                done += hi - lo
                free[c].append(slot)
                progressed = True
            busy = still
            # launch waiting requests on free slots, the class with the oldest waiting request first
            order = []
            for c in self.classes:
                arrived = int(trace.arrived_by[c][nxt])
                if arrived > head[c] and free[c]:
                    order.append((trace.arrival[gid[c][head[c]]], c, arrived))
            for _, c, arrived in sorted(order):
                while free[c] and arrived > head[c]:
                    lo = head[c]
                    hi = min(arrived, lo + self.max_batch[c])
                    if (self.pace and hi - lo < self.max_batch[c] and
                            time.perf_counter() - t0 - last[c] < dur[c] / nslot[c]):
                        break
                    slot = free[c].popleft()
                    try:
                        self.ex.launch(slot, c, lo, hi)
                    except Exception:  # a failed launch fails its requests, the server keeps serving
                        ids = gid[c][lo:hi]
                        finish[ids] = time.perf_counter() - t0
                        failed[ids] = True
                        done += hi - lo
                        free[c].append(slot)
                        head[c] = hi
                        continue
                    tl = time.perf_counter() - t0
                    busy.append((slot, c, lo, hi, tl))
                    batches.append((c, lo, hi, tl))
                    last[c] = tl
                    head[c] = hi
                    progressed = True
            if not progressed:
                if busy or nxt < n:
                    time.sleep(self.idle_sleep)
        return ServeResult(trace, finish, failed, batches)


class ServeResult:
    def __init__(self, trace, finish, failed, batches):
        self.trace, self.finish, self.failed, self.batches = trace, finish, failed, batches

    def stats(self, warmup_frac=0.10):
        tr = self.trace
        k0 = int(tr.n * warmup_frac)
        ok = ~self.failed
        ok[:k0] = False
        lat = (self.finish - tr.arrival)[ok]
        span = np.nanmax(self.finish[k0:]) - tr.arrival[k0] if tr.n > k0 else float("nan")
        sizes = [hi - lo for _, lo, hi, _ in self.batches]
        out = {
            "offered_rate": tr.rate,
            "requests": int(ok.sum()),
            "arrival_span_s": float(tr.arrival[-1]) if tr.n else 0.0,
            "throughput": float(ok.sum() / span) if span > 0 else float("nan"),
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else float("nan"),
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else float("nan"),
            "max_ms": float(lat.max() * 1e3) if lat.size else float("nan"),
            "batches": len(self.batches),
            "mean_batch": float(np.mean(sizes)) if sizes else 0.0,
            "failed": int(self.failed.sum()),
        }
        all_lat = self.finish - tr.arrival
        for c in tr.classes:
            m = ok & (tr.cls == c)
            if m.any():
                out["p50_ms_%d" % c] = float(np.percentile(all_lat[m], 50) * 1e3)
                out["p99_ms_%d" % c] = float(np.percentile(all_lat[m], 99) * 1e3)
        return out


def hw_queues_needed(classes, max_slots):
    """One hardware queue per execution slot, plus the default stream's."""
    return len(tuple(classes)) * max_slots + 1


class GpuExecutor:
    """Batches run through modexp_batch_ws on the trace's device-resident inputs.

    Contexts: one per class holding that class's moduli (resident for the run).
    Slots: preallocated workspaces (and a stream each), as many per class as
    the memory budget allows, at most ``max_slots`` per class.  Batches on
    different streams run concurrently only on different hardware queues:
    HIP's GPU_MAX_HW_QUEUES (read once, when the process first initialises
    the device) must be at least ``hw_queues_needed(classes, max_slots)``, or
    a short batch can wait behind a long one of another class on a shared
    queue.
    """

    def __init__(self, trace, max_batch, mem_budget, windows=None, max_slots=4, device="cuda", one_lane_from=16384,
                 two_lanes_from=None):
        import torch
        self.torch = torch
        self.one_lane_from = one_lane_from
        self.two_lanes_from = one_lane_from if two_lanes_from is None else two_lanes_from
        self.classes = trace.classes
        self.ctx = {c: mx.Context(trace.mods[c], c) for c in self.classes}
        self.windows = windows or {c: 0 for c in self.classes}
        dev = torch.device(device)
        self.base = {c: mx.to_device(trace.base[c], dev) for c in self.classes}
        self.exp = {c: mx.to_device(trace.exp[c], dev) for c in self.classes}
        self.out = {c: torch.zeros_like(self.base[c]) for c in self.classes}
        idx = {c: trace.mod_id[trace.cls == c] for c in self.classes}
        self.cidx = {c: torch.from_numpy(np.ascontiguousarray(idx[c])).to(dev) for c in self.classes}
        self._slots = {c: [] for c in self.classes}
        used = 0
        # one slot per class first (every class must be servable), then round-robin while the budget lasts
        for rnd in range(max_slots):
            for c in self.classes:
                nb = mx.modexp_ws_bytes(self.ctx[c], max_batch[c], self.windows[c])
                if used + nb > mem_budget and rnd > 0:
                    continue
                if used + nb > mem_budget and rnd == 0:
                    raise MemoryError("memory budget %d B cannot hold one %d-bit slot (%d B)" % (mem_budget, c, nb))
                ws = torch.empty(nb, dtype=torch.uint8, device=dev)
                self._slots[c].append({"ws": ws, "stream": torch.cuda.Stream(device=dev), "event": None})
                used += nb
        self.mem_used = used
        torch.cuda.synchronize()

    def slots(self, c):
        return list(self._slots[c])

    def launch(self, slot, c, lo, hi):
        torch = self.torch
        st = slot["stream"]
        # the batch size tells the load: the block kernels keep one lane per instance for
        # large batches (throughput: the other classes' work fills the SIMDs one lane leaves
        # idle) and run four lanes per instance below (latency); two lanes only when asked for
        # (two_lanes_from), four lanes being faster than two at every batch size
        n = hi - lo
        mx.modexp_ws(self.ctx[c], self.base[c][lo:hi], self.exp[c][lo:hi], c, slot["ws"], window=self.windows[c],
                     out=self.out[c][lo:hi], ctx_idx=self.cidx[c][lo:hi], stream=st,
                     one_lane=n >= self.one_lane_from, two_lanes=self.two_lanes_from <= n < self.one_lane_from)
        ev = torch.cuda.Event()
        ev.record(st)
        slot["event"] = ev

    def poll(self, slot):
        return True if slot["event"].query() else None

    def close(self):
        for c in self.classes:
            self.ctx[c].close()
