"""Scheduler logic of the serving loop on the CPU, with a fake executor.

The fake runs the same batch interface as the GPU executor: results by
CPython pow, completion after a simulated service time, optional injected
failures.  Checks: every request served once and correctly, per-class FIFO
batches, continuous batching (batches of a class overlap and late arrivals
join while others run), admission bounded by the slot pool, failures
isolated to their batch.
"""
import time

import numpy as np
import pytest

from paper_2410_18129_amd import serving, workload as wl

CLASSES = (64, 128)


class FakeExecutor:
    def __init__(self, trace, slots_per_class=2, per_req_s=20e-6, fixed_s=2e-3, fail_batches=()):
        self.tr = trace
        self.nslots = slots_per_class
        self.per_req, self.fixed = per_req_s, fixed_s
        self.fail = set(fail_batches)
        self.results = {c: [None] * trace.count[c] for c in trace.classes}
        self.log = []  # (cls, lo, hi, start, end)
        self.inflight = {}
        self.launches = 0
        self.max_inflight = {c: 0 for c in trace.classes}

    def slots(self, c):
        return [(c, k) for k in range(self.nslots)]

    def launch(self, slot, c, lo, hi):
        k = self.launches
        self.launches += 1
        if k in self.fail:
            raise RuntimeError("injected launch failure")
        t = time.perf_counter()
        self.inflight[slot] = (c, lo, hi, t, t + self.fixed + self.per_req * (hi - lo))
        self.max_inflight[c] = max(self.max_inflight[c], sum(1 for s in self.inflight if s[0] == c))

    def poll(self, slot):
        c, lo, hi, t0, t1 = self.inflight[slot]
        if time.perf_counter() < t1:
            return None
        del self.inflight[slot]
        M = wl.words_to_ints(self.tr.mods[c])
        B, E = wl.words_to_ints(self.tr.base[c][lo:hi]), wl.words_to_ints(self.tr.exp[c][lo:hi])
        ids = self.tr.mod_id[self.tr.cls == c][lo:hi]
        for k in range(hi - lo):
            self.results[c][lo + k] = pow(B[k], E[k], M[ids[k]])
        self.log.append((c, lo, hi, t0, time.perf_counter()))
        return True


def _trace(n=3000, rate=60000.0, k=31):
    return serving.Trace(n, rate, k=k, classes=CLASSES, probs=(0.6, 0.4), moduli={64: 50, 128: 30})


def test_trace_mix_and_zipf_reuse():
    tr = serving.Trace(20000, 1e5, k=32, classes=serving.MIX, probs=serving.MIX_P,
                       moduli={1024: 8, 2048: 7, 3072: 3, 4096: 2})
    frac = np.array([np.mean(tr.cls == c) for c in serving.MIX])
    assert np.allclose(frac, serving.MIX_P, atol=0.02)
    assert np.all(np.diff(tr.arrival) >= 0) and abs(tr.n / tr.arrival[-1] - 1e5) < 5e3
    # Zipf(1.1): the most used modulus dominates the least used one
    ids = tr.mod_id[tr.cls == 1024]
    assert np.bincount(ids, minlength=8)[0] > 3 * np.bincount(ids, minlength=8)[7]
    for c in serving.MIX:  # bases below their moduli
        M = wl.words_to_ints(tr.mods[c])
        ids = tr.mod_id[tr.cls == c][:50]
        for b, i in zip(wl.words_to_ints(tr.base[c][:50]), ids):
            assert b < M[i]


def test_every_request_served_once_and_correctly():
    tr = _trace()
    ex = FakeExecutor(tr)
    res = serving.Server(ex, CLASSES, {64: 64, 128: 32}).run(tr)
    assert not np.isnan(res.finish).any() and not res.failed.any()
    assert np.all(res.finish >= tr.arrival)
    for c in CLASSES:
        spans = sorted((lo, hi) for cc, lo, hi, _, _ in ex.log if cc == c)
        assert spans[0][0] == 0 and spans[-1][1] == tr.count[c]
        assert all(a[1] == b[0] for a, b in zip(spans, spans[1:]))  # FIFO, contiguous, no overlap
        assert all(hi - lo <= (64 if c == 64 else 32) for lo, hi in spans)
        M = wl.words_to_ints(tr.mods[c])
        B, E = wl.words_to_ints(tr.base[c]), wl.words_to_ints(tr.exp[c])
        ids = tr.mod_id[tr.cls == c]
        assert ex.results[c] == [pow(b, e, M[i]) for b, e, i in zip(B, E, ids)]
    st = res.stats()
    assert st["requests"] > 0 and st["p99_ms"] >= st["p50_ms"] > 0


def test_continuous_batching_overlaps_batches():
    tr = _trace(n=4000, rate=80000.0)
    ex = FakeExecutor(tr, slots_per_class=3, fixed_s=4e-3)
    serving.Server(ex, CLASSES, {64: 128, 128: 128}).run(tr)
    assert max(ex.max_inflight.values()) >= 2  # batches of one class run concurrently
    # some batch was launched while another batch of the same class was still running
    log = ex.log
    overlaps = sum(1 for a in log for b in log if a is not b and a[0] == b[0] and a[3] < b[3] < a[4])
    assert overlaps > 0


def test_admission_bounded_by_slot_pool():
    tr = _trace(n=2000, rate=200000.0)
    ex = FakeExecutor(tr, slots_per_class=1, fixed_s=3e-3)
    res = serving.Server(ex, CLASSES, {64: 256, 128: 256}).run(tr)
    assert ex.max_inflight == {64: 1, 128: 1}  # never more batches than slots
    assert not res.failed.any()
    # overload queues requests instead of dropping them: latency grows beyond one service time
    assert res.stats()["max_ms"] > 3.0


def test_failures_are_isolated():
    tr = _trace(n=2000)
    ex = FakeExecutor(tr, fail_batches={2, 5})
    res = serving.Server(ex, CLASSES, {64: 64, 128: 64}).run(tr)
    assert res.failed.any() and not res.failed.all()
    assert not np.isnan(res.finish).any()  # the server kept serving and drained
    ok_classes_results = sum(r is not None for c in CLASSES for r in ex.results[c])
    assert ok_classes_results == int((~res.failed).sum())


def test_pacing_staggers_batches_of_a_class():
    # batches cost a fixed 20 ms whatever their size; with 2 slots and a steady trickle of
    # arrivals, a paced class starts a batch about every 10 ms instead of filling both slots
    # with tiny batches, and every request is still served once
    tr = serving.Trace(4000, 40000.0, k=33, classes=(64,), probs=(1.0,), moduli={64: 20})
    ex = FakeExecutor(tr, slots_per_class=2, per_req_s=0.0, fixed_s=20e-3)
    res = serving.Server(ex, tr.classes, {64: 100000}).run(tr, timeout_s=60)
    assert not res.failed.any()
    starts = np.array(sorted(t0 for _, _, _, t0, _ in ex.log))
    gaps = np.diff(starts)[2:]  # after the first batches the duration estimate exists
    # no batch below the size cap starts sooner than (observed duration) / slots after the previous one
    assert np.min(gaps) > 8e-3
    unpaced = FakeExecutor(tr, slots_per_class=2, per_req_s=0.0, fixed_s=20e-3)
    serving.Server(unpaced, tr.classes, {64: 100000}, pace=False).run(tr, timeout_s=60)
    ustarts = np.array(sorted(t0 for _, _, _, t0, _ in unpaced.log))
    # unpaced, both slots are refilled as soon as they free up, together
    assert np.min(np.diff(ustarts)[2:]) < 5e-3
