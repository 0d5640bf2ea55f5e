"""Expected values from the CPU oracle, computed by a pool of worker processes (test infrastructure).

The GPU parity tests check thousands of full-size exponentiations against the oracle, which takes
about 0.5 s per 2048-bit instance on one host core.  The pool spreads that over the host's cores
and starts early: ``conftest.py`` forks it at the end of collection, before any test touches the
GPU (a process that has initialised the GPU must not be forked, and the spawn and forkserver start
methods would exec), and submits each selected test's oracle jobs at once, in the order the tests
run, so the oracle works while earlier GPU tests do.  Workers only call ``oracle.modexp``.

Without a pool (a test module imported outside pytest's collection) the values are computed in
this process, one after another.
"""
import multiprocessing as mp
import os

MAX_WORKERS = 16  # the host share of one GPU on the test machines

_pool = None
_pending = {}
_done = {}


def _modexp(job):
    import oracle
    a, e, N, ebits = job
    return oracle.modexp(a, e, N, ebits)


def start(workers=None):
    """Forks the worker processes (call before the GPU is initialised)."""
    global _pool
    if _pool is None:
        workers = workers or min(MAX_WORKERS, os.cpu_count() or 1)
        _pool = mp.get_context("fork").Pool(workers)
    return _pool


def stop():
    global _pool
    if _pool is not None:
        _pool.terminate()
        _pool.join()
        _pool = None
    _pending.clear()
    _done.clear()


def submit(key, jobs):
    """Queues oracle.modexp(a, e, N, ebits) for every (a, e, N, ebits) in jobs under `key` (once per key)."""
    if key in _pending or key in _done:
        return
    jobs = list(jobs)
    if _pool is None:
        _pending[key] = (jobs, None)
    else:
        _pending[key] = (jobs, _pool.map_async(_modexp, jobs, chunksize=1))


def results(key, jobs_fn=None, timeout=900):
    """The oracle's values for the jobs submitted under `key`, in job order (kept for later calls).

    If nothing was submitted under `key`, the jobs come from jobs_fn() and run here."""
    if key in _done:
        return _done[key]
    if key not in _pending:
        if jobs_fn is None:
            raise KeyError(key)
        submit(key, jobs_fn())
    jobs, res = _pending.pop(key)
    _done[key] = [_modexp(j) for j in jobs] if res is None else res.get(timeout)
    return _done[key]


def spread(n, count, salt=0):
    """`count` instance indices spread over all 64-instance tiles of an n-instance batch.

    Tile t contributes lane (t + salt) mod 64, so the sample visits every lane position as well as
    every tile (every tile when count >= the tile count); the last instance is always included."""
    tiles = (n + 63) // 64
    if count >= tiles:
        picks = range(tiles)
    else:
        picks = sorted({(k * tiles) // count for k in range(count)})
    idx = {min(n - 1, t * 64 + (t + salt) % 64) for t in picks}
    idx.add(n - 1)
    return sorted(idx)
