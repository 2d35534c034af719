"""Worker processes for the oracle's independent loops (test infrastructure).

The oracle's transforms loop over orders m, and each order's Legendre step
is independent of every other (Sec. 2.1: the synthesis factorizes per m).
``run`` hands groups of such independent items to a pool of worker
processes and returns their results in item order.  Each item is computed
by the same function, on the same inputs, as in a plain loop (bit-identical
to that loop run with one BLAS thread; multi-threaded BLAS in the calling
process only reorders the sums of the per-order products); only wall time
changes.

Workers are started with the "spawn" method (fresh interpreters that import
numpy and this package only), hold one BLAS thread each, and live for the
life of the calling process.  Their count is ``ORACLE_WORKERS`` if set, else
the CPUs this process may run on, at most 16.
"""
from __future__ import annotations

import atexit
import concurrent.futures as cf
import multiprocessing as mp
import os

_POOL = None
_NPOOL = 0


def worker_count() -> int:
    env = os.environ.get("ORACLE_WORKERS")
    if env:
        return max(1, int(env))
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:                      # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _init_worker():
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:                           # pragma: no cover
        pass


def _pool(n: int):
    global _POOL, _NPOOL
    if _POOL is None or _NPOOL != n:
        if _POOL is not None:
            _POOL.shutdown(wait=True)
        _POOL = cf.ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn"),
                                       initializer=_init_worker)
        _NPOOL = n
    return _POOL


@atexit.register
def _shutdown():
    global _POOL
    if _POOL is not None:
        _POOL.shutdown(wait=True, cancel_futures=True)
        _POOL = None


def run(fn, groups, workers: int | None = None):
    """[fn(*g) for g in groups], computed by worker processes when workers > 1."""
    n = worker_count() if workers is None else workers
    if n <= 1 or len(groups) <= 1:
        return [fn(*g) for g in groups]
    pool = _pool(n)
    return list(pool.map(fn, *zip(*groups)))


def interleave(count: int, parts: int):
    """Split 0..count-1 into `parts` interleaved index lists (k, k + parts, ...):
    orders m of one list then have similar total length lmax - m + 1."""
    parts = max(1, min(parts, count))
    return [list(range(k, count, parts)) for k in range(parts)]
