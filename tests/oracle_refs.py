"""Oracle optima for many problems at once, for the GPU parity tests.

The FP64 oracle solves one problem at a time; the parity tests need a few
hundred optima, so they are computed in a pool of fresh interpreter processes
(spawned, never forked from a process that holds the GPU), at most 16 of them,
each with single-threaded BLAS.  Only the tests use this module.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import mpcgen

_THREAD_VARS = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")


def _solve_one(p):
    from oracle import qp
    return qp.solve(p)


def solve_many(batch, indices, workers=None):
    """Oracle solutions (dicts of oracle.qp.solve) of problems ``indices`` of a
    generator batch, in the order given."""
    probs = [mpcgen.problem_fp64(batch, int(b)) for b in indices]
    if not probs:
        return []
    if workers is None:
        workers = min(16, os.cpu_count() or 1, len(probs))
    if workers <= 1 or len(probs) < 8:
        return [_solve_one(p) for p in probs]
    saved = {k: os.environ.get(k) for k in _THREAD_VARS}
    for k in _THREAD_VARS:
        os.environ[k] = "1"
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            return pool.map(_solve_one, probs, chunksize=max(1, len(probs) // (4 * workers)))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
