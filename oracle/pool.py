"""Process-parallel evaluation of the oracle's right-hand side over element chunks (oracle, FP64).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.  The arithmetic is the oracle's own
``Operator.rhs`` on element subsets (each element's right-hand side depends only on the state, never on
which other elements are evaluated with it); this module only splits the element loop over forked worker
processes, each writing its chunk into shared memory.  Used to generate stored expected values of long runs
and to time the oracle on all host cores.  Linux only (fork start method).
"""
from __future__ import annotations

import multiprocessing as mp

import numpy as np

_STATE = {}  # operator and shared arrays, inherited by the forked workers


def _chunk(args):
    t, lo, hi = args
    _STATE["out"][lo:hi] = _STATE["op"].rhs(_STATE["q"], t, el=np.arange(lo, hi))
    return hi - lo


class ChunkedRHS:
    """rhs(q, t) of an oracle operator, evaluated by `workers` forked processes (context manager)."""

    def __init__(self, op, shape, workers: int, chunks_per_worker: int = 8):
        if _STATE:
            raise RuntimeError("one ChunkedRHS at a time")
        K = shape[0]
        nbytes = int(np.prod(shape)) * 8
        ctx = mp.get_context("fork")
        self._qbuf, self._obuf = ctx.RawArray("b", nbytes), ctx.RawArray("b", nbytes)
        _STATE["op"] = op
        _STATE["q"] = np.frombuffer(self._qbuf, dtype=np.float64).reshape(shape)
        _STATE["out"] = np.frombuffer(self._obuf, dtype=np.float64).reshape(shape)
        bounds = np.linspace(0, K, max(1, chunks_per_worker * int(workers)) + 1).astype(int)
        self._jobs = [(int(a), int(b)) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
        self.workers = int(workers)
        self._pool = ctx.Pool(self.workers)

    def __call__(self, q, t):
        _STATE["q"][...] = q
        self._pool.map(_chunk, [(t, a, b) for a, b in self._jobs])
        return _STATE["out"].copy()

    def close(self):
        if self._pool is not None:
            self._pool.close()
            self._pool.join()
            self._pool = None
        _STATE.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
