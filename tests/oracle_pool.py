"""The FP64 oracle over many slice tasks at once, in worker processes that
import only numpy and the oracle (test infrastructure; never touches a GPU).
Used where a GPU test compares every task of a full-size launch."""
from __future__ import annotations

import multiprocessing as mp
import os

_CTX = {}


def _init(Js, spins):
    _CTX["J"] = Js
    _CTX["spins"] = spins


def _one(args):
    from threadpoolctl import threadpool_limits

    from oracle import chain as ochain
    inst, c, z, beta, chi, d, seed, key, sweep = args
    margins = []
    with threadpool_limits(1):
        rec = ochain.propose(_CTX["J"][inst], _CTX["spins"][c], z, beta, chi, d, seed=seed, chain=key,
                             sweep=sweep, margins=margins)
    return {"new": rec["new"], "logq_new": rec["logq_new"], "logq_old": rec["logq_old"], "dE": rec["dE"],
            "fault": rec["fault"], "min_margin": min(margins) if margins else 1.0}


def propose_many(Js, spins, tasks, workers: int | None = None):
    """Js: couplings per instance, spins: configuration per chain; tasks: list
    of (instance, chain, z, beta, chi, d, seed, chain key, sweep).  Returns the
    oracle's proposal records in the order of tasks."""
    n = workers or max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("spawn")
    with ctx.Pool(n, initializer=_init, initargs=(Js, spins)) as pool:
        return pool.map(_one, tasks, chunksize=max(1, len(tasks) // (4 * n)))
