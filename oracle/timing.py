"""Timing of the FP64 oracle on all host cores (test infrastructure only).

The positions are split into one shard per worker process; each worker runs the
oracle's forward + adjoint over its shard, in chunks, for a fixed time. Because the
loss and the object/probe gradients of a batch are sums over its positions
(data-parallel section of the paper), the shards together do the same work as one
process over all positions; the shards' partial gradients are not summed here, since
only the rate is measured.

Workers are fresh interpreter processes (spawn start method) that import only NumPy
and this package: they never touch a GPU, also when the parent process has.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time

import numpy as np


def _worker(barrier, queue, obj, probe, positions, I_meas, kw, budget_s, chunk):
    from threadpoolctl import threadpool_limits

    from .ptycho_ref import forward_adjoint

    n = positions.shape[0]
    with threadpool_limits(limits=1):
        barrier.wait()
        t0 = time.perf_counter()
        done, k0 = 0, 0
        while time.perf_counter() - t0 < budget_s:
            k1 = min(k0 + chunk, n)
            forward_adjoint(obj, probe, positions[k0:k1], I_meas[k0:k1], **kw)
            done += k1 - k0
            k0 = 0 if k1 == n else k1
        queue.put((done, time.perf_counter() - t0))


def pool_rate(obj, probe, positions, I_meas, *, workers: int, budget_s: float = 8.0, chunk: int = 25,
              **kw):
    """Patterns/s of ``forward_adjoint`` run concurrently in ``workers`` processes, each
    single-threaded on its own shard of the positions for ``budget_s`` seconds after a
    common start. Returns (rate, patterns done, wall seconds of the slowest worker)."""
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(workers)
    queue = ctx.Queue()
    bounds = np.linspace(0, positions.shape[0], workers + 1).astype(int)
    procs = []
    for w in range(workers):
        a, b = bounds[w], bounds[w + 1]
        p = ctx.Process(target=_worker, args=(barrier, queue, obj, probe, positions[a:b], I_meas[a:b], kw,
                                              budget_s, chunk), daemon=True)
        p.start()
        procs.append(p)
    results = []
    deadline = time.monotonic() + budget_s + 300.0
    while len(results) < workers:
        try:
            results.append(queue.get(timeout=1.0))
        except Exception:  # queue.Empty: check that every worker still runs or has finished cleanly
            if any(p.exitcode not in (None, 0) for p in procs) or time.monotonic() > deadline:
                for p in procs:
                    if p.is_alive():
                        p.terminate()
                barrier.abort()
                raise RuntimeError("an oracle timing worker failed")
    for p in procs:
        p.join(timeout=60.0)
    done = sum(r[0] for r in results)
    wall = max(r[1] for r in results)
    return done / wall, done, wall


HOST_SHARE = 16  # host CPUs allotted to one GPU on the measuring machine


def host_workers(cap: int = HOST_SHARE) -> int:
    """Worker count for the host: the CPUs this process may run on, at most ``cap`` (the
    measuring machine gives each GPU a share of 16 host CPUs, whatever the affinity mask
    or the CPU count of the whole host shows, and caps a job's processes accordingly)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))
