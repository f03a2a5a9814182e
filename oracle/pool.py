"""The float64 oracle over many pixels, in host-core worker processes.

TEST INFRASTRUCTURE ONLY (see the package docstring): used by the tests and
by the benchmark's correctness check and CPU baseline, never by the product.

Each task is one scene: a worker builds its dense matrix and solves for pi
exactly as ``oracle.dtm`` does (Section 3.4's construction, then the linear
solve of Section 2.3's stationarity equations).  Workers are spawned, not
forked (the parent may already hold the GPU), and run one BLAS thread each,
so the pool uses one host core per worker.
"""
from __future__ import annotations

import os

import numpy as np

_BLAS_VARS = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")


def scene_record(s):
    """A scene as a plain tuple (t_r, t_d, tau, sigma, S, B, n_b)."""
    return (float(s["period_ns"]), float(s["dead_time_ns"]), float(s["pulse_center_ns"]),
            float(s["pulse_sigma_ns"]), float(s["signal_flux"]), float(s["background_flux"]),
            int(s["n_bins"]))


def _scene(rec):
    from synth.scenes import make_scenes
    return make_scenes(*rec)


def _pi_one(rec):
    from oracle import dtm
    return dtm.stationary_solve(dtm.transition_matrix(_scene(rec)))


def _l1_one(task):
    rec, v = task
    return float(np.abs(np.asarray(v, dtype=np.float64) - _pi_one(rec)).sum())


def default_workers():
    """One worker per host core, at most 16."""
    return max(1, min(os.cpu_count() or 1, 16))


def _run(fn, tasks, workers):
    """fn over tasks in worker processes; workers == 1 runs them in this
    process (no child processes, e.g. under a profiler that follows them)."""
    if workers == 1:
        return [fn(t) for t in tasks]
    import multiprocessing as mp
    saved = {v: os.environ.get(v) for v in _BLAS_VARS}
    for v in _BLAS_VARS:
        os.environ[v] = "1"
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(workers or default_workers()) as pool:
            # largest first, so the slowest tasks do not start last
            order = sorted(range(len(tasks)), key=lambda i: -tasks[i][0][-1] if fn is _l1_one
                           else -tasks[i][-1])
            res = pool.map(fn, [tasks[i] for i in order], chunksize=1)
    finally:
        for v, old in saved.items():
            if old is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = old
    out = [None] * len(tasks)
    for i, r in zip(order, res):
        out[i] = r
    return out


def stationary_many(scenes, workers=None):
    """The oracle's pi for every scene (list of float64 arrays)."""
    return _run(_pi_one, [scene_record(s) for s in scenes], workers)


def l1_many(scenes, vectors, workers=None):
    """L1 distance of vectors[p] from the oracle's pi of scenes[p], for every p."""
    tasks = [(scene_record(s), np.asarray(v, dtype=np.float64)) for s, v in zip(scenes, vectors)]
    return np.asarray(_run(_l1_one, tasks, workers), dtype=np.float64)
