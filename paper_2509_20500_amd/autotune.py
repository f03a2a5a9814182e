"""Tile-shape autotuner for the batched solver.

Times candidate ``dtm_tile_config`` values on the caller's own scenes (all
of them, or a fixed sample) through the C-ABI and keeps the fastest one that
solves every pixel: first a grid of the one-block and banded launch shapes,
then, for plans with banded pixels, the banded sweep's column vectors per
thread and its hand-off threshold around the best of the grid.  Results are cached as JSON, keyed by the device name,
the dtype, the solver options and the histogram of bin counts, so a workload
is tuned once per machine.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os

import numpy as np

from . import dtm

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "dtm_autotune.json")


def _key(scenes, dtype, solve_opts, device_name):
    n, cnt = np.unique(np.asarray(scenes["n_bins"]), return_counts=True)
    o = solve_opts or dtm.opts()
    raw = json.dumps({"dev": device_name, "dt": dtype, "n": n.tolist(), "c": cnt.tolist(),
                      "tol": o.tol_l1, "safety": o.safety, "max_iter": o.max_iter,
                      "rule": o.stop_rule, "flags": o.flags, "search": 2})
    return hashlib.sha1(raw.encode()).hexdigest()


def candidates(scenes):
    """The search space, pruned to shapes that differ for these scenes."""
    n_max = int(np.max(scenes["n_bins"]))
    out, seen = [], set()
    # dense_sweeps: 0 = the default budget (32 sweeps), 12 = slowly mixing
    # pixels finish on the float64 factored product after twelve dense sweeps;
    # fused_blocks: 0 = one workgroup per one-block pixel, 96 or 128 =
    # persistent workgroups (only differs when banded pixels share the plan)
    n_min = int(np.min(scenes["n_bins"]))
    cpt = 1  # the banded stage varies it
    for threads, unroll, fmax, band, dense, blocks in itertools.product(
            (256, 512), (4, 8), (1024, 2048, 4096), (1024, 8192), (0, 12), (0, 96, 128)):
        eff_fmax = min(fmax, n_max)
        big = n_max > fmax
        mixed = big and n_min <= fmax
        sig = (threads, unroll, eff_fmax, band if big else 0, cpt if big else 0, dense, blocks if mixed else 0)
        if sig in seen:
            continue
        seen.add(sig)
        out.append(dtm.tiles(fused_threads=threads, fused_unroll=unroll, fused_max_bins=fmax,
                             band_rows=band, band_cpt=cpt, dense_sweeps=dense,
                             fused_blocks=blocks if mixed else 0))
    return out


def banded_candidates(scenes, best):
    """Second stage, for plans with banded pixels: column vectors per thread
    of the banded sweep (1, 2, 4) and the hand-off threshold band_min_items
    (0 = never; 128 or 256 work items, below which a sweep's items cannot keep
    HBM busy), around the best first-stage shape."""
    if int(np.max(scenes["n_bins"])) <= best.fused_max_bins:
        return []
    out = []
    for cpt, mi in itertools.product((1, 2, 4), (0, 128, 256)):
        if (cpt, mi) != (best.band_cpt, best.band_min_items):
            out.append(dtm.tiles(**{**best.as_dict(), "band_cpt": cpt, "band_min_items": mi}))
    return out


def time_config(scenes, dtype, solve_opts, tiles, ws, reps=3):
    """Median milliseconds of one batched solve, or None if a pixel failed."""
    import torch
    plan = dtm.Plan(scenes, dtype, solve_opts, tiles)
    try:
        if plan.workspace_bytes > ws.numel():
            return None, plan.workspace_bytes
        plan.bind(ws)
        tdt = torch.float32 if plan.dtype == dtm.DTM_F32 else torch.float64
        pi = torch.empty(plan.pi_elems, dtype=tdt, device=ws.device)
        infos = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device=ws.device)
        plan.solve(pi, infos)
        torch.cuda.synchronize()
        if np.any(dtm.infos_to_numpy(infos)["status"] != 0):
            return None, plan.workspace_bytes
        times = []
        for _ in range(reps):
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            plan.solve(pi, infos)
            e.record()
            torch.cuda.synchronize()
            times.append(s.elapsed_time(e))
        return float(np.median(times)), plan.workspace_bytes
    finally:
        plan.close()


def autotune(scenes, dtype, solve_opts=None, cache_path=DEFAULT_CACHE, reps=3, verbose=False):
    """Returns (TileConfig, report dict).  Uses the cache when it has the key."""
    import torch
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    key = _key(scenes, dtype, solve_opts, dev)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        c = cache[key]["tiles"]
        return dtm.tiles(**c), {"cached": True, **cache[key]}
    max_iter = (solve_opts or dtm.opts()).max_iter
    cands = [t for t in candidates(scenes) if t.dense_sweeps <= max_iter]
    need = 0
    for t in cands:
        p = dtm.Plan(scenes, dtype, solve_opts, t)
        need = max(need, p.workspace_bytes)
        p.close()
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    results = []

    def run(cs):
        for t in cs:
            ms, _ = time_config(scenes, dtype, solve_opts, t, ws, reps)
            results.append((ms, t.as_dict()))
            if verbose:
                print("autotune", t.as_dict(), ms, flush=True)

    def best_of():
        ok = [r for r in results if r[0] is not None]
        if not ok:
            raise RuntimeError("autotune: no candidate solved every pixel")
        return min(ok, key=lambda r: r[0])

    run(cands)
    second = banded_candidates(scenes, dtm.tiles(**best_of()[1]))
    if second:
        extra = 0
        for t in second:  # column chunks change the combine's bookkeeping a little
            p = dtm.Plan(scenes, dtype, solve_opts, t)
            extra = max(extra, p.workspace_bytes)
            p.close()
        if extra > ws.numel():
            del ws
            ws = torch.empty(extra, dtype=torch.uint8, device="cuda")
        run(second)
    del ws
    best_ms, best = best_of()
    entry = {"tiles": best, "ms": best_ms, "device": dev,
             "tried": [{"tiles": t, "ms": ms} for ms, t in results]}
    if cache_path:
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            cache[key] = entry
            json.dump(cache, open(cache_path, "w"), indent=1)
        except OSError:
            pass
    return dtm.tiles(**best), {"cached": False, **entry}
