"""Pixels still running after their dense sweeps (the tile's dense_sweeps)
go on in float64 with the factored product of the same matrix, instead of
ending unconverged: banded pixels and one-block pixels alike.

* The corners of the paper's Section 4 grid where the spectral gap is
  smallest (S = B = 10 and S = B = 9 at t_d = 75 and 95 ns; |lambda_2| up to
  about 0.87, a hundred sweeps and more to 1e-6) at N = 4096 and 8192, in a
  default float32 plan (banded path above 2048 bins, 32 dense sweeps),
  eager and replayed as a HIP graph: every pixel ends DTM_OK within 1e-6 in
  L1 of the float64 reference (the dense oracle at 4096 bins; at 8192 bins
  power iteration with the O(n) factorised product, pinned against the
  dense oracle on the CPU).
* The banded pixels of the uneven batch with only three launched sweeps,
  so that most finish in the continuation: all DTM_OK and within 1e-6 of
  the float64 reference.
* One-block pixels (the headline batch's N = 1024, and a plan mixing both
  paths, eager and graph-replayed) with three dense sweeps: every pixel
  DTM_OK within 1e-6 of the oracle, the continued ones flagged.
* max_iter reached inside the continuation ends DTM_ENOTCONV with the last
  iterate (a probability vector) as pi.
* The banded hand-off (band_min_items): once the running pixels have fewer
  work items than the threshold, the banded sweeps stop and those pixels
  continue in float64.  Every pixel ends DTM_OK within 1e-6 of the float64
  reference, eager and graph-replayed bit for bit alike; a threshold of one
  item changes nothing; a threshold above the batch's items hands every
  pixel over after the building sweep.
* The hand-off in float32 and float64 plans whose two paths do not wait
  for each other, from a caller's warm start: every pixel within the
  dtype's bar.
* Pixels above 8192 bins continue in the four-wave kernel (g, 1/S and the
  vectors in the workspace) rather than in registers.
"""
import numpy as np
import pytest
import torch

from oracle import pool as opool
from synth import scenes as sc

from factored_ref import factored_power
from gpu_helpers import TOL_F32, TOL_F64, default_opts, lib, run_batched, split, tdtype

pytestmark = pytest.mark.gpu


def _slow_scenes():
    levels = []
    for td in (75.0, 95.0):
        for v in (9.0, 10.0):
            levels.append((td, v))
    return np.concatenate([sc.scene(dead_time=td, center=30.0, sigma=0.5, signal=v, background=v, n_bins=n)
                           for n in (4096, 8192) for td, v in levels])


def _solve(scenes, solve_opts, tiles=None, graph=False):
    d = lib()
    plan = d.Plan(scenes, "f32", solve_opts, tiles)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    pi = torch.full((plan.pi_elems,), float("nan"), dtype=tdtype("f32"), device="cuda")
    infos = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
    if graph:
        g = plan.graph(pi, infos)
        g.launch()
        torch.cuda.synchronize()
        g.close()
    else:
        plan.solve(pi, infos)
        torch.cuda.synchronize()
    got = split(pi.cpu().numpy().astype(np.float64), plan.pi_offsets)
    info = d.infos_to_numpy(infos)
    plan.close()
    del ws
    return got, info


@pytest.fixture(scope="module")
def slow_refs():
    scenes = _slow_scenes()
    n = scenes["n_bins"]
    refs = [None] * scenes.size
    dense = np.flatnonzero(n == 4096)
    print(f"dense oracle over {dense.size} pixels of 4096 bins", flush=True)
    for p, r in zip(dense, opool.stationary_many(scenes[dense])):
        refs[p] = r
    for p in np.flatnonzero(n == 8192):
        x, ok = factored_power(scenes[p])
        assert ok
        refs[p] = x
    return scenes, refs


@pytest.mark.parametrize("graph", [False, True])
def test_slow_banded_pixels_continue_to_the_tolerance(slow_refs, graph):
    d = lib()
    scenes, refs = slow_refs
    o = d.opts(tol=1e-6)
    o.flags |= d.DTM_FLAG_START_FLUX
    got, info = _solve(scenes, o, graph=graph)
    assert np.all(info["status"] == 0), info
    cont = (info["flags"] & d.DTM_INFO_CONTINUED) != 0
    assert np.any(cont), info["iterations"]  # some need more than the 32 dense sweeps
    assert np.all(info["iterations"][cont] > 32)
    l1 = np.array([np.abs(g - r).sum() for g, r in zip(got, refs)])
    print(f"graph={graph}: sweeps {info['iterations'].tolist()}, continued {int(cont.sum())}, "
          f"max L1 {l1.max():.3e}", flush=True)
    assert l1.max() <= TOL_F32, (l1, info)


def test_uneven_banded_pixels_with_three_launched_sweeps():
    d = lib()
    scenes = sc.batched_uneven()
    scenes = scenes[scenes["n_bins"] > 2048]
    got, info = _solve(scenes, d.opts(tol=1e-6), tiles=d.tiles(dense_sweeps=3))
    assert np.all(info["status"] == 0), info[info["status"] != 0]
    cont = (info["flags"] & d.DTM_INFO_CONTINUED) != 0
    assert cont.mean() > 0.5  # the others stop within the three launched sweeps
    assert np.all(info["dense_sweeps"][cont] == 3) and np.all(info["iterations"][cont] > 3)
    assert np.all(info["dense_sweeps"][~cont] == info["iterations"][~cont])
    worst = 0.0
    for p in range(scenes.size):
        ref, ok = factored_power(scenes[p])
        assert ok
        worst = max(worst, float(np.abs(got[p] - ref).sum()))
    print(f"{scenes.size} banded pixels, {int(cont.sum())} continued, max L1 {worst:.3e}", flush=True)
    assert worst <= TOL_F32


def test_max_iter_inside_the_continuation():
    d = lib()
    scenes = sc.scene(dead_time=75.0, center=30.0, sigma=0.5, signal=10.0, background=10.0, n_bins=4096)
    got, info = _solve(scenes, d.opts(tol=1e-6, max_iter=12), tiles=d.tiles(dense_sweeps=4))
    assert info["status"][0] == d.DTM_ENOTCONV
    assert info["flags"][0] & d.DTM_INFO_CONTINUED
    assert info["iterations"][0] == 12
    assert np.all(got[0] >= 0) and abs(got[0].sum() - 1.0) < 1e-5


def test_one_block_pixels_with_three_dense_sweeps():
    d = lib()
    scenes = sc.batched_uniform(256, seed=141)
    got, info = _solve(scenes, d.opts(tol=1e-6), tiles=d.tiles(dense_sweeps=3))
    assert np.all(info["status"] == 0), info[info["status"] != 0]
    cont = (info["flags"] & d.DTM_INFO_CONTINUED) != 0
    assert cont.mean() > 0.5 and np.all(info["iterations"][cont] > 3)
    l1 = opool.l1_many(scenes, got)
    print(f"one-block: {int(cont.sum())} of {scenes.size} continued, max L1 {l1.max():.3e}", flush=True)
    assert l1.max() <= TOL_F32


@pytest.mark.parametrize("graph", [False, True])
def test_both_paths_continue_in_one_plan(graph):
    d = lib()
    scenes = sc.batched_uneven(64, seed=142)
    o = d.opts(tol=1e-6)
    o.flags |= d.DTM_FLAG_START_FLUX
    got, info = _solve(scenes, o, tiles=d.tiles(dense_sweeps=3, fused_max_bins=1024), graph=graph)
    assert np.all(info["status"] == 0), info[info["status"] != 0]
    cont = (info["flags"] & d.DTM_INFO_CONTINUED) != 0
    n = scenes["n_bins"]
    assert np.any(cont & (n <= 1024)) and np.any(cont & (n > 1024))
    small = np.flatnonzero(n <= 2048)
    l1 = opool.l1_many(scenes[small], [got[p] for p in small])
    worst = float(l1.max())
    for p in np.flatnonzero(n > 2048):
        ref, ok = factored_power(scenes[p])
        assert ok
        worst = max(worst, float(np.abs(got[p] - ref).sum()))
    print(f"graph={graph}: {int(cont.sum())} of {scenes.size} continued, max L1 {worst:.3e}", flush=True)
    assert worst <= TOL_F32


def _uneven_banded():
    scenes = sc.batched_uneven()
    return scenes[scenes["n_bins"] > 2048]


@pytest.fixture(scope="module")
def uneven_banded_refs():
    scenes = _uneven_banded()
    refs = []
    for s in scenes:
        ref, ok = factored_power(s)
        assert ok
        refs.append(ref)
    return scenes, refs


@pytest.mark.parametrize("min_items", [256, 1 << 20])
def test_banded_hand_off_to_the_continuation(uneven_banded_refs, min_items):
    d = lib()
    scenes, refs = uneven_banded_refs
    o = d.opts(tol=1e-6)
    o.flags |= d.DTM_FLAG_START_FLUX
    tiles = d.tiles(band_min_items=min_items)
    got, info = _solve(scenes, o, tiles=tiles)
    got_g, info_g = _solve(scenes, o, tiles=tiles, graph=True)
    assert all(np.array_equal(a, b) for a, b in zip(got, got_g))
    assert np.array_equal(info, info_g)
    assert np.all(info["status"] == 0), info[info["status"] != 0]
    cont = (info["flags"] & d.DTM_INFO_CONTINUED) != 0
    if min_items > 1000:
        assert np.all(cont), info  # every pixel after the building sweep
        assert np.all(info["dense_sweeps"] == 1)
    else:
        assert np.any(cont) and not np.all(cont)
        # handed over together, after the same sweep
        assert np.unique(info["dense_sweeps"][cont]).size == 1
        assert np.all(info["dense_sweeps"][cont] < info["iterations"][cont])
        assert np.all(info["dense_sweeps"][~cont] <= info["dense_sweeps"][cont][0])
    l1 = np.array([np.abs(g - r).sum() for g, r in zip(got, refs)])
    print(f"band_min_items {min_items}: {int(cont.sum())} of {scenes.size} continued, "
          f"sweeps {np.bincount(info['iterations']).tolist()}, max L1 {l1.max():.3e}", flush=True)
    assert l1.max() <= TOL_F32, (int(np.argmax(l1)), l1.max())


def test_banded_hand_off_of_one_item_changes_nothing():
    """While a pixel runs, the items left are at least one: the threshold
    of one item never stops a sweep, and the bits are the default's."""
    d = lib()
    scenes = sc.batched_uneven(96, seed=143)
    o = d.opts(tol=1e-6)
    ref, ref_info = _solve(scenes, o)
    got, info = _solve(scenes, o, tiles=d.tiles(band_min_items=1))
    assert all(np.array_equal(a, b) for a, b in zip(got, ref))
    assert np.array_equal(info, ref_info)


def test_continuation_above_8192_bins():
    d = lib()
    scenes = sc.scene(dead_time=75.0, center=30.0, sigma=0.5, signal=9.0, background=9.0, n_bins=12288)
    got, info = _solve(scenes, d.opts(tol=1e-6), tiles=d.tiles(dense_sweeps=3))
    assert info["status"][0] == 0 and info["flags"][0] & d.DTM_INFO_CONTINUED
    assert info["iterations"][0] > 3
    ref, ok = factored_power(scenes[0])
    assert ok
    l1 = float(np.abs(got[0] - ref).sum())
    print(f"12288 bins: {info['iterations'][0]} sweeps, L1 {l1:.3e}", flush=True)
    assert l1 <= TOL_F32


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_banded_hand_off_with_warm_start_and_independent_paths(dt):
    """The hand-off in a mixed plan of both dtypes whose paths do not wait
    for each other, from a caller's warm start (the oracle's pi of a nearby
    scene, so some pixels stop early and others run long): every pixel ends
    DTM_OK within the dtype's bar of the float64 reference."""
    d = lib()
    scenes = sc.batched_uneven(160, seed=144)
    near = scenes.copy()
    near["signal_flux"] *= 1.05
    n = scenes["n_bins"]
    small = np.flatnonzero(n <= 2048)
    refs = [None] * scenes.size
    for p, r in zip(small, opool.stationary_many(scenes[small])):
        refs[p] = r
    x0 = []
    warm_small = opool.stationary_many(near[small])
    for p in range(scenes.size):
        if n[p] > 2048:
            refs[p], ok = factored_power(scenes[p])
            assert ok
            x0.append(factored_power(near[p])[0])
        else:
            x0.append(warm_small[int(np.searchsorted(small, p))])
    x0 = torch.tensor(np.concatenate(x0), dtype=tdtype(dt), device="cuda")
    tiles = d.tiles(band_min_items=256, independent_paths=1, dense_sweeps=12)
    pi, info, off = run_batched(scenes, dt, x0=x0, solve_opts=default_opts(dt), tiles=tiles)
    assert np.all(info["status"] == 0), info[info["status"] != 0]
    warm = (info["flags"] & (d.DTM_INFO_WARM_REJECTED | d.DTM_INFO_RESTARTED)) == 0
    assert np.all(warm)
    l1 = np.array([np.abs(v - r).sum() for v, r in zip(split(pi, off), refs)])
    cont = (info["flags"] & d.DTM_INFO_CONTINUED) != 0
    print(f"{dt}: {int(cont.sum())} of {scenes.size} continued, sweeps {np.bincount(info['iterations']).tolist()}, "
          f"max L1 {l1.max():.3e}", flush=True)
    assert l1.max() <= (TOL_F32 if dt == "f32" else TOL_F64), (int(np.argmax(l1)), l1.max())


@pytest.mark.parametrize("case", ["hand-off", "budget of max_iter"])
def test_max_iter_with_the_register_continuation(case):
    """max_iter on either side of the continuation: a slowly mixing
    4096-bin pixel handed off after its building sweep runs out of sweeps
    inside the continuation (flagged continued, one dense sweep); with a
    dense budget of max_iter sweeps the banded launches themselves stop it
    and the continuation leaves it alone.  Both end DTM_ENOTCONV with a
    probability vector, their sweeps counted."""
    d = lib()
    scenes = sc.scene(dead_time=75.0, center=30.0, sigma=0.5, signal=10.0, background=10.0, n_bins=4096)
    if case == "hand-off":
        got, info = _solve(scenes, d.opts(tol=1e-6, max_iter=12), tiles=d.tiles(band_min_items=1 << 20))
        assert info["iterations"][0] == 12 and info["dense_sweeps"][0] == 1
        assert info["flags"][0] & d.DTM_INFO_CONTINUED
    else:
        got, info = _solve(scenes, d.opts(tol=1e-6, max_iter=3), tiles=d.tiles(dense_sweeps=3))
        assert info["iterations"][0] == 3 and info["dense_sweeps"][0] == 3
        assert not info["flags"][0] & d.DTM_INFO_CONTINUED
    assert info["status"][0] == d.DTM_ENOTCONV
    assert np.all(got[0] >= 0) and abs(got[0].sum() - 1.0) < 1e-5
