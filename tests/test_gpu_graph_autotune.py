"""HIP graph replay of the batched solve and the tile autotuner."""
import numpy as np
import pytest
import torch

from synth import scenes as sc

from gpu_helpers import TOL_F32, lib, oracle_pi, split, tdtype

pytestmark = pytest.mark.gpu


def _setup(scenes, dt, tiles=None):
    d = lib()
    plan = d.Plan(scenes, dt, d.opts(tol=1e-6 if dt == "f32" else 1e-10), tiles)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    pi = torch.zeros(plan.pi_elems, dtype=tdtype(dt), device="cuda")
    infos = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
    return d, plan, ws, pi, infos


@pytest.mark.parametrize("banded", [False, True])
def test_graph_replays_match_eager(banded):
    """Several replays, with eager work and synchronisation between them; every
    replay must reproduce the eager result bit for bit."""
    scenes = np.concatenate([sc.batched_uniform(40, seed=101, n_bins=512),
                             sc.random_small(8, seed=102)])
    dt = "f32"
    d = lib()
    tiles = d.tiles(fused_max_bins=128, band_rows=64) if banded else None
    d, plan, ws, pi, infos = _setup(scenes, dt, tiles)
    plan.solve(pi, infos)
    torch.cuda.synchronize()
    ref_pi, ref_info = pi.clone(), infos.clone()
    g = plan.graph(pi, infos)
    for r in range(4):
        pi.fill_(float("nan"))
        infos.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(pi, ref_pi), r
        assert torch.equal(infos, ref_info), r
        del junk
    g.close()
    got = pi.cpu().numpy().astype(np.float64)
    info = d.infos_to_numpy(infos)
    assert np.all(info["status"] == 0)
    for s, v in zip(scenes, split(got, plan.pi_offsets)):
        assert np.abs(v - oracle_pi(s)).sum() <= TOL_F32
    plan.close()


def test_autotune_picks_a_working_shape(tmp_path):
    from paper_2509_20500_amd.autotune import autotune
    d = lib()
    scenes = np.concatenate([sc.batched_uniform(24, seed=111, n_bins=1024),
                             sc.batched_uneven(12, seed=112)])
    scenes = scenes[scenes["n_bins"] <= 4096]
    cache = str(tmp_path / "tune.json")
    tiles, rep = autotune(scenes, "f32", d.opts(tol=1e-6), cache_path=cache, reps=1)
    assert not rep["cached"] and rep["ms"] > 0 and len(rep["tried"]) >= 2
    tiles2, rep2 = autotune(scenes, "f32", d.opts(tol=1e-6), cache_path=cache, reps=1)
    assert rep2["cached"] and tiles2.as_dict() == tiles.as_dict()
    _, plan, ws, pi, infos = _setup(scenes, "f32", tiles)
    plan.solve(pi, infos)
    torch.cuda.synchronize()
    info = d.infos_to_numpy(infos)
    assert np.all(info["status"] == 0)
    got = pi.cpu().numpy().astype(np.float64)
    for p, (s, v) in enumerate(zip(scenes, split(got, plan.pi_offsets))):
        if s["n_bins"] <= 2048:
            assert np.abs(v - oracle_pi(s)).sum() <= TOL_F32
    plan.close()


def test_independent_paths_give_the_same_bits():
    """With one-block and banded pixels in one plan, letting each path sweep
    as soon as its own matrices are written changes only the timing: every
    pixel's kernels and their order are the same, so pi and the reports
    agree bit for bit with the default (eager and graph-replayed)."""
    d = lib()
    scenes = sc.batched_uneven(48, seed=113)
    ref = None
    for indep in (0, 1):
        _, plan, ws, pi, infos = _setup(scenes, "f32", d.tiles(independent_paths=indep))
        plan.solve(pi, infos)
        torch.cuda.synchronize()
        got = (pi.clone(), infos.clone())
        g = plan.graph(pi, infos)
        pi.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(pi, got[0]) and torch.equal(infos, got[1])
        g.close()
        plan.close()
        if ref is None:
            ref = got
        else:
            assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    assert np.all(d.infos_to_numpy(ref[1])["status"] == 0)


@pytest.mark.parametrize("blocks", [1, 7, 64])
def test_persistent_one_block_workgroups_give_the_same_bits(blocks):
    """A few persistent workgroups taking pixels from a counter run the same
    per-pixel code as one workgroup per pixel: the same bits, eager and
    replayed twice as a graph (the build launch resets the counter)."""
    d = lib()
    scenes = np.concatenate([sc.batched_uneven(40, seed=114), sc.random_small(24, seed=115)])
    _, plan, ws, pi, infos = _setup(scenes, "f32", d.tiles(dense_sweeps=6))
    plan.solve(pi, infos)
    torch.cuda.synchronize()
    ref = (pi.clone(), infos.clone())
    plan.close()
    _, plan, ws, pi, infos = _setup(scenes, "f32", d.tiles(dense_sweeps=6, fused_blocks=blocks))
    plan.solve(pi, infos)
    torch.cuda.synchronize()
    assert torch.equal(pi, ref[0]) and torch.equal(infos, ref[1])
    g = plan.graph(pi, infos)
    for _ in range(2):
        pi.fill_(float("nan"))
        infos.zero_()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(pi, ref[0]) and torch.equal(infos, ref[1])
    g.close()
    plan.close()
    assert np.all(d.infos_to_numpy(ref[1])["status"] == 0)


def test_banded_column_chunks_agree():
    """The banded sweep's column vectors per thread (1, 2, 4) change only
    which workgroup adds which columns (every column's partial sum runs over
    the band's rows in order; the building sweep of a plan with 2 or 4
    vectors runs in one-vector column blocks) and how the combine groups
    the column sums of y and |y - x|: the same sweeps and statuses, pi equal
    to float32 rounding, and each plan bit for bit the same eager and
    graph-replayed."""
    d = lib()
    scenes = np.concatenate([sc.batched_uneven(64, seed=116), sc.random_small(8, seed=117)])
    ref = None
    for cpt in (1, 2, 4):
        _, plan, ws, pi, infos = _setup(scenes, "f32", d.tiles(band_cpt=cpt, fused_max_bins=1024))
        plan.solve(pi, infos)
        torch.cuda.synchronize()
        got = (pi.clone(), infos.clone())
        g = plan.graph(pi, infos)
        pi.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(pi, got[0]) and torch.equal(infos, got[1])
        g.close()
        plan.close()
        if ref is None:
            ref = got
        else:
            a, b = d.infos_to_numpy(got[1]), d.infos_to_numpy(ref[1])
            assert np.array_equal(a["iterations"], b["iterations"]) and np.array_equal(a["status"], b["status"])
            assert np.allclose(a["residual_l1"], b["residual_l1"], rtol=1e-9, atol=1e-15), cpt
            assert float((got[0].double() - ref[0].double()).abs().max()) <= 2.0 ** -24, cpt
    assert np.all(d.infos_to_numpy(ref[1])["status"] == 0)
