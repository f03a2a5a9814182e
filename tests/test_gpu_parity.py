"""GPU parity: the HIP path (through the C-ABI) against the float64 CPU
oracle, element by element, on the same seeded inputs.

Tolerances: float64 path L1(pi) <= 1e-9, float32 path L1(pi) <= 1e-6;
matrix entries within a relative 1e-12 (float64) or 1e-6 (float32, a few
float32 roundings per entry)."""
import numpy as np
import pytest
import torch

from oracle import dtm as odtm
from synth import scenes as sc

from gpu_helpers import TOL_F32, TOL_F64, lib, oracle_pi, run_batched, split, tdtype

pytestmark = pytest.mark.gpu

MAT_RTOL = {"f64": 1e-12, "f32": 1e-6}


def _single_build(scene, dt, kind):
    d = lib()
    n = int(np.asarray(scene["n_bins"]).reshape(-1)[0])
    P = torch.empty((n, n), dtype=tdtype(dt), device="cuda")
    ws = d.workspace(n, dt)
    if kind == "base":
        d.build_base(scene, P, ws)
    else:
        d.build_transition(scene, P, ws)
    torch.cuda.synchronize()
    return P


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("idx", range(6))
def test_bin_tables(dt, idx):
    d = lib()
    s = np.concatenate([sc.random_small(4, seed=21), sc.single_pixel_n1000(),
                        sc.batched_uneven(1)])[idx]
    n = int(s["n_bins"])
    lam = torch.empty(n, dtype=tdtype(dt), device="cuda")
    F = torch.empty(n + 1, dtype=torch.float64, device="cuda")
    ws = d.workspace(n, dt)
    d.bin_tables(s, lam, F, ws)
    torch.cuda.synchronize()
    lam_o, F_o, Lam_o, _ = odtm.bin_tables(s)
    rt = 1e-13 if dt == "f64" else 1e-7
    assert np.allclose(lam.cpu().numpy(), lam_o, rtol=rt, atol=0)
    scale = max(1.0, Lam_o)
    assert np.max(np.abs(F.cpu().numpy()[:n] - F_o)) < 1e-13 * scale * max(1, n / 64)
    assert abs(F.cpu().numpy()[n] - Lam_o) < 1e-13 * scale * max(1, n / 64)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["base", "transition"])
def test_single_matrix_matches_oracle(dt, kind):
    for s in np.concatenate([sc.random_small(5, seed=31), sc.single_pixel_n1000()]):
        P = _single_build(s, dt, kind).cpu().numpy().astype(np.float64)
        ref = odtm.transition_matrix(s, shifted=(kind == "transition"))
        assert np.max(np.abs(P - ref) / ref) < MAT_RTOL[dt], s


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_shift_is_exact_row_permutation(dt):
    d = lib()
    for s in np.concatenate([sc.random_small(4, seed=41), sc.single_pixel_n1000()]):
        n = int(s["n_bins"])
        base = _single_build(s, dt, "base")
        P = torch.empty_like(base)
        d.apply_deadtime_shift(s, base, P)
        torch.cuda.synchronize()
        l = odtm.shift_bins(s)
        assert torch.equal(P, torch.roll(base, -l, dims=0))
        # the fused build writes the same bits
        assert torch.equal(P, _single_build(s, dt, "transition"))


def test_single_pixel_n1000_float64_change_rule():
    """Period 100 ns, N=1000, t_d=75 ns, uniform start, stop at change < 1e-12."""
    d = lib()
    s = sc.single_pixel_n1000()
    P = _single_build(s, "f64", "transition")
    pi = torch.empty(1000, dtype=torch.float64, device="cuda")
    ws = d.workspace(1000, "f64")
    info = d.stationary_pdf(P, pi, ws, d.opts(tol=1e-12, stop_rule=d.DTM_STOP_CHANGE))
    assert info.status == d.DTM_OK
    assert info.change_l1 < 1e-12
    assert info.dense_sweeps == info.iterations
    ref = oracle_pi(s)
    assert np.abs(pi.cpu().numpy() - ref).sum() <= TOL_F64
    # the oracle's own power iteration takes about as many sweeps
    _, it_ref, _ = odtm.stationary_power(odtm.transition_matrix(s), tol_change=1e-12)
    assert abs(info.iterations - it_ref) <= 3


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_single_pixel_n4096_dead_time_sweep(dt):
    """N=4096 over 100 ns, t_d in {10, 33, 75, 150} ns; one matrix and one
    solve per sweep point (two scene draws)."""
    d = lib()
    ws = d.workspace(4096, dt)
    pi = torch.empty(4096, dtype=tdtype(dt), device="cuda")
    tol = TOL_F64 if dt == "f64" else TOL_F32
    for s in sc.single_pixel_n4096(n_scenes=2):
        P = _single_build(s, dt, "transition")
        o = d.opts(tol=1e-12, stop_rule=d.DTM_STOP_CHANGE) if dt == "f64" else d.opts(tol=tol)
        info = d.stationary_pdf(P, pi, ws, o)
        assert info.status == d.DTM_OK
        err = np.abs(pi.cpu().numpy() - oracle_pi(s)).sum()
        assert err <= tol, (s, err, info.iterations)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n", [2, 65, 2048, 2049, 2112])
def test_single_pixel_band_shapes(dt, n):
    """Up to 2048 bins the single-pixel sweep takes bands of about 32 rows,
    above about 64.  Both sides of the switch, ragged last bands and the
    two-bin chain, against the oracle and with the iteration count of the
    oracle's own power iteration; a second solve on the same workspace."""
    d = lib()
    s = sc.scene(dead_time=61.7, center=40.0, sigma=0.6, signal=2.0, background=0.3, n_bins=n)
    P = _single_build(s, dt, "transition")
    pi = torch.empty(n, dtype=tdtype(dt), device="cuda")
    ws = d.workspace(n, dt)
    tol = TOL_F64 if dt == "f64" else TOL_F32
    o = d.opts(tol=1e-12, stop_rule=d.DTM_STOP_CHANGE) if dt == "f64" else d.opts(tol=tol)
    for _ in range(2):
        pi.fill_(float("nan"))
        info = d.stationary_pdf(P, pi, ws, o)
        assert info.status == d.DTM_OK
        err = np.abs(pi.cpu().numpy() - oracle_pi(s)).sum()
        assert err <= tol, (n, err, info.iterations)
    if dt == "f64":
        _, it_ref, _ = odtm.stationary_power(odtm.transition_matrix(s), tol_change=1e-12)
        assert abs(info.iterations - it_ref) <= 3


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_single_pixel_on_unaligned_stride(dt):
    """A caller's matrix with an odd row stride takes the scalar path."""
    d = lib()
    s = sc.scene(dead_time=41.3, n_bins=129)
    n, ld = 129, 131
    buf = torch.zeros((n, ld), dtype=tdtype(dt), device="cuda")
    ws = d.workspace(n, dt)
    d.check(d.dtm_build_transition(s, dt, buf.data_ptr(), ld, ws.data_ptr(), ws.numel(),
                                   torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert torch.count_nonzero(buf[:, n:]) == 0  # nothing written past column n
    P = buf[:, :n].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(P / odtm.transition_matrix(s) - 1)) < MAT_RTOL[dt]
    pi = torch.empty(n, dtype=tdtype(dt), device="cuda")
    tol = TOL_F64 if dt == "f64" else TOL_F32
    st, info = d.dtm_stationary_pdf(buf.data_ptr(), n, ld, dt, d.opts(tol=tol), None,
                                    pi.data_ptr(), ws.data_ptr(), ws.numel(),
                                    torch.cuda.current_stream().cuda_stream)
    assert st == 0 and info.status == 0
    assert np.abs(pi.cpu().numpy() - oracle_pi(s)).sum() <= tol


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_batched_small_ragged(dt):
    """Many pixels with ragged N (2..257), dead times above and below a period."""
    scenes = sc.random_small(64, seed=51)
    pi, info, off = run_batched(scenes, dt)
    tol = TOL_F64 if dt == "f64" else TOL_F32
    assert np.all(info["status"] == 0)
    for p, (s, v) in enumerate(zip(scenes, split(pi, off))):
        err = np.abs(v - oracle_pi(s)).sum()
        assert err <= tol, (p, s, err, info[p])


def test_batched_uniform_full_size_float32():
    """64x64 pixels at N=1024, t_d=50 ns, float32 with the float64 check:
    every pixel's residual and normalisation, 64 sampled pixels against the
    oracle."""
    scenes = sc.batched_uniform()
    pi, info, off = run_batched(scenes, "f32")
    assert np.all(info["status"] == 0)
    assert np.all(info["flags"] & 0x4)  # checked in float64
    pis = split(pi, off)
    sums = np.array([v.sum() for v in pis])
    assert np.max(np.abs(sums - 1)) < 1e-5
    assert min(v.min() for v in pis) > 0
    # acceptance is residual x gain <= safety x tol; fast-mixing pixels (gain
    # ~ 5e-3) are accepted at residuals of a few 1e-5
    assert np.max(info["residual_l1"]) < 1e-4
    rng = np.random.default_rng(0)
    for p in rng.choice(len(scenes), 64, replace=False):
        err = np.abs(pis[p] - oracle_pi(scenes[p])).sum()
        assert err <= TOL_F32, (p, err, info[p])


def test_batched_is_deterministic():
    scenes = sc.batched_uniform(256)
    a, ia, _ = run_batched(scenes, "f32")
    b, ib, _ = run_batched(scenes, "f32")
    assert np.array_equal(a, b)
    assert np.array_equal(ia, ib)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_batched_uneven_sizes(dt):
    """N from 512 to 8192 (float64 up to 4096), uneven periods and dead times."""
    scenes = sc.batched_uneven(24, seed=9)
    if dt == "f64":
        scenes = scenes[scenes["n_bins"] <= 4096]
    pi, info, off = run_batched(scenes, dt)
    tol = TOL_F64 if dt == "f64" else TOL_F32
    assert np.all(info["status"] == 0)
    for p, (s, v) in enumerate(zip(scenes, split(pi, off))):
        if s["n_bins"] > 2048:
            continue  # checked by properties below; the dense oracle is slow there
        err = np.abs(v - oracle_pi(s)).sum()
        assert err <= tol, (p, s, err)
    for v in split(pi, off):
        assert abs(v.sum() - 1) < 1e-5 and v.min() > 0


def test_batched_edge_cases():
    """Two bins, three bins, pure background (pi uniform), dead time of whole
    periods (no shift), dead time just under one bin."""
    scenes = np.concatenate([
        sc.scene(n_bins=2, dead_time=30.0, center=20.0, sigma=5.0),
        sc.scene(n_bins=3, dead_time=250.0),
        sc.scene(n_bins=64, signal=0.0, background=2.0, dead_time=33.0),
        sc.scene(n_bins=100, dead_time=300.0),
        sc.scene(n_bins=100, dead_time=0.99),
        sc.scene(n_bins=100, dead_time=0.0),
    ])
    for dt in ("f64", "f32"):
        pi, info, off = run_batched(scenes, dt)
        tol = TOL_F64 if dt == "f64" else TOL_F32
        assert np.all(info["status"] == 0)
        for s, v in zip(scenes, split(pi, off)):
            assert np.abs(v - oracle_pi(s)).sum() <= tol
        u = split(pi, off)[2]
        assert np.max(np.abs(u - 1 / 64)) < (1e-15 if dt == "f64" else 1e-8)


def test_batched_matrices_match_oracle():
    d = lib()
    scenes = sc.random_small(12, seed=61)
    for dt in ("f64", "f32"):
        plan = d.Plan(scenes, dt)
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
        plan.bind(ws)
        base = torch.full((plan.matrix_elems,), float("nan"), dtype=tdtype(dt), device="cuda")
        full = torch.full_like(base, float("nan"))
        shifted = torch.full_like(base, float("nan"))
        plan.build_base(base)
        plan.build_transition(full)
        plan.apply_deadtime_shift(base, shifted)
        torch.cuda.synchronize()
        assert torch.equal(full, shifted)
        B = base.cpu().numpy().astype(np.float64)
        Fm = full.cpu().numpy().astype(np.float64)
        mo = plan.mat_offsets
        for p, s in enumerate(scenes):
            n = int(s["n_bins"])
            got_b = B[mo[p]:mo[p + 1]].reshape(n, n)
            got_f = Fm[mo[p]:mo[p + 1]].reshape(n, n)
            assert np.max(np.abs(got_b / odtm.transition_matrix(s, shifted=False) - 1)) < MAT_RTOL[dt]
            assert np.max(np.abs(got_f / odtm.transition_matrix(s) - 1)) < MAT_RTOL[dt]
        plan.close()


def test_warm_start_and_fallbacks():
    d = lib()
    scenes = sc.batched_uniform(32, seed=71)
    ref = [oracle_pi(s) for s in scenes]
    # a good warm start: the stationary vector itself, slightly perturbed
    rng = np.random.default_rng(1)
    x0 = np.concatenate([r * (1 + 0.01 * rng.standard_normal(r.size)) for r in ref])
    pi_u, info_u, off = run_batched(scenes, "f32")
    pi_w, info_w, _ = run_batched(scenes, "f32", x0=torch.tensor(x0, dtype=torch.float32, device="cuda"))
    assert np.all(info_w["status"] == 0)
    assert info_w["iterations"].sum() < info_u["iterations"].sum()
    for r, v in zip(ref, split(pi_w, off)):
        assert np.abs(v - r).sum() <= TOL_F32
    # garbage warm starts (negative, NaN, all zero) are replaced by uniform
    bad = x0.copy()
    bad[off[0]] = -1.0
    bad[off[1] + 3] = np.nan
    bad[off[2]:off[3]] = 0.0
    pi_b, info_b, _ = run_batched(scenes, "f32", x0=torch.tensor(bad, dtype=torch.float32, device="cuda"))
    assert np.all(info_b["status"] == 0)
    assert np.all(info_b["flags"][:3] & d.DTM_INFO_WARM_REJECTED)
    assert not np.any(info_b["flags"][3:] & d.DTM_INFO_WARM_REJECTED)
    for r, v in zip(ref, split(pi_b, off)):
        assert np.abs(v - r).sum() <= TOL_F32


def test_not_converged_is_soft():
    d = lib()
    scenes = sc.paper_grid(levels=(9.0,), dead_time=75.0, n_bins=256)  # |lambda_2| ~ 0.8
    pi, info, off = run_batched(scenes, "f32", solve_opts=d.opts(max_iter=3))
    assert np.all(info["status"] == d.DTM_ENOTCONV)
    assert np.all(info["iterations"] == 3)
    assert np.all(np.isfinite(pi)) and abs(pi.sum() - 1) < 1e-5


def test_single_pixel_warm_start_and_not_converged():
    d = lib()
    s = sc.scene(signal=9.0, background=9.0, dead_time=75.0, n_bins=256)
    P = _single_build(s, "f64", "transition")
    ws = d.workspace(256, "f64")
    pi = torch.empty(256, dtype=torch.float64, device="cuda")
    info = d.stationary_pdf(P, pi, ws, d.opts(max_iter=2))
    assert info.status == d.DTM_ENOTCONV
    ref = oracle_pi(s)
    x0 = torch.tensor(ref, device="cuda")
    info = d.stationary_pdf(P, pi, ws, d.opts(tol=1e-10), x0=x0)
    assert info.status == d.DTM_OK and info.iterations <= 3
    assert np.abs(pi.cpu().numpy() - ref).sum() <= TOL_F64


def test_float32_paper_grid_with_refinement():
    """The paper's (S, B) grid at t_d = 75 and 95 ns (Section 4), N = 256,
    float32: slowly mixing pixels that float32 cannot certify are re-solved
    in float64 and flagged; every pixel ends within 1e-6 of the oracle."""
    d = lib()
    scenes = np.concatenate([sc.paper_grid(dead_time=75.0), sc.paper_grid(dead_time=95.0),
                             sc.random_small(64, seed=51)])
    pi, info, off = run_batched(scenes, "f32")
    assert np.all(info["status"] == 0)
    for p, (s, v) in enumerate(zip(scenes, split(pi, off))):
        err = np.abs(v - oracle_pi(s)).sum()
        assert err <= TOL_F32, (p, s, err, info[p])
    refined = (info["flags"] & d.DTM_INFO_REFINED) != 0
    print("refined pixels:", int(refined.sum()), "of", len(scenes))
    # the float64 sweeps of a refined or continued pixel regenerate the
    # matrix: they are not dense sweeps
    f64 = refined | ((info["flags"] & d.DTM_INFO_CONTINUED) != 0)
    assert np.all(info["dense_sweeps"][f64] < info["iterations"][f64])
    assert np.all(info["dense_sweeps"][~f64] == info["iterations"][~f64])


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_banded_path_ragged(dt):
    """Pixels above fused_max_bins take the banded multi-block path: ragged
    row bands (64 rows) and, past 4096 (float32) or 2048 (float64) columns,
    several column blocks; mixed with one-block pixels in one plan."""
    d = lib()
    rng = np.random.default_rng(81)
    ns = [300, 1000, 2500, 257, 64, 5000 if dt == "f32" else 3000, 777]
    scenes = np.concatenate([
        sc.scene(period=float(rng.uniform(50, 200)), dead_time=float(rng.uniform(5, 300)),
                 center=float(rng.uniform(10, 40)), sigma=float(rng.uniform(0.2, 2.0)),
                 signal=float(rng.uniform(0.1, 4)), background=float(rng.uniform(0.05, 1.5)), n_bins=n)
        for n in ns])
    tiles = d.tiles(fused_max_bins=256, band_rows=64)
    pi, info, off = run_batched(scenes, dt, tiles=tiles)
    tol = TOL_F64 if dt == "f64" else TOL_F32
    assert np.all(info["status"] == 0), info
    for p, (s, v) in enumerate(zip(scenes, split(pi, off))):
        err = np.abs(v - oracle_pi(s)).sum()
        assert err <= tol, (p, int(s["n_bins"]), err, info[p])


def test_banded_sweep_cap_continues_in_float64():
    """A banded pixel that needs more sweeps than were launched goes on from
    its iterate in float64 (flagged DTM_INFO_CONTINUED) and meets the
    tolerance; with max_iter equal to the launched sweeps it ends with
    DTM_ENOTCONV and its last iterate."""
    d = lib()
    scenes = sc.paper_grid(levels=(9.0,), dead_time=75.0, n_bins=512)
    pi, info, off = run_batched(scenes, "f32", tiles=d.tiles(fused_max_bins=256, dense_sweeps=3))
    assert np.all(info["status"] == 0)
    assert np.all(info["flags"] & d.DTM_INFO_CONTINUED) and np.all(info["iterations"] > 3)
    assert np.abs(pi - oracle_pi(scenes[0])).sum() <= TOL_F32
    pi, info, off = run_batched(scenes, "f32", solve_opts=d.opts(tol=1e-6, max_iter=3),
                                tiles=d.tiles(fused_max_bins=256, dense_sweeps=3))
    assert np.all(info["status"] == d.DTM_ENOTCONV)
    assert np.all(info["iterations"] == 3)
    assert np.all(np.isfinite(pi)) and abs(pi.sum() - 1) < 1e-5


def test_banded_matches_one_block_path():
    """The banded and one-block paths solve the same pixels to the same
    tolerance (they differ only in summation order)."""
    d = lib()
    scenes = sc.batched_uniform(24, seed=91)
    a, ia, off = run_batched(scenes, "f32")
    b, ib, _ = run_batched(scenes, "f32", tiles=d.tiles(fused_max_bins=512, band_rows=128))
    assert np.all(ia["status"] == 0) and np.all(ib["status"] == 0)
    for p in range(len(scenes)):
        assert np.abs(a[off[p]:off[p + 1]] - b[off[p]:off[p + 1]]).sum() < 1e-6


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_batched_stop_rules_and_no_final_check(dt):
    """The batched solve (one-block and banded pixels in one plan) under the
    change rule (config 1's rule) and with the float64 check switched off:
    the change rule at 1e-12 reaches the oracle to 1e-9 in float64; without
    the check, no pixel reports a check sweep (unless it was continued in
    float64 after its dense sweeps) and the iterate still sits within the
    float32 floor of the oracle."""
    d = lib()
    scenes = np.concatenate([sc.random_small(20, seed=171), sc.batched_uniform(4, seed=172)])
    tiles = d.tiles(fused_max_bins=128, band_rows=64)
    if dt == "f64":
        pi, info, off = run_batched(scenes, dt, solve_opts=d.opts(tol=1e-12, stop_rule=d.DTM_STOP_CHANGE),
                                    tiles=tiles)
        assert np.all(info["status"] == 0)
        for p, (s, v) in enumerate(zip(scenes, split(pi, off))):
            assert np.abs(v - oracle_pi(s)).sum() <= 1e-9, (p, s)
    else:
        pi, info, off = run_batched(scenes, dt, solve_opts=d.opts(tol=1e-6, flags=d.DTM_FLAG_NO_FINAL_CHECK),
                                    tiles=tiles)
        assert np.all(info["status"] == 0)
        # only pixels continued in float64 after their dense sweeps (every
        # sweep of the continuation is a float64 one) report a check
        cont = (info["flags"] & d.DTM_INFO_CONTINUED) != 0
        assert not np.any(((info["flags"] & d.DTM_INFO_CHECKED) != 0) & ~cont)
        for p, (s, v) in enumerate(zip(scenes, split(pi, off))):
            assert np.abs(v - oracle_pi(s)).sum() <= 1e-5, (p, s)


def test_banded_warm_start_and_fallbacks():
    """Warm starts on a plan that mixes one-block and banded pixels: a close
    start saves sweeps on both paths; a rejected start (negative, NaN, all
    zero) falls back to uniform and is flagged on the pixel it belongs to."""
    d = lib()
    scenes = np.concatenate([sc.random_small(6, seed=181), sc.batched_uniform(4, seed=182)])
    tiles = d.tiles(fused_max_bins=128, band_rows=64)
    ref = [oracle_pi(s) for s in scenes]
    big = np.array([int(s["n_bins"]) > 128 for s in scenes])
    assert big.any() and (~big).any()
    rng = np.random.default_rng(2)
    x0 = np.concatenate([r * (1 + 0.01 * rng.standard_normal(r.size)) for r in ref])
    _, info_u, off = run_batched(scenes, "f32", tiles=tiles)
    pi_w, info_w, _ = run_batched(scenes, "f32", tiles=tiles,
                                  x0=torch.tensor(x0, dtype=torch.float32, device="cuda"))
    assert np.all(info_w["status"] == 0)
    assert not np.any(info_w["flags"] & d.DTM_INFO_WARM_REJECTED)
    for sel in (big, ~big):
        assert info_w["iterations"][sel].sum() < info_u["iterations"][sel].sum()
    for r, v in zip(ref, split(pi_w, off)):
        assert np.abs(v - r).sum() <= TOL_F32
    bad = x0.copy()
    rejected = [int(np.flatnonzero(~big)[0]), int(np.flatnonzero(big)[0]), int(np.flatnonzero(big)[-1])]
    bad[off[rejected[0]] + 1] = -1.0
    bad[off[rejected[1]] + 5] = np.nan
    bad[off[rejected[2]]:off[rejected[2] + 1]] = 0.0
    pi_b, info_b, _ = run_batched(scenes, "f32", tiles=tiles,
                                  x0=torch.tensor(bad, dtype=torch.float32, device="cuda"))
    assert np.all(info_b["status"] == 0)
    flagged = (info_b["flags"] & d.DTM_INFO_WARM_REJECTED) != 0
    assert sorted(np.flatnonzero(flagged).tolist()) == sorted(rejected)
    for r, v in zip(ref, split(pi_b, off)):
        assert np.abs(v - r).sum() <= TOL_F32
