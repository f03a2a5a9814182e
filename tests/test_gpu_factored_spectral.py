"""GPU tests of the factored solver (O(n) sweeps on the same matrix) and of
the spectral convergence analysis (Section 4) against the float64 oracle."""
import math

import numpy as np
import pytest
import torch

from oracle import dtm as odtm, spectral as ospec
from synth import scenes as sc

from gpu_helpers import lib, oracle_pi, split, tdtype

pytestmark = pytest.mark.gpu


def _plan(scenes, dt, opts, no_dense=True):
    d = lib()
    if no_dense:
        opts.flags |= d.DTM_FLAG_NO_DENSE
    plan = d.Plan(scenes, dt, opts)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    return d, plan, ws


@pytest.mark.parametrize("dt,tol,bar", [("f64", 1e-12, 1e-10), ("f32", 1e-10, 1e-6)])
def test_factored_solver_matches_oracle(dt, tol, bar):
    scenes = np.concatenate([sc.random_small(40, seed=121), sc.batched_uniform(8, seed=122),
                             sc.paper_grid(dead_time=95.0), sc.single_pixel_n1000()])
    d, plan, ws = _plan(scenes, dt, lib().opts(tol=tol))
    pi = torch.full((plan.pi_elems,), float("nan"), dtype=tdtype(dt), device="cuda")
    infos = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
    plan.solve_factored(pi, infos)
    torch.cuda.synchronize()
    info = d.infos_to_numpy(infos)
    got = pi.cpu().numpy().astype(np.float64)
    assert np.all(info["status"] == 0), info[info["status"] != 0]
    assert np.all(info["dense_sweeps"] == 0)  # no matrix is stored
    for p, (s, v) in enumerate(zip(scenes, split(got, plan.pi_offsets))):
        assert np.abs(v - oracle_pi(s)).sum() <= bar, (p, s)
    # the dense solver cannot run on a plan without matrices
    with pytest.raises(d.DtmError):
        plan.solve(pi, infos)
    plan.close()


def _ragged(n_max, seed):
    """Five scenes of varied physics whose largest has n_max bins."""
    scenes = sc.random_small(5, seed=seed).copy()
    scenes["n_bins"] = [n_max, n_max - 37, 3, 64, n_max // 2 + 1]
    return scenes


@pytest.mark.parametrize("n_max", [200, 500, 1000, 1500])
def test_factored_solver_each_launch_shape(n_max):
    """The largest pixel of a plan picks the launch: one wavefront per pixel
    with 4, 8 or 16 bins per lane up to 1024 bins, a block per pixel with its
    vectors in LDS above; smaller ragged pixels share the launch."""
    scenes = _ragged(n_max, seed=140 + n_max)
    d, plan, ws = _plan(scenes, "f64", lib().opts(tol=1e-12))
    pi = torch.full((plan.pi_elems,), float("nan"), dtype=torch.float64, device="cuda")
    infos = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
    plan.solve_factored(pi, infos)
    torch.cuda.synchronize()
    info = d.infos_to_numpy(infos)
    assert np.all(info["status"] == 0), info
    got = pi.cpu().numpy()
    for p, (s, v) in enumerate(zip(scenes, split(got, plan.pi_offsets))):
        assert np.abs(v - oracle_pi(s)).sum() <= 1e-10, (p, s)
    plan.close()


@pytest.mark.parametrize("n_max", [200, 500, 1000, 1100])
def test_mixing_steps_each_launch_shape(n_max):
    """Mixing steps with one wavefront per start state (up to 1024 bins) and
    one thread per start state above, against powers of the dense matrix."""
    scenes = sc.paper_grid((3.0, 9.0), dead_time=75.0, n_bins=n_max).copy()
    scenes["n_bins"][1] = n_max - 37
    d, plan, ws = _plan(scenes, "f64", lib().opts(tol=1e-12))
    scratch = torch.empty(plan.spectral_scratch_bytes(True), dtype=torch.uint8, device="cuda")
    out = torch.zeros(plan.n_pixels * d.SPECTRAL_INFO_BYTES, dtype=torch.uint8, device="cuda")
    plan.spectral(out, scratch, 0.25, 5000)
    torch.cuda.synchronize()
    res = d.spectral_to_numpy(out)
    for p, s in enumerate(scenes):
        Pt = odtm.transition_matrix(s)
        ref = ospec.mixing_steps(Pt, odtm.stationary_solve(Pt), 0.25)
        assert res["mixing_steps"][p] == ref, (p, s, res[p], ref)
    plan.close()


def test_factored_solver_at_large_n():
    """n = 65536 (a 16 GiB float32 matrix if formed): check pi by the residual
    of the factorised left product, written out independently in NumPy."""
    s = sc.scene(dead_time=41.3, center=33.0, sigma=0.3, signal=2.0, background=0.4, n_bins=65536)
    d, plan, ws = _plan(s, "f64", lib().opts(tol=1e-11))
    pi = torch.empty(plan.pi_elems, dtype=torch.float64, device="cuda")
    infos = torch.zeros(40, dtype=torch.uint8, device="cuda")
    plan.solve_factored(pi, infos)
    torch.cuda.synchronize()
    assert d.infos_to_numpy(infos)["status"][0] == 0
    x = pi.cpu().numpy()
    lam, F, Lam, l = odtm.bin_tables(s)
    g = lam * np.exp(-F)
    c = math.exp(-Lam)
    Rh = c * g.sum() + (1 - c) * np.cumsum(g[::-1])[::-1]
    U = np.cumsum(np.roll(x, l) / Rh)
    y = g * (c * U[-1] + (1 - c) * U)
    assert abs(x.sum() - 1) < 1e-12
    assert np.abs(y - x).sum() < 1e-11


def _check_spectral(res, scenes, refs, mod_tol, arg_tol, l3_tol):
    d = lib()
    for p, s in enumerate(scenes):
        lam, third = refs[p]
        r = res[p]
        assert not (r["flags"] & d.DTM_SPECTRAL_UNSETTLED), (p, s, r)
        assert abs(r["lambda2_abs"] - abs(lam)) <= mod_tol * max(1.0, abs(lam)), (p, s, r, lam)
        tied = third >= (1.0 - 1e-9) * abs(lam) and third > 0.0
        assert bool(r["flags"] & d.DTM_SPECTRAL_TIED) == tied, (p, s, r, lam, third)
        if not tied:
            assert abs(r["lambda2_arg"] - abs(np.angle(lam))) <= arg_tol, (p, s, r, lam)
        assert abs(r["lambda3_abs"] - third) <= l3_tol, (p, s, r, third)


def test_spectral_second_eigenvalue_matches_dense_eig():
    """lambda_2 (modulus and phase) and the next modulus of every pixel of the
    paper's Section 4 grid (S, B in {0.1, 1, ..., 10}, t_d = 75 and 95 ns,
    N = 256), of the coarse grid at N = 128 and of random small scenes,
    against LAPACK eigenvalues of the oracle's dense matrix.  The grid holds
    pixels whose third eigenvalue lies within a few per cent of lambda_2 in
    modulus (S, B near 10 at t_d = 95 ns)."""
    levels = (0.1, 3.0, 6.0, 9.0)
    scenes = np.concatenate([sc.paper_rmse_grid(n_bins=256, dead_time=75.0),
                             sc.paper_rmse_grid(n_bins=256, dead_time=95.0),
                             sc.paper_grid(levels, dead_time=75.0, n_bins=128),
                             sc.paper_grid(levels, dead_time=95.0, n_bins=128),
                             sc.random_small(24, seed=131)])
    d, plan, ws = _plan(scenes, "f64", lib().opts(tol=1e-12))
    scratch = torch.empty(plan.spectral_scratch_bytes(False), dtype=torch.uint8, device="cuda")
    out = torch.zeros(plan.n_pixels * d.SPECTRAL_INFO_BYTES, dtype=torch.uint8, device="cuda")
    plan.spectral(out, scratch, 0.0, 5000)
    torch.cuda.synchronize()
    res = d.spectral_to_numpy(out)
    refs = [ospec.second_eigenvalue(odtm.transition_matrix(s)) for s in scenes]
    near = sum(1 for lam, third in refs if third > 0.9 * abs(lam))
    print(f"{scenes.size} pixels, {near} with |lambda_3| > 0.9 |lambda_2|; subspace steps max "
          f"{res['iterations'].max()}, mean {res['iterations'].mean():.1f}", flush=True)
    assert near >= 7
    _check_spectral(res, scenes, refs, 1e-9, 1e-7, 1e-6)
    plan.close()


def test_spectral_slowest_grid_pixels_at_n1024():
    """The Section 4 grid pixels with the smallest spectral gaps and the
    closest third eigenvalues, at N = 1024 and one at 1536 (the plan then
    keeps the subspace in the workspace rather than on chip), against
    LAPACK."""
    cells = [(75.0, 10.0, 10.0, 1024), (75.0, 0.1, 10.0, 1024), (95.0, 10.0, 7.0, 1024),
             (95.0, 10.0, 10.0, 1024), (95.0, 9.0, 9.0, 1024), (95.0, 8.0, 10.0, 1536)]
    scenes = np.concatenate([sc.scene(dead_time=td, center=30.0, sigma=0.5, signal=S, background=B,
                                      n_bins=n) for td, S, B, n in cells])
    d, plan, ws = _plan(scenes, "f64", lib().opts(tol=1e-12))
    scratch = torch.empty(plan.spectral_scratch_bytes(False), dtype=torch.uint8, device="cuda")
    out = torch.zeros(plan.n_pixels * d.SPECTRAL_INFO_BYTES, dtype=torch.uint8, device="cuda")
    plan.spectral(out, scratch, 0.0, 5000)
    torch.cuda.synchronize()
    res = d.spectral_to_numpy(out)
    refs = [ospec.second_eigenvalue(odtm.transition_matrix(s)) for s in scenes]
    _check_spectral(res, scenes, refs, 1e-9, 1e-7, 1e-6)
    plan.close()


def test_mixing_steps_match_dense_powers():
    levels = (0.1, 3.0, 9.0)
    scenes = np.concatenate([sc.paper_grid(levels, dead_time=75.0, n_bins=64),
                             sc.paper_grid(levels, dead_time=95.0, n_bins=96)])
    d, plan, ws = _plan(scenes, "f64", lib().opts(tol=1e-12))
    scratch = torch.empty(plan.spectral_scratch_bytes(True), dtype=torch.uint8, device="cuda")
    out = torch.zeros(plan.n_pixels * d.SPECTRAL_INFO_BYTES, dtype=torch.uint8, device="cuda")
    for eps in (0.25, 1e-3):
        plan.spectral(out, scratch, eps, 5000)
        torch.cuda.synchronize()
        res = d.spectral_to_numpy(out)
        for p, s in enumerate(scenes):
            Pt = odtm.transition_matrix(s)
            ref = ospec.mixing_steps(Pt, odtm.stationary_solve(Pt), eps)
            assert res["mixing_steps"][p] == ref, (p, s, eps, res[p], ref)
    plan.close()
