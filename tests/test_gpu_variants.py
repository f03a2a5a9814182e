"""GPU parity of the discretisation variants (the exact shift-then-quantize
bin, the interpolated shift, bin-mean flux and the bin-integrated
first-arrival mass) against the float64 oracle's variant matrices."""
import numpy as np
import pytest
import torch

from oracle import dtm as odtm, spectral as ospec, variants as ov
from synth import scenes as sc

from gpu_helpers import TOL_F32, TOL_F64, default_opts, lib, split, tdtype

pytestmark = pytest.mark.gpu

MAT_RTOL = {"f64": 1e-12, "f32": 1e-6}


def _flags(d, shift, lam):
    f = 0
    f |= {"ceil": 0, "nearest": d.DTM_FLAG_SHIFT_NEAREST, "interp": d.DTM_FLAG_SHIFT_INTERP}[shift]
    f |= {"point": 0, "bin_mean": d.DTM_FLAG_LAMBDA_BIN_MEAN, "bin_integral": d.DTM_FLAG_BIN_INTEGRAL}[lam]
    return f


def _scenes():
    return np.concatenate([
        sc.random_small(24, seed=171),
        sc.paper_grid((0.1, 3.0, 9.0), dead_time=41.3, n_bins=64),
        sc.scene(dead_time=77.7, center=30.0, sigma=0.1, signal=3.0, background=0.5, n_bins=100),
        sc.scene(dead_time=40.625, center=30.0, sigma=1.0, signal=2.0, background=1.0, n_bins=16),
    ])


DENSE = [("nearest", "point"), ("ceil", "bin_mean"), ("ceil", "bin_integral"), ("nearest", "bin_integral"),
         ("nearest", "bin_mean")]
FACTORED = DENSE + [("interp", "point"), ("interp", "bin_mean"), ("interp", "bin_integral")]


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("shift,lam", DENSE)
def test_dense_solver_variants_match_oracle(dt, shift, lam):
    d = lib()
    scenes = _scenes()
    o = default_opts(dt)
    o.flags |= _flags(d, shift, lam)
    plan = d.Plan(scenes, dt, o)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    pi = torch.full((plan.pi_elems,), float("nan"), dtype=tdtype(dt), device="cuda")
    infos = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
    plan.solve(pi, infos)
    torch.cuda.synchronize()
    info = d.infos_to_numpy(infos)
    assert np.all(info["status"] == 0), info[info["status"] != 0]
    got = split(pi.cpu().numpy().astype(np.float64), plan.pi_offsets)
    bar = TOL_F64 if dt == "f64" else TOL_F32
    for p, s in enumerate(scenes):
        ref = odtm.stationary_solve(ov.transition_matrix_variant(s, shift, lam))
        assert np.abs(got[p] - ref).sum() <= bar, (p, s)
    plan.close()


@pytest.mark.parametrize("shift,lam", FACTORED)
def test_factored_solver_variants_match_oracle(shift, lam):
    d = lib()
    scenes = _scenes()
    o = d.opts(tol=1e-12)
    o.flags |= _flags(d, shift, lam) | d.DTM_FLAG_NO_DENSE
    plan = d.Plan(scenes, "f64", o)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    pi = torch.full((plan.pi_elems,), float("nan"), dtype=torch.float64, device="cuda")
    infos = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
    plan.solve_factored(pi, infos)
    torch.cuda.synchronize()
    info = d.infos_to_numpy(infos)
    assert np.all(info["status"] == 0), info[info["status"] != 0]
    got = split(pi.cpu().numpy(), plan.pi_offsets)
    for p, s in enumerate(scenes):
        ref = odtm.stationary_solve(ov.transition_matrix_variant(s, shift, lam))
        assert np.abs(got[p] - ref).sum() <= 1e-10, (p, s)
    plan.close()


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("shift,lam", DENSE)
def test_variant_matrices_match_oracle(dt, shift, lam):
    d = lib()
    scenes = sc.random_small(12, seed=172)
    o = default_opts(dt)
    o.flags |= _flags(d, shift, lam)
    plan = d.Plan(scenes, dt, o)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    full = torch.full((plan.matrix_elems,), float("nan"), dtype=tdtype(dt), device="cuda")
    plan.build_transition(full)
    torch.cuda.synchronize()
    Fm = full.cpu().numpy().astype(np.float64)
    mo = plan.mat_offsets
    for p, s in enumerate(scenes):
        n = int(s["n_bins"])
        got = Fm[mo[p]:mo[p + 1]].reshape(n, n)
        assert np.max(np.abs(got / ov.transition_matrix_variant(s, shift, lam) - 1)) < MAT_RTOL[dt], (p, s)
    plan.close()


def test_spectral_analysis_of_interpolated_shift():
    d = lib()
    levels = (0.1, 3.0, 6.0, 9.0)
    scenes = np.concatenate([sc.paper_grid(levels, dead_time=41.3, n_bins=96),
                             sc.paper_grid(levels, dead_time=77.7, n_bins=64)])
    o = d.opts(tol=1e-12)
    o.flags |= d.DTM_FLAG_SHIFT_INTERP | d.DTM_FLAG_NO_DENSE
    plan = d.Plan(scenes, "f64", o)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    scratch = torch.empty(plan.spectral_scratch_bytes(True), dtype=torch.uint8, device="cuda")
    out = torch.zeros(plan.n_pixels * d.SPECTRAL_INFO_BYTES, dtype=torch.uint8, device="cuda")
    plan.spectral(out, scratch, 1e-3, 5000)
    torch.cuda.synchronize()
    res = d.spectral_to_numpy(out)
    checked = 0
    for p, s in enumerate(scenes):
        Pt = ov.transition_matrix_variant(s, "interp")
        assert res["mixing_steps"][p] == ospec.mixing_steps(Pt, odtm.stationary_solve(Pt), 1e-3), (p, s)
        lam, third = ospec.second_eigenvalue(Pt)
        checked += 1
        assert abs(res["lambda2_abs"][p] - abs(lam)) < 1e-9 * max(1.0, abs(lam)), (p, s, res[p], lam)
        assert not (res["flags"][p] & d.DTM_SPECTRAL_UNSETTLED), (p, s, res[p])
    assert checked == scenes.size
    plan.close()


def test_variant_flag_errors():
    d = lib()
    s = sc.random_small(3, seed=173)
    for flags in (d.DTM_FLAG_SHIFT_NEAREST | d.DTM_FLAG_SHIFT_INTERP,
                  d.DTM_FLAG_LAMBDA_BIN_MEAN | d.DTM_FLAG_BIN_INTEGRAL, 0x80):
        o = d.opts(tol=1e-10)
        o.flags |= flags | d.DTM_FLAG_NO_DENSE
        with pytest.raises(d.DtmError):
            d.Plan(s, "f64", o)
    o = d.opts(tol=1e-10)
    o.flags |= d.DTM_FLAG_SHIFT_INTERP  # the dense kernels take whole shifted rows
    with pytest.raises(d.DtmError):
        d.Plan(s, "f64", o)
