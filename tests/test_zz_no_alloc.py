"""dtm_stationary_pdf_noalloc (the single-pixel solver with its workspace in
the library's static device array) against dtm_stationary_pdf with a
caller's workspace: the same kernels on the same matrix, so pi and the
solver report must agree exactly.  Two calls in a row per dtype, the first
at the largest accepted size, the second smaller, so that the second call
runs on scratch the first one left behind."""
import numpy as np
import pytest
import torch

from synth import scenes as sc

from gpu_helpers import TOL_F32, TOL_F64, lib, oracle_pi, tdtype

pytestmark = pytest.mark.gpu


def _matrix(d, scene, dt):
    n = int(scene["n_bins"][0])
    P = torch.empty((n, n), dtype=tdtype(dt), device="cuda")
    d.build_transition(scene, P, d.workspace(n, dt))
    return P


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_noalloc_matches_workspace_solver(dt):
    d = lib()
    big = sc.scene(dead_time=75.0, center=30.0, sigma=0.5, signal=0.5, background=0.1,
                   n_bins=d.DTM_NOALLOC_MAX_BINS)
    small = sc.scene(dead_time=75.0, center=30.0, sigma=0.5, signal=0.5, background=0.1, n_bins=1000)
    o = d.opts(tol=1e-6) if dt == "f32" else d.opts(tol=1e-10)
    for scene in (big, small):
        n = int(scene["n_bins"][0])
        print(f"noalloc {dt} n={n}", flush=True)
        P = _matrix(d, scene, dt)
        ref = torch.full((n,), float("nan"), dtype=tdtype(dt), device="cuda")
        ws = d.workspace(n, dt)
        info_ref = d.stationary_pdf(P, ref, ws, o)
        got = torch.full((n,), float("nan"), dtype=tdtype(dt), device="cuda")
        info = d.stationary_pdf_noalloc(P, got, o)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (dt, n, float((got - ref).abs().max()))
        for f in ("iterations", "status", "flags", "change_l1", "residual_l1", "rho_hat"):
            assert getattr(info, f) == getattr(info_ref, f), (dt, n, f)
        assert info.status == d.DTM_OK
        if n <= 1024:
            err = np.abs(got.cpu().numpy().astype(np.float64) - oracle_pi(scene)).sum()
            assert err <= (TOL_F32 if dt == "f32" else TOL_F64), (dt, n, err)
        del P, ws
