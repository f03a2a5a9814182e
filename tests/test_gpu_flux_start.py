"""Batched dense solver started from lambda / sum(lambda), the stationary
vector without dead time (Section 2.2), instead of the uniform vector: same
answers to the parity bars on one-block and banded pixels, a caller's warm
start still takes precedence, and fewer sweeps on the headline pixels."""
import numpy as np
import pytest
import torch

from oracle import dtm as odtm
from synth import scenes as sc

from gpu_helpers import TOL_F32, TOL_F64, default_opts, lib, oracle_pi, run_batched, split

pytestmark = pytest.mark.gpu


def _flux_opts(dt):
    o = default_opts(dt)
    o.flags |= lib().DTM_FLAG_START_FLUX
    return o


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("banded", [False, True])
def test_flux_start_matches_oracle(dt, banded):
    d = lib()
    scenes = np.concatenate([sc.random_small(10, seed=81), sc.batched_uniform(6, seed=82, n_bins=300),
                             sc.scene(n_bins=2, dead_time=30.0, center=20.0, sigma=5.0),
                             sc.scene(n_bins=64, signal=0.0, background=2.0, dead_time=33.0)])
    tiles = d.tiles(fused_max_bins=128, band_rows=64) if banded else None
    pi, info, off = run_batched(scenes, dt, solve_opts=_flux_opts(dt), tiles=tiles)
    assert np.all(info["status"] == 0), info
    tol = TOL_F32 if dt == "f32" else TOL_F64
    for p, (s, v) in enumerate(zip(scenes, split(pi, off))):
        assert np.abs(v - oracle_pi(s)).sum() <= tol, (p, s)
    # S = 0: lambda is flat, so the flux start is the uniform vector and pi
    # (uniform) is reached at once
    assert np.max(np.abs(split(pi, off)[-1] - 1 / 64)) < (1e-15 if dt == "f64" else 1e-8)


def test_flux_start_yields_to_a_warm_start():
    scenes = sc.batched_uniform(16, seed=83)
    x0 = torch.tensor(np.concatenate([oracle_pi(s) for s in scenes]), dtype=torch.float32, device="cuda")
    a, ia, _ = run_batched(scenes, "f32", x0=x0)
    b, ib, _ = run_batched(scenes, "f32", x0=x0, solve_opts=_flux_opts("f32"))
    assert np.array_equal(a, b) and np.array_equal(ia["iterations"], ib["iterations"])


def test_flux_start_saves_sweeps_on_headline_pixels():
    """The first 256 pixels of the 64 x 64 headline batch (N = 1024, t_d = 50
    ns): every pixel within 1e-6 of the oracle on a sample, and fewer
    matrix passes in total than from uniform."""
    scenes = sc.batched_uniform()[:256]
    pu, iu, off = run_batched(scenes, "f32")
    pf, jf, _ = run_batched(scenes, "f32", solve_opts=_flux_opts("f32"))
    assert np.all(jf["status"] == 0)
    assert jf["iterations"].sum() < iu["iterations"].sum()
    vs = split(pf, off)
    for p in range(0, 256, 16):
        assert np.abs(vs[p] - oracle_pi(scenes[p])).sum() <= TOL_F32, p


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_flux_start_falls_back_to_uniform_without_flux_at_the_centres(dt):
    """B = 0 and a pulse 50 sigma from the nearest centres: lambda(s_j) is zero
    at every centre, but the bin-averaged variants keep the pulse's mass and
    define the chain.  The flux start then has nothing to normalise and must
    fall back to the uniform vector (one-block and banded pixels)."""
    from oracle import variants as ovar
    d = lib()
    s = sc.scene(period=100.0, dead_time=33.0, center=30.0, sigma=0.01, signal=1.0, background=0.0,
                 n_bins=100)
    scenes = np.concatenate([s, s])
    tol = TOL_F32 if dt == "f32" else TOL_F64
    for flag, lam in ((d.DTM_FLAG_LAMBDA_BIN_MEAN, "bin_mean"), (d.DTM_FLAG_BIN_INTEGRAL, "bin_integral")):
        o = _flux_opts(dt)
        o.flags |= flag
        ref = odtm.stationary_solve(ovar.transition_matrix_variant(s, "ceil", lam))
        for tiles in (None, d.tiles(fused_max_bins=64, band_rows=32)):
            pi, info, off = run_batched(scenes, dt, solve_opts=o, tiles=tiles)
            assert np.all(info["status"] == 0), info
            for v in split(pi, off):
                assert np.all(np.isfinite(v)) and np.abs(v - ref).sum() <= tol
