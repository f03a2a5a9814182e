"""Every pixel of the benchmarked workloads against the float64 oracle.

* The 64 x 64 headline batch (N = 1024 over 100 ns, t_d = 50 ns, float32
  build and sweeps with the float64 check, default tiles), from
  lambda / sum(lambda) exactly as the benchmark runs it and from the uniform
  start: all 4096 pixels within 1e-6 in L1 of the oracle's pi (Section 2.3:
  the stationary vector of the matrix of Section 3.4).
* The paper's Section 4 grid, S, B in {0.1, 1, ..., 10} at t_d = 75 and 95 ns
  (242 pixels, N = 1024, float32 from the flux start), where the slowest
  chains of the method live (|lambda_2| up to about 0.87): all pixels.
* The uneven batch (2048 pixels, N from 512 to 8192) replayed as a HIP graph
  with the default tiles (the autotuner's pick): every pixel of up to 2048
  bins and eight each of 4096 and 8192 bins against the dense oracle, and
  every pixel above 2048 bins (the banded launches) against float64 power
  iteration with the O(n) factorised product of the same matrix, started
  from the uniform vector.
* 2048 wide parameter draws at N = 1024 (dead time up to three periods,
  a quarter within 2 % of a whole number of periods, S and B log-uniform
  up to 10), float32 from both starts: all pixels.

The oracle runs in a pool of host-core processes (``oracle.pool``).
"""
import numpy as np
import pytest
import torch

from oracle import pool as opool
from synth import scenes as sc

from factored_ref import factored_power, residual_l1
from gpu_helpers import TOL_F32, lib, run_batched, split, tdtype

pytestmark = pytest.mark.gpu


def _opts(flux):
    d = lib()
    o = d.opts(tol=1e-6)
    if flux:
        o.flags |= d.DTM_FLAG_START_FLUX
    return o


@pytest.fixture(scope="module")
def headline():
    scenes = sc.batched_uniform()
    print(f"oracle over {scenes.size} headline pixels", flush=True)
    return scenes, opool.stationary_many(scenes)


@pytest.mark.parametrize("start", ["flux", "uniform"])
def test_headline_batch_every_pixel(headline, start):
    scenes, ref = headline
    print(f"headline batch, start {start}", flush=True)
    pi, info, off = run_batched(scenes, "f32", solve_opts=_opts(start == "flux"))
    assert np.all(info["status"] == 0)
    l1 = np.array([np.abs(v - r).sum() for v, r in zip(split(pi, off), ref)])
    worst = int(np.argmax(l1))
    print(f"start {start}: max L1 {l1.max():.3e} (pixel {worst}), median {np.median(l1):.3e}, "
          f"mean sweeps {info['iterations'].mean():.3f}", flush=True)
    assert l1.max() <= TOL_F32, (worst, l1[worst], info[worst])


def test_section4_grid_every_pixel():
    scenes = np.concatenate([sc.paper_rmse_grid(n_bins=1024, dead_time=75.0),
                             sc.paper_rmse_grid(n_bins=1024, dead_time=95.0)])
    pi, info, off = run_batched(scenes, "f32", solve_opts=_opts(True))
    assert np.all(info["status"] == 0), info[info["status"] != 0]
    l1 = opool.l1_many(scenes, split(pi, off))
    worst = int(np.argmax(l1))
    print(f"Section 4 grid: max L1 {l1.max():.3e} (pixel {worst}), max sweeps "
          f"{info['iterations'].max()}, refined {int(np.sum(info['flags'] & 0x10 != 0))}", flush=True)
    assert l1.max() <= TOL_F32, (worst, scenes[worst], l1[worst], info[worst])


@pytest.mark.parametrize("flux", [True, False])
def test_wide_scene_draws_every_pixel(flux):
    """2048 wide draws at N = 1024 (dead times up to three periods, a
    quarter of them within 2 % of a whole number of periods, S up to 10 and
    B up to 10 photons per period): whatever the stop rule accepted, float32
    from the flux start and from uniform, is within 1e-6 of the oracle."""
    d = lib()
    scenes = sc.stress_n1024()
    pi, info, off = run_batched(scenes, "f32", solve_opts=_opts(flux))
    assert np.all(info["status"] == 0), info[info["status"] != 0]
    l1 = opool.l1_many(scenes, split(pi, off))
    worst = int(np.argmax(l1))
    print(f"wide draws ({'flux' if flux else 'uniform'} start): max L1 {l1.max():.3e} (pixel {worst}), "
          f"sweeps mean {info['iterations'].mean():.2f} max {info['iterations'].max()}, "
          f"{int(np.sum((info['flags'] & d.DTM_INFO_CONTINUED) != 0))} continued", flush=True)
    assert l1.max() <= TOL_F32, (worst, scenes[worst], l1[worst], info[worst])


def test_uneven_batch_graph_every_pixel():
    d = lib()
    scenes = sc.batched_uneven()
    n = scenes["n_bins"]
    plan = d.Plan(scenes, "f32", _opts(True))
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    pi = torch.full((plan.pi_elems,), float("nan"), dtype=tdtype("f32"), device="cuda")
    infos = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
    graph = plan.graph(pi, infos)
    graph.launch()
    torch.cuda.synchronize()
    got = split(pi.cpu().numpy().astype(np.float64), plan.pi_offsets)
    info = d.infos_to_numpy(infos)
    graph.close()
    plan.close()
    del ws
    assert np.all(info["status"] == 0), info[info["status"] != 0]

    rng = np.random.default_rng(11)
    dense = list(np.flatnonzero(n <= 2048))
    for size in (4096, 8192):
        dense += list(rng.choice(np.flatnonzero(n == size), 8, replace=False))
    print(f"uneven batch: oracle over {len(dense)} pixels", flush=True)
    l1 = opool.l1_many(scenes[dense], [got[p] for p in dense])
    worst = int(np.argmax(l1))
    print(f"uneven batch: dense oracle max L1 {l1.max():.3e} (pixel {dense[worst]}, n {n[dense[worst]]})",
          flush=True)
    assert l1.max() <= TOL_F32, (dense[worst], scenes[dense[worst]], l1[worst])

    big = np.flatnonzero(n > 2048)
    worst_f, worst_r = 0.0, 0.0
    for p in big:
        ref, ok = factored_power(scenes[p])
        assert ok, p
        worst_f = max(worst_f, float(np.abs(got[p] - ref).sum()))
        worst_r = max(worst_r, residual_l1(scenes[p], got[p]))
    print(f"uneven batch: {big.size} banded pixels, max L1 vs float64 factored power {worst_f:.3e}, "
          f"max residual {worst_r:.3e}", flush=True)
    assert worst_f <= TOL_F32
