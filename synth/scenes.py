"""Seeded synthetic scene generators.

This module only draws scene parameters; it holds none of the method's
arithmetic (no flux, no cumulative flux, no matrix, no shift rule).  Both the
CPU oracle (through the tests) and the GPU path take their inputs from here.

A scene is the problem statement theta = (t_r, t_d, sigma_t, tau, S, B, n_b)
of the paper's Section 2.2 (distortion of the timestamp distribution), with
the flux model of Eq. (arrival_flux): time in ns, S and B in expected photons
per laser period.  Scenes are returned as a NumPy structured array whose field
order and widths match the C struct ``dtm_scene`` (6 float64, 2 int32), so the
array's buffer can be handed to the C-ABI unchanged.

Workloads (all synthetic; the paper's own evaluation is synthetic too, its
Section 3.5 sweeps S, B over {0.1, 3, 6, 9} and over [0, 10]):

* ``single_pixel_n1000``   period 100 ns, N=1000, pulse sigma 0.5 ns at 30 ns,
  S=0.5, B=0.1, dead time 75 ns (deterministic).
* ``single_pixel_n4096``   period 100 ns, N=4096, sigma 0.2 ns, depth U[5,95],
  S log-uniform [0.05,5], B log-uniform [0.01,1], dead time swept over
  {10,33,75,150} ns; ``n_scenes`` draws per dead time (seed 2).
* ``batched_uniform``      64x64 pixels, N=1024, period 100 ns, dead time 50 ns,
  sigma 0.4 ns, depth U[5,95], S, B as above (seed 3).
* ``batched_uneven``       2048 pixels, N from {512,...,8192} with weights
  16:8:4:2:1, period U[50,200] ns, dead time period*U[0.2,1.5],
  sigma U[0.1,1] ns, depth U[5, period-5], S, B as above (seed 4).
* ``warm_start_train`` / ``warm_start_eval``  batched_uniform sampling with
  seeds 5 and 6 (200,000 and 4,096 scenes).
* ``paper_grid``           the (S, B) grid of the paper's Section 3.5 /
  Section 4, period 100 ns, pulse at 30 ns.
"""
from __future__ import annotations

import numpy as np

SCENE_DTYPE = np.dtype(
    [
        ("period_ns", "<f8"),
        ("dead_time_ns", "<f8"),
        ("pulse_center_ns", "<f8"),
        ("pulse_sigma_ns", "<f8"),
        ("signal_flux", "<f8"),
        ("background_flux", "<f8"),
        ("n_bins", "<i4"),
        ("reserved", "<i4"),
    ],
    align=False,
)
assert SCENE_DTYPE.itemsize == 56

UNEVEN_SIZES = np.array([512, 1024, 2048, 4096, 8192], dtype=np.int64)
UNEVEN_WEIGHTS = np.array([16.0, 8.0, 4.0, 2.0, 1.0]) / 31.0


def make_scenes(period, dead_time, center, sigma, signal, background, n_bins):
    """Pack per-field arrays (broadcast to a common length) into scenes."""
    arrays = np.broadcast_arrays(
        np.asarray(period, dtype=np.float64),
        np.asarray(dead_time, dtype=np.float64),
        np.asarray(center, dtype=np.float64),
        np.asarray(sigma, dtype=np.float64),
        np.asarray(signal, dtype=np.float64),
        np.asarray(background, dtype=np.float64),
        np.asarray(n_bins, dtype=np.int64),
    )
    n = arrays[0].size
    out = np.zeros(n, dtype=SCENE_DTYPE)
    for name, a in zip(SCENE_DTYPE.names[:7], arrays):
        out[name] = a.reshape(-1)
    return out


def scene(period=100.0, dead_time=75.0, center=30.0, sigma=0.5, signal=0.5,
          background=0.1, n_bins=1000):
    """One scene (a length-1 structured array)."""
    return make_scenes(period, dead_time, center, sigma, signal, background, n_bins)


def _log_uniform(rng, lo, hi, n):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))


def single_pixel_n1000():
    """Period 100 ns, N=1000 (100 ps bins), sigma 0.5 ns at 30 ns, S=0.5,
    B=0.1, dead time 75 ns."""
    return scene(100.0, 75.0, 30.0, 0.5, 0.5, 0.1, 1000)


def single_pixel_n4096(n_scenes=8, seed=2, dead_times=(10.0, 33.0, 75.0, 150.0)):
    """N=4096 over 100 ns, sigma 0.2 ns; draws (tau, S, B) ``n_scenes`` times
    and crosses them with the dead-time sweep (scene-major order)."""
    rng = np.random.default_rng(seed)
    tau = rng.uniform(5.0, 95.0, n_scenes)
    sig = _log_uniform(rng, 0.05, 5.0, n_scenes)
    bg = _log_uniform(rng, 0.01, 1.0, n_scenes)
    td = np.asarray(dead_times, dtype=np.float64)
    return make_scenes(100.0, np.tile(td, n_scenes), np.repeat(tau, td.size), 0.2,
                       np.repeat(sig, td.size), np.repeat(bg, td.size), 4096)


def batched_uniform(n_pixels=4096, seed=3, n_bins=1024, dead_time=50.0, sigma=0.4):
    """64x64 array: N=1024 over 100 ns, dead time 50 ns, sigma 0.4 ns,
    depth U[5,95], S log-U[0.05,5], B log-U[0.01,1]."""
    rng = np.random.default_rng(seed)
    tau = rng.uniform(5.0, 95.0, n_pixels)
    sig = _log_uniform(rng, 0.05, 5.0, n_pixels)
    bg = _log_uniform(rng, 0.01, 1.0, n_pixels)
    return make_scenes(100.0, dead_time, tau, sigma, sig, bg, n_bins)


def batched_uneven(n_pixels=2048, seed=4, sizes=UNEVEN_SIZES, weights=UNEVEN_WEIGHTS):
    """2048 pixels with N drawn from {512..8192} (weights 16:8:4:2:1), period
    U[50,200], dead time period*U[0.2,1.5], sigma U[0.1,1], depth
    U[5, period-5], S and B as in ``batched_uniform``."""
    rng = np.random.default_rng(seed)
    n = rng.choice(np.asarray(sizes), size=n_pixels, p=np.asarray(weights))
    period = rng.uniform(50.0, 200.0, n_pixels)
    td = period * rng.uniform(0.2, 1.5, n_pixels)
    sigma = rng.uniform(0.1, 1.0, n_pixels)
    tau = 5.0 + rng.uniform(0.0, 1.0, n_pixels) * (period - 10.0)
    sig = _log_uniform(rng, 0.05, 5.0, n_pixels)
    bg = _log_uniform(rng, 0.01, 1.0, n_pixels)
    return make_scenes(period, td, tau, sigma, sig, bg, n)


def stress_n1024(n_pixels=2048, seed=7):
    """Wide parameter draws at N=1024 over 100 ns, for every-pixel stop-rule
    checks: dead time 100 ns x U[0, 3] with a quarter of the draws within
    2 % of a whole number of periods (the nearly periodic, slowly mixing
    chains), sigma U[0.1, 2] ns, depth U[5, 95], S log-uniform [0.01, 10],
    B log-uniform [0.001, 10]."""
    rng = np.random.default_rng(seed)
    td = 100.0 * rng.uniform(0.0, 3.0, n_pixels)
    near = rng.uniform(size=n_pixels) < 0.25
    whole = rng.integers(1, 3, n_pixels) + rng.uniform(-0.02, 0.02, n_pixels)
    td = np.where(near, 100.0 * whole, td)
    sigma = rng.uniform(0.1, 2.0, n_pixels)
    tau = rng.uniform(5.0, 95.0, n_pixels)
    sig = _log_uniform(rng, 0.01, 10.0, n_pixels)
    bg = _log_uniform(rng, 0.001, 10.0, n_pixels)
    return make_scenes(100.0, td, tau, sigma, sig, bg, 1024)


def warm_start_train(n_pixels=200_000, seed=5):
    return batched_uniform(n_pixels=n_pixels, seed=seed)


def warm_start_eval(n_pixels=4096, seed=6):
    return batched_uniform(n_pixels=n_pixels, seed=seed)


def paper_grid(levels=(0.1, 3.0, 6.0, 9.0), dead_time=75.0, n_bins=256, sigma=0.5,
               center=30.0):
    """Cross product of signal and background levels (S outer, B inner)."""
    s, b = np.meshgrid(np.asarray(levels, float), np.asarray(levels, float), indexing="ij")
    return make_scenes(100.0, dead_time, center, sigma, s.ravel(), b.ravel(), n_bins)


def paper_rmse_grid(n_bins=256, dead_time=75.0):
    """The (S, B) grid over [0, 10] of the RMSE study: levels 0.1, 1, 2, ...,
    10 (0.1 stands for the empty end, where S = B = 0 has no photons)."""
    return paper_grid(levels=(0.1,) + tuple(float(v) for v in range(1, 11)), dead_time=dead_time,
                      n_bins=n_bins)


def random_small(n_scenes, seed, n_bins_choices=(2, 3, 5, 8, 17, 31, 64, 100, 129, 257)):
    """Varied small scenes for parity at sizes the oracle finishes quickly:
    ragged N, dead time below and above one period, wide flux range."""
    rng = np.random.default_rng(seed)
    n = rng.choice(np.asarray(n_bins_choices), size=n_scenes)
    period = rng.uniform(20.0, 200.0, n_scenes)
    td = period * rng.uniform(0.0, 2.5, n_scenes)
    sigma = period * rng.uniform(0.002, 0.05, n_scenes)
    tau = period * rng.uniform(0.05, 0.95, n_scenes)
    sig = _log_uniform(rng, 0.01, 10.0, n_scenes)
    bg = _log_uniform(rng, 0.005, 10.0, n_scenes)
    return make_scenes(period, td, tau, sigma, sig, bg, n)


def warm_start_vector(n_bins, seed):
    """A positive random start vector (sums to one) for solver tests."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.1, 1.0, n_bins)
    return v / v.sum()
