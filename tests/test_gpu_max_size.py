"""The dense batched solver at the largest pixel the library accepts
(n_b = 65536: a 16 GiB float32 matrix per pixel, swept by the banded
launches).  The dense oracle cannot be formed at this size, so each pixel is
checked against a reference that holds at any size and is pinned to the
oracle at small n in the CPU tests:

* t_d = 0 (l = 0): the O(n) recurrence for pi;
* S = 0: pi is exactly uniform (the base matrix is circulant), here at the
  ragged n_b = 65535 (last row band and column block partly filled);
* a general dead time: float64 power iteration with the factorised O(n)
  left product of the same matrix, written out in NumPy, and the residual
  of the GPU's pi under that product.
"""
import numpy as np
import pytest

from oracle import dtm as odtm
from synth import scenes as sc

from gpu_helpers import TOL_F32, run_batched, split
from factored_ref import factored_power, factored_product
from test_oracle_pins import _recurrence_pi

pytestmark = pytest.mark.gpu

N_MAX = 65536


def test_dense_solver_at_maximum_bins():
    scenes = np.concatenate([
        sc.scene(dead_time=0.0, center=40.0, sigma=2.0, signal=4.0, background=0.8, n_bins=N_MAX),
        sc.scene(dead_time=33.0, signal=0.0, background=2.5, n_bins=N_MAX - 1),
        sc.scene(dead_time=41.3, center=33.0, sigma=0.3, signal=2.0, background=0.4, n_bins=N_MAX),
    ])
    pi, info, off = run_batched(scenes, "f32")
    assert np.all(info["status"] == 0), info
    assert np.all(info["flags"] & 0x4)  # certified by the float64 check sweep
    v0, v1, v2 = split(pi, off)

    ref0, v_last = _recurrence_pi(scenes[0])
    assert abs(v_last - 1.0) < 1e-9
    assert np.abs(v0 - ref0).sum() <= TOL_F32

    n1 = N_MAX - 1
    assert np.max(np.abs(v1 - 1.0 / n1)) <= 1e-6 / n1

    ref2, ok2 = factored_power(scenes[2])
    assert ok2
    assert np.abs(v2 - ref2).sum() <= TOL_F32
    y = factored_product(scenes[2])(v2)
    assert np.abs(y / y.sum() - v2).sum() <= TOL_F32
    for v in (v0, v1, v2):
        assert abs(v.sum() - 1.0) < 1e-5 and v.min() > 0
