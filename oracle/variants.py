"""Discretisation variants of the dead-time chain.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``).

Theorem 2 replaces the bin of the shifted centre, D(s_i (+) x_d) ("shift then
quantize"), by the centre s_i moved by ceil(x_d / Delta) whole bins
("quantize then shift"); Remark 2 notes that the error vanishes as the bins
shrink.  Section 3.4 samples the flux at the bin centres, lambda_j =
lambda(s_j).  The variants here change one of those two steps and nothing
else (same exponent matrix of Theorem 1, same row normalisation):

* ``shift="nearest"``: the exact shift-then-quantize bin.  With bins
  (j Delta, (j + 1) Delta] and q = x_d / Delta, s_i + x_d = (i + 1/2 + q) Delta
  lies in bin i + ceil(q - 1/2), one bin fewer than Theorem 2 whenever the
  fractional part of q is in (0, 1/2].
* ``shift="interp"``: the reactivation point s_i + x_d lies between the
  centres s_{i+m} and s_{i+m+1} (q = m + f, 0 <= f < 1); row i of the matrix
  is (1 - f) times base row i + m plus f times base row i + m + 1 (linear
  interpolation in the reactivation time; rows stay stochastic).
* ``lam="bin_mean"``: lambda_j = (F(e_{j+1}) - F(e_j)) / Delta, the flux
  averaged over bin j, in place of the point value at its centre (matters
  when the pulse is narrower than a bin).
* ``lam="bin_integral"``: the product lambda_j e^{-F(s_j)} (the density of
  the first arrival, up to the row factor) replaced by its average over bin
  j, (e^{-F(e_j)} - e^{-F(e_{j+1})}) / Delta: the exact probability that the
  first arrival after a reactivation before the bin falls in it.

``shift="ceil"``, ``lam="point"`` is the paper's model and reproduces
``dtm.transition_matrix``.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ndtr

from .dtm import (SHIFT_SNAP_RTOL, _fields, base_exponent_matrix, bin_centres, cumulative_flux, flux,
                  relative_dead_time, shift_bins, total_flux)


def _snap(p):
    """Nearest integer when p is one up to a relative 1e-9, else None."""
    r = round(p)
    return int(r) if abs(p - r) <= SHIFT_SNAP_RTOL * max(1.0, abs(p)) else None


def shift_bins_nearest(scene):
    """ceil(x_d / Delta - 1/2) mod n_b: the bin the shifted centre falls in
    (a centre shifted exactly onto a bin edge belongs to the lower bin)."""
    t_r, *_, n = _fields(scene)
    p = relative_dead_time(scene) * n / t_r - 0.5
    r = _snap(p)
    return (r if r is not None else int(math.ceil(p))) % n


def fractional_shift(scene):
    """(m, f) with x_d / Delta = m + f, 0 <= f < 1 (f = 0 when x_d / Delta
    is an integer up to a relative 1e-9); m is taken mod n_b."""
    t_r, *_, n = _fields(scene)
    q = relative_dead_time(scene) * n / t_r
    r = _snap(q)
    if r is not None:
        return r % n, 0.0
    m = int(math.floor(q))
    return m % n, q - m


def bin_flux(scene):
    """F(e_{j+1}) - F(e_j), the flux integrated over each bin, without
    subtracting the cumulative values: S times the Gaussian mass of the bin
    (taken between upper-tail probabilities right of the pulse centre, where
    the cdf differences would cancel) plus B Delta / t_r."""
    t_r, _, tau, sigma, S, B, n = _fields(scene)
    delta = t_r / n
    e = np.arange(n + 1, dtype=np.float64) * delta
    z = (e - tau) / sigma
    za, zb = z[:-1], z[1:]
    mass = np.where(za >= 0.0, ndtr(-za) - ndtr(-zb), ndtr(zb) - ndtr(za))
    return S * mass + B * delta / t_r


def bin_mean_flux(scene):
    """lambda averaged over each bin: (F(e_{j+1}) - F(e_j)) / Delta."""
    t_r, *_, n = _fields(scene)
    return bin_flux(scene) / (t_r / n)


def bin_integral_density(scene):
    """(e^{-F(e_j)} - e^{-F(e_{j+1})}) / Delta for every bin j, evaluated as
    e^{-F(e_j)} (1 - e^{-(F(e_{j+1}) - F(e_j))}) / Delta so that narrow
    bins lose no digits."""
    t_r, *_, n = _fields(scene)
    delta = t_r / n
    F_lo = cumulative_flux(np.arange(n, dtype=np.float64) * delta, scene)
    return np.exp(-F_lo) * -np.expm1(-bin_flux(scene)) / delta


def base_transition_matrix(scene, lam="point"):
    """Row-normalised base matrix: row k is the next-registration pmf for a
    reactivation at the centre s_k (no dead-time shift)."""
    E = base_exponent_matrix(scene)
    if lam == "point":
        P = flux(bin_centres(scene), scene)[None, :] * E
    elif lam == "bin_mean":
        P = bin_mean_flux(scene)[None, :] * E
    elif lam == "bin_integral":
        # E_kj = e^{-Lambda [s_k > s_j]} e^{F(s_k)} e^{-F(s_j)}: the column
        # factor e^{-F(s_j)} goes into the bin average, the row factor cancels
        c = np.exp(-total_flux(scene))
        s = bin_centres(scene)
        P = bin_integral_density(scene)[None, :] * np.where(s[:, None] > s[None, :], c, 1.0)
    else:
        raise ValueError(lam)
    return P / P.sum(axis=1, keepdims=True)


def transition_matrix_variant(scene, shift="ceil", lam="point"):
    """The row-stochastic matrix of a variant (see the module docstring)."""
    B = base_transition_matrix(scene, lam)
    n = B.shape[0]
    i = np.arange(n)
    if shift == "ceil":
        return B[(i + shift_bins(scene)) % n]
    if shift == "nearest":
        return B[(i + shift_bins_nearest(scene)) % n]
    if shift == "interp":
        m, f = fractional_shift(scene)
        return (1.0 - f) * B[(i + m) % n] + f * B[(i + m + 1) % n]
    raise ValueError(shift)
