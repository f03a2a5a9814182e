"""Element-wise transition matrix, Eq. (transition_pmf), by numerical
integration.

TEST INFRASTRUCTURE ONLY.  This is the slow formulation the paper accelerates:
for every pair (s_i, s_j) the exponent is an integral of the periodic flux
replica between the quantised reactivation point D(a) and the quantised next
registration D(b), with

    a = s_i + x_d,   b = ceil((a - s_j) / t_r) * t_r + s_j     (Section 3.1)

and D(t) = (ceil(t / Delta) - 1/2) Delta applied on the whole real line (it
commutes with shifts by t_r because t_r = n_b * Delta).  The integral is
evaluated by adaptive quadrature of lambda itself, never through the closed
form of F, so it pins Theorem 1 (the cumulative-flux exponent) and Theorem 2
(quantize-then-shift) independently of the oracle's construction.

Only small n_b (tens of bins) are practical: n_b^2 quadratures.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad

from .dtm import _fields, flux


def quantize(t, delta):
    """D(t) = (ceil(t / Delta) - 1/2) Delta (Section 3.1)."""
    return (math.ceil(t / delta) - 0.5) * delta


def periodic_flux_integral(u, v, scene):
    """Integral of the periodic replica of lambda over [u, v], u <= v, by
    quadrature over each period piece (break points at the pulse centre)."""
    t_r, _, tau, sigma, *_ = _fields(scene)
    if v <= u:
        return 0.0
    total = 0.0
    k = math.floor(u / t_r)
    while k * t_r < v:
        lo = max(u, k * t_r) - k * t_r
        hi = min(v, (k + 1) * t_r) - k * t_r
        if hi > lo:
            pts = [p for p in (tau - 8 * sigma, tau, tau + 8 * sigma) if lo < p < hi]
            val, _ = quad(lambda t: float(flux(t, scene)), lo, hi, points=pts or None,
                          epsabs=1e-14, epsrel=1e-13, limit=400)
            total += val
        k += 1
    return total


def exponent_elementwise(scene):
    """E_ij = exp(-int_{D(a)}^{D(b)} lambda~) for all i, j (Eq. transition_pmf)."""
    t_r, t_d, *_, n = _fields(scene)
    delta = t_r / n
    x_d = math.fmod(t_d, t_r)
    s = (np.arange(n) + 0.5) * delta
    E = np.empty((n, n))
    for i in range(n):
        a = s[i] + x_d
        lo = quantize(a, delta)
        for j in range(n):
            b = math.ceil((a - s[j]) / t_r) * t_r + s[j]
            hi = quantize(b, delta)
            E[i, j] = math.exp(-periodic_flux_integral(lo, hi, scene))
    return E


def transition_matrix_elementwise(scene):
    """P_ij proportional to lambda(s_j) E_ij, rows normalised (Eq. transition_pmf)."""
    t_r, *_, n = _fields(scene)
    s = (np.arange(n) + 0.5) * (t_r / n)
    P = flux(s, scene)[None, :] * exponent_elementwise(scene)
    return P / P.sum(axis=1, keepdims=True)


def reactivation_bins_exact(scene):
    """Index of D(s_i (+) x_d), the exact shift-then-quantize bin (Thm 2's
    left-hand side), for every state i."""
    t_r, t_d, *_, n = _fields(scene)
    delta = t_r / n
    x_d = math.fmod(t_d, t_r)
    out = np.empty(n, dtype=np.int64)
    for i in range(n):
        a = math.fmod((i + 0.5) * delta + x_d, t_r)
        out[i] = (math.ceil(a / delta) - 1) % n
    return out
