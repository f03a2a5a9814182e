"""An O(n) float64 reference for pixels too large for the dense oracle
(test infrastructure).

The left product with the dead-time matrix of Section 3.4 factorises (the
row factor exp(F_k) cancels in the row normalisation, and row i is base row
(i + l) mod n by Theorem 2): with g_j = lambda_j exp(-F_j), c = exp(-Lambda)
and the base row normalisers Rh_k = c sum(g) + (1 - c) sum_{j >= k} g_j,

    (x P~)_j = g_j (c U_{n-1} + (1 - c) U_j),   U_j = sum_{k <= j} x_{(k-l) mod n} / Rh_k.

The tables come from the oracle (``oracle.dtm.bin_tables``); the product is
pinned against the oracle's dense matrix in ``test_oracle_pins.py``.
"""
import math

import numpy as np

from oracle import dtm as odtm


def factored_product(s):
    """x -> x P~ for the scene's dead-time matrix, in O(n)."""
    lam, F, Lam, l = odtm.bin_tables(s)
    g = lam * np.exp(-F)
    c = math.exp(-Lam)
    Rh = c * g.sum() + (1 - c) * np.cumsum(g[::-1])[::-1]

    def apply(x):
        U = np.cumsum(np.roll(x, l) / Rh)
        return g * (c * U[-1] + (1 - c) * U)
    return apply


def factored_power(s, x0=None, tol=1e-14, max_iter=20000):
    """Float64 power iteration with the factorised product from x0 (uniform
    when None) until the L1 change is below tol.  Returns (x, converged)."""
    apply = factored_product(s)
    n = int(np.asarray(s).reshape(-1)[0]["n_bins"])
    x = np.full(n, 1.0 / n) if x0 is None else np.asarray(x0, dtype=np.float64) / np.sum(x0)
    for _ in range(max_iter):
        y = apply(x)
        y /= y.sum()
        done = np.abs(y - x).sum() < tol
        x = y
        if done:
            return x, True
    return x, False


def residual_l1(s, x):
    """||x P~ - x||_1 for x normalised to sum 1, in float64."""
    x = np.asarray(x, dtype=np.float64)
    x = x / x.sum()
    return float(np.abs(factored_product(s)(x) - x).sum())
