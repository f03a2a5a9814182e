"""Spectral convergence quantities of the transition matrix (Section 4).

TEST INFRASTRUCTURE ONLY.  Dense float64 definitions: the eigenvalues of
P~ by LAPACK, the second one by magnitude (its modulus sets the spectral gap
1 - |lambda_2|, its phase the oscillation of the convergence), and the
empirical mixing steps from explicit matrix powers.
"""
from __future__ import annotations

import numpy as np


def second_eigenvalue(Pt):
    """lambda_2: the eigenvalue of largest modulus after the Perron value 1
    (for a conjugate pair, the member with nonnegative imaginary part), and
    the largest modulus among the remaining eigenvalues once lambda_2's
    conjugate is left out (0 when none remain)."""
    w = np.linalg.eigvals(np.asarray(Pt, dtype=np.float64))
    k = int(np.argmin(np.abs(w - 1.0)))
    rest = list(np.delete(w, k)[np.argsort(-np.abs(np.delete(w, k)), kind="stable")])
    first = rest.pop(0)
    if first.imag != 0.0 and rest:
        # a complex eigenvalue comes with its conjugate: leave that one out
        rest.pop(int(np.argmin([abs(z - np.conj(first)) for z in rest])))
    lam = first if first.imag >= 0 else np.conj(first)
    third = max((abs(z) for z in rest), default=0.0)
    return complex(lam), float(third)


def mixing_steps(Pt, pi, eps=0.25, max_steps=10000):
    """Smallest n >= 1 with d(n) <= eps (rows of P~^n advanced one step at a
    time), or -1 if not reached within max_steps."""
    Pt = np.asarray(Pt, dtype=np.float64)
    M = Pt.copy()
    for n in range(1, max_steps + 1):
        if 0.5 * np.abs(M - pi[None, :]).sum(axis=1).max() <= eps:
            return n
        M = M @ Pt
    return -1
