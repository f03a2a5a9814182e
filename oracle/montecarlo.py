"""Monte Carlo simulator of an asynchronous SPAD with dead time.

TEST INFRASTRUCTURE ONLY.  It simulates the physics of Section 2.1 directly,
with no Markov chain: photons arrive as an inhomogeneous Poisson process of
rate lambda(t) on each laser period (Eq. arrival_flux); the free-running
detector registers a photon, is blind for a fixed non-paralyzable dead time
t_d, and rearms the moment the dead time ends, without waiting for the laser
sync; the TCSPC records X_k = T_k mod t_r and a histogram of n_b bins is
formed.  The histogram of the stationary regime estimates the registration
PDF that the Markov chain predicts.

Per period: Poisson(S) pulse photons at tau + sigma*N(0,1) (those outside
[0, t_r) are dropped: the pulse is truncated to one period, like the flux
model) and Poisson(B) background photons uniform on [0, t_r).  The first 1%
of cycles are discarded as burn-in.  Bins are right-closed,
bin j = (j Delta, (j+1) Delta], matching the quantiser D of Section 3.1.
"""
from __future__ import annotations

import math

import numpy as np

from .dtm import _fields


def arrival_times(scene, n_cycles, rng):
    """Sorted absolute photon arrival times over ``n_cycles`` periods."""
    t_r, _, tau, sigma, S, B, _ = _fields(scene)
    n_sig = rng.poisson(S, n_cycles)
    n_bg = rng.poisson(B, n_cycles)
    cyc_sig = np.repeat(np.arange(n_cycles), n_sig)
    cyc_bg = np.repeat(np.arange(n_cycles), n_bg)
    t_sig = tau + sigma * rng.standard_normal(cyc_sig.size)
    keep = (t_sig >= 0.0) & (t_sig < t_r)
    t_bg = rng.uniform(0.0, t_r, cyc_bg.size)
    T = np.concatenate([cyc_sig[keep] * t_r + t_sig[keep], cyc_bg * t_r + t_bg])
    T.sort()
    return T


def register(T, dead_time):
    """Non-paralyzable dead time: the first photon is registered; afterwards
    a photon is registered iff it arrives at or after the previous
    registration plus the dead time.  Returns the registered times."""
    out = []
    i = 0
    n = T.size
    while i < n:
        t = T[i]
        out.append(t)
        i = max(i + 1, int(np.searchsorted(T, t + dead_time, side="left")))
    return np.asarray(out)


def registration_histogram(scene, n_cycles, seed, burn_in=0.01):
    """Normalised histogram (sums to 1) of X_k = T_k mod t_r over n_b bins."""
    t_r, t_d, *_, n = _fields(scene)
    rng = np.random.default_rng(seed)
    T = register(arrival_times(scene, n_cycles, rng), t_d)
    T = T[T >= burn_in * n_cycles * t_r]
    X = np.mod(T, t_r)
    delta = t_r / n
    idx = (np.ceil(X / delta).astype(np.int64) - 1) % n
    h = np.bincount(idx, minlength=n).astype(np.float64)
    return h / h.sum(), int(T.size)


def noise_floor_l1(n_bins, n_registrations):
    """Expected L1 error of a multinomial histogram estimate with the given
    number of samples, sum_j sqrt(2 p_j (1-p_j) / (pi n)) <= sqrt(2 N / (pi n))
    (mean absolute deviation of a binomial count, normal approximation)."""
    return math.sqrt(2.0 * n_bins / (math.pi * n_registrations))
