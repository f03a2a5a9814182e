"""Monte Carlo dead-time detector driven by a counter-based generator.

TEST INFRASTRUCTURE ONLY.  The same physics as ``montecarlo`` (Section 2.1:
Poisson arrivals of rate lambda(t) per period, non-paralyzable dead time,
free-running rearm, X_k = T_k mod t_r), but every random number comes from
Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC 2011), written here from its published definition, and
the sampling steps are spelled out so that another implementation of the
same steps (the GPU simulator) can be compared count for count:

* stream of a period: key = (seed low word, seed high word), counter =
  (draw block, period c, run, pixel); a block gives four 32-bit words w,
  each read as the uniform (w + 0.5) / 2^32.  Periods draw from streams of
  their own, so a simulator may generate them in any order.  Block 0: the
  pulse count and the background count (words 0 and 1), each a Poisson draw
  by inversion: the first k with u <= C_k, where C_0 = p_0 = exp(-S) (resp.
  exp(-B)), p_k = p_{k-1} * S / k, C_k = C_{k-1} + p_k, summed in that order
  in float64 (k < 128; a u beyond C_127 counts as 127).  Then one block per
  four pulse photons: words (0, 1) and (2, 3) are two Box-Muller pairs,
  r = sqrt(-2 ln u1), theta = 2 pi u2, giving tau + sigma r cos(theta) and
  tau + sigma r sin(theta) in that order, as far as the count goes; a time is
  kept when 0 <= t < t_r.  Then one block per four background photons,
  t = t_r u per word, as far as the count goes;
* the detector state is the rearm time a, measured from the start of the
  current period (0 at the start of a run: armed).  The period's photons are
  sorted by time and visited in order; a photon at t >= a is registered and
  sets a = t + t_d.  At the end of the period a becomes max(a - t_r, 0);
* registrations in the first `burn` periods are not counted; the bin of a
  count is ceil(t / Delta) - 1 (0 maps to the last bin).
"""
from __future__ import annotations

import math

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Ten Philox rounds on a 4-word counter with a 2-word key."""
    c0, c1, c2, c3 = (int(x) & MASK for x in ctr)
    k0, k1 = (int(x) & MASK for x in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniforms(seed, block, cycle, run, pixel):
    """The four uniforms of one draw block of a period's stream."""
    w = philox4x32_10((block & MASK, cycle & MASK, run & MASK, pixel & MASK), (seed & MASK, (seed >> 32) & MASK))
    return [(x + 0.5) / 4294967296.0 for x in w]


KMAX = 128


def poisson_cdf(mean, p0):
    """C_0..C_{KMAX-1} of a Poisson law with p_0 = exp(-mean) given."""
    p, c, out = p0, p0, [p0]
    for k in range(1, KMAX):
        p = p * mean / k
        c = c + p
        out.append(c)
    return out


def poisson(u, cdf):
    k = 0
    while k < KMAX - 1 and u > cdf[k]:
        k += 1
    return k


def simulate_run(scene_fields, cycles, burn, seed, run, pixel, hist):
    """Adds the registrations of one run to ``hist`` (n_b integer counts)."""
    t_r, t_d, tau, sigma, S, B, n = scene_fields
    cdf_s, cdf_b = poisson_cdf(S, math.exp(-S)), poisson_cdf(B, math.exp(-B))
    delta = t_r / n
    a = 0.0
    for c in range(cycles):
        u = uniforms(seed, 0, c, run, pixel)
        ns = poisson(u[0], cdf_s)
        nb = poisson(u[1], cdf_b)
        ts = []
        block = 1
        for i in range(0, ns, 4):
            u = uniforms(seed, block, c, run, pixel)
            block += 1
            pulse = []
            for u1, u2 in ((u[0], u[1]), (u[2], u[3])):
                r = math.sqrt(-2.0 * math.log(u1))
                theta = 2.0 * math.pi * u2
                pulse += [tau + sigma * (r * math.cos(theta)), tau + sigma * (r * math.sin(theta))]
            for t in pulse[:min(4, ns - i)]:
                if 0.0 <= t < t_r:
                    ts.append(t)
        for i in range(0, nb, 4):
            u = uniforms(seed, block, c, run, pixel)
            block += 1
            ts += [t_r * x for x in u[:min(4, nb - i)]]
        ts.sort()
        for t in ts:
            if t >= a:
                a = t + t_d
                if c >= burn:
                    j = math.ceil(t / delta) - 1
                    hist[j % n] += 1
        a = max(a - t_r, 0.0)
    return hist


def histograms(scenes, runs, cycles, burn, seed):
    """Counts per pixel (list of int arrays), runs summed."""
    out = []
    for p, s in enumerate(np.asarray(scenes).reshape(-1)):
        f = (float(s["period_ns"]), float(s["dead_time_ns"]), float(s["pulse_center_ns"]),
             float(s["pulse_sigma_ns"]), float(s["signal_flux"]), float(s["background_flux"]),
             int(s["n_bins"]))
        h = np.zeros(f[6], dtype=np.int64)
        for r in range(runs):
            simulate_run(f, cycles, burn, seed, r, p, h)
        out.append(h)
    return out
