"""Pins of the discretisation variants (Theorem 2's shift, the flux sampling
of Section 3.4) in the oracle, against independent routes: the element-wise
quadrature model, the paper model at neighbouring dead times, numerical
integration, and a Monte Carlo detector."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import dtm, elementwise as ew, montecarlo as mc, variants as V
from synth import scenes as sc


@pytest.mark.parametrize("n,td", [(8, 41.3), (13, 12.34), (10, 73.0), (9, 160.0), (16, 40.625)])
def test_theorem2_matrix_is_the_elementwise_model_for_any_dead_time(n, td):
    """Eq. (transition_pmf) integrated element by element, with the quantised
    reactivation D(s_i + x_d), is Theorem 2's matrix for every dead time, not
    only for whole-bin ones.  The nearest-shift variant (Eq. (Eij_ori) with
    the exact D(x_k (+) x_d)) agrees with it everywhere but in one corner:
    when the reactivation point lies after the centre s_k of its bin, Eq.
    (transition_pmf) puts a next registration at s_k one period later
    (b = s_k + t_r), a factor e^{-Lambda} on that element, while the indicator
    of Eq. (Eij_ori) compares s_k with s_k and gives 1.  Base row k with that
    factor is base row k + 1, the row Theorem 2 picks: the approximation of
    Theorem 2 and the corner of Theorem 1 cancel."""
    s = sc.scene(period=100.0, dead_time=td, center=37.0, sigma=4.0, signal=1.5, background=0.6, n_bins=n)
    P_slow = ew.transition_matrix_elementwise(s)
    assert np.max(np.abs(dtm.transition_matrix(s) - P_slow)) < 1e-10
    P_near = V.transition_matrix_variant(s, "nearest")
    delta = 100.0 / n
    c = math.exp(-dtm.total_flux(s))
    corners = 0
    for i in range(n):
        a = math.fmod((i + 0.5) * delta + math.fmod(td, 100.0), 100.0)
        k = (math.ceil(a / delta) - 1) % n
        row = P_near[i].copy()
        if 0.0 < math.fmod(a - (k + 0.5) * delta + 100.0, 100.0) < delta:  # after the centre
            row[k] *= c
            row /= row.sum()
            corners += 1
        assert np.max(np.abs(row - P_slow[i])) < 1e-10, i
    q = math.fmod(td, 100.0) * n / 100.0
    f = q - math.floor(q)
    assert corners == (n if 0.0 < f <= 0.5 else 0)


def test_nearest_shift_bins_are_the_exact_reactivation_bins():
    rng = np.random.default_rng(31)
    for _ in range(300):
        n = int(rng.integers(2, 300))
        s = sc.scene(period=float(rng.uniform(20, 200)), dead_time=float(rng.uniform(0, 400)), n_bins=n)
        exact = (ew.reactivation_bins_exact(s) - np.arange(n)) % n
        assert np.all(exact == V.shift_bins_nearest(s))
    # a shifted centre exactly on a bin edge belongs to the lower bin:
    # period 64, 16 bins of 4, x_d = 6 moves centre 4i + 2 to the edge 4(i + 2)
    s = sc.scene(period=64.0, dead_time=6.0, n_bins=16)
    assert V.shift_bins_nearest(s) == 1
    assert np.all((ew.reactivation_bins_exact(s) - np.arange(16)) % 16 == 1)


@pytest.mark.parametrize("f", [0.0, 0.25, 0.5, 0.9])
def test_interpolated_shift_between_whole_bin_dead_times(f):
    """Row i of the interpolated matrix at x_d = (m + f) Delta is the mix of
    the paper's matrices at x_d = m Delta and (m + 1) Delta (whole bins, where
    Theorem 2 is exact)."""
    n, m = 24, 7
    kw = dict(period=120.0, center=50.0, sigma=2.0, signal=2.0, background=0.7, n_bins=n)
    delta = 120.0 / n
    P = V.transition_matrix_variant(sc.scene(dead_time=(m + f) * delta, **kw), "interp")
    A = dtm.transition_matrix(sc.scene(dead_time=m * delta, **kw))
    B = dtm.transition_matrix(sc.scene(dead_time=(m + 1) * delta, **kw))
    assert np.max(np.abs(P - ((1.0 - f) * A + f * B))) < 1e-12
    if f == 0.0:
        assert np.array_equal(P, A)


def test_bin_mean_flux_by_quadrature():
    s = sc.scene(period=100.0, center=30.0, sigma=0.3, signal=4.0, background=0.8, n_bins=50)
    lam = V.bin_mean_flux(s)
    for j in range(50):
        val, _ = quad(lambda t: float(dtm.flux(t, s)), 2.0 * j, 2.0 * (j + 1), points=[30.0],
                      epsabs=1e-14, epsrel=1e-13, limit=200)
        assert abs(lam[j] - val / 2.0) <= 1e-12 * max(1.0, abs(lam[j]))


def test_bin_integral_density_by_quadrature():
    s = sc.scene(period=100.0, center=30.0, sigma=0.3, signal=4.0, background=0.8, n_bins=50)
    g = V.bin_integral_density(s)
    for j in range(50):
        val, _ = quad(lambda t: float(dtm.flux(t, s) * np.exp(-dtm.cumulative_flux(np.array([t]), s)[0])),
                      2.0 * j, 2.0 * (j + 1), points=[30.0], epsabs=1e-15, epsrel=1e-12, limit=200)
        assert abs(g[j] - val / 2.0) <= 1e-11 * max(1e-3, abs(g[j]))


def test_flux_variants_agree_for_constant_flux():
    """S = 0: lambda is constant, so the bin mean is the centre value, and the
    bin integral is e^{-F(s_j)} times one factor common to every bin, which
    the row normalisation removes."""
    s = sc.scene(dead_time=31.7, signal=0.0, background=2.5, n_bins=40)
    P = V.transition_matrix_variant(s)
    for lam in ("bin_mean", "bin_integral"):
        assert np.max(np.abs(V.transition_matrix_variant(s, "ceil", lam) - P)) < 1e-14


def test_variants_converge_together_as_bins_shrink():
    base = dict(period=100.0, dead_time=41.3, center=60.0, sigma=0.5, signal=6.0, background=3.0)
    for shift, lam in (("nearest", "point"), ("interp", "point"), ("ceil", "bin_mean"),
                       ("ceil", "bin_integral"), ("interp", "bin_integral")):
        d = []
        for n in (32, 128, 512):
            s = sc.scene(n_bins=n, **base)
            a = dtm.stationary_solve(V.transition_matrix_variant(s, shift, lam))
            b = dtm.stationary_solve(dtm.transition_matrix(s))
            d.append(np.abs(a - b).sum())
        assert d[2] < 0.01 and d[0] > d[2], (shift, lam, d)


@pytest.mark.slow
def test_bin_integral_fixes_an_under_resolved_pulse():
    """sigma = 0.1 ns against bins of 3.1 and 1.6 ns: sampling lambda at the
    centres misses or overweights the pulse; the bin-integrated first-arrival
    mass brings the model to the Monte Carlo detector."""
    base = dict(period=100.0, dead_time=77.7, center=30.0, sigma=0.1, signal=3.0, background=0.5)
    rng = np.random.default_rng(8)
    T = mc.register(mc.arrival_times(sc.scene(n_bins=16, **base), 400_000, rng), 77.7)
    T = T[T >= 0.01 * 400_000 * 100.0]
    X = np.mod(T, 100.0)
    for n in (32, 64):
        h = np.bincount((np.ceil(X / (100.0 / n)).astype(int) - 1) % n, minlength=n).astype(float)
        h /= h.sum()
        s = sc.scene(n_bins=n, **base)
        e_point = np.abs(dtm.stationary_solve(dtm.transition_matrix(s)) - h).sum()
        e_int = np.abs(dtm.stationary_solve(V.transition_matrix_variant(s, "ceil", "bin_integral")) - h).sum()
        assert e_point > 0.3
        assert e_int < 3 * mc.noise_floor_l1(n, T.size) + 0.03, (n, e_int)
