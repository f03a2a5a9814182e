"""Pins for the CPU oracle: every check compares it with something other than
itself (quadrature, the per-element integral form, closed forms, a different
eigen-solver, invariants, Monte Carlo physics).  CPU only."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import dtm, elementwise as ew, montecarlo as mc
from synth import scenes as sc


# ---------------------------------------------------------------------------
# Cumulative flux: closed form vs adaptive quadrature of lambda (Theorem 1's F)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("params", [
    dict(period=100.0, center=30.0, sigma=0.5, signal=0.5, background=0.1),
    dict(period=100.0, center=2.0, sigma=1.5, signal=5.0, background=1.0),   # pulse cut at t=0
    dict(period=50.0, center=49.0, sigma=0.7, signal=3.0, background=0.01),  # cut at t_r
])
def test_cumulative_flux_matches_quadrature(params):
    s = sc.scene(n_bins=64, dead_time=10.0, **params)
    t_r, tau, sigma = params["period"], params["center"], params["sigma"]
    for t in np.linspace(0.0, t_r, 23)[1:]:
        pts = [p for p in (tau - 5 * sigma, tau, tau + 5 * sigma) if 0 < p < t]
        ref, _ = quad(lambda u: float(dtm.flux(u, s)), 0.0, t, points=pts or None,
                      epsabs=1e-14, epsrel=1e-13, limit=400)
        assert abs(dtm.cumulative_flux(t, s) - ref) <= 1e-12 * (1 + params["signal"])


def test_total_flux_is_s_plus_b_for_interior_pulse():
    s = sc.single_pixel_n1000()
    assert abs(dtm.total_flux(s) - 0.6) < 1e-15


def test_total_flux_loses_truncated_pulse_mass():
    # Pulse centred on t=0: half of it lies outside [0, t_r).
    s = sc.scene(center=0.0, sigma=1.0, signal=2.0, background=0.3, n_bins=32)
    assert abs(dtm.total_flux(s) - (1.0 + 0.3)) < 1e-14


# ---------------------------------------------------------------------------
# Shift rule (Theorem 2) on the documented workloads
# ---------------------------------------------------------------------------
def test_shift_values_of_the_workloads():
    assert dtm.shift_bins(sc.single_pixel_n1000()) == 750
    got = [dtm.shift_bins(s) for s in sc.single_pixel_n4096(n_scenes=1)]
    assert got == [410, 1352, 3072, 2048]
    assert dtm.shift_bins(sc.batched_uniform(n_pixels=1)) == 512
    # dead time of exactly k periods: no shift
    assert dtm.shift_bins(sc.scene(dead_time=300.0, n_bins=1000)) == 0
    # q just below n_b wraps to 0
    assert dtm.shift_bins(sc.scene(dead_time=99.99, n_bins=1000)) == 0


def test_shift_golden_table():
    """tests/golden/shift_bins.txt: hand-computed l = ceil(x_d n_b / t_r)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "shift_bins.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(rows) >= 8
    for t_r, t_d, n, l in rows:
        s = sc.scene(period=float(t_r), dead_time=float(t_d), n_bins=int(n))
        assert dtm.shift_bins(s) == int(l), (t_r, t_d, n)


# ---------------------------------------------------------------------------
# Theorems 1 and 2 against the per-element integral form (Eq. transition_pmf)
# ---------------------------------------------------------------------------
def _dyadic_scene(n, q, signal=2.0, background=0.5, center=9.0, sigma=1.25):
    # Delta = 2 ns, t_r = 2n: dead times that are whole or 3/4 bins are exact.
    delta = 2.0
    return sc.scene(period=n * delta, dead_time=q * delta, center=center, sigma=sigma,
                    signal=signal, background=background, n_bins=n)


@pytest.mark.parametrize("n,q", [(16, 5.0), (16, 5.75), (16, 21.0), (24, 13.625), (24, 0.0),
                                 (24, 23.75)])
def test_theorems_match_elementwise_integrals(n, q):
    """frac(x_d/Delta) in {0} U (1/2, 1): quantize-then-shift equals
    shift-then-quantize, so Eq. (Eij_ours) must equal Eq. (transition_pmf)."""
    s = _dyadic_scene(n, q)
    P_fast = dtm.transition_matrix(s)
    P_slow = ew.transition_matrix_elementwise(s)
    assert np.max(np.abs(P_fast - P_slow)) < 1e-10
    E_fast = dtm.exponent_matrix(s)
    E_slow = ew.exponent_elementwise(s)
    assert np.max(np.abs(E_fast - E_slow)) < 1e-10


@pytest.mark.parametrize("n,q,equal", [(16, 5.75, True), (16, 5.0, True), (16, 5.25, False),
                                       (16, 5.5, False), (32, 17.9, True), (32, 17.1, False),
                                       (32, 31.6, True)])
def test_theorem2_reactivation_bin(n, q, equal):
    """Thm 2's bin r(i) = (i + ceil(x_d/Delta)) mod n equals D(s_i (+) x_d)
    when frac in {0} U (1/2, 1) and is one bin later when frac in (0, 1/2]."""
    s = _dyadic_scene(n, q)
    exact = ew.reactivation_bins_exact(s)
    thm2 = (np.arange(n) + dtm.shift_bins(s)) % n
    if equal:
        assert np.array_equal(exact, thm2)
    else:
        assert np.array_equal((exact + 1) % n, thm2)


# ---------------------------------------------------------------------------
# Structure of the transition matrix
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1])
def test_matrix_invariants(seed):
    for s in sc.random_small(6, seed=seed):
        Pt = dtm.transition_matrix(s)
        n = int(s["n_bins"])
        assert Pt.shape == (n, n)
        assert np.all(Pt > 0)
        assert np.max(np.abs(Pt.sum(axis=1) - 1.0)) < 1e-14
        # un-normalised entries P_ij / lambda_j are exp of a value in [-Lambda, 0]
        lam = dtm.flux(dtm.bin_centres(s), s)
        E = dtm.unnormalized_matrix(s) / lam[None, :]
        Lam = dtm.total_flux(s)
        assert np.all(E <= 1.0 + 1e-15) and np.all(E >= math.exp(-Lam) * (1 - 1e-12))
        # exactly one E = 1 per row: the reactivation bin itself (no wrap)
        l = dtm.shift_bins(s)
        r = (np.arange(n) + l) % n
        assert np.allclose(E[np.arange(n), r], 1.0, rtol=0, atol=1e-15)


def test_row_shift_is_a_roll_of_the_base_matrix():
    s = sc.scene(dead_time=37.3, n_bins=64)
    base = dtm.transition_matrix(s, shifted=False)
    l = dtm.shift_bins(s)
    assert l == math.ceil(37.3 * 64 / 100)
    full = dtm.transition_matrix(s)
    for i in range(64):
        assert np.array_equal(full[i], base[(i + l) % 64])


def test_whole_period_dead_time_is_bitwise_the_no_dead_time_matrix():
    a = dtm.transition_matrix(sc.scene(dead_time=0.0, n_bins=128))
    for td in (100.0, 200.0, 300.0):
        b = dtm.transition_matrix(sc.scene(dead_time=td, n_bins=128))
        assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# Stationary vector: solve vs eig vs GTH, closed forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [17, 64, 257])
def test_solve_eig_gth_agree(n):
    s = sc.scene(dead_time=61.7, sigma=1.0, signal=3.0, background=0.7, n_bins=n)
    Pt = dtm.transition_matrix(s)
    a = dtm.stationary_solve(Pt)
    b = dtm.stationary_eig(Pt)
    c = dtm.stationary_gth(Pt)
    assert np.abs(a - b).sum() < 1e-12
    assert np.abs(a - c).sum() < 1e-12
    assert np.abs(a @ Pt - a).sum() < 1e-13
    assert np.all(a > 0)


def test_solve_matches_brute_force_eig_at_config_size():
    Pt = dtm.transition_matrix(sc.single_pixel_n1000())
    a = dtm.stationary_solve(Pt)
    b = dtm.stationary_eig(Pt)
    assert np.abs(a - b).sum() < 1e-11


def test_two_state_closed_form():
    for td in (0.0, 13.0, 70.0, 140.0):
        s = sc.scene(dead_time=td, center=20.0, sigma=5.0, signal=1.3, background=0.4, n_bins=2)
        Pt = dtm.transition_matrix(s)
        p01, p10 = Pt[0, 1], Pt[1, 0]
        ref = np.array([p10, p01]) / (p01 + p10)
        assert np.abs(dtm.stationary_solve(Pt) - ref).max() < 1e-15


@pytest.mark.parametrize("td", [0.0, 7.3, 50.0, 99.0, 250.0])
def test_pure_background_is_uniform(td):
    """S = 0: the base matrix is circulant, so pi is exactly uniform."""
    s = sc.scene(dead_time=td, signal=0.0, background=2.5, n_bins=200)
    pi = dtm.stationary_pdf(s)
    assert np.abs(pi - 1.0 / 200).max() < 1e-15


def _recurrence_pi(s):
    """Stationary vector of the l = 0 chain by an O(N) recurrence derived from
    the factorised matrix: with g_j = lambda_j exp(-F_j), c = exp(-Lambda),
    Rh_k = c sum(g) + (1-c) sum_{j>=k} g_j and V_j accumulating pi_k / Rh_k,
    V_j = (V_{j-1} + c g_j/Rh_j) / (1 - (1-c) g_j/Rh_j) with V = 1, and
    pi_j is proportional to g_j (c + (1-c) V_j)."""
    lam, F, Lam, l = dtm.bin_tables(s)
    assert l == 0
    g = lam * np.exp(-F)
    c = math.exp(-Lam)
    T = np.cumsum(g[::-1])[::-1]
    Rh = c * g.sum() + (1 - c) * T
    V = np.empty_like(g)
    prev = 0.0
    for j in range(g.size):
        h = g[j] / Rh[j]
        prev = (prev + c * h) / (1.0 - (1.0 - c) * h)
        V[j] = prev
    pi = g * (c + (1 - c) * V)
    return pi / pi.sum(), V[-1]


@pytest.mark.parametrize("n", [8, 100, 512])
def test_no_dead_time_recurrence(n):
    s = sc.scene(dead_time=0.0, center=40.0, sigma=2.0, signal=4.0, background=0.8, n_bins=n)
    ref, v_last = _recurrence_pi(s)
    assert abs(v_last - 1.0) < 1e-12
    assert np.abs(dtm.stationary_pdf(s) - ref).sum() < 1e-13


def test_no_dead_time_continuum_limit():
    """t_d = 0: the registrations are the arrivals, pi -> lambda / Lambda
    (Section 2.2).  The discrete chain approaches it at rate O(1/N)."""
    errs = []
    for n in (256, 1024):
        s = sc.scene(dead_time=0.0, center=30.0, sigma=0.5, signal=2.0, background=0.5, n_bins=n)
        lam = dtm.flux(dtm.bin_centres(s), s)
        errs.append(np.abs(dtm.stationary_pdf(s) - lam / lam.sum()).sum())
    assert errs[1] < 0.05
    assert 3.0 < errs[0] / errs[1] < 5.0


# ---------------------------------------------------------------------------
# Power iteration and the factorised matrix-vector product
# ---------------------------------------------------------------------------
def test_factorised_left_product_matches_dense():
    """(x P~)_j = g_j [c U_{N-1} + (1-c) U_j] with u_k = x_{(k-l) mod N}/Rh_k
    and U the prefix sum of u (derived from Eqs. (Eij_ours) and the row shift),
    as the O(n) reference of the large-pixel GPU tests writes it."""
    from factored_ref import factored_power, factored_product, residual_l1
    rng = np.random.default_rng(7)
    scenes = np.concatenate([sc.random_small(5, seed=3),
                             sc.scene(dead_time=41.3, center=33.0, sigma=0.3, signal=2.0,
                                      background=0.4, n_bins=300),
                             sc.scene(dead_time=130.0, period=80.0, center=5.0, sigma=1.0,
                                      signal=0.3, background=3.0, n_bins=97)])
    for s in scenes:
        n = int(s["n_bins"])
        Pt = dtm.transition_matrix(s)
        x = rng.uniform(0, 1, n)
        y = factored_product(s)(x)
        ref = x @ Pt
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
        pi = dtm.stationary_solve(Pt)
        xp, ok = factored_power(s, tol=1e-15)
        assert ok and np.abs(xp - pi).sum() < 1e-12
        assert residual_l1(s, pi) < 1e-13
        # the same product with the roll the wrong way round disagrees with
        # the dense matrix (whenever the two directions differ)
        lam, F, Lam, l = dtm.bin_tables(s)
        if l != 0 and 2 * l != n:
            g = lam * np.exp(-F)
            c = math.exp(-Lam)
            Rh = c * g.sum() + (1 - c) * np.cumsum(g[::-1])[::-1]
            U = np.cumsum(np.roll(x, -l) / Rh)
            wrong = g * (c * U[-1] + (1 - c) * U)
            assert np.abs(wrong - ref).max() > 1e-6 * np.abs(ref).max()


def test_power_iteration_reaches_solve():
    s = sc.single_pixel_n1000()
    Pt = dtm.transition_matrix(s)
    x, it, change = dtm.stationary_power(Pt, tol_change=1e-12)
    assert change < 1e-12 and it < 50
    assert np.abs(x - dtm.stationary_solve(Pt)).sum() < 1e-11


# ---------------------------------------------------------------------------
# Model vs physics: Monte Carlo dead-time detector
# ---------------------------------------------------------------------------
@pytest.mark.slow
def test_markov_model_approaches_monte_carlo():
    base = dict(period=100.0, dead_time=75.0, center=30.0, sigma=2.0, signal=2.0, background=0.5)
    rng = np.random.default_rng(11)
    T = mc.register(mc.arrival_times(sc.scene(n_bins=16, **base), 200_000, rng), 75.0)
    T = T[T >= 0.01 * 200_000 * 100.0]
    X = np.mod(T, 100.0)
    errs = []
    for n in (16, 32, 64):
        h = np.bincount((np.ceil(X / (100.0 / n)).astype(int) - 1) % n, minlength=n).astype(float)
        h /= h.sum()
        pi = dtm.stationary_pdf(sc.scene(n_bins=n, **base))
        errs.append(np.abs(pi - h).sum())
    noise = mc.noise_floor_l1(64, T.size)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < noise + 2.5 / 64
    # a wrong shift direction would not approach the physics
    s = sc.scene(n_bins=64, **base)
    bad = dtm.transition_matrix(s, shifted=False)
    bad = np.roll(bad, dtm.shift_bins(s), axis=0)
    h = np.bincount((np.ceil(X / (100.0 / 64)).astype(int) - 1) % 64, minlength=64).astype(float)
    h /= h.sum()
    assert np.abs(dtm.stationary_solve(bad) - h).sum() > 5 * errs[2]


def test_monte_carlo_without_dead_time_is_the_arrival_pdf():
    s = sc.scene(dead_time=0.0, sigma=3.0, signal=1.0, background=1.0, n_bins=20)
    h, n_reg = mc.registration_histogram(s, 40_000, seed=3)
    edges = np.arange(21) * 5.0
    F = dtm.cumulative_flux(edges, s)
    ref = np.diff(F) / F[-1]
    assert np.abs(h - ref).sum() < 3 * mc.noise_floor_l1(20, n_reg)


# ---------------------------------------------------------------------------
# Spectral quantities (Section 4)
# ---------------------------------------------------------------------------
def test_second_eigenvalue_two_state_closed_form():
    from oracle import spectral
    s = sc.scene(dead_time=13.0, center=20.0, sigma=5.0, signal=1.3, background=0.4, n_bins=2)
    Pt = dtm.transition_matrix(s)
    lam, third = spectral.second_eigenvalue(Pt)
    assert abs(lam - (1.0 - Pt[0, 1] - Pt[1, 0])) < 1e-15
    assert third == 0.0  # two states: no eigenvalue besides 1 and lambda_2


def test_second_eigenvalue_of_pure_background_is_a_dft_value():
    """S = 0: P~ is circulant, so its eigenvalues are the discrete Fourier
    transform of its first row."""
    from oracle import spectral
    s = sc.scene(dead_time=31.0, signal=0.0, background=3.0, n_bins=64)
    Pt = dtm.transition_matrix(s)
    row = Pt[0]
    k = np.arange(64)
    dft = np.array([np.sum(row * np.exp(2j * np.pi * k * m / 64)) for m in range(64)])
    dft = dft[np.argsort(-np.abs(dft))]
    lam, third = spectral.second_eigenvalue(Pt)
    assert abs(abs(lam) - abs(dft[1])) < 1e-12
    # the first row is real, so DFT values m and 64 - m are conjugate: the
    # moduli after the Perron value come in equal pairs (m = 32 aside), and
    # the next modulus once lambda_2's pair is set aside is the third one
    mods = np.sort(np.abs(dft[1:]))[::-1]
    assert abs(mods[0] - mods[1]) < 1e-12 and mods[2] < mods[1] - 1e-6
    assert abs(third - mods[2]) < 1e-12


def test_mixing_steps_two_state_closed_form():
    """Two states: d(n) = |lambda_2|^n max(pi_0, pi_1)."""
    from oracle import spectral
    s = sc.scene(dead_time=45.0, center=20.0, sigma=5.0, signal=3.0, background=2.0, n_bins=2)
    Pt = dtm.transition_matrix(s)
    pi = dtm.stationary_solve(Pt)
    lam = abs(1.0 - Pt[0, 1] - Pt[1, 0])
    for eps in (0.25, 1e-3, 1e-6):
        ref = next(n for n in range(1, 10000) if lam ** n * pi.max() <= eps)
        assert spectral.mixing_steps(Pt, pi, eps) == ref


# ---------------------------------------------------------------------------
# Counter-based Monte Carlo (Philox4x32-10)
# ---------------------------------------------------------------------------
def test_philox_known_answers():
    import os
    from oracle.mc_philox import philox4x32_10
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert list(philox4x32_10(v[0:4], v[4:6])) == v[6:10]


@pytest.mark.slow
def test_philox_monte_carlo_agrees_with_numpy_monte_carlo_and_model():
    """Two independent simulators of the same detector (different generators
    and sampling code) agree within their noise, and both approach the
    Markov model."""
    from oracle import mc_philox
    s = sc.scene(period=100.0, dead_time=75.0, center=30.0, sigma=2.0, signal=2.0, background=0.5,
                 n_bins=32)
    hp = mc_philox.histograms(s, runs=2, cycles=15000, burn=150, seed=12345)[0].astype(float)
    hp /= hp.sum()
    hn, n_reg = mc.registration_histogram(s, 60000, seed=4)
    noise = mc.noise_floor_l1(32, 30000) + mc.noise_floor_l1(32, n_reg)
    assert np.abs(hp - hn).sum() < 2.0 * noise
    pi = dtm.stationary_pdf(s)
    assert np.abs(hp - pi).sum() < 0.1 + 2 * mc.noise_floor_l1(32, 30000)
