"""Pins for the float64 warm-start network: closed-form features and
central finite differences of the cross-entropy gradients.  CPU only."""
import numpy as np

from oracle import mlp
from synth import scenes as sc


def _params(rng, scale=0.3):
    return {
        "W1": rng.normal(0, scale, (mlp.IN, mlp.HIDDEN)), "b1": rng.normal(0, 0.1, mlp.HIDDEN),
        "W2": rng.normal(0, scale / 4, (mlp.HIDDEN, mlp.HIDDEN)), "b2": rng.normal(0, 0.1, mlp.HIDDEN),
        "W3": rng.normal(0, scale / 4, (mlp.HIDDEN, mlp.OUT)), "b3": rng.normal(0, 0.1, mlp.OUT),
    }


def test_features_closed_form():
    # tau = 30 ns is at 307.2 bins of 100/1024 ns: bin 307, 0.3 bins before
    # that bin's centre at 307.5
    s = sc.scene(period=100.0, dead_time=150.0, center=30.0, sigma=0.4, signal=0.05, background=1.0)
    assert mlp.pulse_bin(s) == 307
    assert np.allclose(mlp.features(s), [-0.6, 0.4, -1.0, 1.0, 0.5], atol=1e-12)
    # tau on a bin edge (25 ns = bin 512 of 1024 over 50 ns): offset -1/2
    s = sc.scene(period=50.0, dead_time=10.0, center=25.0, sigma=1.0, signal=5.0, background=0.01)
    assert mlp.pulse_bin(s) == 512
    assert np.allclose(mlp.features(s), [-1.0, 1.0, 1.0, -1.0, 0.2], atol=1e-15)


def test_rotation_is_a_roll_of_the_bins():
    """Bin j takes the network's output (j - k) mod 1024: with no prior the
    rotated PDF is the unrotated one rolled forward by k bins, row by row,
    and the cross-entropy against a target rolled the same way is unchanged."""
    rng = np.random.default_rng(6)
    P = _params(rng)
    X = rng.normal(size=(3, mlp.IN))
    k = np.array([0, 5, 1023])
    Q0, _ = mlp.forward(P, X)
    Qk, _ = mlp.forward(P, X, shift=k)
    for i in range(3):
        assert np.allclose(Qk[i], np.roll(Q0[i], k[i]), atol=1e-15)
    T = rng.uniform(size=(3, mlp.OUT))
    T /= T.sum(axis=1, keepdims=True)
    Tk = np.stack([np.roll(T[i], k[i]) for i in range(3)])
    assert abs(mlp.loss(P, X, Tk, shift=k) - mlp.loss(P, X, T)) < 1e-12


def test_stationary_pdf_rotates_with_the_pulse():
    """What the rotation relies on: moving the pulse by whole bins rotates
    the model's stationary PDF by as many bins (the flux, its integral and
    the dead-time shift are periodic in the arrival time), so two such scenes
    have the same features and pulse bins that differ by the move."""
    from oracle import dtm as odtm
    n, t_r = mlp.OUT, 100.0
    d = t_r / n
    a = sc.scene(period=t_r, dead_time=50.0, center=300.3 * d, sigma=0.4, signal=2.0, background=0.3, n_bins=n)
    b = sc.scene(period=t_r, dead_time=50.0, center=(300.3 + 377) * d, sigma=0.4, signal=2.0, background=0.3,
                 n_bins=n)
    assert mlp.pulse_bin(b) - mlp.pulse_bin(a) == 377
    assert np.allclose(mlp.features(a), mlp.features(b), atol=1e-12)
    pa = odtm.stationary_solve(odtm.transition_matrix(a))
    pb = odtm.stationary_solve(odtm.transition_matrix(b))
    assert np.abs(np.roll(pa, 377) - pb).sum() < 1e-11


def test_gelu_matches_its_definition():
    from scipy.stats import norm
    x = np.linspace(-6, 6, 101)
    assert np.allclose(mlp.gelu(x), x * norm.cdf(x), atol=1e-15)
    h = 1e-6
    assert np.allclose(mlp.gelu_grad(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h), atol=1e-8)


def test_softmax_rows_sum_to_one():
    rng = np.random.default_rng(0)
    Q, _ = mlp.forward(_params(rng), rng.normal(size=(4, mlp.IN)))
    assert np.allclose(Q.sum(axis=1), 1.0, atol=1e-14) and np.all(Q > 0)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    P = _params(rng)
    X = rng.normal(size=(3, mlp.IN))
    T = rng.uniform(size=(3, mlp.OUT))
    T /= T.sum(axis=1, keepdims=True)
    G = mlp.grads(P, X, T)
    h = 1e-6
    for name, arr in P.items():
        flat = arr.reshape(-1)
        for idx in rng.choice(flat.size, 12, replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(P, X, T)
            flat[idx] = old - h
            lm = mlp.loss(P, X, T)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = G[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)) + 1e-9, (name, idx, fd, an)


def test_gradients_with_prior_match_finite_differences():
    """The prior is a constant shift of the logits: the chain rule is the
    same, only Q moves."""
    rng = np.random.default_rng(4)
    P = _params(rng)
    X = rng.normal(size=(2, mlp.IN))
    prior = rng.normal(0, 2.0, size=(2, mlp.OUT))
    T = rng.uniform(size=(2, mlp.OUT))
    T /= T.sum(axis=1, keepdims=True)
    G = mlp.grads(P, X, T, prior)
    h = 1e-6
    for name, arr in P.items():
        flat = arr.reshape(-1)
        for idx in rng.choice(flat.size, 6, replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(P, X, T, prior)
            flat[idx] = old - h
            lm = mlp.loss(P, X, T, prior)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = G[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)) + 1e-9, (name, idx, fd, an)
    # a prior constant along a row changes nothing
    Q0, _ = mlp.forward(P, X)
    Q1, _ = mlp.forward(P, X, np.full((2, mlp.OUT), 3.7))
    assert np.allclose(Q0, Q1, atol=1e-15)


def test_gradients_with_prior_and_rotation_match_finite_differences():
    """With the rotation each bin's error goes back to the output it took."""
    rng = np.random.default_rng(7)
    P = _params(rng)
    X = rng.normal(size=(2, mlp.IN))
    prior = rng.normal(0, 2.0, size=(2, mlp.OUT))
    k = np.array([300, 1021])
    T = rng.uniform(size=(2, mlp.OUT))
    T /= T.sum(axis=1, keepdims=True)
    G = mlp.grads(P, X, T, prior, k)
    h = 1e-6
    for name, arr in P.items():
        flat = arr.reshape(-1)
        for idx in rng.choice(flat.size, 6, replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(P, X, T, prior, k)
            flat[idx] = old - h
            lm = mlp.loss(P, X, T, prior, k)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = G[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)) + 1e-9, (name, idx, fd, an)


def test_flux_prior_special_cases():
    # pure background: the flux is constant, the prior uniform
    s = sc.scene(period=80.0, dead_time=30.0, center=20.0, sigma=0.5, signal=0.0, background=0.7)
    assert np.allclose(mlp.flux_prior(s), -np.log(mlp.OUT), atol=1e-13)
    # no background: a sampled Gaussian whose height S / (sigma sqrt(2 pi))
    # drops out, so the prior does not depend on S
    a = mlp.flux_prior(sc.scene(period=100.0, center=40.0, sigma=2.0, signal=0.3, background=0.0))
    b = mlp.flux_prior(sc.scene(period=100.0, center=40.0, sigma=2.0, signal=3.0, background=0.0))
    assert np.allclose(a, b, atol=1e-12)
    z = ((np.arange(mlp.OUT) + 0.5) * 100.0 / mlp.OUT - 40.0) / 2.0
    ref = -0.5 * z * z - np.log(np.exp(-0.5 * z * z).sum())
    assert np.allclose(a, ref, atol=1e-12)
    # every prior is a log-distribution
    for s in sc.batched_uniform(8, seed=12):
        assert abs(np.exp(mlp.flux_prior(s)).sum() - 1.0) < 1e-12
