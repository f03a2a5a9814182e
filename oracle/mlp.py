"""Float64 reference of the warm-start network (test infrastructure only).

Not from the paper: the warm start is a project addition that predicts the
stationary PDF pi from the scene parameters to seed power iteration.  The
network is
    phi (5) -> Linear(5, 256) -> GELU -> Linear(256, 256) -> GELU
            -> Linear(256, 1024) -> (+ prior logits) -> softmax,
with GELU(x) = x Phi(x) (erf form), an optional fixed prior added to the
logits (the log of the flux start lambda_j / sum_k lambda_k at the 1024 bin
centres, ``flux_prior``), trained by cross-entropy
-sum_j t_j log q_j against target PDFs t.  Weights are row-major
(in x out), so a layer is X W + b.  Gradients are the written-out chain rule
and are pinned by central finite differences in the CPU tests.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

IN, HIDDEN, OUT = 5, 256, 1024


def features(scene):
    """phi(theta): fixed affine maps of (tau, sigma, ln S, ln B, x_d) onto
    about [-1, 1] for the warm-start workload's ranges."""
    s = np.asarray(scene).reshape(-1)[0]
    t_r = float(s["period_ns"])
    return np.array([
        2.0 * float(s["pulse_center_ns"]) / t_r - 1.0,
        float(s["pulse_sigma_ns"]),
        2.0 * (math.log(max(float(s["signal_flux"]), 1e-30)) - math.log(0.05)) / math.log(100.0) - 1.0,
        2.0 * (math.log(max(float(s["background_flux"]), 1e-30)) - math.log(0.01)) / math.log(100.0) - 1.0,
        math.fmod(float(s["dead_time_ns"]), t_r) / t_r,
    ])


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def flux_prior(scene, n_out=OUT):
    """log(lambda_j / sum_k lambda_k) at the centres (j + 1/2) t_r / n_out of
    the scene's period, lambda the flux of Eq. (arrival_flux) (the oracle's
    ``dtm.flux``)."""
    from oracle import dtm
    s = np.asarray(scene).reshape(-1)[0]
    centres = (np.arange(n_out) + 0.5) * float(s["period_ns"]) / n_out
    lam = dtm.flux(centres, s)
    return np.log(lam) - np.log(lam.sum())


def forward(params, X, prior=None):
    """Returns (Q, cache).  params: dict W1 (5x256), b1, W2 (256x256), b2,
    W3 (256x1024), b3; X: batch x 5; prior: batch x 1024 logits added
    before the softmax, or None."""
    A1 = X @ params["W1"] + params["b1"]
    H1 = gelu(A1)
    A2 = H1 @ params["W2"] + params["b2"]
    H2 = gelu(A2)
    Z = H2 @ params["W3"] + params["b3"]
    if prior is not None:
        Z = Z + prior
    Zs = Z - Z.max(axis=1, keepdims=True)
    E = np.exp(Zs)
    Q = E / E.sum(axis=1, keepdims=True)
    logQ = Zs - np.log(E.sum(axis=1, keepdims=True))
    return Q, dict(X=X, A1=A1, H1=H1, A2=A2, H2=H2, logQ=logQ, Q=Q)


def loss(params, X, T, prior=None):
    """Mean over rows of -sum_j T_j log Q_j."""
    _, c = forward(params, X, prior)
    return float(-(T * c["logQ"]).sum(axis=1).mean())


def grads(params, X, T, prior=None):
    """Gradients of the mean cross-entropy with respect to every parameter
    (the prior is a constant: it shifts Q, not the form of dZ)."""
    _, c = forward(params, X, prior)
    B = X.shape[0]
    dZ = (c["Q"] - T) / B  # softmax + cross-entropy; rows of T sum to 1
    g = {}
    g["W3"] = c["H2"].T @ dZ
    g["b3"] = dZ.sum(axis=0)
    dA2 = (dZ @ params["W3"].T) * gelu_grad(c["A2"])
    g["W2"] = c["H1"].T @ dA2
    g["b2"] = dA2.sum(axis=0)
    dA1 = (dA2 @ params["W2"].T) * gelu_grad(c["A1"])
    g["W1"] = c["X"].T @ dA1
    g["b1"] = dA1.sum(axis=0)
    return g
