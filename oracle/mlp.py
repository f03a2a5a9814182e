"""Float64 reference of the warm-start network (test infrastructure only).

Not from the paper: the warm start is a project addition that predicts the
stationary PDF pi from the scene parameters to seed power iteration.  The
network is
    phi (5) -> Linear(5, 256) -> GELU -> Linear(256, 256) -> GELU
            -> Linear(256, 1024) -> (rotation by the pulse bin k)
            -> (+ prior logits) -> softmax,
with GELU(x) = x Phi(x) (erf form), the rotation making output m the logit
of bin (m + k) mod 1024 (``pulse_bin``; the model is periodic in the arrival
time, so moving the pulse by whole bins rotates pi), an optional fixed prior
added to the logits (the log of the flux start lambda_j / sum_k lambda_k at
the 1024 bin centres, ``flux_prior``), trained by cross-entropy
-sum_j t_j log q_j against target PDFs t.  Weights are row-major
(in x out), so a layer is X W + b.  Gradients are the written-out chain rule
and are pinned by central finite differences in the CPU tests.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

IN, HIDDEN, OUT = 5, 256, 1024


def pulse_bin(scene, n_out=OUT):
    """The bin of n_out over the period that holds the pulse centre tau."""
    s = np.asarray(scene).reshape(-1)[0]
    return int(math.floor(float(s["pulse_center_ns"]) / (float(s["period_ns"]) / n_out)))


def features(scene):
    """phi(theta): fixed affine maps onto about [-1, 1] for the warm-start
    workload's ranges: twice the pulse centre's offset from the centre of its
    bin (in bins), sigma, ln S, ln B, x_d."""
    s = np.asarray(scene).reshape(-1)[0]
    t_r = float(s["period_ns"])
    pos = float(s["pulse_center_ns"]) / (t_r / OUT)
    return np.array([
        2.0 * (pos - pulse_bin(s) - 0.5),
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


def _rotation(shift, batch):
    """idx[i, j] = (j - k_i) mod OUT: the network output that bin j takes."""
    k = np.zeros(batch, dtype=np.int64) if shift is None else np.asarray(shift, dtype=np.int64)
    return (np.arange(OUT)[None, :] - k[:, None]) % OUT


def forward(params, X, prior=None, shift=None):
    """Returns (Q, cache).  params: dict W1 (5x256), b1, W2 (256x256), b2,
    W3 (256x1024), b3; X: batch x 5; prior: batch x 1024 logits added
    before the softmax, or None; shift: the batch's pulse bins, or None (no
    rotation)."""
    A1 = X @ params["W1"] + params["b1"]
    H1 = gelu(A1)
    A2 = H1 @ params["W2"] + params["b2"]
    H2 = gelu(A2)
    Z = np.take_along_axis(H2 @ params["W3"] + params["b3"], _rotation(shift, X.shape[0]), axis=1)
    if prior is not None:
        Z = Z + prior
    Zs = Z - Z.max(axis=1, keepdims=True)
    E = np.exp(Zs)
    Q = E / E.sum(axis=1, keepdims=True)
    logQ = Zs - np.log(E.sum(axis=1, keepdims=True))
    return Q, dict(X=X, A1=A1, H1=H1, A2=A2, H2=H2, logQ=logQ, Q=Q)


def loss(params, X, T, prior=None, shift=None):
    """Mean over rows of -sum_j T_j log Q_j."""
    _, c = forward(params, X, prior, shift)
    return float(-(T * c["logQ"]).sum(axis=1).mean())


def grads(params, X, T, prior=None, shift=None):
    """Gradients of the mean cross-entropy with respect to every parameter
    (the prior is a constant: it shifts Q, not the form of dZ; the rotation
    sends each bin's dZ back to the output it took)."""
    _, c = forward(params, X, prior, shift)
    B = X.shape[0]
    dZb = (c["Q"] - T) / B  # softmax + cross-entropy, per bin; rows of T sum to 1
    dZ = np.empty_like(dZb)
    np.put_along_axis(dZ, _rotation(shift, B), dZb, axis=1)
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
