"""Float64 CPU oracle: transition matrix and stationary distribution.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function follows
the paper step by step, in its notation, with no blocking, fusion or
factorisation:

1. photon flux lambda(t) on one period, Eq. (arrival_flux);
2. cumulative flux F(t), defined in Theorem 1;
3. bin centres s_j and the shift l = ceil(x_d / Delta) of Theorem 2;
4. E_base = exp(-Lambda*L - D) and E = J_l E_base (Section 3.4);
5. P = (1 lambda^T) (.) E, then row normalisation (Section 3.4);
6. the leading left eigenvector of the normalised matrix (Section 2.3,
   "Markov chain pipeline").

Readings where the paper is silent (each is also listed in the design notes):

* Lambda in the wrap term is the one-period integral F(t_r).  The paper
  writes Lambda = S + B (Section 2.1); the two differ only by the pulse mass
  that falls outside [0, t_r), because lambda is defined on one period only.
* The pulse is the unit-area normal pdf truncated to [0, t_r) and replicated
  periodically (not wrapped).
* Bins are 0-based with centres s_j = (j + 1/2) Delta.
* x_d = t_d mod t_r; l = ceil(x_d / Delta) evaluated as q = x_d * N / t_r with
  integer snapping: if |q - round(q)| <= 1e-9 * max(1, q) then l = round(q),
  else l = ceil(q); finally l mod N.
* Row i of E is row (i + l) mod N of E_base (Theorem 2: the reactivation bin
  of state s_i is s_i shifted forward by l bins), i.e. J_l rolls rows up by l.
* The indicator is strict: no wrap when the reactivation bin equals the
  next-state bin.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ndtr

SHIFT_SNAP_RTOL = 1e-9


def _fields(scene):
    """Unpack one scene record (structured array element or length-1 array)."""
    sc = np.asarray(scene).reshape(-1)[0]
    return (float(sc["period_ns"]), float(sc["dead_time_ns"]), float(sc["pulse_center_ns"]),
            float(sc["pulse_sigma_ns"]), float(sc["signal_flux"]), float(sc["background_flux"]),
            int(sc["n_bins"]))


def flux(t, scene):
    """lambda(t) = S * N(t - tau; 0, sigma^2) + B / t_r on [0, t_r).

    Eq. (arrival_flux) with s(t) = calE * N(t; 0, sigma_t^2), S = alpha*calE
    and B = t_r * lambda_b (Section 2.1).  Units: photons per ns.
    """
    t_r, _, tau, sigma, S, B, _ = _fields(scene)
    t = np.asarray(t, dtype=np.float64)
    z = (t - tau) / sigma
    return S * np.exp(-0.5 * z * z) / (sigma * math.sqrt(2.0 * math.pi)) + B / t_r


def cumulative_flux(t, scene):
    """F(t) = integral_0^t lambda (Theorem 1), in closed form:

    F(t) = S [Phi((t - tau)/sigma) - Phi(-tau/sigma)] + B t / t_r,
    Phi the standard normal cdf.
    """
    t_r, _, tau, sigma, S, B, _ = _fields(scene)
    t = np.asarray(t, dtype=np.float64)
    return S * (ndtr((t - tau) / sigma) - ndtr(-tau / sigma)) + B * t / t_r


def total_flux(scene):
    """Lambda := F(t_r), the flux integrated over one period (wrap term of
    Theorem 1 and normaliser of Eq. (transition_pdf))."""
    t_r = _fields(scene)[0]
    return float(cumulative_flux(t_r, scene))


def bin_centres(scene):
    """s_j = (j + 1/2) Delta, Delta = t_r / n_b (Section 2.3; the operator D
    of Section 3.1 maps times to these centres)."""
    t_r, *_, n = _fields(scene)
    delta = t_r / n
    return (np.arange(n, dtype=np.float64) + 0.5) * delta


def relative_dead_time(scene):
    """x_d = t_d mod t_r (Section 3.1)."""
    t_r, t_d, *_ = _fields(scene)
    return math.fmod(t_d, t_r)


def shift_bins(scene):
    """l = ceil(x_d / Delta) mod n_b (Theorem 2), with integer snapping.

    q = x_d * n_b / t_r.  When q is an integer up to a relative 1e-9 (the dead
    time is a whole number of bins, so the shifted centre is itself a centre),
    l = round(q); otherwise l = ceil(q).  A shift of n_b bins is no shift.
    """
    t_r, *_, n = _fields(scene)
    q = relative_dead_time(scene) * n / t_r
    r = round(q)
    if abs(q - r) <= SHIFT_SNAP_RTOL * max(1.0, q):
        l = int(r)
    else:
        l = int(math.ceil(q))
    return l % n


def base_exponent_matrix(scene):
    """E_base = exp(-Lambda * L - D) (Section 3.4).

    L = 1{s 1^T > 1 s^T} is strictly lower triangular (L_ij = 1 iff s_i > s_j)
    and D = 1 F(s)^T - F(s) 1^T, i.e. D_ij = F(s_j) - F(s_i).
    """
    s = bin_centres(scene)
    F = cumulative_flux(s, scene)
    Lam = total_flux(scene)
    L = (s[:, None] > s[None, :]).astype(np.float64)
    D = F[None, :] - F[:, None]
    return np.exp(-Lam * L - D)


def permutation_matrix(scene):
    """J_l: the row permutation with (J_l M)[i, :] = M[(i + l) mod n_b, :]."""
    n = _fields(scene)[6]
    l = shift_bins(scene)
    J = np.zeros((n, n))
    J[np.arange(n), (np.arange(n) + l) % n] = 1.0
    return J


def exponent_matrix(scene):
    """E = J_l E_base (Section 3.4, Theorem 2): Eq. (Eij_ours) for all i, j."""
    return permutation_matrix(scene) @ base_exponent_matrix(scene)


def unnormalized_matrix(scene, shifted=True):
    """P = (1 lambda^T) (.) E with lambda_j = lambda(s_j) (Section 3.4)."""
    lam = flux(bin_centres(scene), scene)
    E = exponent_matrix(scene) if shifted else base_exponent_matrix(scene)
    return lam[None, :] * E


def transition_matrix(scene, shifted=True):
    """The row-stochastic P~: P with each row divided by its sum
    (Section 2.3).  ``shifted=False`` gives the dead-time-free base matrix."""
    P = unnormalized_matrix(scene, shifted)
    return P / P.sum(axis=1, keepdims=True)


def stationary_solve(Pt):
    """pi with pi P~ = pi, sum(pi) = 1, by a dense linear solve.

    The equations (P~^T - I) pi = 0 are rank n-1 for an irreducible chain; the
    last one is replaced by sum(pi) = 1.
    """
    Pt = np.asarray(Pt, dtype=np.float64)
    n = Pt.shape[0]
    A = Pt.T - np.eye(n)
    A[-1, :] = 1.0
    rhs = np.zeros(n)
    rhs[-1] = 1.0
    return np.linalg.solve(A, rhs)


def stationary_eig(Pt):
    """pi as the left eigenvector of P~ whose eigenvalue is closest to 1,
    normalised to sum 1 (Section 2.3: the leading left eigenvector)."""
    w, V = np.linalg.eig(np.asarray(Pt, dtype=np.float64).T)
    k = int(np.argmin(np.abs(w - 1.0)))
    v = np.real(V[:, k])
    return v / v.sum()


def stationary_gth(Pt):
    """pi by Grassmann-Taksar-Heyman state reduction (subtraction-free
    Gaussian elimination for stochastic matrices).  An independent route to
    the same vector, used to pin the dense solve."""
    A = np.array(Pt, dtype=np.float64, copy=True)
    n = A.shape[0]
    for k in range(n - 1, 0, -1):
        s = A[k, :k].sum()
        A[:k, k] /= s
        A[:k, :k] += np.outer(A[:k, k], A[k, :k])
    pi = np.zeros(n)
    pi[0] = 1.0
    for k in range(1, n):
        pi[k] = pi[:k] @ A[:k, k]
    return pi / pi.sum()


def stationary_power(Pt, x0=None, tol_change=1e-12, max_iter=100000):
    """Power iteration x_{t+1} = x_t P~ / sum(x_t P~) from x0 (uniform when
    None) until ||x_{t+1} - x_t||_1 < tol_change.  Returns (x, iterations,
    last change)."""
    Pt = np.asarray(Pt, dtype=np.float64)
    n = Pt.shape[0]
    x = np.full(n, 1.0 / n) if x0 is None else np.asarray(x0, dtype=np.float64) / np.sum(x0)
    change = np.inf
    it = 0
    while it < max_iter:
        y = x @ Pt
        y = y / y.sum()
        change = float(np.abs(y - x).sum())
        x = y
        it += 1
        if change < tol_change:
            break
    return x, it, change


def stationary_pdf(scene, method="solve"):
    """The registration PDF over bins: the stationary vector of P~."""
    Pt = transition_matrix(scene)
    if method == "solve":
        return stationary_solve(Pt)
    if method == "eig":
        return stationary_eig(Pt)
    if method == "gth":
        return stationary_gth(Pt)
    if method == "power":
        return stationary_power(Pt)[0]
    raise ValueError(method)


def bin_tables(scene):
    """(lambda_j, F_j, Lambda, l): the per-bin inputs of the construction."""
    s = bin_centres(scene)
    return flux(s, scene), cumulative_flux(s, scene), total_flux(scene), shift_bins(scene)
