"""Stochastic Chebyshev (KPM) density of states and equal-count shift placement.

The paper (Section 3.1) estimates the DOS phi and the cumulative DOS Phi of the
pencil to place all shifts at once, roots of Phi at evenly spaced counts
(eq. cdos_root), with one shift per interval at its midpoint.  Its estimator is a
Gaussian-broadened Lanczos DOS (eq. dos / cdos); here the estimator is the kernel
polynomial method, a reading recorded with the build's design notes:

* operator H = L_B^{-1} A L_B^{-T} with B = L_B L_B^T (the Cholesky form the
  paper gives for the generalized problem);
* spectral bounds [a, b] from a 30-step Lanczos on H (full reorthogonalisation),
  extreme Ritz values widened by their residual norm plus 1% of (b - a);
* H~ = (H - c) / d with c = (a + b) / 2, d = (b - a) / 2;
* mu_k = (1 / (N n_v)) sum_v v^T T_k(H~) v over n_v Rademacher vectors;
* Jackson damping g_k for M moments;
* Phi(omega) = N [ g_0 mu_0 (1 - theta/pi) - (2/pi) sum_{k>=1} g_k mu_k sin(k theta)/k ],
  theta = arccos t, t = (omega - c)/d  (the integral of the damped Chebyshev series).

Shift placement (reading of eq. cdos_root, whose printed form mixes a spectral
point with a count): the region to slice is [a, omega_top] with
omega_top = root of Phi = n_e + top_margin * n_e / n_s (the lowest n_e plus a
margin, because the estimate is only accurate to the kernel resolution); its
equal-count points omega_j solve Phi(omega) = j K', K' = Phi(omega_top) / n_s,
j = 0..n_s, and sigma_j = (omega_{j-1} + omega_j) / 2 is the midpoint of the
j-th interval (the paper's "midpoint", printed as (u_j - l_j)/2).  The top slice
[sigma_ns, omega_top) is then half an interval wide, like the bottom one.
Roots by bisection.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import prng


def jackson(M):
    """Jackson damping factors g_0..g_{M-1} (g_0 = 1)."""
    k = np.arange(M, dtype=np.float64)
    q = math.pi / (M + 1)
    return ((M - k + 1) * np.cos(q * k) + np.sin(q * k) / math.tan(q)) / (M + 1)


class Operator:
    """H = L_B^{-1} A L_B^{-T} applied to a block."""

    def __init__(self, A, B):
        self.A = np.asarray(A, dtype=np.float64)
        self.LB = np.linalg.cholesky(np.asarray(B, dtype=np.float64))
        self.n = self.A.shape[0]

    def __call__(self, X):
        y = sla.solve_triangular(self.LB.T, X, lower=False)
        y = self.A @ y
        return sla.solve_triangular(self.LB, y, lower=True)


def lanczos_bounds(op, seed, steps=30):
    """Extreme Ritz values of H after ``steps`` Lanczos steps, widened by the Ritz
    residual norms and 1% of the Ritz range.  Returns (a, b)."""
    n = op.n
    v = prng.gauss(prng.derive(seed, prng.TAG_BOUNDS), 0, n)
    v = v / np.linalg.norm(v)
    m = min(steps, n)
    V = np.zeros((n, m + 1))
    V[:, 0] = v
    alpha = np.zeros(m)
    beta = np.zeros(m)
    for j in range(m):
        w = op(V[:, j:j + 1])[:, 0]
        alpha[j] = V[:, j] @ w
        w = w - V[:, : j + 1] @ (V[:, : j + 1].T @ w)      # full reorthogonalisation
        w = w - V[:, : j + 1] @ (V[:, : j + 1].T @ w)
        beta[j] = np.linalg.norm(w)
        if beta[j] == 0.0:
            m = j + 1
            break
        V[:, j + 1] = w / beta[j]
    T = np.diag(alpha[:m]) + np.diag(beta[: m - 1], 1) + np.diag(beta[: m - 1], -1)
    th, S = np.linalg.eigh(T)
    res = np.abs(beta[m - 1] * S[m - 1, :])
    lo = th[0] - res[0]
    hi = th[-1] + res[-1]
    pad = 0.01 * (th[-1] - th[0])
    return lo - pad, hi + pad


def rademacher_block(seed, n, nv):
    """n x nv Rademacher probe vectors: column c, row i uses stream index c*n + i."""
    s = prng.derive(seed, prng.TAG_KPM)
    return prng.rademacher(s, 0, n * nv).reshape(nv, n).T.copy()


def moments(op, a, b, M, nv, seed):
    """mu_0..mu_{M-1} by the three-term recurrence, one operator application per moment."""
    n = op.n
    c = 0.5 * (a + b)
    d = 0.5 * (b - a)
    V = rademacher_block(seed, n, nv)

    def Ht(X):
        return (op(X) - c * X) / d

    mu = np.zeros(M)
    t_prev = V
    mu[0] = np.sum(V * t_prev) / (n * nv)
    if M > 1:
        t_cur = Ht(V)
        mu[1] = np.sum(V * t_cur) / (n * nv)
        for k in range(2, M):
            t_next = 2.0 * Ht(t_cur) - t_prev
            mu[k] = np.sum(V * t_next) / (n * nv)
            t_prev, t_cur = t_cur, t_next
    return mu


def cdos(omega, mu, g, a, b, n):
    """Closed-form cumulative DOS Phi(omega) (number of eigenvalues below omega)."""
    c = 0.5 * (a + b)
    d = 0.5 * (b - a)
    t = np.clip((np.asarray(omega, dtype=np.float64) - c) / d, -1.0, 1.0)
    th = np.arccos(t)
    M = mu.size
    acc = g[0] * mu[0] * (1.0 - th / math.pi)
    for k in range(1, M):
        acc = acc - (2.0 / math.pi) * g[k] * mu[k] * np.sin(k * th) / k
    return n * acc


def cdos_root(target, mu, g, a, b, n, rtol=1e-12):
    lo, hi = a, b
    while hi - lo > rtol * (b - a):
        mid = 0.5 * (lo + hi)
        if cdos(mid, mu, g, a, b, n) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def place_shifts(mu, a, b, n, n_e, n_s, top_margin=2.0):
    """Equal-count roots and interval midpoints; returns (sigmas, omegas, omega_top)."""
    g = jackson(mu.size)
    K = n_e / n_s
    top_count = n_e + top_margin * K
    top = cdos_root(top_count, mu, g, a, b, n)
    Kp = top_count / n_s
    omegas = [a] + [cdos_root(j * Kp, mu, g, a, b, n) for j in range(1, n_s + 1)]
    sig = np.array([0.5 * (omegas[j - 1] + omegas[j]) for j in range(1, n_s + 1)])
    return sig, np.array(omegas), top


def plan(A, B, n_e, n_s, M=64, nv=20, seed=0, top_margin=2.0):
    """Full KPM planner: bounds, moments, roots, midpoints."""
    op = Operator(A, B)
    a, b = lanczos_bounds(op, seed)
    mu = moments(op, a, b, M, nv, seed)
    sig, omegas, top = place_shifts(mu, a, b, op.n, n_e, n_s, top_margin)
    return dict(a=a, b=b, mu=mu, sigmas=sig, omegas=omegas, omega_top=top)
