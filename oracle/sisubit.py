"""Shift-invert subspace iteration (Algorithm 2), CholeskyQR, Rayleigh-Ritz, residuals.

Section 2.1: V_0 is B-orthonormalised by CholeskyQR (G = V^T B V = R R^T,
V <- V R^{-T}); C = A - sigma B is factored as L D L^T; then M times
V <- L^{-T} D^{-1} L^{-1} B V followed by CholeskyQR; finally Rayleigh-Ritz:
solve (V^T A V) Q = Q Omega and set V <- V Q.  Residuals R = A X - B X Lambda,
judged column by column (the paper uses the raw 2-norm; the tolerance used here
is the normalised ||A x - lambda B x||_2 / (||A||_2 ||x||_2)).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import bk


def cholesky_qr(V, B):
    """B-orthonormalise V: G = V^T B V = R R^T (R lower), V <- V R^{-T}."""
    G = V.T @ (B @ V)
    G = 0.5 * (G + G.T)
    R = np.linalg.cholesky(G)            # G = R R^T, R lower triangular
    # V R^{-T}: solve R Y^T = V^T
    return sla.solve_triangular(R, V.T, lower=True).T


def rayleigh_ritz(A, B, V):
    """Ritz pairs of (A, B) on span(V), V B-orthonormal: (V^T A V) Q = Q Omega, X = V Q."""
    H = V.T @ (A @ V)
    H = 0.5 * (H + H.T)
    om, Qh = np.linalg.eigh(H)
    return om, V @ Qh


def residual_norms(A, B, X, lam, anorm):
    """||A x_i - lam_i B x_i||_2 / (||A||_2 ||x_i||_2) for each column."""
    R = A @ X - (B @ X) * lam[None, :]
    return np.linalg.norm(R, axis=0) / (anorm * np.linalg.norm(X, axis=0))


def sisubit(A, B, V0, sigma, M, fac=None):
    """Algorithm 2 exactly: returns (lam, X, fac).  ``fac`` may carry a precomputed
    factorization of A - sigma B (its computation is the algorithm's second step)."""
    V = cholesky_qr(np.asarray(V0, dtype=np.float64), B)
    if fac is None:
        fac = bk.bk_ldlt(bk.shifted(A, B, sigma))
    for _ in range(M):
        V = bk.ldlt_solve(fac, B @ V)
        V = cholesky_qr(V, B)
    lam, X = rayleigh_ritz(A, B, V)
    return lam, X, fac


def norm2_sym(A, iters=200, seed=12345):
    """||A||_2 of a symmetric matrix: exact for small n, power iteration otherwise."""
    A = np.asarray(A)
    n = A.shape[0]
    if n <= 1500:
        return float(np.max(np.abs(np.linalg.eigvalsh(A))))
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n)
    x /= np.linalg.norm(x)
    val = 0.0
    for _ in range(iters):
        y = A @ x
        val = float(np.linalg.norm(y))
        x = y / val
    return val
